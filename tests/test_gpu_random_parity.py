"""Seeded randomized GPU-vs-oracle parity over every entry point: random
shapes (20 .. 1500), ranks, team sizes, FP64 / FP32 / BF16 inputs, all four
starts of the C-A path (random, abridged SRHT, bidiagonal product, abridged
Fourier), the r-projective-volume generators, the uniform-score CUR and the
cynical CUR.  Each case is drawn up front from a fixed seed, so the list is
the same on every run.

Bars, as in the per-path tests: where the oracle's smallest decision margin
is at least 1e-6 the index sets are equal and the reconstructions agree to
1e-6 (FP64 input) or 1e-4 (FP32 / BF16); below that margin equal sets are
held to the same bar, and differing sets must be dominant (C-A paths) with
an error against the input within the tolerance of the oracle's; the
r-projective runs also make the same number of exchanges; the uniform-score draws are integer work and are
equal always, and its reconstructions agree within the truncated
pseudo-inverse's own condition.  A launch the layout cannot hold (a team of
one with too large a panel) returns LRA_EUNSUPPORTED and the case is
skipped."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import as_f64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PATHS = ["plain", "asrht", "bidiag", "fourier", "projective", "uniform", "cynical"]


def draw_cases(count, seed):
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < count:
        path = PATHS[int(rng.integers(0, len(PATHS)))]
        hi = 1500 if rng.random() < 0.25 else 600
        m, n = int(rng.integers(20, hi)), int(rng.integers(20, hi))
        c = dict(path=path, m=m, n=n, dt=["f64", "f32", "bf16"][int(rng.integers(0, 3))],
                 kind=int(rng.integers(0, 2)), seed=int(rng.integers(0, 1 << 40)),
                 gen=int(rng.integers(0, 1 << 30)))
        if path in ("plain", "asrht", "bidiag", "fourier"):
            r = int(rng.integers(1, min(16, m, n) + 1))
            c.update(r=r, sweeps=int(rng.integers(1, 4)), team=int(rng.choice([0, 1, 2, 3, 5, 8])), kw={})
            if path != "plain":
                d = int(rng.integers(0, 4))
                l = int(rng.integers(max(1, (r + 1) // 2), 40))
                pre = {"asrht": 1, "bidiag": 2, "fourier": 3}[path]
                dim = max(m, n)
                if pre != 3:
                    l = max(l, r)
                if pre == 3 and 2 * l < r:
                    l = r
                if pre == 2:
                    l = min(l, dim)
                if pre in (1, 3) and l > (1 << d) * ((dim + (1 << d) - 1) >> d):
                    continue
                c["kw"] = dict(preprocess=pre, ah_depth=d, ah_samples=l)
        elif path == "projective":
            r = int(rng.integers(1, min(10, m, n) + 1))
            c.update(r=r, k=int(rng.integers(r, min(64, m) + 1)), l=int(rng.integers(r, min(64, n) + 1)),
                     team=int(rng.choice([0, 2, 3, 5])), delta=float(rng.choice([0.0, 0.01])))
        elif path == "uniform":
            r = int(rng.integers(1, 12))
            c.update(r=r, k=int(rng.integers(r, 65)), l=int(rng.integers(r, 65)))
        else:
            r = int(rng.integers(1, min(8, m, n) + 1))
            c.update(r=r, k=int(rng.integers(r, min(40, m, n) + 1)), loops=int(rng.integers(0, 3)))
        cases.append(c)
    return cases


CASES = draw_cases(70, 20261203)


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


def make(c):
    g = np.random.default_rng(c["gen"])
    m, n, r = c["m"], c["n"], c["r"]
    if c["kind"] == 0:
        A = workloads.orthogonal_lowrank(m, n, r, noise=10.0 ** g.uniform(-9, -3),
                                         seeds=tuple(int(v) for v in g.integers(0, 1 << 30, 3)))
    else:
        A = g.standard_normal((m, n))
    if c["dt"] == "f32":
        A = A.astype(np.float32)
    elif c["dt"] == "bf16":
        A = (A.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return np.ascontiguousarray(A)


def to_dev(A):
    if A.dtype == np.uint16:
        return torch.from_numpy(A.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(A).cuda()


def recon(A64, I, J, U):
    return A64[:, J] @ U @ A64[I]


def check_sets(A, I, J, U, info, o, tol, dominant_rows=False, delta=0.01):
    """Where the oracle's decisions are stable (margin >= 1e-6), or the sets
    agree anyway, the sets and reconstructions must match.  Otherwise (a
    near-tie the two sides may break differently) the GPU's own result must
    still be a valid answer: J dominant in A[I, :] after the last row step
    of a converged C-A run, and an error against A that agrees with the
    oracle's to tol * max(err_oracle, 1)."""
    assert info["status"] == o.status, (info, o.status)
    if o.status != 0:
        return
    A64 = as_f64(A)
    same = I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
    if o.min_margin >= 1e-6:
        assert same
    if same:
        Xo, Xg = recon(A64, o.I, o.J, o.U), recon(A64, I, J, U)
        den = np.linalg.norm(Xo)
        assert (np.linalg.norm(Xg - Xo) / den if den > 0 else np.linalg.norm(Xg)) <= tol
        return
    print("low margin %.3e: sets differ, checking validity" % o.min_margin, flush=True)
    if dominant_rows and info["converged"]:
        R = A64[I]
        assert np.abs(np.linalg.solve(R[:, J], R)).max() <= 1.0 + delta + 1e-9
    nA = np.linalg.norm(A64)
    err_o = np.linalg.norm(A64 - recon(A64, o.I, o.J, o.U)) / nA
    err_g = np.linalg.norm(A64 - recon(A64, I, J, U)) / nA
    assert abs(err_g - err_o) <= tol * max(err_o, 1.0), (err_g, err_o)


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_random_case(lra, idx):
    c = CASES[idx]
    print("case", idx, c, flush=True)
    A = make(c)
    tol = 1e-6 if c["dt"] == "f64" else 1e-4
    path = c["path"]
    try:
        if path in ("plain", "asrht", "bidiag", "fourier"):
            o = oracle.ca_cur(A, c["r"], c["sweeps"], c["seed"], **c["kw"])
            out = lra.lra_cur(to_dev(A), c["r"], c["sweeps"], c["seed"], team_size=c["team"], track_margin=True,
                              **c["kw"])
        elif path == "projective":
            o = oracle.projective_cur(A, c["r"], c["k"], c["l"], 2, c["seed"], delta=c["delta"])
            out = lra.lra_cur_projective(to_dev(A), c["r"], c["k"], c["l"], 2, c["seed"], delta=c["delta"],
                                         team_size=c["team"])
        elif path == "uniform":
            o = oracle.uniform_cur(A, c["r"], c["k"], c["l"], c["seed"])
            out = lra.lra_cur_uniform(to_dev(A), c["r"], c["k"], c["l"], c["seed"])
        else:
            o = oracle.cynical(A, c["r"], c["k"], c["loops"], 2, c["seed"])
            out = lra.lra_cur_cynical(to_dev(A), c["r"], c["k"], c["loops"], 2, c["seed"])
        torch.cuda.synchronize()
    except lra.LraError as e:
        if e.status == lra.LRA_EUNSUPPORTED:
            pytest.skip("panel layout does not fit this team size")
        raise
    I, J, U, info = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()
    if path == "uniform":
        assert info["status"] == o.status
        if o.status == 0:
            assert I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
            A64 = as_f64(A)
            s = np.linalg.svd(A64[np.ix_(I, J)], compute_uv=False)
            r = c["r"]
            gap = s[r - 1] if r == len(s) else min(s[r - 1], s[r - 1] - s[r])
            bar = max(1e-6, 1e4 * 2.0 ** -52 * s[0] / max(gap, 1e-300))
            Xo, Xg = recon(A64, o.I, o.J, o.U), recon(A64, I, J, U)
            assert np.linalg.norm(Xg - Xo) / max(np.linalg.norm(Xo), 1e-300) <= bar
        return
    check_sets(A, I, J, U, info, o, tol, dominant_rows=path in ("plain", "asrht", "bidiag", "fourier"))
    if path == "projective" and o.status == 0 and o.min_margin >= 1e-6:
        assert info["swaps_total"] == o.swaps_total
    # lra_cur reports the decisions' smallest margin; with the same decisions
    # (stable, or taken alike) it is the oracle's exactly
    if path in ("plain", "asrht", "bidiag", "fourier") and o.status == 0:
        if I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist() and info["swaps_total"] == o.swaps_total:
            assert info["min_margin"] == o.min_margin, (info["min_margin"], o.min_margin)
    elif path != "uniform":
        assert np.isnan(info["min_margin"])
