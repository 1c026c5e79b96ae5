"""GPU parity of the refinement of a CUR LRA by its leverage scores (section
on refining an LRA with leverage scores; Algorithm algcurlevsc; canonical
nucleus) against the oracle, both given the same crude sets I0, J0.

Bar: the scores, their running sums and the draws are formed in the
oracle's order of operations, so I and J equal the oracle's exactly; the
nucleus agrees to 1000 eps sigma_1 / d (d the smaller of sigma_r and the gaps
beside it; at least 1e-9) and the reconstructions to 1e-6, as for the
uniform-score CUR; the kept rank exactly."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import as_f64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


def to_dev(A):
    if A.dtype == np.uint16:
        return torch.from_numpy(A.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(A).cuda()


def run(lra, A, I0, J0, k, l, seed, Ad=None):
    print("leverage", A.shape, A.dtype, "r=%d k=%d l=%d seed=%d" % (len(I0), k, l, seed), flush=True)
    Ad = to_dev(A) if Ad is None else Ad
    out = lra.lra_cur_leverage(Ad, torch.tensor(np.asarray(I0), dtype=torch.int64, device="cuda"),
                               torch.tensor(np.asarray(J0), dtype=torch.int64, device="cuda"), k, l, seed)
    torch.cuda.synchronize()
    return out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()


def check(A, g, o, r, rows=None):
    I, J, U, info = g
    assert info["status"] == o.status, (info, o.status)
    if o.status != 0:
        assert (I == -1).all() and (J == -1).all() and np.isnan(U).all()
        return
    assert I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
    A64 = as_f64(A) if rows is None else None
    G = (A64[np.ix_(I, J)] if A64 is not None else A[np.ix_(I, J)].astype(np.float64))
    s = np.linalg.svd(G, compute_uv=False)
    d = s[r - 1]
    if r > 1:
        d = min(d, s[r - 2] - s[r - 1])
    if r < len(s):
        d = min(d, s[r - 1] - s[r])
    tol = max(1e-9, 1000 * 2.0 ** -52 * s[0] / d)
    err = np.abs(U - o.U).max() / np.abs(o.U).max()
    if rows is None:
        Xg, Xo = A64[:, J] @ U @ A64[I], A64[:, o.J] @ o.U @ A64[o.I]
    else:
        Xg = A[np.ix_(rows, J)].astype(np.float64) @ U @ A[I].astype(np.float64)
        Xo = A[np.ix_(rows, o.J)].astype(np.float64) @ o.U @ A[o.I].astype(np.float64)
    perr = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print("nucleus rel diff %.3e (bar %.3e)  recon diff %.3e" % (err, tol, perr), flush=True)
    assert err <= tol and perr <= 1e-6
    assert info["nucleus_rank"] == o.nucleus_rank


def test_512_fp64_from_a_one_sweep_ca(lra):
    A = workloads.orthogonal_lowrank()
    base = oracle.ca_cur(A, 10, 1, 2001)
    o = oracle.leverage_cur(A, base.I, base.J, 24, 20, 5)
    check(A, run(lra, A, base.I, base.J, 24, 20, 5), o, 10)


@pytest.mark.parametrize("r,k,l", [(1, 1, 1), (3, 12, 7), (16, 64, 64), (8, 9, 40)])
def test_shapes_fp32(lra, r, k, l):
    A = workloads.factor_gaussian(900, 700, 8, 1e-5, seeds=(7, 8, 9)).astype(np.float32)
    base = oracle.ca_cur(A, r, 1, 31)
    o = oracle.leverage_cur(A, base.I, base.J, k, l, 13)
    check(A, run(lra, A, base.I, base.J, k, l, 13), o, r)


@pytest.mark.parametrize("k,l", [(65, 130), (128, 128), (200, 96), (256, 256), (256, 20)])
def test_samples_beyond_64(lra, k, l):
    # more than 64 draws on a side: the nucleus's rotations run in the
    # global workspace with 8 or 16 rows per lane
    A = workloads.factor_gaussian(900, 700, 16, 1e-5, seeds=(17, 18, 19)).astype(np.float32)
    base = oracle.ca_cur(A, 16, 1, 41)
    o = oracle.leverage_cur(A, base.I, base.J, k, l, 23)
    check(A, run(lra, A, base.I, base.J, k, l, 23), o, 16)


def test_bf16_with_repeated_draws(lra):
    A32 = workloads.orthogonal_lowrank(30, 25, 3, noise=1e-3, seeds=(1, 2, 3)).astype(np.float32)
    A = (A32.view(np.uint32) >> 16).astype(np.uint16)
    base = oracle.ca_cur(A, 3, 2, 4)
    o = oracle.leverage_cur(A, base.I, base.J, 40, 33, 6)
    g = run(lra, A, base.I, base.J, 40, 33, 6)
    assert len(set(g[0].tolist())) < 40
    check(A, g, o, 3)


def test_zero_row_is_singular_and_nan_is_invalid(lra):
    A = workloads.orthogonal_lowrank(120, 100, 4, noise=1e-6, seeds=(1, 2, 3))
    A[17, :] = 0.0
    o = oracle.leverage_cur(A, [3, 17, 40, 90], [1, 2, 3, 4], 8, 8, 1)
    assert o.status == oracle.ESINGULAR
    check(A, run(lra, A, [3, 17, 40, 90], [1, 2, 3, 4], 8, 8, 1), o, 4)
    A[17, :] = 1.0
    A[40, 55] = np.nan
    o = oracle.leverage_cur(A, [3, 17, 40, 90], [1, 2, 3, 4], 8, 8, 1)
    assert o.status == oracle.EINVAL
    check(A, run(lra, A, [3, 17, 40, 90], [1, 2, 3, 4], 8, 8, 1), o, 4)


def test_out_of_range_sets_are_rejected_on_the_host(lra):
    A = torch.zeros((50, 40), dtype=torch.float64, device="cuda")
    bad = torch.tensor([0, 50], dtype=torch.int64, device="cuda")
    good = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    with pytest.raises(lra.LraError):
        lra.lra_cur_leverage(A, bad, good, 4, 4, 0)
    with pytest.raises(lra.LraError):
        lra.lra_cur_leverage(A, good, torch.tensor([0, 40], dtype=torch.int64, device="cuda"), 4, 4, 0)


def test_headline_size_sampled(lra):
    # the benchmark's refinement: the 20000 x 20000 headline matrix, crude
    # sets from its C-A CUR, k = l = 200 (4 r); reconstruction parity on 2000
    # rows
    m = n = 20000
    Ad = workloads.factor_gaussian_device(m, n, 50, 1e-6, 1011, "cuda")
    base = lra.lra_cur(Ad, 50, 4, 2011, preprocess=lra.LRA_PRE_ASRHT, ah_depth=3, ah_samples=100)
    I0, J0 = base.I.cpu().numpy(), base.J.cpu().numpy()
    out = lra.lra_cur_leverage(Ad, base.I, base.J, 200, 200, 7)
    torch.cuda.synchronize()
    g = (out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info())
    A = Ad.cpu().numpy()
    del Ad
    torch.cuda.empty_cache()
    o = oracle.leverage_cur(A, I0, J0, 200, 200, 7)
    rows = np.sort(np.random.default_rng(0).choice(m, 2000, replace=False))
    check(A, g, o, 50, rows=rows)


def draw_cases(count, seed):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        hi = 1500 if rng.random() < 0.3 else 400
        m, n = int(rng.integers(20, hi)), int(rng.integers(20, hi))
        r = int(rng.integers(1, min(64, m, n) + 1))
        cases.append(dict(m=m, n=n, r=r, k=int(rng.integers(r, 65)), l=int(rng.integers(r, 65)),
                          dt=["f64", "f32", "bf16"][int(rng.integers(0, 3))], kind=int(rng.integers(0, 2)),
                          seed=int(rng.integers(0, 1 << 40)), gen=int(rng.integers(0, 1 << 30))))
    # the largest rank and sample sizes on a ragged shape
    cases.append(dict(m=1037, n=771, r=64, k=64, l=64, dt="f32", kind=1, seed=99, gen=5))
    return cases


CASES = draw_cases(24, 20261204)


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_random_case(lra, idx):
    # random shapes (ragged against the 64-item chunks), ranks up to 64 (Gram
    # matrices over several wavefronts), FP64 / FP32 / BF16; crude sets drawn
    # uniformly without repetition
    c = CASES[idx]
    g = np.random.default_rng(c["gen"])
    m, n, r = c["m"], c["n"], c["r"]
    if c["kind"] == 0:
        A = workloads.orthogonal_lowrank(m, n, r, noise=10.0 ** g.uniform(-6, -2),
                                         seeds=tuple(int(v) for v in g.integers(0, 1 << 30, 3)))
    else:
        A = g.standard_normal((m, n))
    if c["dt"] == "f32":
        A = A.astype(np.float32)
    elif c["dt"] == "bf16":
        A = (A.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    A = np.ascontiguousarray(A)
    I0 = np.sort(g.choice(m, r, replace=False))
    J0 = np.sort(g.choice(n, r, replace=False))
    print("case", idx, c, flush=True)
    o = oracle.leverage_cur(A, I0, J0, c["k"], c["l"], c["seed"])
    check(A, run(lra, A, I0, J0, c["k"], c["l"], c["seed"]), o, r)


@pytest.mark.parametrize("m,n,k,l", [(1, 1, 1, 1), (1, 300, 3, 5), (257, 1, 6, 2), (64, 64, 64, 64)])
def test_degenerate_shapes(lra, m, n, k, l):
    # a single row or column (every draw on the same item, the generator of
    # rank one), a 1 x 1 matrix, and k = l = m = n = 64 with r = 1
    g = np.random.default_rng(m * 1000 + n)
    A = np.ascontiguousarray(g.standard_normal((m, 1)) @ g.standard_normal((1, n)) + 0.5)
    I0, J0 = [m // 2], [n // 3]
    o = oracle.leverage_cur(A, I0, J0, k, l, 3)
    assert o.status == 0
    check(A, run(lra, A, I0, J0, k, l, 3), o, 1)
