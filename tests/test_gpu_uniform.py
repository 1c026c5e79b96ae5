"""GPU parity of the CUR with uniform leverage scores (Algorithm algcurlevsc
with p_j = 1/n, pbar_i = 1/m; canonical nucleus of Algorithm algcnnncl)
against the oracle on the same seeded inputs.

Bar: the draws are integer work, so I and J equal the oracle's exactly.
The two one-sided Jacobi runs sum in different orders, so the nucleus agrees
to the rounding level amplified by the truncated pseudo-inverse's own
condition: |U_g - U_o| / |U_o| <= 1000 eps sigma_1 / d, d the smaller of
sigma_r and the gaps on either side of it (a singular vector moves by about
eps sigma_1 / gap, and 1 / sigma_r by eps sigma_1 / sigma_r), and no looser
than 1e-9 when that figure is smaller; the reconstructions W[:, J] U W[I, :]
agree to 1e-6; the kept rank exactly; log v_{2,r}(M), a sum of r logs each
moved by about eps sigma_1 / sigma_j, to r 1000 eps sigma_1 / sigma_r (at
least 1e-9)."""
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


def check(g, o, A, r):
    I, J, U, info = g
    assert info["status"] == o.status, (info, o.status)
    if o.status != 0:
        assert (I == -1).all() and (J == -1).all() and np.isnan(U).all()
        return
    assert I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
    A64 = as_f64(A)
    s = np.linalg.svd(A64[np.ix_(I, J)], compute_uv=False)
    d = s[r - 1]
    if r > 1:
        d = min(d, s[r - 2] - s[r - 1])
    if r < len(s):
        d = min(d, s[r - 1] - s[r])
    tol = max(1e-9, 1000 * 2.0 ** -52 * s[0] / d)
    err = np.abs(U - o.U).max() / np.abs(o.U).max()
    Xg = A64[:, J] @ U @ A64[I]
    Xo = A64[:, o.J] @ o.U @ A64[o.I]
    perr = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print("nucleus rel diff %.3e (bar %.3e)  recon diff %.3e" % (err, tol, perr), flush=True)
    assert err <= tol
    assert perr <= 1e-6
    assert info["nucleus_rank"] == o.nucleus_rank
    assert info["det_log_abs"] == pytest.approx(o.det_log_abs, abs=max(1e-9, r * 1000 * 2.0 ** -52 * s[0] / s[r - 1]))


def test_single_512_fp64(lra):
    A = workloads.orthogonal_lowrank()
    print("uniform 512x512 r=10 k=l=40", flush=True)
    out = lra.lra_cur_uniform(torch.from_numpy(A).cuda(), 10, 40, 40, 2001)
    torch.cuda.synchronize()
    g = (out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info())
    check(g, oracle.uniform_cur(A, 10, 40, 40, 2001), A, 10)


@pytest.mark.parametrize("r,k,l", [(16, 64, 64), (16, 32, 48), (5, 64, 9), (1, 1, 1), (3, 12, 7)])
def test_batched_fmm_blocks(lra, r, k, l):
    count = 20
    flat, desc = workloads.fmm_batch(count, shape_seed=5, block_seed0=700)
    print("uniform batched fmm", count, "r=%d k=%d l=%d" % (r, k, l), flush=True)
    out = lra.lra_cur_uniform_batched(torch.from_numpy(flat).cuda(), desc, r, k, l, 1000)
    torch.cuda.synchronize()
    I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()
    infos = out.info()
    for b in range(count):
        o0, m, n, ld = desc[b]
        blk = flat[o0:o0 + m * n].reshape(m, n)
        check((I[b], J[b], U[b], infos[b]), oracle.uniform_cur(blk, r, k, l, 1000 + b), blk, r)


def test_repeated_draws_and_bf16(lra):
    # k > m and l > n: draws repeat; BF16 entries upcast exactly
    A32 = workloads.orthogonal_lowrank(9, 7, 3, noise=1e-3, seeds=(1, 2, 3)).astype(np.float32)
    A = (A32.view(np.uint32) >> 16).astype(np.uint16)
    dev = torch.from_numpy(A.view(np.int16)).view(torch.bfloat16).cuda()
    print("uniform bf16 9x7 k=20 l=16", flush=True)
    out = lra.lra_cur_uniform(dev, 3, 20, 16, 4)
    torch.cuda.synchronize()
    g = (out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info())
    assert len(set(g[0].tolist())) < 20
    check(g, oracle.uniform_cur(A, 3, 20, 16, 4), A, 3)


def test_non_finite_generator_entry_fails_only_its_block(lra):
    flat, desc = workloads.fmm_batch(3, shape_seed=5, block_seed0=700)
    o = oracle.uniform_cur(flat[desc[1, 0]:desc[1, 0] + desc[1, 1] * desc[1, 2]].reshape(desc[1, 1], desc[1, 2]),
                           4, 8, 8, 51)
    i0, j0 = o.I[2], o.J[5]
    flat = flat.copy()
    flat[desc[1, 0] + i0 * desc[1, 3] + j0] = np.nan
    print("uniform non-finite entry in block 1", flush=True)
    out = lra.lra_cur_uniform_batched(torch.from_numpy(flat).cuda(), desc, 4, 8, 8, 50)
    torch.cuda.synchronize()
    infos = out.info()
    assert [i["status"] for i in infos] == [0, oracle.EINVAL, 0]
    assert (out.I[1].cpu().numpy() == -1).all() and torch.isnan(out.U[1]).all()


def test_4096_fmm_blocks_sampled(lra):
    """The benchmark's launch: 4096 device-evaluated FMM blocks, r = 16,
    k = l = 64; 24 blocks over the size range checked against the oracle."""
    count = 4096
    base, desc = workloads.fmm_batch_device(count, "cuda")
    print("uniform batched 4096 fmm r=16 k=l=64", flush=True)
    out = lra.lra_cur_uniform_batched(base, desc, 16, 64, 64, 1000)
    torch.cuda.synchronize()
    infos = out.info()
    assert all(i["status"] == 0 for i in infos)
    I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()
    order = np.argsort(desc[:, 1] * desc[:, 2])
    picks = sorted(set(order[np.linspace(0, count - 1, 24).astype(int)].tolist()))
    flat = base.cpu().numpy()
    for b in picks:
        o0, m, n, _ = (int(v) for v in desc[b])
        blk = flat[o0:o0 + m * n].reshape(m, n)
        check((I[b], J[b], U[b], infos[b]), oracle.uniform_cur(blk, 16, 64, 64, 1000 + b), blk, 16)
