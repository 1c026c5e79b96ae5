"""GPU parity of C-A with DMM08 leverage-score sampling of every sketch
(Section "Testing C-A acceleration of the algorithms of DMM08", Tables 7
and 8) against the oracle on the same seeded inputs.

Bar.  The kernel takes the rank-r scores of each sketch from its Gram
matrix, the oracle from a one-sided Jacobi SVD of the sketch itself: the
scores agree to about eps sigma_1^2 / (sigma_r^2 gap), far inside the
oracle's reported sampling margin (the smallest relative distance of a draw
from the boundary of the item it picked).  So where that margin exceeds
1e-9 every draw is the same: I and J equal the oracle's exactly and the
kept nucleus rank too; the rescalings differ at rounding level, so the
reconstructions W[:, J] U W[I, :] agree to 1e-9 relative.  Where the
margin is smaller, the sets are checked for validity and the error against
W for being within 1e-4 (FP32 entries) of max(err_oracle, 1e-3)."""
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


def to_device(flat):
    if flat.dtype == np.uint16:
        return torch.from_numpy(flat.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(np.ascontiguousarray(flat)).cuda()


def pack(blocks):
    parts, desc, off = [], [], 0
    for B in blocks:
        m, n = B.shape
        desc.append((off, m, n, n))
        parts.append(np.ascontiguousarray(B).ravel())
        off += m * n
    return np.concatenate(parts), np.array(desc, dtype=np.int64)


def check(g, o, A):
    I, J, U, info = g
    assert info["status"] == o.status, (info, o.status)
    if o.status != 0:
        assert (I == -1).all() and (J == -1).all() and np.isnan(U).all()
        return
    assert info["sweeps_run"] == o.sweeps_run
    A64 = as_f64(A)
    Xg = A64[:, J] @ U @ A64[I]
    if o.min_margin > 1e-9:
        assert I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
        assert info["nucleus_rank"] == o.nucleus_rank
        # the sampling margin: the same draws, running sums equal to rounding
        assert abs(info["min_margin"] - o.min_margin) <= 1e-12, (info["min_margin"], o.min_margin)
        Xo = A64[:, o.J] @ o.U @ A64[o.I]
        d = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
        print("  sets equal, recon diff %.2e (margin %.1e)" % (d, o.min_margin), flush=True)
        assert d <= 1e-9
    else:
        m, n = A.shape
        assert np.all(np.diff(I) >= 0) and np.all(np.diff(J) >= 0)
        assert 0 <= I.min() and I.max() < m and 0 <= J.min() and J.max() < n
        eg = np.linalg.norm(A64 - Xg) / np.linalg.norm(A64)
        eo = oracle.rel_fro(A, o.I, o.J, o.U)
        print("  low margin %.1e: err gpu %.3e oracle %.3e" % (o.min_margin, eg, eo), flush=True)
        assert eg <= eo + 1e-4 * max(eo, 1e-3)


@pytest.mark.parametrize("r,k,l,iters", [(4, 8, 12, 3), (8, 32, 32, 8), (16, 64, 64, 8), (5, 5, 5, 2), (1, 3, 2, 4)])
def test_blocks_of_several_shapes(lra, r, k, l, iters):
    # items below, at and above the 64-row staging chunk and the 512-item scan
    # chunk, with ragged tails; rows and columns both the longer side
    shapes = [(64, 64), (130, 200), (600, 257), (300, 1000), (1000, 513)]
    blocks = [workloads.graded_lowrank(m, n, r, 1e-6, 900 + b) for b, (m, n) in enumerate(shapes)]
    flat, desc = pack(blocks)
    print("dmm r=%d k=%d l=%d iters=%d" % (r, k, l, iters), flush=True)
    out = lra.lra_cur_dmm_batched(to_device(flat), desc, r, k, l, iters, 77)
    torch.cuda.synchronize()
    I, J, U, infos = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()
    for b, B in enumerate(blocks):
        check((I[b], J[b], U[b], infos[b]), oracle.dmm_ca(B, r, k, l, iters, 77 + b), B)


@pytest.mark.parametrize("dtype", [np.float64, "bf16"])
def test_dtypes(lra, dtype):
    B = workloads.graded_lowrank(400, 350, 6, 1e-5, 17, np.float64 if dtype is np.float64 else np.float32)
    if dtype == "bf16":
        B = (B.view(np.uint32) >> 16).astype(np.uint16)
    flat, desc = pack([B])
    print("dmm dtype", dtype, flush=True)
    out = lra.lra_cur_dmm_batched(to_device(flat), desc, 6, 24, 24, 8, 5)
    torch.cuda.synchronize()
    check((out.I[0].cpu().numpy(), out.J[0].cpu().numpy(), out.U[0].cpu().numpy(), out.info()),
          oracle.dmm_ca(B, 6, 24, 24, 8, 5), B)


def test_more_blocks_than_workgroups(lra):
    # 300 blocks over a grid of at most 256 workgroups: some take two blocks
    count = 300
    blocks = [workloads.graded_lowrank(70 + b % 5, 90 + b % 7, 3, 1e-6, 5000 + b) for b in range(count)]
    flat, desc = pack(blocks)
    print("dmm 300 small blocks", flush=True)
    out = lra.lra_cur_dmm_batched(to_device(flat), desc, 3, 9, 9, 4, 1)
    torch.cuda.synchronize()
    I, J, U, infos = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()
    assert all(i["status"] == 0 for i in infos)
    for b in list(range(0, count, 23)) + [count - 1]:
        check((I[b], J[b], U[b], infos[b]), oracle.dmm_ca(blocks[b], 3, 9, 9, 4, 1 + b), blocks[b])


def test_failures_stay_in_their_block(lra):
    good = workloads.graded_lowrank(100, 120, 4, 1e-6, 1)
    nan = workloads.graded_lowrank(100, 120, 4, 1e-6, 2)
    nan[:, 37] = np.nan            # a whole column: the first row sketch or a later one reads it
    zero = np.zeros((90, 80), np.float32)
    blocks = [good, nan, zero, good]
    flat, desc = pack(blocks)
    print("dmm failures", flush=True)
    out = lra.lra_cur_dmm_batched(to_device(flat), desc, 4, 8, 8, 3, 40)
    torch.cuda.synchronize()
    infos = out.info()
    assert [i["status"] for i in infos] == [0, oracle.EINVAL, oracle.ESINGULAR, 0]
    for b, B in enumerate(blocks):
        check((out.I[b].cpu().numpy(), out.J[b].cpu().numpy(), out.U[b].cpu().numpy(), infos[b]),
              oracle.dmm_ca(B, 4, 8, 8, 3, 40 + b), B)


def test_argument_checks(lra):
    base = torch.zeros(100 * 100, dtype=torch.float32, device="cuda")
    desc = [[0, 100, 100, 100]]
    for args in ((4, 3, 8, 2), (4, 8, 65, 2), (4, 8, 8, 0), (0, 8, 8, 2)):
        with pytest.raises(lra.LraError):
            lra.lra_cur_dmm_batched(base, desc, *args, 1)
    with pytest.raises(lra.LraError):   # r above a block's side
        lra.lra_cur_dmm_batched(base, [[0, 3, 100, 100]], 4, 8, 8, 2, 1)


def test_benchmark_launch_sampled(lra):
    """The benchmark's launch: 256 blocks 1000 x 1000 FP32 of numerical rank
    16, r = 16, k = l = 64, 8 iterations; three blocks against the oracle."""
    count, m, n = 256, 1000, 1000
    base, desc = workloads.graded_lowrank_batch_device(count, m, n, 16, 1e-6, 8000, "cuda")
    print("dmm 256 x 1000 x 1000 r=16 k=l=64 8 iterations", flush=True)
    out = lra.lra_cur_dmm_batched(base, desc, 16, 64, 64, 8, 3000)
    torch.cuda.synchronize()
    infos = out.info()
    assert all(i["status"] == 0 for i in infos)
    for b in (0, 101, 255):
        blk = base[b * m * n:(b + 1) * m * n].cpu().numpy().reshape(m, n)
        check((out.I[b].cpu().numpy(), out.J[b].cpu().numpy(), out.U[b].cpu().numpy(), infos[b]),
              oracle.dmm_ca(blk, 16, 64, 64, 8, 3000 + b), blk)
