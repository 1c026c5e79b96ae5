"""GPU parity of the far-field batched path, whose entries K_ij = 1/|x_i - y_j|
are evaluated on the fly from the point sets (the Superfast Multipole setting,
Section "Some Implications and Extensions of Our Study"), against the FP64
oracle run on the oracle's own entries.  Bar as in test_gpu_parity: exact
index sets and a nucleus within 1e-12 where the oracle's decision margins are
at least 1e-6, reconstructions within 1e-6 (the entries are FP64)."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


def block_entries(pts, d):
    xo, yo, m, n = (int(v) for v in d)
    return oracle.fmm_entries(pts[xo:xo + m], pts[yo:yo + n])


def test_points_match_oracle(lra):
    count, r = 24, 16
    pts, desc = workloads.fmm_points(count, shape_seed=5, block_seed0=700)
    print("points batch", count, "blocks, r=16, 3 sweeps", flush=True)
    out = lra.lra_cur_batched_points(torch.from_numpy(pts).cuda(), desc, r, 3, 1000, track_margin=True)
    torch.cuda.synchronize()
    I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()
    infos = out.info()
    for b in range(count):
        K = block_entries(pts, desc[b])
        o = oracle.ca_cur(K, r, 3, 1000 + b)
        assert_parity(K, (I[b], J[b], U[b], infos[b]), o, 1e-6)


def test_points_equal_the_dense_path_on_oracle_entries(lra):
    """The same blocks stored densely in FP64 (entries written by the oracle)
    through the dense batched kernel: identical sets and nucleus bit for bit,
    so every entry the points kernel formed equals the oracle's."""
    count, r = 8, 16
    pts, desc = workloads.fmm_points(count, shape_seed=11, block_seed0=900)
    blocks, parts, off = [], [], 0
    for b in range(count):
        K = block_entries(pts, desc[b])
        m, n = K.shape
        blocks.append((off, m, n, n))
        parts.append(K.ravel())
        off += m * n
    flat = torch.from_numpy(np.concatenate(parts)).cuda()
    print("dense twin of", count, "point blocks", flush=True)
    dense = lra.lra_cur_batched(flat, np.array(blocks, np.int64), r, 3, 1000, track_margin=True)
    pt = lra.lra_cur_batched_points(torch.from_numpy(pts).cuda(), desc, r, 3, 1000, track_margin=True)
    torch.cuda.synchronize()
    assert torch.equal(dense.I, pt.I) and torch.equal(dense.J, pt.J)
    assert torch.equal(dense.U, pt.U)
    assert all(i["status"] == 0 for i in pt.info())


def test_points_4096_blocks_sampled(lra):
    """The benchmark's launch: the 4096 FMM blocks' point sets (64..1024 points
    per side), r = 16, 3 sweeps, one persistent launch; 24 blocks spread over
    the size range checked against the oracle."""
    count, r = 4096, 16
    pts, desc = workloads.fmm_points(count)
    print("points batch 4096 blocks", flush=True)
    out = lra.lra_cur_batched_points(torch.from_numpy(pts).cuda(), desc, r, 3, 1000, track_margin=True)
    torch.cuda.synchronize()
    infos = out.info()
    assert all(i["status"] == 0 for i in infos)
    I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()
    sizes = desc[:, 2] * desc[:, 3]
    order = np.argsort(sizes)
    picks = sorted(set(order[np.linspace(0, count - 1, 24).astype(int)].tolist()))
    for b in picks:
        K = block_entries(pts, desc[b])
        o = oracle.ca_cur(K, r, 3, 1000 + b)
        assert_parity(K, (I[b], J[b], U[b], infos[b]), o, 1e-6)


def test_coinciding_points_flag_only_their_block(lra):
    """A row point equal to a column point makes an infinite entry: that block
    reports LRA_EINVAL with -1 sets, the others are unaffected."""
    pts, desc = workloads.fmm_points(3, shape_seed=5, block_seed0=700)
    pts = pts.copy()
    xo, yo, _, n = (int(v) for v in desc[1])
    j0 = int(oracle.draw_distinct(1001, 0, n, 8)[0])  # a column of block 1's start set
    pts[yo + j0] = pts[xo + 7]
    print("points batch with a coinciding pair in block 1", flush=True)
    out = lra.lra_cur_batched_points(torch.from_numpy(pts).cuda(), desc, 8, 2, 1000, track_margin=True)
    torch.cuda.synchronize()
    infos = out.info()
    assert infos[1]["status"] == lra.LRA_EINVAL
    assert oracle.ca_cur(block_entries(pts, desc[1]), 8, 2, 1001).status == lra.LRA_EINVAL
    assert (out.I[1] == -1).all().item() and (out.J[1] == -1).all().item()
    for b in (0, 2):
        assert infos[b]["status"] == 0
        K = block_entries(pts, desc[b])
        o = oracle.ca_cur(K, 8, 2, 1000 + b)
        assert_parity(K, (out.I[b].cpu().numpy(), out.J[b].cpu().numpy(), out.U[b].cpu().numpy(), infos[b]),
                      o, 1e-6)
