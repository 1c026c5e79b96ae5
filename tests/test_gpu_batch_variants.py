"""Batched C-A launch variants against each other and against the oracle.

Every register-panel variant (items per lane x wavefronts per workgroup) and
the LDS-panel kernel run the same arithmetic in the same order, so for every
block they must return identical index sets, nucleus and info; with the
built-in bin table the results also meet the oracle's bar (exact sets and a
nucleus within 1e-12 where the oracle's decision margins are at least 1e-6,
reconstructions within 1e-4 for FP32 entries, 1e-6 for FP64).
"""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import as_f64, assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = [(2, 1), (2, 2), (2, 4), (2, 8)]
# rows and columns spanning every bin, with ragged tails (r = 16 needs >= 16)
SHAPES = [(16, 16), (17, 130), (64, 64), (128, 128), (129, 60), (200, 256), (256, 257), (300, 513),
          (511, 512), (513, 100), (640, 700), (767, 768), (800, 1000), (1000, 999), (40, 1000), (1000, 33)]


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    yield lra
    lra.lra_batch_set_rules([])


def pack(blocks):
    """Flat FP array and (offset, m, n, lda) descriptors of a list of 2-D arrays."""
    parts, desc, off = [], [], 0
    for B in blocks:
        m, n = B.shape
        desc.append((off, m, n, n))
        parts.append(np.ascontiguousarray(B).ravel())
        off += m * n
    return np.concatenate(parts), np.array(desc, dtype=np.int64)


def fmm_blocks(shapes, seed, dtype=np.float32):
    return [workloads.fmm_block(m, n, seed + b, dtype) for b, (m, n) in enumerate(shapes)]


def to_device(flat):
    if flat.dtype == np.uint16:
        return torch.from_numpy(flat.view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(flat).cuda()


def run(lra, base, desc, r, sweeps, seed, rules, **kw):
    lra.lra_batch_set_rules(rules)
    out = lra.lra_cur_batched(base, desc, r, sweeps, seed, track_margin=True, **kw)
    torch.cuda.synchronize()
    return out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()


LDS_ONLY = [(1 << 20, 16, 0, 0)]


def same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2], equal_nan=True)
    assert a[3] == b[3]


def test_every_variant_equals_the_lds_kernel(lra):
    flat, desc = pack(fmm_blocks(SHAPES, 4100))
    base = to_device(flat)
    ref = run(lra, base, desc, 16, 3, 77, LDS_ONLY)
    assert all(i["status"] == 0 for i in ref[3])
    for P, W in VARIANTS:
        print("variant items_per_lane=%d waves=%d" % (P, W), flush=True)
        got = run(lra, base, desc, 16, 3, 77, [(64 * P * W, 16, P, W)])
        same(got, ref)


def test_builtin_table_meets_the_oracle(lra):
    blocks = fmm_blocks(SHAPES, 4200)
    flat, desc = pack(blocks)
    base = to_device(flat)
    I, J, U, infos = run(lra, base, desc, 16, 3, 1000, [])
    for b, B in enumerate(blocks):
        o = oracle.ca_cur(B, 16, 3, 1000 + b)
        assert_parity(B, (I[b], J[b], U[b], infos[b]), o, 1e-4)


@pytest.mark.parametrize("dtype", [np.float64, "bf16"])
def test_dtypes(lra, dtype):
    rng = np.random.default_rng(5)
    shapes = [(int(rng.integers(16, 900)), int(rng.integers(16, 900))) for _ in range(12)]
    blocks = fmm_blocks(shapes, 4300, np.float64 if dtype is np.float64 else np.float32)
    if dtype == "bf16":
        blocks = [(B.view(np.uint32) >> 16).astype(np.uint16) for B in blocks]
    flat, desc = pack(blocks)
    base = to_device(flat)
    ref = run(lra, base, desc, 16, 3, 5, LDS_ONLY)
    got = run(lra, base, desc, 16, 3, 5, [])
    same(got, ref)
    for b in (0, 5, 11):
        o = oracle.ca_cur(blocks[b], 16, 3, 5 + b)
        assert_parity(blocks[b], (got[0][b], got[1][b], got[2][b], got[3][b]), o,
                      1e-6 if dtype is np.float64 else 1e-4)


def test_failures_caps_and_delta(lra):
    good = workloads.fmm_block(300, 200, 4400, np.float32)
    nan = workloads.fmm_block(150, 400, 4401, np.float32)
    nan[77, :] = np.nan  # a whole row: every column panel reads it
    low = np.zeros((500, 260), np.float32)  # five equal non-zero columns: every panel has rank <= 1
    low[:, :5] = 1.0
    big = workloads.fmm_block(700, 600, 4402, np.float32)
    blocks = [good, nan, low, big]
    flat, desc = pack(blocks)
    base = to_device(flat)
    for kw in ({}, {"max_swaps": 1}, {"delta": 0.0}):
        ref = run(lra, base, desc, 16, 3, 9, LDS_ONLY, **kw)
        got = run(lra, base, desc, 16, 3, 9, [], **kw)
        print("options", kw, [i["status"] for i in got[3]], [i["converged"] for i in got[3]], flush=True)
        same(got, ref)
        assert [i["status"] for i in got[3]] == [0, 1, 2, 0]
        for b in (0, 2, 3):
            o = oracle.ca_cur(blocks[b], 16, 3, 9 + b, **kw)
            assert_parity(blocks[b], (got[0][b], got[1][b], got[2][b], got[3][b]), o, 1e-4)


def test_points_variants_equal_the_lds_kernel(lra):
    pts, desc = workloads.fmm_points(20, shape_seed=31, block_seed0=4500)
    dpts = torch.from_numpy(pts).cuda()
    outs = []
    for rules in (LDS_ONLY, []):
        lra.lra_batch_set_rules(rules)
        out = lra.lra_cur_batched_points(dpts, desc, 16, 3, 300, track_margin=True)
        torch.cuda.synchronize()
        outs.append((out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()))
    same(outs[1], outs[0])


def test_blocks_at_the_largest_variant(lra):
    """Up to 1024 items: the largest register variant (8 wavefronts x 64 lanes x 2 items)."""
    shapes = [(1024, 1000), (1024, 1024), (1000, 64)]
    blocks = fmm_blocks(shapes, 4600)
    flat, desc = pack(blocks)
    base = to_device(flat)
    I, J, U, infos = run(lra, base, desc, 16, 3, 11, [])
    for b, B in enumerate(blocks):
        o = oracle.ca_cur(B, 16, 3, 11 + b)
        assert_parity(B, (I[b], J[b], U[b], infos[b]), o, 1e-4)


def test_truncated_nucleus(lra):
    """Exactly rank 15 plus rounding-level noise: full-rank panels, a
    numerically singular 16 x 16 generator, the truncated pseudo-inverse."""
    g = np.random.default_rng(7)
    blocks = [g.standard_normal((m, 15)) @ g.standard_normal((15, n)) + 1e-15 * g.standard_normal((m, n))
              for m, n in [(200, 150), (600, 90), (90, 1000)]]
    flat, desc = pack(blocks)
    base = to_device(flat)
    ref = run(lra, base, desc, 16, 2, 21, LDS_ONLY)
    got = run(lra, base, desc, 16, 2, 21, [])
    same(got, ref)
    assert [i["nucleus_rank"] for i in got[3]] == [15, 15, 15]
