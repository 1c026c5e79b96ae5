"""The entry point that allocates nothing (lra_cur_noalloc), called through
the C ABI, against lra_cur on the same inputs: the two run the same kernels
on the same data, so index sets, nucleus and info must be identical.  Two
calls in a row share the per-GPU scratch; the second is smaller, so stale
contents of the first would show."""
import ctypes as ct

import numpy as np
import pytest

import paper_1710_07946_amd as lra
from paper_1710_07946_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _call(name, A, r, sweeps, seed, **kw):
    """One call of `name` through ctypes; returns (status, I, J, U, info)."""
    L = lra.load()
    dev = A.device
    I = torch.full((r,), -7, dtype=torch.int64, device=dev)
    J = torch.full((r,), -7, dtype=torch.int64, device=dev)
    U = torch.full((r, r), float("nan"), dtype=torch.float64, device=dev)
    info = torch.zeros(lra.INFO_BYTES, dtype=torch.uint8, device=dev)
    o = lra.lra_default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    m, n = A.shape
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = getattr(L, name)(ct.c_void_p(A.data_ptr()), lra._dtype_code(A), m, n, A.stride(0), r, sweeps,
                          ct.c_uint64(seed), ct.byref(o), ct.c_void_p(I.data_ptr()), ct.c_void_p(J.data_ptr()),
                          ct.c_void_p(U.data_ptr()), ct.c_void_p(info.data_ptr()), stream)
    torch.cuda.synchronize()
    return st, I.cpu().numpy(), J.cpu().numpy(), U.cpu().numpy(), lra.parse_info(info)[0]


def _same(A, r, sweeps, seed, **kw):
    kw.setdefault("track_margin", 1)   # every info field, the team's margin word included
    print("noalloc case: %s %s r=%d sweeps=%d seed=%d %s" % (tuple(A.shape), A.dtype, r, sweeps, seed, kw), flush=True)
    ref = _call("lra_cur", A, r, sweeps, seed, **kw)
    got = _call("lra_cur_noalloc", A, r, sweeps, seed, **kw)
    assert ref[0] == lra.LRA_OK and got[0] == lra.LRA_OK, (ref[0], got[0])
    assert ref[4]["status"] == lra.LRA_OK, ref[4]
    assert got[1].tolist() == ref[1].tolist()
    assert got[2].tolist() == ref[2].tolist()
    assert np.array_equal(got[3], ref[3])
    assert got[4] == ref[4]
    return got


def _lowrank(m, n, r, seed, dtype):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 1e-6 * g.standard_normal((m, n))
    return torch.from_numpy(A).to(dtype).cuda()


def test_two_calls_second_smaller():
    A1 = torch.from_numpy(workloads.orthogonal_lowrank()).cuda()  # 512 x 512 FP64, four workgroups
    _same(A1, 10, 3, 2001)
    A2 = _lowrank(300, 700, 8, 11, torch.float32)  # smaller; post-multiplied sketch start
    _same(A2, 8, 2, 77, preprocess=lra.LRA_PRE_ASRHT, ah_depth=2, ah_samples=20)


def test_global_sketch_panel_and_bidiagonal_table():
    # l = 256 sampled columns do not fit on chip: the sketch panel lives in the scratch
    A = _lowrank(3000, 3000, 16, 12, torch.float32)
    _same(A, 16, 2, 5, preprocess=lra.LRA_PRE_ASRHT, ah_depth=3, ah_samples=256)
    # then a smaller call whose bidiagonal column table lives in the scratch
    B = _lowrank(400, 400, 8, 13, torch.float64)
    _same(B, 8, 2, 9, preprocess=lra.LRA_PRE_BIDIAG, ah_depth=3, ah_samples=24)
    # and a one-workgroup launch (no exchange words)
    C = _lowrank(100, 90, 4, 14, torch.float64)
    _same(C, 4, 3, 3)


def test_rejections_launch_nothing():
    A = _lowrank(64, 64, 4, 15, torch.float64)
    start = (ct.c_int64 * 4)(0, 1, 2, 3)
    st = _call("lra_cur_noalloc", A, 4, 2, 1, init_cols=ct.cast(start, ct.POINTER(ct.c_int64)))[0]
    assert st == lra.LRA_EINVAL
    # 8000 x 8000 with l = 256: 50 workgroups x 161 x 256 doubles of sketch panel, above the 8 MiB scratch
    big = torch.zeros((8000, 8000), dtype=torch.float32, device="cuda")
    st, I, _, _, _ = _call("lra_cur_noalloc", big, 16, 1, 1, preprocess=lra.LRA_PRE_ASRHT, ah_depth=3,
                           ah_samples=256)
    assert st == lra.LRA_EUNSUPPORTED
    assert I.tolist() == [-7] * 16  # nothing was launched
