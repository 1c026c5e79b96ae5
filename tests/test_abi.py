"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments on the host before touching a device."""
import ctypes as ct
import os
import subprocess

import pytest

import paper_1710_07946_amd as lra


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lra.library_path()):
        pytest.skip("library not built")
    return lra.load()


def test_exports_every_declared_symbol(lib):
    names = lra.declared_functions()
    assert {"lra_cur", "lra_cur_batched", "lra_default_opts", "lra_release", "lra_strerror"} <= set(names)
    out = subprocess.check_output(["nm", "-D", "--defined-only", lra.library_path()], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_default_opts(lib):
    o = lra.lra_default_opts()
    assert o.delta == 0.01 and o.max_swaps == -1 and o.preprocess == 0 and o.ah_depth == 3
    assert o.ah_samples == 0 and o.refine_steps == 0 and o.team_size == 0 and not o.init_cols


def test_strerror(lib):
    for s in range(6):
        assert lra.lra_strerror(s)
    assert "rank" in lra.lra_strerror(lra.LRA_ESINGULAR)


def test_struct_layouts():
    assert ct.sizeof(lra.lra_info) == 48
    assert ct.sizeof(lra.lra_block) == 32
    assert ct.sizeof(lra.lra_pts_block) == 32
    assert ct.sizeof(lra.lra_opts) == 48
    assert lra.lra_opts.track_margin.offset == 32 and lra.lra_opts.init_cols.offset == 40
    assert lra.lra_info.min_margin.offset == 40
    assert lra.lra_default_opts().track_margin == 0      # margins are opt-in


def _call(lib, m=100, n=80, lda=80, r=5, sweeps=2, dt=1, opts=None, ptr=0x1000):
    fake = ct.c_void_p(ptr)
    return lib.lra_cur(fake, dt, m, n, lda, r, sweeps, 1, opts, fake, fake, fake, None, None)


def test_invalid_arguments_rejected_on_host(lib):
    E = lra.LRA_EINVAL
    assert _call(lib, r=0) == E
    assert _call(lib, r=81) == E           # r > min(m, n)
    assert _call(lib, r=65, m=200, n=200, lda=200) == E  # r > 64
    assert _call(lib, sweeps=0) == E
    assert _call(lib, lda=79) == E
    assert _call(lib, dt=7) == E
    assert _call(lib, ptr=0) == E          # null pointers
    o = lra.lra_default_opts()
    o.delta = -1.0
    assert _call(lib, opts=ct.byref(o)) == E
    o = lra.lra_default_opts()
    o.preprocess = 1
    o.ah_samples = 3                       # l < r
    assert _call(lib, opts=ct.byref(o)) == E
    o = lra.lra_default_opts()
    bad = (ct.c_int64 * 5)(0, 1, 2, 2, 4)  # duplicate warm-start column
    o.init_cols = ct.cast(bad, ct.POINTER(ct.c_int64))
    assert _call(lib, opts=ct.byref(o)) == E
    bad2 = (ct.c_int64 * 5)(0, 1, 2, 3, 80)  # out of range
    o.init_cols = ct.cast(bad2, ct.POINTER(ct.c_int64))
    assert _call(lib, opts=ct.byref(o)) == E


def test_batched_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    blocks = (lra.lra_block * 2)(lra.lra_block(0, 10, 10, 10), lra.lra_block(100, 10, 9, 8))  # lda < n
    assert lib.lra_cur_batched(fake, 1, blocks, 2, 3, 1, 0, None, fake, fake, fake, None, None) == lra.LRA_EINVAL
    blocks = (lra.lra_block * 1)(lra.lra_block(0, 2, 10, 10))  # r > m
    assert lib.lra_cur_batched(fake, 1, blocks, 1, 3, 1, 0, None, fake, fake, fake, None, None) == lra.LRA_EINVAL
    o = lra.lra_default_opts()
    o.preprocess = 1
    blocks = (lra.lra_block * 1)(lra.lra_block(0, 20, 20, 20))
    assert lib.lra_cur_batched(fake, 1, blocks, 1, 3, 1, 0, ct.byref(o), fake, fake, fake, None,
                               None) == lra.LRA_EINVAL
    # an empty batch is a no-op
    assert lib.lra_cur_batched(fake, 1, blocks, 0, 3, 1, 0, None, fake, fake, fake, None, None) == lra.LRA_OK


def test_points_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(blocks, npts=100, r=3, count=None, opts=None, pts=fake):
        arr = (lra.lra_pts_block * max(len(blocks), 1))(*blocks)
        return lib.lra_cur_batched_points(pts, npts, arr, len(blocks) if count is None else count, r, 1, 0, opts,
                                          fake, fake, fake, None, None)

    B = lra.lra_pts_block
    assert call([B(0, 50, 40, 51)], npts=100) == E   # columns end past the buffer: 50 + 51 > 100
    assert call([B(61, 0, 40, 40)], npts=100) == E   # 61 + 40 > 100
    assert call([B(-1, 0, 10, 10)]) == E
    assert call([B(0, 10, 2, 10)]) == E              # r > m
    assert call([B(0, 10, 10, 10)], r=0) == E
    assert call([B(0, 10, 10, 10)], r=65) == E
    assert call([B(0, 10, 10, 10)], npts=0) == E
    assert call([B(0, 10, 10, 10)], pts=None) == E
    o = lra.lra_default_opts()
    o.preprocess = 1
    assert call([B(0, 10, 10, 10)], opts=ct.byref(o)) == E
    # an empty batch is a no-op
    assert call([B(0, 10, 10, 10)], count=0) == lra.LRA_OK


def test_cynical_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(m=100, n=80, lda=80, r=4, k=16, loops=1, sweeps=2, dt=1, opts=None, W=fake):
        return lib.lra_cur_cynical(W, dt, m, n, lda, r, k, loops, sweeps, 1, opts, fake, fake, fake, None, None)

    assert call(k=3) == E            # k < r
    assert call(k=65) == E           # k > 64
    assert call(m=10, k=16) == E     # k > m
    assert call(n=12, lda=12) == E   # k > n
    assert call(loops=-1) == E
    assert call(sweeps=0) == E
    assert call(r=0) == E
    assert call(lda=79) == E
    assert call(dt=7) == E
    assert call(W=None) == E
    o = lra.lra_default_opts()
    o.preprocess = 1
    assert call(opts=ct.byref(o)) == E


def test_fourier_start_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(d=3, l=20, r=8, m=500, n=400):
        o = lra.lra_default_opts()
        o.preprocess = lra.LRA_PRE_ASRFT
        o.ah_depth = d
        o.ah_samples = l
        return lib.lra_cur(fake, 1, m, n, n, r, 2, 1, ct.byref(o), fake, fake, fake, None, None)

    assert call(d=4) == E            # more than three abridged stages
    assert call(d=-1) == E
    assert call(l=127) == E          # l 2^d above the coefficient table
    assert call(l=3) == E            # 2l < r
    assert call(d=0, l=129) == E     # 2l above the sketch width limit
    assert call(l=100, d=0, m=60, n=50) == E    # more samples than columns of the multiplier


def test_leverage_invalid_arguments_rejected_on_host(lib):
    # every check here runs before the call reads the device sets
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(m=100, n=80, lda=80, r=4, k=8, l=8, dt=1, W=fake, I0=fake):
        return lib.lra_cur_leverage(W, dt, m, n, lda, r, I0, fake, k, l, 1, fake, fake, fake, None, None)

    assert call(k=3) == E            # k < r
    assert call(l=3) == E            # l < r
    assert call(k=257) == E          # more than 256 draws on a side
    assert call(l=257) == E
    assert call(r=0) == E
    assert call(r=65, k=65, l=65) == E   # rank above 64
    assert call(m=3, r=4) == E       # r > m
    assert call(lda=79) == E
    assert call(dt=7) == E
    assert call(W=None) == E
    assert call(I0=None) == E


def test_projective_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(m=100, n=80, lda=80, r=4, k=16, l=12, sweeps=2, dt=1, opts=None, W=fake):
        return lib.lra_cur_projective(W, dt, m, n, lda, r, k, l, sweeps, 1, opts, fake, fake, fake, None, None)

    assert call(k=3) == E            # k < r
    assert call(l=3) == E            # l < r
    assert call(k=65) == E           # k > 64
    assert call(l=65) == E           # l > 64
    assert call(m=10, k=16) == E     # k > m
    assert call(n=10, lda=10) == E   # l > n
    assert call(sweeps=0) == E
    assert call(r=0) == E
    assert call(lda=79) == E
    assert call(dt=7) == E
    assert call(W=None) == E
    o = lra.lra_default_opts()
    o.preprocess = 1
    assert call(opts=ct.byref(o)) == E


def test_uniform_invalid_arguments_rejected_on_host(lib):
    fake = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL
    B = lra.lra_block

    def call(blocks, r=4, k=8, l=8, count=None, dt=1, base=fake):
        arr = (B * max(1, len(blocks)))(*blocks)
        cnt = len(blocks) if count is None else count
        return lib.lra_cur_uniform_batched(base, dt, arr, cnt, r, k, l, 1, fake, fake, fake, None, None)

    good = [B(0, 10, 10, 10)]
    assert call(good, k=3) == E      # k < r
    assert call(good, l=3) == E      # l < r
    assert call(good, k=65) == E     # k > 64
    assert call(good, l=65) == E     # l > 64
    assert call(good, r=0) == E
    assert call(good, dt=7) == E
    assert call(good, base=None) == E
    assert call(good, count=-1) == E
    assert call([B(0, 10, 10, 9)]) == E    # lda < n
    assert call([B(-1, 10, 10, 10)]) == E  # negative offset
    assert call([B(0, 0, 10, 10)]) == E    # empty block
    assert call(good, count=0) == lra.LRA_OK  # an empty batch is a no-op


def test_residual_invalid_arguments_rejected_on_host(lib):
    f = ct.c_void_p(0x1000)
    E = lra.LRA_EINVAL

    def call(W=f, dt=1, m=100, n=80, lda=80, r=5, q=0, s=0, prec=0, out=f):
        return lib.lra_residual(W, dt, m, n, lda, r, f, f, f, q, s, 0, prec, out, None)

    assert call(W=None) == E
    assert call(out=None) == E
    assert call(dt=9) == E
    assert call(lda=79) == E
    assert call(r=0) == E
    assert call(r=81) == E                 # r > min(m, n)
    assert call(q=10, s=0) == E            # q and s are both zero or both positive
    assert call(q=0, s=10) == E
    assert call(q=257, s=10) == E          # at most 256 sampled rows
    assert call(q=10, s=81) == E           # s > n
    assert call(prec=2) == E               # unknown precision
    assert call(m=128 * 65535 + 1, n=80) == lra.LRA_EUNSUPPORTED  # more rows than the launch grid covers


def test_adjoint_invalid_arguments_rejected_on_host(lib):
    f = ct.c_void_p(0x1000)

    def call(count=1, m=20, n=20, r=4, nnz=10, C=f, om=f):
        return lib.lra_cur_adjoint(count, m, n, r, C, f, f, nnz, om, om, om, f, f, f, f, f, f, None)

    assert call(count=-1) == lra.LRA_EINVAL
    assert call(r=0) == lra.LRA_EINVAL
    assert call(r=65) == lra.LRA_EINVAL
    assert call(nnz=-1) == lra.LRA_EINVAL
    assert call(C=None) == lra.LRA_EINVAL
    assert call(om=None) == lra.LRA_EINVAL
    assert call(m=1 << 31) == lra.LRA_EINVAL  # Omega indices are int32
    assert call(count=0) == lra.LRA_OK        # an empty batch is a no-op


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(lra, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(lra, "_lib", None)
    with pytest.raises(ImportError):
        lra.load()


def test_caller_outputs_are_checked_before_any_call():
    """A caller-supplied out= must hold exactly what the kernels write; an
    undersized or mistyped buffer is refused on the host (ValueError)."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cpu")
    r = 5

    def outs(nI=r, nJ=r, nU=r * r, ninfo=1, dtI=torch.int64, dtU=torch.float64):
        return lra.CurOut(torch.empty(nI, dtype=dtI), torch.empty(nJ, dtype=torch.int64),
                          torch.empty(nU, dtype=dtU), torch.empty(ninfo * lra.INFO_BYTES, dtype=torch.uint8))

    lra._check_out(outs(), r, r, r * r, 1, dev)
    for bad in (outs(nI=r - 1), outs(nJ=r + 1), outs(nU=r * r - 1), outs(ninfo=0), outs(dtI=torch.int32),
                outs(dtU=torch.float32)):
        with pytest.raises(ValueError):
            lra._check_out(bad, r, r, r * r, 1, dev)
    # a non-contiguous view of the right size
    o = outs()
    o.U = torch.empty((r, 2 * r), dtype=torch.float64)[:, ::2]
    with pytest.raises(ValueError):
        lra._check_out(o, r, r, r * r, 1, dev)
    # the k x l generators: I has k entries, J l, U l x k
    k, l = 7, 9
    o = lra.CurOut(torch.empty(k, dtype=torch.int64), torch.empty(l, dtype=torch.int64),
                   torch.empty((l, k), dtype=torch.float64), torch.empty(lra.INFO_BYTES, dtype=torch.uint8))
    lra._check_out(o, k, l, l * k, 1, dev)
    with pytest.raises(ValueError):
        lra._check_out(o, l, k, l * k, 1, dev)


def test_batch_rule_table_checked_on_host(lib):
    """The bin table API validates its rules without touching a device."""
    assert ct.sizeof(lra.lra_batch_rule) == 16
    default = lra.lra_batch_get_rules()
    assert default and all(q[2] in (0, 2) for q in default)
    E, U = lra.LRA_EINVAL, lra.LRA_EUNSUPPORTED

    def status(rules):
        arr = (lra.lra_batch_rule * max(1, len(rules)))(*[lra.lra_batch_rule(*q) for q in rules])
        return lib.lra_batch_set_rules(arr, len(rules))

    assert status([(512, 16, 2, 2)]) == E         # 2 x 2 x 64 = 256 item slots < 512
    assert status([(512, 16, 2, 9)]) == E         # at most 8 wavefronts
    assert status([(0, 16, 2, 1)]) == E
    assert status([(128, 65, 2, 1)]) == E         # rank above 64
    assert status([(256, 8, 2, 2)]) == U          # no register variant for rank 8
    assert status([(256, 16, 3, 2)]) == U         # nor for 3 items per lane
    assert lib.lra_batch_set_rules(None, -1) == E
    assert status([(1 << 20, 16, 0, 0), (256, 16, 2, 2)]) == lra.LRA_OK
    assert lra.lra_batch_get_rules() == [(256, 16, 2, 2), (1 << 20, 16, 0, 0)]  # sorted by max_dim
    lra.lra_batch_set_rules([])
    assert lra.lra_batch_get_rules() == default
