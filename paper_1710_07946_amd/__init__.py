"""Python binding of the MI355X cross-approximation CUR library.

The functions here carry the names of the C ABI in ``include/lra_cur.h`` and
only marshal arguments: PyTorch supplies device memory and the current HIP
stream, and every step of the computation runs in the library's HIP kernels
(``_build/liblra_cur.so``, built by ``build.py``).  There is no fallback: if
the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as ct
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "_build", "liblra_cur.so")
HEADER = os.path.join(ROOT, "include", "lra_cur.h")

LRA_OK, LRA_EINVAL, LRA_ESINGULAR, LRA_EDEVICE, LRA_ENOMEM, LRA_EUNSUPPORTED = range(6)
LRA_F64, LRA_F32, LRA_BF16 = 0, 1, 2
LRA_PRE_NONE, LRA_PRE_ASRHT, LRA_PRE_BIDIAG, LRA_PRE_ASRFT = 0, 1, 2, 3
LRA_PREC_PLAIN, LRA_PREC_MIXED = 0, 1


class LraError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, lra_strerror(status), status))
        self.status = status


class lra_opts(ct.Structure):
    _fields_ = [("delta", ct.c_double), ("max_swaps", ct.c_int32), ("preprocess", ct.c_int32),
                ("ah_depth", ct.c_int32), ("ah_samples", ct.c_int32), ("refine_steps", ct.c_int32),
                ("team_size", ct.c_int32), ("track_margin", ct.c_int32), ("init_cols", ct.POINTER(ct.c_int64))]


class lra_info(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("sweeps_run", ct.c_int32), ("swaps_total", ct.c_int32),
                ("converged", ct.c_int32), ("rank_found", ct.c_int32), ("team_size", ct.c_int32),
                ("nucleus_rank", ct.c_int32), ("reserved", ct.c_int32), ("det_log_abs", ct.c_double),
                ("min_margin", ct.c_double)]


class lra_block(ct.Structure):
    _fields_ = [("offset", ct.c_int64), ("m", ct.c_int64), ("n", ct.c_int64), ("lda", ct.c_int64)]


class lra_pts_block(ct.Structure):
    _fields_ = [("x_off", ct.c_int64), ("y_off", ct.c_int64), ("m", ct.c_int64), ("n", ct.c_int64)]


class lra_posterior(ct.Structure):
    _fields_ = [("K", ct.c_int64), ("mean", ct.c_double), ("mean_abs", ct.c_double), ("var", ct.c_double),
                ("threshold", ct.c_double), ("accept", ct.c_int32), ("reserved", ct.c_int32)]


class lra_batch_rule(ct.Structure):
    _fields_ = [("max_dim", ct.c_int32), ("r", ct.c_int32), ("items_per_lane", ct.c_int32), ("waves", ct.c_int32)]


INFO_BYTES = ct.sizeof(lra_info)
_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> ct.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library not built: %s (run paper_1710_07946_amd/build.py)" % LIB_PATH)
        # torch first: the library must bind to the HIP runtime torch loads,
        # or the process holds two runtimes and torch's device pointers are
        # foreign to the library's (its first call fails with LRA_EDEVICE)
        import torch  # noqa: F401
        L = ct.CDLL(LIB_PATH)
        P, i64, i32 = ct.c_void_p, ct.c_int64, ct.c_int32
        L.lra_default_opts.argtypes = [ct.POINTER(lra_opts)]
        L.lra_default_opts.restype = None
        L.lra_strerror.argtypes = [ct.c_int]
        L.lra_strerror.restype = ct.c_char_p
        L.lra_release.argtypes = []
        L.lra_release.restype = None
        L.lra_cur.argtypes = [P, ct.c_int, i64, i64, i64, i32, i32, ct.c_uint64, ct.POINTER(lra_opts), P, P, P, P,
                              P]
        L.lra_cur.restype = ct.c_int
        L.lra_cur_noalloc.argtypes = L.lra_cur.argtypes
        L.lra_cur_noalloc.restype = ct.c_int
        L.lra_cur_batched.argtypes = [P, ct.c_int, ct.POINTER(lra_block), i64, i32, i32, ct.c_uint64,
                                      ct.POINTER(lra_opts), P, P, P, P, P]
        L.lra_cur_batched.restype = ct.c_int
        L.lra_cur_batched_points.argtypes = [P, i64, ct.POINTER(lra_pts_block), i64, i32, i32, ct.c_uint64,
                                             ct.POINTER(lra_opts), P, P, P, P, P]
        L.lra_cur_batched_points.restype = ct.c_int
        L.lra_batch_set_rules.argtypes = [ct.POINTER(lra_batch_rule), ct.c_int32]
        L.lra_batch_set_rules.restype = ct.c_int
        L.lra_batch_get_rules.argtypes = [ct.POINTER(lra_batch_rule), ct.c_int32]
        L.lra_batch_get_rules.restype = ct.c_int32
        L.lra_cur_cynical.argtypes = [P, ct.c_int, i64, i64, i64, i32, i32, i32, i32, ct.c_uint64,
                                      ct.POINTER(lra_opts), P, P, P, P, P]
        L.lra_cur_cynical.restype = ct.c_int
        L.lra_cur_projective.argtypes = [P, ct.c_int, i64, i64, i64, i32, i32, i32, i32, ct.c_uint64,
                                         ct.POINTER(lra_opts), P, P, P, P, P]
        L.lra_cur_projective.restype = ct.c_int
        L.lra_cur_leverage.argtypes = [P, ct.c_int, i64, i64, i64, i32, P, P, i32, i32, ct.c_uint64, P, P, P, P, P]
        L.lra_cur_leverage.restype = ct.c_int
        L.lra_cur_uniform_batched.argtypes = [P, ct.c_int, ct.POINTER(lra_block), i64, i32, i32, i32, ct.c_uint64,
                                              P, P, P, P, P]
        L.lra_cur_uniform_batched.restype = ct.c_int
        L.lra_cur_dmm_batched.argtypes = [P, ct.c_int, ct.POINTER(lra_block), i64, i32, i32, i32, i32, ct.c_uint64,
                                          P, P, P, P, P]
        L.lra_cur_dmm_batched.restype = ct.c_int
        L.lra_cur_hadamard.argtypes = [P, ct.c_int, i64, i64, i64, i32, i32, ct.c_uint64, i32,
                                       ct.POINTER(lra_opts), P, P, P, P, P]
        L.lra_cur_hadamard.restype = ct.c_int
        L.lra_residual.argtypes = [P, ct.c_int, i64, i64, i64, i32, P, P, P, i32, i32, ct.c_uint64, i32, P, P]
        L.lra_residual.restype = ct.c_int
        L.lra_posterior_test.argtypes = [P, ct.c_int, i64, i64, i64, i32, P, P, P, i32, i32, ct.c_uint64, i32,
                                         ct.c_double, ct.c_double, P, P]
        L.lra_posterior_test.restype = ct.c_int
        L.lra_probe_exchange.argtypes = [i32, ct.POINTER(ct.c_double), P]
        L.lra_probe_exchange.restype = ct.c_int
        L.lra_cur_adjoint.argtypes = [i64, i64, i64, i32, P, P, P, i64, P, P, P, P, P, P, P, P, P, P]
        L.lra_cur_adjoint.restype = ct.c_int
        _lib = L
        # free the cached device workspaces while the HIP runtime is still up
        # (interpreter exit runs this before the runtime's own teardown)
        atexit.register(L.lra_release)
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions the public header declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lra_[a-z_]+)\s*\(", text)))


def lra_strerror(status: int) -> str:
    try:
        return load().lra_strerror(int(status)).decode()
    except ImportError:
        return "status %d" % status


def lra_release() -> None:
    load().lra_release()


def lra_batch_set_rules(rules) -> None:
    """Replace the batched launch's bin table: rules are (max_dim, r,
    items_per_lane, waves) tuples; an empty list restores the built-in table."""
    arr = (lra_batch_rule * max(1, len(rules)))()
    for i, q in enumerate(rules):
        arr[i] = lra_batch_rule(*(int(v) for v in q))
    st = load().lra_batch_set_rules(arr, len(rules))
    if st != LRA_OK:
        raise LraError(st, "lra_batch_set_rules")


def lra_batch_get_rules() -> list:
    """The current bin table as (max_dim, r, items_per_lane, waves) tuples."""
    L = load()
    n = L.lra_batch_get_rules(None, 0)
    arr = (lra_batch_rule * max(1, n))()
    L.lra_batch_get_rules(arr, n)
    return [(q.max_dim, q.r, q.items_per_lane, q.waves) for q in arr[:n]]


def lra_default_opts() -> lra_opts:
    o = lra_opts()
    load().lra_default_opts(ct.byref(o))
    return o


# ------------------------------------------------------------------ helpers
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return LRA_F64
    if t.dtype == torch.float32:
        return LRA_F32
    if t.dtype == torch.bfloat16:
        return LRA_BF16
    raise TypeError("unsupported dtype %s" % t.dtype)


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _make_opts(delta, max_swaps, preprocess, ah_depth, ah_samples, refine_steps, team_size, init_cols,
               track_margin=False):
    o = lra_default_opts()
    o.track_margin = 1 if track_margin else 0
    o.delta = delta
    o.max_swaps = max_swaps
    o.preprocess = preprocess
    o.ah_depth = ah_depth
    o.ah_samples = ah_samples
    o.refine_steps = refine_steps
    o.team_size = team_size
    keep = None
    if init_cols is not None:
        keep = np.ascontiguousarray(init_cols, np.int64)
        o.init_cols = keep.ctypes.data_as(ct.POINTER(ct.c_int64))
    return o, keep


def parse_info(raw) -> dict:
    """Decode lra_info records from a uint8 tensor/array of INFO_BYTES each."""
    b = np.ascontiguousarray(raw.cpu().numpy() if hasattr(raw, "cpu") else raw, np.uint8).reshape(-1, INFO_BYTES)
    out = []
    for row in b:
        inf = lra_info.from_buffer_copy(row.tobytes())
        out.append({k: getattr(inf, k) for k, _ in lra_info._fields_})
    return out


@dataclass
class CurOut:
    I: object       # device int64[r] (or [count, r])
    J: object
    U: object       # device float64[r, r] (or [count, r, r])
    info_raw: object

    def info(self):
        recs = parse_info(self.info_raw)
        return recs[0] if len(recs) == 1 else recs


def _check_out(out: CurOut, n_i: int, n_j: int, n_u: int, n_info: int, dev) -> None:
    """A caller-supplied output set must hold exactly what the kernels write:
    contiguous device tensors of n_i and n_j int64 indices, n_u float64
    nucleus entries and n_info lra_info records, on the input's device."""
    torch = _torch()
    for name, t, numel, dt in (("I", out.I, n_i, torch.int64), ("J", out.J, n_j, torch.int64),
                               ("U", out.U, n_u, torch.float64), ("info_raw", out.info_raw, n_info * INFO_BYTES,
                                                                  torch.uint8)):
        if not hasattr(t, "device") or t.device != dev:
            raise ValueError("out.%s must be a tensor on %s" % (name, dev))
        if t.dtype != dt or t.numel() != numel or not t.is_contiguous():
            raise ValueError("out.%s must be a contiguous %s tensor of %d elements (got %s, %d)"
                             % (name, dt, numel, t.dtype, t.numel()))


# ------------------------------------------------------------------ entry points
def _cur_entry(name: str, A, r, sweeps, seed, delta, max_swaps, preprocess, ah_depth, ah_samples, refine_steps,
               team_size, init_cols, out, stream, track_margin=False) -> CurOut:
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    dev = A.device
    if out is None:
        out = CurOut(torch.empty(r, dtype=torch.int64, device=dev), torch.empty(r, dtype=torch.int64, device=dev),
                     torch.empty((r, r), dtype=torch.float64, device=dev),
                     torch.empty(INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, r, r, r * r, 1, dev)
    o, keep = _make_opts(delta, max_swaps, preprocess, ah_depth, ah_samples, refine_steps, team_size, init_cols,
                         track_margin)
    st = getattr(load(), name)(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r, sweeps,
                               ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.byref(o), ct.c_void_p(out.I.data_ptr()),
                               ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                               ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    del keep
    if st != LRA_OK:
        raise LraError(st, name)
    return out


def lra_cur(A, r: int, sweeps: int, seed: int, *, delta: float = 0.01, max_swaps: int = -1,
            preprocess: int = LRA_PRE_NONE, ah_depth: int = 3, ah_samples: int = 0, refine_steps: int = 0,
            team_size: int = 0, init_cols=None, out: CurOut | None = None, stream=None,
            track_margin: bool = False) -> CurOut:
    """C-A CUR of a 2-D device tensor (row-major rows, unit column stride).

    Asynchronous on the current (or given) stream; the returned tensors are
    filled when the stream reaches the launch.  ``CurOut.info()`` syncs.
    ``track_margin`` reports the decisions' smallest margin in the info.
    """
    return _cur_entry("lra_cur", A, r, sweeps, seed, delta, max_swaps, preprocess, ah_depth, ah_samples,
                      refine_steps, team_size, init_cols, out, stream, track_margin)


def lra_cur_noalloc(A, r: int, sweeps: int, seed: int, *, delta: float = 0.01, max_swaps: int = -1,
                    preprocess: int = LRA_PRE_NONE, ah_depth: int = 3, ah_samples: int = 0, refine_steps: int = 0,
                    team_size: int = 0, out: CurOut | None = None, stream=None,
                    track_margin: bool = False) -> CurOut:
    """``lra_cur`` with every work buffer in the library's fixed per-GPU scratch
    (no device allocation by the library; pass ``out`` to allocate nothing
    here either).  Calls that overlap on one GPU race."""
    return _cur_entry("lra_cur_noalloc", A, r, sweeps, seed, delta, max_swaps, preprocess, ah_depth, ah_samples,
                      refine_steps, team_size, None, out, stream, track_margin)


def lra_cur_hadamard(A, r: int, sweeps: int, seed: int, d: int, *, delta: float = 0.01, max_swaps: int = -1,
                     refine_steps: int = 0, team_size: int = 0, out: CurOut | None = None, stream=None,
                     track_margin: bool = False) -> CurOut:
    """C-A CUR of the pre-processed matrix W' = W D (H_{2^d} (x) I_s) (m x N, N the
    multiple of 2^d at or above n), its entries formed on the fly; J indexes the
    columns of W'.  Asynchronous like ``lra_cur``."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    dev = A.device
    if out is None:
        out = CurOut(torch.empty(r, dtype=torch.int64, device=dev), torch.empty(r, dtype=torch.int64, device=dev),
                     torch.empty((r, r), dtype=torch.float64, device=dev),
                     torch.empty(INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, r, r, r * r, 1, dev)
    o, keep = _make_opts(delta, max_swaps, LRA_PRE_NONE, 3, 0, refine_steps, team_size, None, track_margin)
    st = load().lra_cur_hadamard(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r, sweeps,
                                 ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), d, ct.byref(o), ct.c_void_p(out.I.data_ptr()),
                                 ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                 ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    del keep
    if st != LRA_OK:
        raise LraError(st, "lra_cur_hadamard")
    return out


def lra_cur_cynical(A, r: int, k: int, loops: int, sweeps: int, seed: int, *, delta: float = 0.01,
                    max_swaps: int = -1, refine_steps: int = 0, team_size: int = 0, out: CurOut | None = None,
                    stream=None) -> CurOut:
    """Cynical CUR: an r x r generator of locally maximal volume inside a k x k
    sketch W[K, L], with K, L random (loops = 0, Tests 3) or from `loops` C-A
    loops at rank k (loops = 1: Tests 4).  Asynchronous like ``lra_cur``."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    dev = A.device
    if out is None:
        out = CurOut(torch.empty(r, dtype=torch.int64, device=dev), torch.empty(r, dtype=torch.int64, device=dev),
                     torch.empty((r, r), dtype=torch.float64, device=dev),
                     torch.empty(INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, r, r, r * r, 1, dev)
    o, keep = _make_opts(delta, max_swaps, LRA_PRE_NONE, 3, 0, refine_steps, team_size, None)
    st = load().lra_cur_cynical(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r, k, loops, sweeps,
                                ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.byref(o), ct.c_void_p(out.I.data_ptr()),
                                ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    del keep
    if st != LRA_OK:
        raise LraError(st, "lra_cur_cynical")
    return out


def lra_cur_projective(A, r: int, k: int, l: int, sweeps: int, seed: int, *, delta: float = 0.01,
                       max_swaps: int = -1, team_size: int = 0, out: CurOut | None = None,
                       stream=None) -> CurOut:
    """C-A with k x l generators of large r-projective volume and the
    canonical nucleus: I has k rows, J l columns, U is l x k (W ~ W[:, J] U
    W[I, :]).  delta and max_swaps govern each step's exchanges (max_swaps
    -1: 16 r).  Asynchronous like ``lra_cur``."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    dev = A.device
    if out is None:
        out = CurOut(torch.empty(k, dtype=torch.int64, device=dev), torch.empty(l, dtype=torch.int64, device=dev),
                     torch.empty((l, k), dtype=torch.float64, device=dev),
                     torch.empty(INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, k, l, l * k, 1, dev)
    o, keep = _make_opts(delta, max_swaps, LRA_PRE_NONE, 3, 0, 0, team_size, None)
    st = load().lra_cur_projective(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r, k, l, sweeps,
                                   ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.byref(o), ct.c_void_p(out.I.data_ptr()),
                                   ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                   ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    del keep
    if st != LRA_OK:
        raise LraError(st, "lra_cur_projective")
    return out


def lra_cur_batched(base, blocks, r: int, sweeps: int, seed: int, *, delta: float = 0.01, max_swaps: int = -1,
                    refine_steps: int = 0, out: CurOut | None = None, stream=None,
                    track_margin: bool = False) -> CurOut:
    """C-A CUR of `count` blocks stored in the flat device tensor `base`.

    ``blocks`` is an int64 array of shape (count, 4): (offset, m, n, lda) in
    elements.  Block b uses seed + b.  Asynchronous like ``lra_cur``.
    """
    torch = _torch()
    if base.dim() != 1 or not base.is_cuda:
        raise ValueError("base must be a flat device tensor")
    desc = np.ascontiguousarray(blocks, np.int64).reshape(-1, 4)
    count = desc.shape[0]
    if count:
        off, m, n, ld = desc.T
        end = off + (m - 1) * ld + n
        if (off < 0).any() or (m < 1).any() or (n < 1).any() or (ld < n).any() or int(end.max()) > base.numel():
            raise ValueError("block descriptors reach outside the base tensor")
    dev = base.device
    if out is None:
        out = CurOut(torch.empty((count, r), dtype=torch.int64, device=dev),
                     torch.empty((count, r), dtype=torch.int64, device=dev),
                     torch.empty((count, r, r), dtype=torch.float64, device=dev),
                     torch.empty(count * INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, count * r, count * r, count * r * r, count, dev)
    arr = (lra_block * max(count, 1))()
    ct.memmove(arr, desc.ctypes.data, desc.nbytes)
    o, keep = _make_opts(delta, max_swaps, LRA_PRE_NONE, 3, 0, refine_steps, 0, None, track_margin)
    st = load().lra_cur_batched(ct.c_void_p(base.data_ptr()), _dtype_code(base), arr, count, r, sweeps,
                                ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.byref(o), ct.c_void_p(out.I.data_ptr()),
                                ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_batched")
    return out


def lra_cur_uniform_batched(base, blocks, r: int, k: int, l: int, seed: int, *, out: CurOut | None = None,
                            stream=None) -> CurOut:
    """CUR with uniform leverage scores of `count` blocks of the flat device
    tensor `base` (descriptors as in ``lra_cur_batched``): per block k rows and
    l columns drawn with replacement and U = D M_r^+ Dbar (l x k).  Block b
    uses seed + b.  Asynchronous like ``lra_cur``."""
    torch = _torch()
    if base.dim() != 1 or not base.is_cuda:
        raise ValueError("base must be a flat device tensor")
    desc = np.ascontiguousarray(blocks, np.int64).reshape(-1, 4)
    count = desc.shape[0]
    if count:
        off, m, n, ld = desc.T
        end = off + (m - 1) * ld + n
        if (off < 0).any() or (m < 1).any() or (n < 1).any() or (ld < n).any() or int(end.max()) > base.numel():
            raise ValueError("block descriptors reach outside the base tensor")
    dev = base.device
    if out is None:
        out = CurOut(torch.empty((count, k), dtype=torch.int64, device=dev),
                     torch.empty((count, l), dtype=torch.int64, device=dev),
                     torch.empty((count, l, k), dtype=torch.float64, device=dev),
                     torch.empty(count * INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, count * k, count * l, count * l * k, count, dev)
    arr = (lra_block * max(count, 1))()
    ct.memmove(arr, desc.ctypes.data, desc.nbytes)
    st = load().lra_cur_uniform_batched(ct.c_void_p(base.data_ptr()), _dtype_code(base), arr, count, r, k, l,
                                        ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.c_void_p(out.I.data_ptr()),
                                        ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                        ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_uniform_batched")
    return out


def lra_cur_dmm_batched(base, blocks, r: int, k: int, l: int, iters: int, seed: int, *, out: CurOut | None = None,
                        stream=None) -> CurOut:
    """C-A with DMM08 leverage-score sampling of every sketch for `count`
    blocks of the flat device tensor `base` (descriptors as in
    ``lra_cur_batched``): per block k rows, l columns (sorted, duplicates
    kept) and U (l x k) after `iters` iterations.  Block b uses seed + b.
    Asynchronous like ``lra_cur``."""
    torch = _torch()
    if base.dim() != 1 or not base.is_cuda:
        raise ValueError("base must be a flat device tensor")
    desc = np.ascontiguousarray(blocks, np.int64).reshape(-1, 4)
    count = desc.shape[0]
    if count:
        off, m, n, ld = desc.T
        end = off + (m - 1) * ld + n
        if (off < 0).any() or (m < 1).any() or (n < 1).any() or (ld < n).any() or int(end.max()) > base.numel():
            raise ValueError("block descriptors reach outside the base tensor")
    dev = base.device
    if out is None:
        out = CurOut(torch.empty((count, k), dtype=torch.int64, device=dev),
                     torch.empty((count, l), dtype=torch.int64, device=dev),
                     torch.empty((count, l, k), dtype=torch.float64, device=dev),
                     torch.empty(count * INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, count * k, count * l, count * l * k, count, dev)
    arr = (lra_block * max(count, 1))()
    ct.memmove(arr, desc.ctypes.data, desc.nbytes)
    st = load().lra_cur_dmm_batched(ct.c_void_p(base.data_ptr()), _dtype_code(base), arr, count, r, k, l, iters,
                                    ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.c_void_p(out.I.data_ptr()),
                                    ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                    ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_dmm_batched")
    return out


def lra_cur_dmm(A, r: int, k: int, l: int, iters: int, seed: int, *, stream=None) -> CurOut:
    """C-A with DMM08 sampling of one 2-D device tensor (row-major rows, unit
    column stride): a batch of one block covering A."""
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    flat = A.as_strided(((m - 1) * A.stride(0) + n,), (1,))
    out = lra_cur_dmm_batched(flat, [[0, m, n, A.stride(0)]], r, k, l, iters, seed, stream=stream)
    return CurOut(out.I[0], out.J[0], out.U[0], out.info_raw)


def lra_cur_uniform(A, r: int, k: int, l: int, seed: int, *, stream=None) -> CurOut:
    """CUR with uniform leverage scores of one 2-D device tensor (row-major
    rows, unit column stride): a batch of one block covering A."""
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    flat = A.as_strided(((m - 1) * A.stride(0) + n,), (1,))
    out = lra_cur_uniform_batched(flat, [[0, m, n, A.stride(0)]], r, k, l, seed, stream=stream)
    return CurOut(out.I[0], out.J[0], out.U[0], out.info_raw)


def lra_cur_leverage(A, I0, J0, k: int, l: int, seed: int, *, out: CurOut | None = None, stream=None) -> CurOut:
    """Refinement of the CUR LRA of (I0, J0) (device int64 tensors of r
    entries) by its leverage scores: k rows and l columns drawn by the crude
    LRA's scores, U = D M_r^+ Dbar (l x k).  Synchronizes the stream once to
    check I0 and J0."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    for t in (I0, J0):
        if not t.is_cuda or t.dtype != torch.int64 or not t.is_contiguous():
            raise ValueError("I0 and J0 must be contiguous int64 device tensors")
    if I0.numel() != J0.numel():
        raise ValueError("I0 and J0 must have the same length")
    m, n = A.shape
    dev = A.device
    if out is None:
        out = CurOut(torch.empty(k, dtype=torch.int64, device=dev), torch.empty(l, dtype=torch.int64, device=dev),
                     torch.empty((l, k), dtype=torch.float64, device=dev),
                     torch.empty(INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, k, l, l * k, 1, dev)
    st = load().lra_cur_leverage(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), int(I0.numel()),
                                 ct.c_void_p(I0.data_ptr()), ct.c_void_p(J0.data_ptr()), k, l,
                                 ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.c_void_p(out.I.data_ptr()),
                                 ct.c_void_p(out.J.data_ptr()), ct.c_void_p(out.U.data_ptr()),
                                 ct.c_void_p(out.info_raw.data_ptr()), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_leverage")
    return out


def lra_cur_batched_points(pts, blocks, r: int, sweeps: int, seed: int, *, delta: float = 0.01,
                           max_swaps: int = -1, refine_steps: int = 0, out: CurOut | None = None,
                           stream=None, track_margin: bool = False) -> CurOut:
    """C-A CUR of `count` far-field blocks K_ij = 1/|x_i - y_j| evaluated on the
    fly from the device float64 point tensor `pts` of shape (npts, 2).

    ``blocks`` is an int64 array of shape (count, 4): (x_off, y_off, m, n) in
    points.  Block b uses seed + b.  Asynchronous like ``lra_cur``.
    """
    torch = _torch()
    if pts.dim() != 2 or pts.shape[1] != 2 or not pts.is_cuda or pts.dtype != torch.float64 \
            or not pts.is_contiguous():
        raise ValueError("pts must be a contiguous (npts, 2) float64 device tensor")
    desc = np.ascontiguousarray(blocks, np.int64).reshape(-1, 4)
    count = desc.shape[0]
    dev = pts.device
    if out is None:
        out = CurOut(torch.empty((count, r), dtype=torch.int64, device=dev),
                     torch.empty((count, r), dtype=torch.int64, device=dev),
                     torch.empty((count, r, r), dtype=torch.float64, device=dev),
                     torch.empty(count * INFO_BYTES, dtype=torch.uint8, device=dev))
    else:
        _check_out(out, count * r, count * r, count * r * r, count, dev)
    arr = (lra_pts_block * max(count, 1))()
    ct.memmove(arr, desc.ctypes.data, desc.nbytes)
    o, keep = _make_opts(delta, max_swaps, LRA_PRE_NONE, 3, 0, refine_steps, 0, None, track_margin)
    st = load().lra_cur_batched_points(ct.c_void_p(pts.data_ptr()), pts.shape[0], arr, count, r, sweeps,
                                       ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ct.byref(o),
                                       ct.c_void_p(out.I.data_ptr()), ct.c_void_p(out.J.data_ptr()),
                                       ct.c_void_p(out.U.data_ptr()), ct.c_void_p(out.info_raw.data_ptr()),
                                       _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_batched_points")
    return out


def lra_residual(A, I, J, U, q: int = 0, s: int = 0, seed: int = 0, prec: int = 0, out=None, stream=None):
    """Residual moments [sum e, sum e^2, sum |e|, sum w^2] of E = A - A[:, J] U A[I, :]
    over all entries (q = s = 0) or a seeded q x s sample; a device float64[4].
    prec = LRA_PREC_MIXED computes the product on BF16 matrix cores (hi/lo split)."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    r = int(I.numel())
    for t, dt in ((I, torch.int64), (J, torch.int64), (U, torch.float64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("I, J must be contiguous int64 and U contiguous float64 device tensors")
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=A.device)
    st = load().lra_residual(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r,
                             ct.c_void_p(I.data_ptr()), ct.c_void_p(J.data_ptr()), ct.c_void_p(U.data_ptr()), q, s,
                             ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), prec, ct.c_void_p(out.data_ptr()),
                             _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_residual")
    return out


def lra_posterior_test(A, I, J, U, q: int, s: int, seed: int, tau: float, z: float, prec: int = 0, out=None,
                       stream=None):
    """The a-posteriori variance test on a seeded q x s sample of the error of
    the CUR (I, J, U); returns the device-resident lra_posterior record as a
    uint8 tensor (decode with ``parse_posterior``)."""
    torch = _torch()
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    m, n = A.shape
    r = int(I.numel())
    for t, dt in ((I, torch.int64), (J, torch.int64), (U, torch.float64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("I, J must be contiguous int64 and U contiguous float64 device tensors")
    nbytes = ct.sizeof(lra_posterior)
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    elif out.dtype != torch.uint8 or out.numel() != nbytes or not out.is_contiguous() or out.device != A.device:
        raise ValueError("out must be a contiguous uint8 tensor of %d bytes on %s" % (nbytes, A.device))
    st = load().lra_posterior_test(ct.c_void_p(A.data_ptr()), _dtype_code(A), m, n, A.stride(0), r,
                                   ct.c_void_p(I.data_ptr()), ct.c_void_p(J.data_ptr()), ct.c_void_p(U.data_ptr()),
                                   q, s, ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), prec, ct.c_double(tau),
                                   ct.c_double(z), ct.c_void_p(out.data_ptr()), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_posterior_test")
    return out


def lra_probe_exchange(rounds: int = 20000, stream=None) -> float:
    """One-way latency (ns) of a hand-off between workgroups on different XCDs."""
    ns = ct.c_double(0)
    st = load().lra_probe_exchange(rounds, ct.byref(ns), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_probe_exchange")
    return ns.value


def parse_posterior(raw) -> dict:
    """Decode an lra_posterior record (uint8 tensor or array)."""
    b = np.ascontiguousarray(raw.cpu().numpy() if hasattr(raw, "cpu") else raw, np.uint8)
    p = lra_posterior.from_buffer_copy(b.tobytes())
    return {"K": p.K, "mean": p.mean, "mean_abs": p.mean_abs, "var": p.var, "threshold": p.threshold,
            "accept": bool(p.accept)}


def omega_column_order(om_row, om_col):
    """Stable permutation sorting each block's Omega entries by column (int32).
    Part of the sparse input format of lra_cur_adjoint (like building CSC from CSR)."""
    torch = _torch()
    cols = om_col.to(torch.int64)
    rows = om_row.to(torch.int64)
    # entries are sorted by (row, col); sorting by col * (max_row + 1) + row keeps row order within a column
    key = cols * (int(rows.max().item()) + 1 if rows.numel() else 1) + rows
    return torch.argsort(key, dim=-1).to(torch.int32).contiguous()


def lra_cur_adjoint(C, R, G, om_row, om_col, col_order, a_om, stream=None):
    """Loss and gradients of sum over Omega of (a - C G^{-1} R)^2 for a batch of blocks.

    C (count, m, r), R (count, r, n), G (count, r, r): float64 device tensors;
    om_row, om_col, col_order (count, nnz) int32; a_om (count, nnz) float64.
    Returns (loss (count,), dC, dR, dG, status (count,) int32)."""
    torch = _torch()
    count, m, r = C.shape
    n = R.shape[2]
    nnz = om_row.shape[1] if om_row.dim() == 2 else 0
    for t in (C, R, G, a_om):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("C, R, G, a_om must be contiguous float64 device tensors")
    for t in (om_row, om_col, col_order):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("om_row, om_col, col_order must be contiguous int32 device tensors")
    if R.shape != (count, r, n) or G.shape != (count, r, r) or a_om.shape != (count, nnz):
        raise ValueError("inconsistent shapes")
    dev = C.device
    loss = torch.empty(count, dtype=torch.float64, device=dev)
    dC, dR, dG = torch.empty_like(C), torch.empty_like(R), torch.empty_like(G)
    status = torch.empty(count, dtype=torch.int32, device=dev)
    P = lambda t: ct.c_void_p(t.data_ptr())  # noqa: E731
    st = load().lra_cur_adjoint(count, m, n, r, P(C), P(R), P(G), nnz, P(om_row), P(om_col), P(col_order), P(a_om),
                                P(loss), P(dC), P(dR), P(dG), P(status), _stream_ptr(stream))
    if st != LRA_OK:
        raise LraError(st, "lra_cur_adjoint")
    return loss, dC, dR, dG, status


def _make_autograd():
    torch = _torch()

    class CURReconLoss(torch.autograd.Function):
        """loss_b = sum over Omega_b of (a - C_b G_b^{-1} R_b)^2, differentiable in
        C, R and G; forward and backward both come from lra_cur_adjoint."""

        @staticmethod
        def forward(ctx, C, R, G, om_row, om_col, col_order, a_om):
            loss, dC, dR, dG, status = lra_cur_adjoint(C.detach().contiguous(), R.detach().contiguous(),
                                                       G.detach().contiguous(), om_row, om_col, col_order, a_om)
            ctx.save_for_backward(dC, dR, dG)
            ctx.status = status
            return loss

        @staticmethod
        def backward(ctx, gloss):
            dC, dR, dG = ctx.saved_tensors
            g = gloss.to(torch.float64)
            return (g[:, None, None] * dC, g[:, None, None] * dR, g[:, None, None] * dG, None, None, None, None)

    return CURReconLoss


_autograd_fn = None


def cur_recon_loss(C, R, G, om_row, om_col, col_order, a_om):
    """torch.autograd entry point of the CUR adjoint (see CURReconLoss)."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn.apply(C, R, G, om_row, om_col, col_order, a_om)
