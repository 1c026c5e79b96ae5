"""FP64 CPU oracle for cross-approximation CUR (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it.  Everything here is a thin ctypes layer over
``lra_oracle.c``, a plain C reading of Pan, Luan, Svadlenka and Zhao,
"Superfast Accurate Low Rank Approximation"; each C routine cites the passage
it follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lra_oracle.c")
_OUT = os.path.join(_HERE, "_build", "liblra_oracle.so")

OK, EINVAL, ESINGULAR = 0, 1, 2
F64, F32, BF16 = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/_build`` and return the path."""
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_OUT), exist_ok=True)
        tmp = _OUT + ".tmp%d" % os.getpid()
        # no contraction of a * b + c into a fused multiply-add: every
        # operation rounds once, whatever the host compiler's default target
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


class _Opts(ct.Structure):
    _fields_ = [("delta", ct.c_double), ("max_swaps", ct.c_int32), ("preprocess", ct.c_int32),
                ("ah_depth", ct.c_int32), ("ah_samples", ct.c_int32), ("refine_steps", ct.c_int32),
                ("init_cols", ct.POINTER(ct.c_int64))]


class _Info(ct.Structure):
    _fields_ = [("sweeps_run", ct.c_int32), ("swaps_total", ct.c_int32), ("converged", ct.c_int32),
                ("rank_found", ct.c_int32), ("nucleus_rank", ct.c_int32), ("pad", ct.c_int32),
                ("min_margin", ct.c_double), ("det_log_abs", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ct.CDLL(build())
        P = ct.c_void_p
        i64, i32, u64, dbl = ct.c_int64, ct.c_int32, ct.c_uint64, ct.c_double
        L.orc_rng_u64.argtypes = [u64, u64, u64]
        L.orc_rng_u64.restype = u64
        L.orc_draw_distinct.argtypes = [u64, u64, i64, i64, P]
        L.orc_sign.argtypes = [u64, i64]
        L.orc_sign.restype = dbl
        L.orc_panel_lu.argtypes = [P, i64, ct.c_int, P, P, P, P]
        L.orc_maxvol.argtypes = [P, i64, ct.c_int, dbl, i32, P, P, P, P, P, P, P, P]
        L.orc_sketch.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, u64, P, P]
        L.orc_qrp.argtypes = [P, i64, ct.c_int, ct.c_int, P, P, P]
        L.orc_inverse.argtypes = [P, ct.c_int, P, ct.c_int, P]
        L.orc_refine_inverse.argtypes = [P, ct.c_int, P, ct.c_int]
        L.orc_default_opts.argtypes = [P]
        L.orc_ca_cur.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, u64, P, P, P, P, P]
        L.orc_residual.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, P, P, P, P, P]
        L.orc_cur_adjoint.argtypes = [P, P, P, i64, i64, ct.c_int, P, P, P, i64, P, P, P, P]
        L.orc_residual_moments.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, P, P, P, i64, i64, u64, P]
        L.orc_posterior_test.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, P, P, P, i64, i64, u64, dbl, dbl, P]
        L.orc_fmm_entries.argtypes = [P, i64, P, i64, P]
        L.orc_hadamard_apply.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, u64, P]
        L.orc_feistel.argtypes = [u64, ct.c_int, i64, i64]
        L.orc_feistel.restype = i64
        L.orc_bidiag_column.argtypes = [u64, i64, ct.c_int, i64, P, P, P]
        L.orc_sketch_bidiag.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, u64, P, P]
        L.orc_sketch_fourier.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, u64, P, P]
        L.orc_unit_root.argtypes = [i64, i64, P, P]
        L.orc_leverage_scores.argtypes = [P, i64, ct.c_int, P, P]
        L.orc_leverage_cur.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, P, P, ct.c_int, ct.c_int, u64, P, P, P,
                                       P]
        L.orc_unit_root.restype = None
        L.orc_cynical.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, ct.c_int, u64, P, P, P,
                                  P, P]
        L.orc_pinv_trunc.argtypes = [P, ct.c_int, ct.c_int, ct.c_int, P, P, P]
        L.orc_projective_select.argtypes = [P, i64, ct.c_int, ct.c_int, ct.c_int, dbl, i32, P, P, P, P, P]
        L.orc_projective_cur.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, ct.c_int, u64,
                                         dbl, i32, P, P, P, P]
        L.orc_draw_uniform.argtypes = [u64, u64, i64, i64, P]
        L.orc_uniform_cur.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, u64, P, P, P, P]
        L.orc_sketch_scores.argtypes = [P, i64, ct.c_int, ct.c_int, P, P]
        L.orc_dmm_ca.argtypes = [P, ct.c_int, i64, i64, i64, ct.c_int, ct.c_int, ct.c_int, ct.c_int, u64, P, P, P, P]
        for f in ("orc_draw_distinct", "orc_panel_lu", "orc_maxvol", "orc_sketch", "orc_qrp",
                  "orc_inverse", "orc_refine_inverse", "orc_ca_cur", "orc_residual", "orc_cur_adjoint", "orc_residual_moments",
                  "orc_fmm_entries", "orc_cynical", "orc_bidiag_column", "orc_sketch_bidiag",
                  "orc_hadamard_apply", "orc_pinv_trunc", "orc_projective_select", "orc_projective_cur",
                  "orc_draw_uniform", "orc_uniform_cur", "orc_sketch_fourier", "orc_leverage_scores",
                  "orc_leverage_cur", "orc_posterior_test", "orc_sketch_scores", "orc_dmm_ca"):
            getattr(L, f).restype = ct.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float64:
        return F64
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.uint16:  # bfloat16 bit patterns
        return BF16
    raise TypeError("oracle input must be float64, float32 or uint16 (bf16 bits)")


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def rng_u64(seed: int, stream: int, i: int) -> int:
    return int(lib().orc_rng_u64(seed, stream, i))


def draw_distinct(seed: int, stream: int, n: int, k: int) -> np.ndarray:
    out = np.zeros(k, np.int64)
    st = lib().orc_draw_distinct(seed, stream, n, k, _p(out))
    if st:
        raise ValueError("draw_distinct: status %d" % st)
    return out


def sign(seed: int, c: int) -> float:
    return float(lib().orc_sign(seed, c))


# --------------------------------------------------------------------------
# panel routines
# --------------------------------------------------------------------------
def panel_lu(P: np.ndarray):
    """Pivoted LU of a tall items x r panel: returns (status, piv, LU, rank, margin)."""
    P = np.ascontiguousarray(P, np.float64)
    items, r = P.shape
    piv = np.full(r, -1, np.int64)
    LU = np.zeros_like(P)
    rank = ct.c_int32(0)
    mm = ct.c_double(1.0)
    st = lib().orc_panel_lu(_p(P), items, r, _p(piv), _p(LU), ct.byref(rank), ct.byref(mm))
    return st, piv, LU, rank.value, mm.value


@dataclass
class MaxvolResult:
    status: int
    slots: np.ndarray
    B: np.ndarray
    swaps: int
    converged: int
    rank: int
    min_margin: float
    trace_idx: np.ndarray
    trace_val: np.ndarray


def maxvol(P: np.ndarray, delta: float = 0.01, max_swaps: int | None = None) -> MaxvolResult:
    """Dominant r x r submatrix of a tall panel (GEPP start + swaps)."""
    P = np.ascontiguousarray(P, np.float64)
    items, r = P.shape
    if max_swaps is None:
        max_swaps = 16 * r
    slots = np.full(r, -1, np.int64)
    B = np.zeros_like(P)
    tr_i = np.full(2 * max(max_swaps, 1), -1, np.int64)
    tr_v = np.zeros(max(max_swaps, 1))
    sw, cv, rk = ct.c_int32(0), ct.c_int32(0), ct.c_int32(0)
    mm = ct.c_double(1.0)
    st = lib().orc_maxvol(_p(P), items, r, delta, max_swaps, _p(slots), _p(B), _p(tr_i), _p(tr_v),
                          ct.byref(sw), ct.byref(cv), ct.byref(rk), ct.byref(mm))
    return MaxvolResult(st, slots, B, sw.value, cv.value, rk.value, mm.value,
                        tr_i[: 2 * sw.value].reshape(-1, 2), tr_v[: sw.value])


def sketch(A: np.ndarray, side: int, d: int, l: int, seed: int):
    """Abridged SRHT sketch: returns (Y items x l, samples)."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    items = n if side else m
    Y = np.zeros((items, l))
    smp = np.zeros(l, np.int64)
    st = lib().orc_sketch(_p(A), _dtype_code(A), m, n, n, side, d, l, seed, _p(Y), _p(smp))
    if st:
        raise ValueError("sketch: status %d" % st)
    return Y, smp


def unit_root(m: int, N: int):
    """(cos, sin) of 2 pi m / N by the oracle's fixed-order evaluation."""
    c, s = ct.c_double(0.0), ct.c_double(0.0)
    lib().orc_unit_root(m, N, ct.byref(c), ct.byref(s))
    return c.value, s.value


def sketch_fourier(A: np.ndarray, side: int, d: int, l: int, seed: int):
    """Abridged randomized Fourier sketch in real form: (Y items x 2l with
    Re y_q at q and Im y_q at l + q, sampled columns)."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    items = n if side else m
    Y = np.zeros((items, 2 * l))
    smp = np.zeros(l, np.int64)
    st = lib().orc_sketch_fourier(_p(A), _dtype_code(A), m, n, n, side, d, l, seed, _p(Y), _p(smp))
    if st:
        raise ValueError("sketch_fourier: status %d" % st)
    return Y, smp


def qrp(Z: np.ndarray, k: int):
    """Greedy Householder QRP over the items (rows) of Z: returns (status, piv, rank, margin)."""
    Z = np.array(Z, np.float64, order="C", copy=True)
    items, w = Z.shape
    piv = np.full(k, -1, np.int64)
    rank = ct.c_int32(0)
    mm = ct.c_double(1.0)
    st = lib().orc_qrp(_p(Z), items, w, k, _p(piv), ct.byref(rank), ct.byref(mm))
    return st, piv, rank.value, mm.value


def pinv_jacobi(G: np.ndarray, rtol: float = 1e-14):
    """Truncated pseudo-inverse by one-sided Jacobi SVD: (status, X, kept rank)."""
    G = np.ascontiguousarray(G, np.float64)
    r = G.shape[0]
    X = np.zeros_like(G)
    rk = ct.c_int(0)
    st = lib().orc_pinv_jacobi(_p(G), r, ct.c_double(rtol), _p(X), ct.byref(rk))
    return st, X, rk.value


def pinv_trunc(G: np.ndarray, r: int):
    """Pseudo-inverse of the rank-r SVD truncation of a k x l generator:
    (status, X (l x k), kept rank, log of the product of the kept sigmas)."""
    G = np.ascontiguousarray(G, np.float64)
    k, l = G.shape
    X = np.zeros((l, k))
    rk = ct.c_int(0)
    lv = ct.c_double(0.0)
    st = lib().orc_pinv_trunc(_p(G), k, l, r, _p(X), ct.byref(rk), ct.byref(lv))
    return st, X, rk.value, lv.value


def projective_select(P: np.ndarray, r: int, k: int, delta: float = 0.01, max_swaps: int = 0, full: bool = False):
    """k items (rows of P) chosen for r-projective volume: (status, items,
    rank reached, min margin), plus (swaps, converged) when full.  The
    default max_swaps = 0 stops after the greedy stages."""
    P = np.ascontiguousarray(P, np.float64)
    items, w = P.shape
    out = np.full(k, -1, np.int64)
    rank = ct.c_int32(0)
    mm = ct.c_double(1.0)
    sw = ct.c_int32(0)
    cv = ct.c_int32(0)
    st = lib().orc_projective_select(_p(P), items, w, r, k, ct.c_double(delta), max_swaps, _p(out), ct.byref(rank),
                                     ct.byref(mm), ct.byref(sw), ct.byref(cv))
    if full:
        return st, out, rank.value, mm.value, sw.value, cv.value
    return st, out, rank.value, mm.value


def nucleus(G: np.ndarray, refine_steps: int = 0):
    """The nucleus routine of the C-A driver: (status, U, log|det G|, kept rank)."""
    G = np.ascontiguousarray(G, np.float64)
    r = G.shape[0]
    U = np.zeros_like(G)
    ld = ct.c_double(0.0)
    rk = ct.c_int(0)
    st = lib().orc_nucleus(_p(G), r, refine_steps, _p(U), ct.byref(ld), ct.byref(rk))
    return st, U, ld.value, rk.value


def refine_inverse(G: np.ndarray, X0: np.ndarray, steps: int):
    """`steps` refinement steps X <- X + X (I - G X) from the start X0."""
    G = np.ascontiguousarray(G, np.float64)
    X = np.array(X0, dtype=np.float64, order="C", copy=True)
    st = lib().orc_refine_inverse(_p(G), G.shape[0], _p(X), steps)
    assert st == OK, st
    return X


def inverse(G: np.ndarray, refine_steps: int = 0):
    G = np.ascontiguousarray(G, np.float64)
    r = G.shape[0]
    U = np.zeros_like(G)
    ld = ct.c_double(0.0)
    st = lib().orc_inverse(_p(G), r, _p(U), refine_steps, ct.byref(ld))
    return st, U, ld.value


# --------------------------------------------------------------------------
# the whole path
# --------------------------------------------------------------------------
@dataclass
class CurResult:
    status: int
    I: np.ndarray
    J: np.ndarray
    U: np.ndarray
    sweeps_run: int
    swaps_total: int
    converged: int
    rank_found: int
    min_margin: float
    det_log_abs: float
    nucleus_rank: int = 0


def ca_cur(A: np.ndarray, r: int, sweeps: int, seed: int, delta: float = 0.01, max_swaps: int = -1,
           preprocess: int = 0, ah_depth: int = 3, ah_samples: int = 0, refine_steps: int = 0,
           init_cols=None) -> CurResult:
    """C-A CUR of a row-major matrix (float64, float32 or uint16 bf16 bits)."""
    A = np.ascontiguousarray(A)
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    m, n = A.shape
    o = _Opts()
    lib().orc_default_opts(ct.byref(o))
    o.delta = delta
    o.max_swaps = max_swaps
    o.preprocess = preprocess
    o.ah_depth = ah_depth
    o.ah_samples = ah_samples
    o.refine_steps = refine_steps
    ic = None
    if init_cols is not None:
        ic = np.ascontiguousarray(init_cols, np.int64)
        o.init_cols = ic.ctypes.data_as(ct.POINTER(ct.c_int64))
    I = np.full(r, -1, np.int64)
    J = np.full(r, -1, np.int64)
    U = np.zeros((r, r))
    info = _Info()
    st = lib().orc_ca_cur(_p(A), _dtype_code(A), m, n, n, r, sweeps, seed, ct.byref(o),
                          _p(I), _p(J), _p(U), ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def cynical(A: np.ndarray, r: int, k: int, loops: int, sweeps: int, seed: int, delta: float = 0.01,
            max_swaps: int = -1, refine_steps: int = 0) -> CurResult:
    """Cynical CUR on a k x k sketch (Tests 3, loops = 0) or after `loops` C-A
    loops at rank k (Tests 4, loops = 1); see orc_cynical."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    o = _Opts()
    lib().orc_default_opts(ct.byref(o))
    o.delta = delta
    o.max_swaps = max_swaps
    o.refine_steps = refine_steps
    I = np.full(r, -1, np.int64)
    J = np.full(r, -1, np.int64)
    U = np.zeros((r, r))
    info = _Info()
    st = lib().orc_cynical(_p(A), _dtype_code(A), m, n, n, r, k, loops, sweeps, seed, ct.byref(o),
                           _p(I), _p(J), _p(U), ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def projective_cur(A: np.ndarray, r: int, k: int, l: int, sweeps: int, seed: int, delta: float = 0.01,
                   max_swaps: int = -1) -> CurResult:
    """C-A with k x l generators of large r-projective volume and the
    canonical nucleus (see orc_projective_cur): I has k rows, J l columns,
    U is l x k."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.full(k, -1, np.int64)
    J = np.full(l, -1, np.int64)
    U = np.zeros((l, k))
    info = _Info()
    st = lib().orc_projective_cur(_p(A), _dtype_code(A), m, n, n, r, k, l, sweeps, seed, ct.c_double(delta),
                                  max_swaps, _p(I), _p(J), _p(U), ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def draw_uniform(seed: int, stream: int, n: int, k: int) -> np.ndarray:
    """k uniform draws from [0, n) with replacement, in draw order."""
    out = np.zeros(k, np.int64)
    st = lib().orc_draw_uniform(seed, stream, n, k, _p(out))
    if st:
        raise ValueError("draw_uniform: status %d" % st)
    return out


def uniform_cur(A: np.ndarray, r: int, k: int, l: int, seed: int) -> CurResult:
    """CUR with uniform leverage scores (see orc_uniform_cur): I has k rows,
    J l columns (sorted, duplicates kept), U is l x k."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.full(k, -1, np.int64)
    J = np.full(l, -1, np.int64)
    U = np.zeros((l, k))
    info = _Info()
    st = lib().orc_uniform_cur(_p(A), _dtype_code(A), m, n, n, r, k, l, seed, _p(I), _p(J), _p(U), ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def leverage_scores(P: np.ndarray):
    """(status, q, cdf): leverage scores of the rows of P (items x r) in its
    column space and their running sums."""
    P = np.ascontiguousarray(P, np.float64)
    items, r = P.shape
    q = np.zeros(items)
    cdf = np.zeros(items)
    st = lib().orc_leverage_scores(_p(P), items, r, _p(q), _p(cdf))
    return st, q, cdf


def leverage_cur(A: np.ndarray, I0, J0, k: int, l: int, seed: int) -> CurResult:
    """Refinement of the CUR of (I0, J0) by its leverage scores (see
    orc_leverage_cur): I has k rows, J l columns, U is l x k."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I0 = np.ascontiguousarray(I0, np.int64)
    J0 = np.ascontiguousarray(J0, np.int64)
    r = len(I0)
    I = np.full(k, -1, np.int64)
    J = np.full(l, -1, np.int64)
    U = np.zeros((l, k))
    info = _Info()
    st = lib().orc_leverage_cur(_p(A), _dtype_code(A), m, n, n, r, _p(I0), _p(J0), k, l, seed, _p(I), _p(J),
                                _p(U), ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def sketch_scores(P: np.ndarray, r: int):
    """(status, q, cdf): rank-r leverage scores of the rows of the sketch P
    (items x w), q_i = |row i of its r dominant left singular vectors|^2
    (summing to r), and their running sums."""
    P = np.ascontiguousarray(P, np.float64)
    items, w = P.shape
    q = np.zeros(items)
    cdf = np.zeros(items)
    st = lib().orc_sketch_scores(_p(P), items, w, r, _p(q), _p(cdf))
    return st, q, cdf


def dmm_ca(A: np.ndarray, r: int, k: int, l: int, iters: int, seed: int) -> CurResult:
    """C-A with DMM08 leverage-score sampling of every sketch (see
    orc_dmm_ca): I has k rows, J l columns (sorted, duplicates kept), U is
    l x k; min_margin is the smallest relative distance of a draw from the
    boundary of the item it picked."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.full(k, -1, np.int64)
    J = np.full(l, -1, np.int64)
    U = np.zeros((l, k))
    info = _Info()
    st = lib().orc_dmm_ca(_p(A), _dtype_code(A), m, n, n, r, k, l, iters, seed, _p(I), _p(J), _p(U),
                          ct.byref(info))
    return CurResult(st, I, J, U, info.sweeps_run, info.swaps_total, info.converged, info.rank_found,
                     info.min_margin, info.det_log_abs, info.nucleus_rank)


def residual(A: np.ndarray, I, J, U):
    """(||A - C U R||_F^2, ||A||_F^2) in FP64."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.ascontiguousarray(I, np.int64)
    J = np.ascontiguousarray(J, np.int64)
    U = np.ascontiguousarray(U, np.float64)
    e2, w2 = ct.c_double(0), ct.c_double(0)
    st = lib().orc_residual(_p(A), _dtype_code(A), m, n, n, len(I), _p(I), _p(J), _p(U), ct.byref(e2),
                            ct.byref(w2))
    if st:
        raise ValueError("residual: status %d" % st)
    return e2.value, w2.value


def residual_moments(A, I, J, U, q: int = 0, s: int = 0, seed: int = 0) -> np.ndarray:
    """[sum e, sum e^2, sum |e|, sum w^2] over all entries (q = s = 0) or a seeded q x s sample."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.ascontiguousarray(I, np.int64)
    J = np.ascontiguousarray(J, np.int64)
    U = np.ascontiguousarray(U, np.float64)
    out = np.zeros(4)
    st = lib().orc_residual_moments(_p(A), _dtype_code(A), m, n, n, len(I), _p(I), _p(J), _p(U), q, s, seed,
                                    _p(out))
    if st:
        raise ValueError("residual_moments: status %d" % st)
    return out


def posterior_test(A, I, J, U, q: int, s: int, seed: int, tau: float, z: float) -> dict:
    """The a-posteriori variance test on a seeded q x s sample of E = A - C U R
    (orc_posterior_test): K, mean, mean_abs, var, threshold, accept."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    I = np.ascontiguousarray(I, np.int64)
    J = np.ascontiguousarray(J, np.int64)
    U = np.ascontiguousarray(U, np.float64)
    out = np.zeros(6)
    st = lib().orc_posterior_test(_p(A), _dtype_code(A), m, n, n, len(I), _p(I), _p(J), _p(U), q, s, seed,
                                  ct.c_double(tau), ct.c_double(z), _p(out))
    if st:
        raise ValueError("posterior_test: status %d" % st)
    return {"K": int(out[0]), "mean": out[1], "mean_abs": out[2], "var": out[3], "threshold": out[4],
            "accept": bool(out[5])}


def rel_fro(A, I, J, U) -> float:
    e2, w2 = residual(A, I, J, U)
    return float(np.sqrt(e2 / w2)) if w2 > 0 else float(np.sqrt(e2))


def cur_adjoint(C, R, G, om_i, om_j, aval):
    """Loss and (dC, dR, dG) of sum over Omega of (a - C G^{-1} R)^2, all FP64."""
    C = np.ascontiguousarray(C, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    om_i = np.ascontiguousarray(om_i, np.int64)
    om_j = np.ascontiguousarray(om_j, np.int64)
    aval = np.ascontiguousarray(aval, np.float64)
    m, r = C.shape
    n = R.shape[1]
    dC = np.zeros_like(C)
    dR = np.zeros_like(R)
    dG = np.zeros_like(G)
    loss = ct.c_double(0)
    st = lib().orc_cur_adjoint(_p(C), _p(R), _p(G), m, n, r, _p(om_i), _p(om_j), _p(aval), len(om_i),
                               ct.byref(loss), _p(dC), _p(dR), _p(dG))
    if st:
        raise ValueError("cur_adjoint: status %d" % st)
    return loss.value, dC, dR, dG


def fmm_entries(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """K_ij = 1/|x_i - y_j| in FP64 for planar points x (m, 2) and y (n, 2)
    (far-field block of the Superfast Multipole discussion, Section "Some
    Implications and Extensions of Our Study")."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    m, n = x.shape[0], y.shape[0]
    K = np.empty((m, n), np.float64)
    st = lib().orc_fmm_entries(_p(x), m, _p(y), n, _p(K))
    if st != 0:
        raise ValueError("orc_fmm_entries: status %d" % st)
    return K


def feistel(seed: int, factor: int, N: int, x: int) -> int:
    """pi_factor(x): the random permutation of [0, N) of bidiagonal factor `factor` (1-based)."""
    return int(lib().orc_feistel(seed, factor, N, x))


def bidiag_column(seed: int, N: int, q: int, c: int):
    """Column c of G_q = B_1 P_1 ... B_q P_q as (positions, integer coefficients), ascending."""
    pos = np.zeros(64, np.int64)
    coef = np.zeros(64, np.int64)
    cnt = ct.c_int(0)
    st = lib().orc_bidiag_column(seed, N, q, c, _p(pos), _p(coef), ct.byref(cnt))
    if st != 0:
        raise ValueError("orc_bidiag_column: status %d" % st)
    return pos[:cnt.value].copy(), coef[:cnt.value].copy()


def sketch_bidiag(A: np.ndarray, side: int, q: int, l: int, seed: int):
    """Sketch with l sampled columns of the bidiagonal-product multiplier (see orc_sketch_bidiag)."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    items = n if side else m
    Y = np.zeros((items, l))
    smp = np.zeros(l, np.int64)
    st = lib().orc_sketch_bidiag(_p(A), _dtype_code(A), m, n, n, side, q, l, seed, _p(Y), _p(smp))
    if st != 0:
        raise ValueError("orc_sketch_bidiag: status %d" % st)
    return Y, smp


def hadamard_apply(A: np.ndarray, d: int, seed: int) -> np.ndarray:
    """W' = W D (H_{2^d} (x) I_s) for the pre-processed C-A (see orc_hadamard_apply); m x N."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    q2 = 1 << d
    N = q2 * ((n + q2 - 1) // q2)
    Wp = np.zeros((m, N))
    st = lib().orc_hadamard_apply(_p(A), _dtype_code(A), m, n, n, d, seed, _p(Wp))
    if st != 0:
        raise ValueError("orc_hadamard_apply: status %d" % st)
    return Wp
