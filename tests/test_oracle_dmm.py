"""Pins of the oracle's C-A with DMM08 leverage-score sampling of every
sketch (Section "Testing C-A acceleration of the algorithms of DMM08",
Tables 7 and 8; Algorithm algcurlevsc, Algorithm algsmplex, eq. eqlevsc).

The rank-r sketch scores are checked against LAPACK's SVD, against their
trace identity, against the exact leverage scores of the oracle's Cholesky
route when the sketch has exactly r columns, and against the column space
of an exactly rank-r sketch; the whole iteration against an independent
numpy evaluation of the same chain of steps (LAPACK SVD for the scores and
the nucleus, numpy's sorted search for the draws), and against exact
recovery of rank-r inputs."""
import numpy as np
import pytest

import oracle


def spread_sketch(items, w, seed, decay=3.0):
    """items x w with singular values 10^0 .. 10^-decay (a clear gap at every r)."""
    g = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(g.standard_normal((items, w)))
    Q2, _ = np.linalg.qr(g.standard_normal((w, w)))
    return (Q1 * np.logspace(0, -decay, w)) @ Q2.T


def lapack_scores(P, r):
    Us, s, _ = np.linalg.svd(P, full_matrices=False)
    kept = min(r, int((s * s > 1e-13 * s[0] ** 2).sum()))
    return (Us[:, :kept] ** 2).sum(axis=1)


@pytest.mark.parametrize("items,w,r", [(200, 24, 6), (90, 10, 10), (64, 40, 1), (500, 64, 16)])
def test_scores_match_the_svd(items, w, r):
    P = spread_sketch(items, w, items + w + r)
    st, q, cdf = oracle.sketch_scores(P, r)
    assert st == 0
    assert np.allclose(q, lapack_scores(P, r), atol=1e-12)
    assert cdf[-1] == pytest.approx(r, rel=1e-12)                  # each singular vector has unit norm
    assert np.allclose(np.cumsum(q), cdf, rtol=0, atol=1e-12)


def test_scores_are_invariant_under_a_right_rotation():
    P = spread_sketch(150, 20, 3)
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((20, 20)))
    q0 = oracle.sketch_scores(P, 5)[1]
    q1 = oracle.sketch_scores(P @ Q, 5)[1]
    assert np.allclose(q0, q1, atol=1e-12)


def test_full_width_scores_are_the_exact_leverage_scores():
    # w = r: the dominant subspace is the whole column space
    P = np.random.default_rng(8).standard_normal((120, 7))
    st, q, _ = oracle.sketch_scores(P, 7)
    st2, q2, _ = oracle.leverage_scores(P)
    assert st == st2 == 0
    assert np.allclose(q, q2, atol=1e-12)


def test_rank_r_sketch_scores_are_those_of_its_column_space():
    g = np.random.default_rng(9)
    X = g.standard_normal((300, 4))
    P = X @ g.standard_normal((4, 16))
    Qx, _ = np.linalg.qr(X)
    assert np.allclose(oracle.sketch_scores(P, 4)[1], (Qx * Qx).sum(axis=1), atol=1e-11)


def test_rank_deficient_sketch_gives_the_scores_of_its_whole_range():
    # rank 1 < r = 2: the scores of the one dominant direction (summing to 1)
    g = np.random.default_rng(2)
    x = g.standard_normal(30)
    P = np.zeros((30, 6))
    P[:, 0] = x
    P[:, 3] = 2.0 * x
    st, q, cdf = oracle.sketch_scores(P, 2)
    assert st == 0
    assert np.allclose(q, x * x / (x @ x), atol=1e-14)
    assert oracle.sketch_scores(np.zeros((30, 6)), 2)[0] == oracle.ESINGULAR


def numpy_dmm_ca(A, r, k, l, iters, seed):
    """The same chain of steps evaluated with LAPACK and numpy only."""
    m, n = A.shape

    def draws(q, cnt, stream):
        cdf = np.cumsum(q)
        S = cdf[-1]
        u = np.array([(oracle.rng_u64(seed, stream, t) >> 11) * 2.0 ** -53 for t in range(cnt)])
        idx = np.searchsorted(cdf, u * S, side="right")
        order = np.argsort(idx, kind="stable")
        idx = idx[order]
        return idx, 1.0 / np.sqrt(cnt * q[idx] / S)

    J = np.sort(oracle.draw_uniform(seed, 8, n, l))
    d = np.full(l, np.sqrt(n / l))
    for t in range(iters):
        I, dbar = draws(lapack_scores(A[:, J] * d, r), k, 16 + 2 * t)
        J, d = draws(lapack_scores((dbar[:, None] * A[I, :]).T, r), l, 17 + 2 * t)
    M = dbar[:, None] * A[np.ix_(I, J)] * d
    Us, s, Vt = np.linalg.svd(M)
    Mp = (Vt[:r].T / s[:r]) @ Us[:, :r].T
    return I, J, d[:, None] * Mp * dbar


@pytest.mark.parametrize("m,n,r,k,l,iters", [(120, 90, 4, 8, 12, 3), (200, 260, 6, 24, 24, 8), (80, 80, 5, 5, 5, 2)])
def test_iteration_matches_an_independent_evaluation(m, n, r, k, l, iters):
    g = np.random.default_rng(m + n + k)
    A = (g.standard_normal((m, r)) * np.logspace(0, -1, r)) @ g.standard_normal((r, n))
    A += 1e-4 * g.standard_normal((m, n))
    o = oracle.dmm_ca(A, r, k, l, iters, 31)
    assert o.status == 0 and o.sweeps_run == iters
    assert o.min_margin > 1e-9          # no draw within rounding of a boundary
    I, J, U = numpy_dmm_ca(A, r, k, l, iters, 31)
    assert np.array_equal(o.I, I)
    assert np.array_equal(o.J, J)
    assert np.allclose(o.U, U, rtol=1e-8, atol=1e-10 * np.abs(U).max())


@pytest.mark.parametrize("k", [6, 12, 24])
def test_exact_rank_r_inputs_are_reproduced(k):
    g = np.random.default_rng(k)
    A = g.standard_normal((150, 6)) @ g.standard_normal((6, 170))
    o = oracle.dmm_ca(A, 6, k, k, 8, 2)
    assert o.status == 0
    if k > 6:
        assert o.nucleus_rank == 6
    if o.nucleus_rank == 6:
        assert oracle.rel_fro(A, o.I, o.J, o.U) < 1e-10


def test_oversampling_reaches_the_noise_level():
    # the pattern of Tables 7 and 8: k = l = 4r is far more accurate than k = l = r
    g = np.random.default_rng(12)
    A = g.standard_normal((400, 8)) @ g.standard_normal((8, 400)) + 1e-6 * g.standard_normal((400, 400))
    errs = {}
    for k in (8, 32):
        e = [oracle.rel_fro(A, o.I, o.J, o.U) for o in (oracle.dmm_ca(A, 8, k, k, 8, s) for s in range(6))]
        errs[k] = np.median(e)
    assert errs[32] < 1e-5
    assert errs[32] < errs[8]


def test_invalid_arguments():
    A = np.ones((20, 20))
    assert oracle.dmm_ca(A, 4, 3, 8, 8, 1).status == oracle.EINVAL      # k < r
    assert oracle.dmm_ca(A, 4, 8, 8, 0, 1).status == oracle.EINVAL      # no iteration
    B = np.random.default_rng(0).standard_normal((20, 20))
    B[:, :] = np.where(np.arange(20)[None, :] == 11, np.nan, B)       # a whole column: every row sketch reads it
    assert oracle.dmm_ca(B, 4, 8, 20, 2, 1).status == oracle.EINVAL
