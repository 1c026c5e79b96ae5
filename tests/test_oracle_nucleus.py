"""Pins of the oracle's nucleus: the LU inverse, and the truncated
pseudo-inverse (one-sided Jacobi SVD) that replaces it for singular or badly
conditioned generators (Algorithm algcnnncl, Section 3)."""
import numpy as np
import pytest


@pytest.mark.parametrize("r", [1, 2, 5, 7, 33, 64])
def test_pinv_of_nonsingular_is_inverse(orc, r):
    G = np.random.default_rng(r).standard_normal((r, r))
    st, X, rk = orc.pinv_jacobi(G)
    assert st == 0 and rk == r
    Ginv = np.linalg.inv(G)
    assert np.max(np.abs(X - Ginv)) <= 1e-11 * np.max(np.abs(Ginv))


@pytest.mark.parametrize("r,k", [(2, 1), (6, 3), (17, 16), (40, 5)])
def test_pinv_of_rank_deficient_matches_lapack(orc, r, k):
    g = np.random.default_rng(100 + r)
    G = g.standard_normal((r, k)) @ g.standard_normal((k, r))
    st, X, rk = orc.pinv_jacobi(G)
    assert st == 0 and rk == k
    P = np.linalg.pinv(G, rcond=1e-14)
    assert np.max(np.abs(X - P)) <= 1e-10 * np.max(np.abs(P))
    # the four Penrose conditions
    sc = np.max(np.abs(G))
    assert np.max(np.abs(G @ X @ G - G)) <= 1e-11 * sc
    assert np.max(np.abs(X @ G @ X - X)) <= 1e-11 * np.max(np.abs(X))
    assert np.allclose(G @ X, (G @ X).T, atol=1e-11)
    assert np.allclose(X @ G, (X @ G).T, atol=1e-11)


def test_pinv_of_zero_matrix(orc):
    st, X, rk = orc.pinv_jacobi(np.zeros((4, 4)))
    assert st == 0 and rk == 0 and not X.any()


def test_nucleus_is_the_lu_inverse_when_well_conditioned(orc):
    G = np.random.default_rng(3).standard_normal((12, 12))
    st, U, ld, rk = orc.nucleus(G)
    st2, Uinv, ld2 = orc.inverse(G)
    assert st == 0 and rk == 12 and np.array_equal(U, Uinv) and ld == ld2


def test_nucleus_falls_back_on_exact_singularity(orc):
    g = np.random.default_rng(4)
    G = g.standard_normal((8, 5)) @ g.standard_normal((5, 8))
    G[:, 7] = G[:, 0]  # keep it exactly singular whatever the rounding
    st, U, ld, rk = orc.nucleus(G)
    assert st == 0 and rk < 8 and ld == -np.inf
    assert np.max(np.abs(U - np.linalg.pinv(G, rcond=1e-14))) <= 1e-9 * np.max(np.abs(U))


def test_nucleus_falls_back_on_bad_conditioning(orc):
    # singular values 1 .. 1e-16: the pivot spread exceeds 1e14, the smallest
    # singular value is truncated (below 1e-14 of the largest)
    g = np.random.default_rng(5)
    Q1, _ = np.linalg.qr(g.standard_normal((6, 6)))
    Q2, _ = np.linalg.qr(g.standard_normal((6, 6)))
    s = np.array([1.0, 0.5, 0.3, 0.2, 0.1, 1e-16])
    G = (Q1 * s) @ Q2.T
    st, U, ld, rk = orc.nucleus(G)
    assert st == 0 and rk == 5
    P = np.linalg.pinv(G, rcond=1e-14)
    assert np.max(np.abs(U - P)) <= 1e-9 * np.max(np.abs(P))


def test_ca_cur_reports_truncated_nucleus(orc):
    # an exactly rank-(r-1) matrix plus rounding-level noise: the panels keep
    # full rank, the final generator is numerically singular
    g = np.random.default_rng(6)
    m, n, r = 120, 100, 6
    A = g.standard_normal((m, r - 1)) @ g.standard_normal((r - 1, n)) + 1e-15 * g.standard_normal((m, n))
    res = orc.ca_cur(A, r, 2, 11)
    assert res.status == 0 and res.nucleus_rank == r - 1
    # C U R with the truncated nucleus reproduces the rank-(r-1) part
    rec = A[:, res.J] @ res.U @ A[res.I]
    assert np.linalg.norm(rec - A) <= 1e-8 * np.linalg.norm(A)
