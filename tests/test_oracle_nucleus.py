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


# ---------------------------------------------------------------------------
# Iterative refinement of the nucleus inverse, X <- X + X (I - G X) (the
# refined nucleus of Section 3, Algorithm algcnnncl with k = l = r).  With
# E = I - G X one step leaves I - G (X + X E) = E^2 exactly, so the pins
# below drive the oracle's step from a deliberately perturbed start: a wrong
# sign (X - X E leaves 2E - E^2), a transposed operand or the other residual
# (I - X G) all break the matrix identity, not just a norm.
# ---------------------------------------------------------------------------
def _conditioned(r, cond, seed):
    """G = Q1 diag(s) Q2^T with singular values spread log-uniformly from 1 down to 1/cond."""
    g = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(g.standard_normal((r, r)))
    Q2, _ = np.linalg.qr(g.standard_normal((r, r)))
    s = np.logspace(0.0, -np.log10(cond), r)
    return (Q1 * s) @ Q2.T


def _exact_inverse(G):
    """Inverse of the FP64 matrix G in exact rational arithmetic (Gauss-Jordan)."""
    from fractions import Fraction
    r = G.shape[0]
    M = [[Fraction(float(G[i, j])) for j in range(r)] + [Fraction(int(i == j)) for j in range(r)]
         for i in range(r)]
    for k in range(r):
        p = max(range(k, r), key=lambda i: abs(M[i][k]))
        M[k], M[p] = M[p], M[k]
        piv = M[k][k]
        M[k] = [x / piv for x in M[k]]
        for i in range(r):
            if i != k and M[i][k] != 0:
                f = M[i][k]
                M[i] = [a - f * b for a, b in zip(M[i], M[k])]
    return np.array([[float(M[i][r + j]) for j in range(r)] for i in range(r)])


@pytest.mark.parametrize("r,cond", [(5, 10.0), (12, 1e3), (33, 1e2)])
def test_refinement_squares_the_residual(orc, r, cond):
    G = _conditioned(r, cond, 40 + r)
    Ginv = np.linalg.inv(G)
    P = np.random.default_rng(50 + r).standard_normal((r, r))
    # a start whose residual has norm about 1e-2 (E0 = -G D for the perturbation D)
    X0 = Ginv + (1e-2 / cond) * np.linalg.norm(Ginv, 2) * P / np.linalg.norm(P, 2)
    E0 = np.eye(r) - G @ X0
    assert 1e-4 < np.linalg.norm(E0, 2) < 1e-1
    X1 = orc.refine_inverse(G, X0, 1)
    E1 = np.eye(r) - G @ X1
    # the identity E1 = E0^2, up to the rounding of forming X1 and E1
    rnd = 64 * r * np.finfo(float).eps * np.linalg.norm(G, 2) * np.linalg.norm(X1, 2)
    assert np.linalg.norm(E1 - E0 @ E0, 2) <= 1e-6 * np.linalg.norm(E0, 2) ** 2 + rnd
    # and it is the residual that shrinks: quadratically down to the rounding floor
    norms = [np.linalg.norm(E0, 2)]
    X = X0
    for _ in range(4):
        X = orc.refine_inverse(G, X, 1)
        norms.append(np.linalg.norm(np.eye(r) - G @ X, 2))
    for a, b in zip(norms, norms[1:]):
        assert b <= 1.01 * a * a + rnd
    assert norms[-1] <= rnd


def test_refinement_steps_compose(orc):
    # two calls of one step equal one call of two steps, bit for bit
    G = _conditioned(9, 1e4, 7)
    X0 = np.linalg.inv(G) * (1.0 + 1e-4)
    a = orc.refine_inverse(G, orc.refine_inverse(G, X0, 1), 1)
    b = orc.refine_inverse(G, X0, 2)
    assert np.array_equal(a, b)
    # zero steps leave the start untouched
    assert np.array_equal(orc.refine_inverse(G, X0, 0), X0)


def test_refinement_of_a_scaled_inverse_is_newton(orc):
    # X0 = c G^{-1} gives E0 = (1 - c) I, so every step maps c -> c (2 - c)
    # (the scalar Newton iteration for 1/x at x = 1): 0.5 -> 0.75 -> 0.9375
    G = _conditioned(6, 10.0, 8)
    Ginv = _exact_inverse(G)
    X = orc.refine_inverse(G, 0.5 * Ginv, 2)
    assert np.max(np.abs(X - 0.9375 * Ginv)) <= 1e-12 * np.max(np.abs(Ginv))


@pytest.mark.parametrize("cond", [1e8, 1e10])
def test_refined_inverse_of_ill_conditioned_generator(orc, cond):
    # the LU inverse with two refinement steps (the nucleus of the tall
    # rank-64 workload) against the exact inverse of the same FP64 numbers
    r = 8
    G = _conditioned(r, cond, int(np.log10(cond)))
    Xe = _exact_inverse(G)
    eps = np.finfo(float).eps
    st, X2, _ = orc.inverse(G, refine_steps=2)
    assert st == 0
    bound = 10 * r * cond * eps
    assert np.linalg.norm(X2 - Xe, 2) <= bound * np.linalg.norm(Xe, 2)
    assert np.linalg.norm(X2 - np.linalg.inv(G), 2) <= bound * np.linalg.norm(Xe, 2)
    # refinement does not leave a larger residual than the plain LU inverse
    st, X0, _ = orc.inverse(G, refine_steps=0)
    res = lambda X: np.linalg.norm(np.eye(r) - G @ X, 2)
    assert res(X2) <= 2 * res(X0) + 4 * r * eps * cond
    # and from a start far from the inverse, two steps reach the rounding floor
    P = np.random.default_rng(9).standard_normal((r, r))
    Xs = Xe + 1e-5 * np.linalg.norm(Xe, 2) * P / np.linalg.norm(P, 2)
    e0 = res(Xs)
    assert e0 > 1e-3 * cond / 1e8
    Xr = orc.refine_inverse(G, Xs, 2)
    assert res(Xr) <= max(1.1 * e0 ** 4, 0.0) + 64 * r * eps * cond
