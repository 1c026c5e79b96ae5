"""Pins of the oracle's CUR adjoint: finite differences and the least-squares special case."""
import numpy as np
import pytest

from paper_1710_07946_amd import workloads


def _problem(seed, m=40, n=36, r=4, frac=0.3):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 1e-2 * g.standard_normal((m, n))
    I = np.sort(g.choice(m, r, replace=False))
    J = np.sort(g.choice(n, r, replace=False))
    oi, oj = workloads.sample_omega(m, n, int(frac * m * n), seed + 1)
    return A, A[:, J].copy(), A[I].copy(), A[np.ix_(I, J)].copy(), oi, oj


@pytest.mark.parametrize("seed", range(4))
def test_adjoint_matches_central_differences(orc, seed):
    A, C, R, G, oi, oj = _problem(seed)
    aval = A[oi, oj]
    loss, dC, dR, dG = orc.cur_adjoint(C, R, G, oi, oj, aval)
    g = np.random.default_rng(seed + 50)

    def fd(name, X, idx, h):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        args_p = {"C": C, "R": R, "G": G}
        args_m = dict(args_p)
        args_p[name], args_m[name] = Xp, Xm
        lp = orc.cur_adjoint(args_p["C"], args_p["R"], args_p["G"], oi, oj, aval)[0]
        lm = orc.cur_adjoint(args_m["C"], args_m["R"], args_m["G"], oi, oj, aval)[0]
        return (lp - lm) / (2 * h)

    for name, X, dX in (("C", C, dC), ("R", R, dR), ("G", G, dG)):
        for _ in range(8):
            idx = tuple(int(g.integers(0, s)) for s in X.shape)
            # central differences at h = 1e-3 and h/2, Richardson-combined to
            # cancel the h^2 term (the loss is quadratic in C and R, so there
            # the plain central difference is already exact up to rounding)
            f1, f2 = fd(name, X, idx, 1e-3), fd(name, X, idx, 5e-4)
            est = (4 * f2 - f1) / 3
            assert abs(est - dX[idx]) <= 1e-6 * max(1.0, abs(est)), (name, idx, est, dX[idx])


def test_adjoint_reduces_to_least_squares_gradient(orc):
    # G = I and Omega = every entry: L = ||A - C R||_F^2 with the textbook
    # gradients dC = -2 (A - C R) R^T, dR = -2 C^T (A - C R).
    g = np.random.default_rng(9)
    m, n, r = 12, 10, 3
    A = g.standard_normal((m, n))
    C = g.standard_normal((m, r))
    R = g.standard_normal((r, n))
    oi, oj = np.divmod(np.arange(m * n), n)
    loss, dC, dR, dG = orc.cur_adjoint(C, R, np.eye(r), oi, oj, A[oi, oj])
    E = A - C @ R
    assert np.isclose(loss, (E ** 2).sum(), rtol=1e-13)
    assert np.allclose(dC, -2 * E @ R.T, atol=1e-12)
    assert np.allclose(dR, -2 * C.T @ E, atol=1e-12)
    # dG = -G^-T dZ Z^T with Z = R and dZ = dR at G = I
    assert np.allclose(dG, -dR @ R.T, atol=1e-12)


def test_adjoint_zero_at_exact_fit(orc):
    g = np.random.default_rng(10)
    A = g.standard_normal((20, 3)) @ g.standard_normal((3, 18))
    I, J = np.array([1, 5, 9]), np.array([0, 7, 11])
    oi, oj = workloads.sample_omega(20, 18, 100, 3)
    loss, dC, dR, dG = orc.cur_adjoint(A[:, J], A[I], A[np.ix_(I, J)], oi, oj, A[oi, oj])
    assert loss < 1e-20
    assert np.abs(dC).max() < 1e-9 and np.abs(dR).max() < 1e-9 and np.abs(dG).max() < 1e-9
