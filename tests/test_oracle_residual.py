"""Pins of the oracle's residual moments (the a-posteriori error check of Section 4).

The moments are [sum e, sum e^2, sum |e|, sum w^2] over the entries of
E = W - W[:, J] U W[I, :] that are used: every entry, or the q x s submatrix
on seeded random rows (stream 3) and columns (stream 4).
"""
import itertools

import numpy as np
import pytest

from paper_1710_07946_amd import workloads


def _sets(g, m, n, r):
    return np.sort(g.choice(m, r, replace=False)), np.sort(g.choice(n, r, replace=False))


def test_zero_nucleus_gives_plain_sums(orc):
    # With U = 0 the residual is W itself, so the moments are numpy's plain sums,
    # over all entries and over the drawn sample.
    g = np.random.default_rng(1)
    m, n, r = 37, 29, 3
    A = g.standard_normal((m, n))
    I, J = _sets(g, m, n, r)
    U = np.zeros((r, r))
    full = orc.residual_moments(A, I, J, U)
    assert np.allclose(full, [A.sum(), (A ** 2).sum(), np.abs(A).sum(), (A ** 2).sum()], rtol=1e-13)
    q, s, seed = 7, 5, 77
    rows = orc.draw_distinct(seed, 3, m, q)
    cols = orc.draw_distinct(seed, 4, n, s)
    S = A[np.ix_(rows, cols)]
    samp = orc.residual_moments(A, I, J, U, q, s, seed)
    assert np.allclose(samp, [S.sum(), (S ** 2).sum(), np.abs(S).sum(), (S ** 2).sum()], rtol=1e-13)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_entries_are_schur_determinant_ratios(orc, r):
    # E = W - W[:, J] W[I, J]^-1 W[I, :] is the Schur complement of W[I, J]:
    # E_kl = det W[I + k, J + l] / det W[I, J] (zero when k in I or l in J).
    g = np.random.default_rng(10 + r)
    m, n = 9, 8
    A = g.standard_normal((m, n))
    I, J = _sets(g, m, n, r)
    U = np.linalg.inv(A[np.ix_(I, J)])
    d0 = np.linalg.det(A[np.ix_(I, J)])
    E = np.zeros((m, n))
    for k, l in itertools.product(range(m), range(n)):
        if k in I or l in J:
            continue
        E[k, l] = np.linalg.det(A[np.ix_(list(I) + [k], list(J) + [l])]) / d0
    mom = orc.residual_moments(A, I, J, U)
    assert np.isclose(mom[0], E.sum(), rtol=1e-10, atol=1e-12)
    assert np.isclose(mom[1], (E ** 2).sum(), rtol=1e-10)
    assert np.isclose(mom[2], np.abs(E).sum(), rtol=1e-10)
    assert np.isclose(mom[3], (A ** 2).sum(), rtol=1e-13)


def test_full_row_set_interpolates_everything(orc):
    # m = r: the generator is W[:, J] itself, C U R = W[:, J] W[:, J]^-1 W = W
    # for any matrix, so the residual vanishes to round-off.
    g = np.random.default_rng(3)
    r, n = 5, 40
    A = g.standard_normal((r, n))
    J = np.sort(g.choice(n, r, replace=False))
    U = np.linalg.inv(A[:, J])
    mom = orc.residual_moments(A, np.arange(r), J, U)
    assert mom[1] <= 1e-26 * mom[3]


def test_exact_rank_residual_vanishes(orc):
    A = workloads.orthogonal_lowrank(200, 150, 6, noise=0.0)
    res = orc.ca_cur(A, 6, 3, 5)
    mom = orc.residual_moments(A, res.I, res.J, res.U)
    assert mom[1] <= 1e-24 * mom[3]
    assert np.isclose(mom[3], np.linalg.norm(A) ** 2, rtol=1e-13)


def test_sample_of_everything_equals_full(orc):
    # q = m, s = n draws every row and column once, in some order
    g = np.random.default_rng(4)
    m, n, r = 50, 40, 4
    A = g.standard_normal((m, n))
    I, J = _sets(g, m, n, r)
    U = np.linalg.inv(A[np.ix_(I, J)])
    assert np.allclose(orc.residual_moments(A, I, J, U, m, n, 9), orc.residual_moments(A, I, J, U), rtol=1e-12)


def test_sampled_estimate_is_unbiased(orc):
    # Section 4: the sampled mean square, scaled by mn / (qs), estimates
    # ||E||_F^2; averaged over seeds it approaches the full value.
    A = workloads.orthogonal_lowrank(120, 100, 5, noise=1e-3)
    res = orc.ca_cur(A, 5, 3, 1)
    full = orc.residual_moments(A, res.I, res.J, res.U)[1]
    est = [orc.residual_moments(A, res.I, res.J, res.U, 20, 20, s)[1] * (120 * 100) / 400 for s in range(300)]
    assert abs(np.mean(est) / full - 1) < 0.05


def test_invalid_sample_sizes(orc):
    A = np.ones((8, 8))
    I = J = np.arange(2)
    U = np.eye(2)
    for q, s in ((1, 0), (0, 1), (9, 2), (2, 9), (-1, -1)):
        with pytest.raises(ValueError):
            orc.residual_moments(A, I, J, U, q, s, 0)
