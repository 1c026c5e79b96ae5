"""Pins of the oracle's a-posteriori variance test (Section 4, the subsection
on LRA of a matrix filled with i.i.d. values of a single variable): the
entries of a random q x s submatrix of E = W - C U R are taken as observed
values of one Gaussian variable, and a customary test for its variance
decides whether the LRA meets a tolerance tau.

With U = 0 the error matrix is W itself, so a W of i.i.d. Gaussian entries
with known mean and variance pins the statistics (central limit bounds), a
constant W pins them exactly, and repeated seeds pin the test's level.
"""
import math

import numpy as np
import pytest

import oracle


def zero_cur(A, r=2):
    """A CUR with U = 0: C U R = 0 and E = A."""
    return np.arange(r), np.arange(r), np.zeros((r, r))


def test_constant_error_has_zero_variance():
    A = np.full((40, 30), -0.375)
    I, J, U = zero_cur(A)
    t = oracle.posterior_test(A, I, J, U, 10, 12, 3, tau=1.0, z=2.0)
    assert t["K"] == 120
    assert t["mean"] == -0.375 and t["mean_abs"] == 0.375 and t["var"] == 0.0
    assert t["accept"]


@pytest.mark.parametrize("mu,sigma", [(0.0, 1e-3), (0.5, 2.0), (-3e-7, 1e-7)])
def test_gaussian_statistics_follow_the_central_limit(mu, sigma):
    g = np.random.default_rng(11)
    A = mu + sigma * g.standard_normal((1000, 900))
    I, J, U = zero_cur(A)
    t = oracle.posterior_test(A, I, J, U, 200, 150, 5, tau=sigma, z=0.0)
    K = t["K"]
    assert K == 30000
    assert abs(t["mean"] - mu) <= 5 * sigma / math.sqrt(K)
    assert abs(t["var"] - sigma ** 2) <= 5 * sigma ** 2 * math.sqrt(2.0 / K)
    if mu == 0.0:  # E|g| = sigma sqrt(2 / pi) for a centred Gaussian
        assert abs(t["mean_abs"] - sigma * math.sqrt(2 / math.pi)) <= 5 * sigma / math.sqrt(K)


def test_sample_is_the_drawn_submatrix():
    """The statistics are those of the entries at the drawn rows and columns
    (streams 3 and 4 of the seed), whatever the rest of W holds."""
    g = np.random.default_rng(12)
    A = g.standard_normal((60, 50))
    I, J, U = zero_cur(A)
    q, s, seed = 7, 9, 21
    rows = oracle.draw_distinct(seed, 3, 60, q)
    cols = oracle.draw_distinct(seed, 4, 50, s)
    B = A.copy()
    mask = np.ones_like(B, bool)
    mask[np.ix_(rows, cols)] = False
    B[mask] = 1e6  # outside the sample
    t1 = oracle.posterior_test(A, I, J, U, q, s, seed, 1.0, 1.0)
    t2 = oracle.posterior_test(B, I, J, U, q, s, seed, 1.0, 1.0)
    assert t1 == t2
    sub = A[np.ix_(rows, cols)]
    assert abs(t1["mean"] - sub.mean()) <= 1e-15 and abs(t1["var"] - sub.var()) <= 1e-14


def test_error_of_an_exact_cur_is_its_residual():
    """A real CUR: the sampled errors are the entries of W - C U R."""
    g = np.random.default_rng(13)
    A = g.standard_normal((80, 6)) @ g.standard_normal((6, 70)) + 1e-4 * g.standard_normal((80, 70))
    res = oracle.ca_cur(A, 6, 2, 7)
    t = oracle.posterior_test(A, res.I, res.J, res.U, 20, 30, 9, tau=1e-3, z=2.0)
    E = A - A[:, res.J] @ res.U @ A[res.I]
    rows = oracle.draw_distinct(9, 3, 80, 20)
    cols = oracle.draw_distinct(9, 4, 70, 30)
    sub = E[np.ix_(rows, cols)]
    assert abs(t["var"] - sub.var()) <= 1e-12 * sub.var()
    assert t["accept"]  # errors of order 1e-4, well inside tau = 1e-3
    assert not oracle.posterior_test(A, res.I, res.J, res.U, 20, 30, 9, tau=1e-5, z=2.0)["accept"]


def test_level_of_the_test():
    """At sigma = tau the test accepts with probability about Phi(-z); well
    inside the tolerance it always accepts, well outside never."""
    g = np.random.default_rng(14)
    z = 1.6449  # one-sided 5 %
    runs, acc = 400, 0
    for k in range(runs):
        A = g.standard_normal((30, 30))
        I, J, U = zero_cur(A)
        acc += oracle.posterior_test(A, I, J, U, 20, 20, 100 + k, tau=1.0, z=z)["accept"]
    p = 0.05
    assert abs(acc / runs - p) <= 4 * math.sqrt(p * (1 - p) / runs) + 0.01
    A = 0.8 * g.standard_normal((100, 100))
    I, J, U = zero_cur(A)
    assert oracle.posterior_test(A, I, J, U, 100, 100, 1, tau=1.0, z=z)["accept"]
    assert not oracle.posterior_test(A, I, J, U, 100, 100, 1, tau=0.75, z=z)["accept"]


def test_invalid_arguments():
    A = np.ones((10, 10))
    I, J, U = zero_cur(A)
    for kw in ({"q": 0, "s": 3}, {"q": 11, "s": 3}, {"q": 1, "s": 1}):
        with pytest.raises(ValueError):
            oracle.posterior_test(A, I, J, U, kw["q"], kw["s"], 1, 1.0, 1.0)
    with pytest.raises(ValueError):
        oracle.posterior_test(A, I, J, U, 3, 3, 1, 0.0, 1.0)
