"""Pins of the oracle's pre-processed matrix W' = W D (H_{2^d} (x) I_s) (Tests 2
with abridged randomized Hadamard pre-processing, Section 13; Appendix B):
the full-depth case is SciPy's Hadamard matrix, the general case the
Kronecker product, depth 0 the sign flips, and C-A on W' yields an LRA of W
through M M^T = 2^d I."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle


def signs(seed, n):
    return np.array([oracle.sign(seed, c) for c in range(n)])


def test_full_depth_is_the_hadamard_transform():
    g = np.random.default_rng(1)
    A = g.standard_normal((7, 32))
    Wp = oracle.hadamard_apply(A, 5, 9)
    assert np.abs(Wp - (A * signs(9, 32)) @ sl.hadamard(32)).max() <= 1e-12


def test_depth_zero_flips_signs():
    g = np.random.default_rng(2)
    A = g.standard_normal((5, 13))
    assert np.array_equal(oracle.hadamard_apply(A, 0, 4), A * signs(4, 13))


@pytest.mark.parametrize("n,d", [(24, 3), (30, 2), (37, 3), (64, 1)])
def test_kronecker_structure_with_padding(n, d):
    g = np.random.default_rng(n)
    A = g.standard_normal((6, n))
    q2 = 1 << d
    s = -(-n // q2)
    N = q2 * s
    Ap = np.zeros((6, N))
    Ap[:, :n] = A * signs(11, n)
    ref = Ap @ np.kron(sl.hadamard(q2), np.eye(s))
    Wp = oracle.hadamard_apply(A, d, 11)
    assert Wp.shape == (6, N)
    assert np.abs(Wp - ref).max() <= 1e-12


@pytest.mark.parametrize("d", [0, 2, 3])
def test_ca_on_the_preprocessed_matrix_gives_an_lra_of_w(d):
    # Theorem thdcmp on W' (rank r like W), then W = W' M^T / 2^d
    m, n, r, seed = 120, 90, 5, 3
    g = np.random.default_rng(5)
    W = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    Wp = oracle.hadamard_apply(W, d, seed)
    res = oracle.ca_cur(Wp, r, 2, seed)
    assert res.status == 0
    q2 = 1 << d
    s = -(-n // q2)
    N = q2 * s
    M = np.zeros((N, N))
    M[:n, :] = (signs(seed, n)[:, None] * np.kron(sl.hadamard(q2), np.eye(s))[:n, :])
    approx = Wp[:, res.J] @ res.U @ Wp[res.I, :] @ M.T / q2
    assert np.linalg.norm(approx[:, :n] - W) <= 1e-10 * np.linalg.norm(W)
