"""Pins of the oracle's refinement of a CUR LRA by leverage scores (section
on refining an LRA with leverage scores; Algorithm algcurlevsc with the crude
LRA's scores, sampling by Algorithm algsmplex, canonical nucleus).

The scores are checked against LAPACK (squared row norms of an orthonormal
basis of the panel's column space) and against their trace identity (they
sum to r); the sampling against the score distribution (chi-square); the
rescaled nucleus against a direct LAPACK evaluation of D M_r^+ Dbar; the
whole refinement against exact recovery of rank-r inputs and its effect on a
crude C-A."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


@pytest.mark.parametrize("items,r", [(50, 3), (200, 7), (33, 1)])
def test_scores_are_squared_row_norms_of_an_orthonormal_basis(items, r):
    P = np.random.default_rng(items + r).standard_normal((items, r))
    st, q, cdf = oracle.leverage_scores(P)
    Q, _ = np.linalg.qr(P)
    assert st == 0
    assert np.allclose(q, (Q * Q).sum(axis=1), atol=1e-13)
    assert cdf[-1] == pytest.approx(r, rel=1e-13)                 # trace of the projector
    assert np.all(np.diff(cdf) >= 0) and np.all(q <= 1 + 1e-13)
    # invariant under a change of basis of the column space
    T = np.random.default_rng(1).standard_normal((r, r))
    assert np.allclose(oracle.leverage_scores(P @ T)[1], q, atol=1e-10)


def test_rank_deficient_panel_is_singular():
    P = np.zeros((10, 2))
    P[:, 0] = 1.0
    assert oracle.leverage_scores(P)[0] == oracle.ESINGULAR


def test_draws_follow_the_scores():
    # concentrated scores: most draws land on the heavy rows, in proportion
    g = np.random.default_rng(5)
    A = g.standard_normal((400, 3)) @ g.standard_normal((3, 300))
    A[7] *= 30.0
    A[123] *= 10.0
    I0 = np.array([7, 123, 5])
    J0 = np.array([0, 1, 2])
    counts = np.zeros(400)
    for seed in range(40):
        c = oracle.leverage_cur(A, I0, J0, 50, 3, seed)
        assert c.status == 0
        np.add.at(counts, c.I, 1)
    C = A[:, J0]
    Q, _ = np.linalg.qr(C)
    p = (Q * Q).sum(axis=1) / 3
    expect = 40 * 50 * p
    heavy = expect > 20
    chi2 = float(((counts[heavy] - expect[heavy]) ** 2 / expect[heavy]).sum())
    assert chi2 < 3 * heavy.sum() + 20


def test_nucleus_is_the_rescaled_truncated_pseudo_inverse():
    W = workloads.orthogonal_lowrank(120, 90, 4, noise=1e-3, seeds=(3, 4, 5))
    I0, J0 = np.array([3, 40, 77, 101]), np.array([2, 30, 55, 80])
    c = oracle.leverage_cur(W, I0, J0, 12, 10, 9)
    assert c.status == 0 and c.nucleus_rank == 4
    qc = oracle.leverage_scores(W[I0].T.copy())[1]
    qr = oracle.leverage_scores(W[:, J0].copy())[1]
    D = 1 / np.sqrt(10 * qc[c.J] / qc.sum())
    Db = 1 / np.sqrt(12 * qr[c.I] / qr.sum())
    M = Db[:, None] * W[np.ix_(c.I, c.J)] * D[None, :]
    u, s, vt = np.linalg.svd(M, full_matrices=False)
    Mp = vt[:4].T @ np.diag(1 / s[:4]) @ u[:, :4].T
    ref = D[:, None] * Mp * Db[None, :]
    assert np.linalg.norm(c.U - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.all(np.diff(c.I) >= 0) and np.all(np.diff(c.J) >= 0)


@pytest.mark.parametrize("k,l", [(8, 8), (20, 12), (5, 30)])
def test_exact_rank_r_inputs_are_reproduced(k, l):
    g = np.random.default_rng(k * l)
    W = g.standard_normal((150, 5)) @ g.standard_normal((5, 130))
    base = oracle.ca_cur(W, 5, 1, 3)
    c = oracle.leverage_cur(W, base.I, base.J, k, l, 11)
    assert c.status == 0
    E = W - W[:, c.J] @ c.U @ W[c.I]
    assert np.linalg.norm(E) <= 1e-11 * np.linalg.norm(W)


def test_refinement_of_a_crude_ca_stays_near_the_noise_level():
    # one C-A sweep from a random start is crude; leverage-score sampling
    # with k = l = 4r from its factors gives an error near the perturbation
    W = workloads.factor_gaussian(1200, 1000, 8, 1e-6, seeds=(11, 12, 13))
    base = oracle.ca_cur(W, 8, 1, 4)
    errs = []
    for seed in range(4):
        c = oracle.leverage_cur(W, base.I, base.J, 32, 32, seed)
        assert c.status == 0
        errs.append(np.linalg.norm(W - W[:, c.J] @ c.U @ W[c.I]) / np.linalg.norm(W))
    noise = 1e-6 * np.sqrt(1200 * 1000) / np.linalg.norm(W)
    assert max(errs) < 5 * noise


def test_invalid_arguments():
    W = np.ones((10, 8))
    assert oracle.leverage_cur(W, [0, 1], [0, 1], 1, 4, 0).status == oracle.EINVAL    # k < r
    assert oracle.leverage_cur(W, [0, 11], [0, 1], 4, 4, 0).status == oracle.EINVAL   # row out of range
    W[2, 5] = np.nan
    assert oracle.leverage_cur(W, [2, 3], [0, 1], 4, 4, 0).status == oracle.EINVAL    # non-finite in R
