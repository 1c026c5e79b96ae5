"""Pins of the oracle's CUR with uniform leverage scores (Algorithm
algcurlevsc with p_j = 1/n and pbar_i = 1/m; sampling by Algorithm
algsmplex; canonical nucleus of Algorithm algcnnncl).

The draws are checked against the published SplitMix64 outputs and the
rejection rule, and for uniformity; the nucleus against LAPACK's SVD (the
rescalings D and Dbar are multiples of the identity, so D M_r^+ Dbar is the
truncated pseudo-inverse of W[I, J]); the whole CUR against exact recovery
(Theorem thcandec) and the error level of perturbed factor-Gaussian inputs,
for which uniform scores are the superfast case of the paper."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


def test_draws_follow_the_stream_with_rejection():
    # n = 3 * 2^61 rejects the top 2^64 mod n = 2^62 words; every accepted
    # word is reduced mod n, duplicates kept, in draw order
    n = 3 << 61
    lim = (1 << 64) - ((1 << 64) % n)
    want, ctr = [], 0
    while len(want) < 40:
        u = oracle.rng_u64(123, 8, ctr)
        ctr += 1
        if u < lim:
            want.append(u % n)
    assert oracle.draw_uniform(123, 8, n, 40).tolist() == want
    assert ctr > 40  # some words were rejected at this n


def test_draws_are_uniform_and_repeat():
    n = 10
    d = oracle.draw_uniform(7, 9, n, 20000)
    counts = np.bincount(d, minlength=n)
    chi2 = float(((counts - 2000) ** 2 / 2000).sum())
    assert chi2 < 30.0  # 9 degrees of freedom: p < 1e-3 above 27.9
    small = oracle.draw_uniform(7, 9, 5, 12)
    assert len(set(small.tolist())) < 12  # with replacement


def test_nucleus_is_the_truncated_pseudo_inverse_of_the_generator():
    g = np.random.default_rng(4)
    W = g.standard_normal((90, 70))
    c = oracle.uniform_cur(W, 5, 12, 9, 31)
    assert c.status == 0 and c.nucleus_rank == 5
    assert c.I.tolist() == sorted(oracle.draw_uniform(31, 9, 90, 12).tolist())
    assert c.J.tolist() == sorted(oracle.draw_uniform(31, 8, 70, 9).tolist())
    G = W[np.ix_(c.I, c.J)]
    u, s, vt = np.linalg.svd(G, full_matrices=False)
    ref = vt[:5].T @ np.diag(1.0 / s[:5]) @ u[:, :5].T
    assert np.linalg.norm(c.U - ref) <= 1e-12 * np.linalg.norm(ref)
    scale = np.sqrt(90 / 12) * np.sqrt(70 / 9)
    assert c.det_log_abs == pytest.approx(np.sum(np.log(s[:5] * scale)), rel=1e-12)


@pytest.mark.parametrize("m,n,k,l", [(120, 100, 10, 10), (6, 200, 12, 12), (300, 4, 9, 7)])
def test_exact_rank_r_inputs_are_reproduced(m, n, k, l):
    # duplicates (k > m or l > n) leave the generator's rank at r
    g = np.random.default_rng(m + n)
    r = 3
    W = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    c = oracle.uniform_cur(W, r, k, l, 5)
    assert c.status == 0 and len(c.I) == k and len(c.J) == l and c.U.shape == (l, k)
    E = W - W[:, c.J] @ c.U @ W[c.I]
    assert np.linalg.norm(E) <= 1e-12 * np.linalg.norm(W)


def test_factor_gaussian_error_is_near_the_noise_level():
    # uniform scores suit perturbed factor-Gaussian inputs: with k = l = 4r
    # the error stays within a small factor of the perturbation
    W = workloads.factor_gaussian(1500, 1200, 8, 1e-6, seeds=(3, 4, 5))
    errs = []
    for seed in range(5):
        c = oracle.uniform_cur(W, 8, 32, 32, seed)
        assert c.status == 0
        errs.append(np.linalg.norm(W - W[:, c.J] @ c.U @ W[c.I]) / np.linalg.norm(W))
    noise = 1e-6 * np.sqrt(1500 * 1200) / np.linalg.norm(W)
    assert max(errs) < 5.0 * noise


def test_only_the_generator_is_read():
    W = np.random.default_rng(1).standard_normal((50, 40))
    c = oracle.uniform_cur(W, 2, 4, 4, 8)
    W2 = np.full_like(W, np.nan)
    W2[np.ix_(c.I, c.J)] = W[np.ix_(c.I, c.J)]
    c2 = oracle.uniform_cur(W2, 2, 4, 4, 8)
    assert c2.status == 0 and np.array_equal(c.U, c2.U)
    W2[c.I[0], c.J[0]] = np.inf
    assert oracle.uniform_cur(W2, 2, 4, 4, 8).status == oracle.EINVAL


def test_invalid_arguments():
    W = np.ones((10, 8))
    assert oracle.uniform_cur(W, 3, 2, 4, 0).status == oracle.EINVAL
    assert oracle.uniform_cur(W, 3, 4, 2, 0).status == oracle.EINVAL
    assert oracle.uniform_cur(W, 0, 4, 4, 0).status == oracle.EINVAL
