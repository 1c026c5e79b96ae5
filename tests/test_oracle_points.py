"""Pins of the oracle's far-field entries K_ij = 1/|x_i - y_j| (the Superfast
Multipole discussion, Section "Some Implications and Extensions of Our
Study") and of C-A on such blocks: closed forms, exact invariants, an
independent distance routine, and the accuracy the smooth kernel allows."""
import math

import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


def test_pythagorean_triples_give_exact_reciprocals():
    # |(0,0) - (3,4)| = 5, |(0,0) - (5,12)| = 13, |(1,1) - (1,3)| = 2, |(2,0) - (0,0)| = 2
    x = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 0.0]])
    y = np.array([[3.0, 4.0], [5.0, 12.0], [1.0, 3.0], [0.0, 0.0]])
    K = oracle.fmm_entries(x, y)
    assert K[0, 0] == 1.0 / 5.0 and K[0, 1] == 1.0 / 13.0
    assert K[1, 2] == 0.5 and K[2, 3] == 0.5
    assert K.shape == (3, 4)


def test_scaling_by_two_halves_every_entry_exactly():
    # doubling the points doubles dx, dy exactly, quadruples the square sum
    # exactly, doubles the correctly rounded root and halves the reciprocal
    g = np.random.default_rng(5)
    x = g.uniform(0, 1, (37, 2))
    y = g.uniform(0, 1, (29, 2)) + [3.0, 0.0]
    K = oracle.fmm_entries(x, y)
    K2 = oracle.fmm_entries(2 * x, 2 * y)
    assert np.array_equal(K2 * 2, K)


def test_swapping_the_point_sets_transposes():
    g = np.random.default_rng(6)
    x = g.uniform(0, 1, (11, 2))
    y = g.uniform(0, 1, (7, 2)) + [2.5, 0.0]
    assert np.array_equal(oracle.fmm_entries(y, x), oracle.fmm_entries(x, y).T)


def test_within_one_ulp_of_hypot():
    # math.hypot is a different distance algorithm (scaled, compensated)
    g = np.random.default_rng(7)
    x = g.uniform(0, 1, (23, 2))
    y = g.uniform(0, 1, (19, 2)) + [3.2, 0.0]
    K = oracle.fmm_entries(x, y)
    for i in range(23):
        for j in range(19):
            ref = 1.0 / math.hypot(x[i, 0] - y[j, 0], x[i, 1] - y[j, 1])
            assert abs(K[i, j] - ref) <= 2 * math.ulp(ref)


def test_coinciding_points_give_infinity():
    K = oracle.fmm_entries(np.array([[0.5, 0.5]]), np.array([[0.5, 0.5], [1.5, 0.5]]))
    assert math.isinf(K[0, 0]) and K[0, 1] == 1.0


def test_points_reproduce_the_fmm_blocks():
    # the point sets behind the stored FP32 blocks: same shapes, and the FP64
    # entries round to the stored FP32 values
    pts, desc = workloads.fmm_points(4, shape_seed=5, block_seed0=700)
    flat, bdesc = workloads.fmm_batch(4, shape_seed=5, block_seed0=700)
    for b in range(4):
        xo, yo, m, n = (int(v) for v in desc[b])
        K = oracle.fmm_entries(pts[xo:xo + m], pts[yo:yo + n])
        o0, bm, bn, _ = (int(v) for v in bdesc[b])
        assert (bm, bn) == (m, n)
        blk = flat[o0:o0 + m * n].reshape(m, n)
        assert np.array_equal(K.astype(np.float32), blk)


@pytest.mark.parametrize("b", [0, 1, 3])
def test_ca_on_a_far_field_block_meets_the_volume_bound(b):
    # well separated clusters: the kernel is smooth and its singular values
    # decay geometrically.  Theorem th12 bounds the Chebyshev norm of the CUR
    # error by h f(r, r) sigma_{r+1} with f(r, r) = r + 1 (h: volume ratio to
    # the maximum); the C-A sets meet it with h = 1 here
    pts, desc = workloads.fmm_points(4, shape_seed=5, block_seed0=700)
    xo, yo, m, n = (int(v) for v in desc[b])
    K = oracle.fmm_entries(pts[xo:xo + m], pts[yo:yo + n])
    r = 16
    res = oracle.ca_cur(K, r, 3, 1000 + b)
    E = K - K[:, res.J] @ res.U @ K[res.I, :]
    s = np.linalg.svd(K, compute_uv=False)
    assert np.abs(E).max() <= (r + 1) * s[r]
    assert oracle.rel_fro(K, res.I, res.J, res.U) < 1e-6
