"""Pins of the oracle's cynical CUR (Section 1.3 and Fig. 3; Section 13,
Tests 3 and Tests 4): special cases that reduce to C-A, exact recovery of
rank-r inputs, dominance of the inner generator inside its sketch, and the
error level of the paper's Table tb_ranrc."""
import numpy as np
import pytest

import oracle
from conftest import read_golden
from paper_1710_07946_amd import workloads


def test_whole_matrix_sketch_reduces_to_ca():
    # k = m = n: the random k-sets are all rows and columns, so the sketch is W
    # and the inner C-A (seed + 1) is the plain C-A of W
    W = workloads.orthogonal_lowrank(40, 40, 6, noise=1e-6, seeds=(1, 2, 3))
    c = oracle.cynical(W, 6, 40, 0, 3, 77)
    o = oracle.ca_cur(W, 6, 3, 78)
    assert c.status == 0 and o.status == 0
    assert c.I.tolist() == o.I.tolist() and c.J.tolist() == o.J.tolist()
    assert np.array_equal(c.U, o.U)


@pytest.mark.parametrize("loops", [0, 1, 2])
def test_exact_rank_r_inputs_are_reproduced(loops):
    # any nonsingular r x r generator reproduces a rank-r matrix (Theorem thdcmp)
    g = np.random.default_rng(9)
    W = g.standard_normal((200, 5)) @ g.standard_normal((5, 150))
    c = oracle.cynical(W, 5, 20, loops, 3, 5)
    assert c.status == 0
    assert oracle.rel_fro(W, c.I, c.J, c.U) < 1e-12


def test_inner_generator_is_dominant_in_the_sketch():
    # loops = 0: the sketch rows and columns are the seeded draws (streams 5
    # and 0); the final row step leaves J dominant in S[I, :]
    m, n, r, k, seed = 300, 260, 7, 28, 31
    W = workloads.orthogonal_lowrank(m, n, r, noise=1e-4, seeds=(4, 5, 6))
    c = oracle.cynical(W, r, k, 0, 4, seed)
    assert c.status == 0
    K = np.sort(oracle.draw_distinct(seed, 5, m, k))
    L = np.sort(oracle.draw_distinct(seed, 0, n, k))
    assert set(c.I.tolist()) <= set(K.tolist()) and set(c.J.tolist()) <= set(L.tolist())
    R = W[c.I][:, L]
    Jpos = np.searchsorted(L, c.J)
    B = np.linalg.solve(R[:, Jpos], R)
    assert np.abs(B).max() <= 1.0 + 0.01 + 1e-9


def test_loops_make_the_outer_sets_dominant():
    # loops = 1: L is dominant at rank k in W[K, :], so the C-A generator W[K, L]
    # is dominant in its rows; with k = r the cynical CUR is one C-A loop
    m, n, r = 220, 180, 6
    W = workloads.orthogonal_lowrank(m, n, r, noise=1e-3, seeds=(7, 8, 9))
    c = oracle.cynical(W, r, r, 1, 2, 11)
    o = oracle.ca_cur(W, r, 1, 11)
    assert c.status == 0 and o.status == 0
    assert c.I.tolist() == o.I.tolist() and c.J.tolist() == o.J.tolist()
    assert np.array_equal(c.U, o.U)


def test_invalid_arguments():
    W = np.ones((30, 20))
    assert oracle.cynical(W, 5, 4, 0, 1, 0).status == 1     # k < r
    assert oracle.cynical(W, 5, 21, 0, 1, 0).status == 1    # k > min(m, n)
    assert oracle.cynical(W, 5, 10, -1, 1, 0).status == 1   # loops < 0
    assert oracle.cynical(W, 5, 10, 0, 0, 0).status == 1    # sweeps < 1


def test_error_statistics_sanity_band():
    # Table tb_ranrc, Tests 3 and Tests 4 (n = 256, k = l = 4r): mean relative
    # spectral error on perturbed factor-Gaussian inputs.  The paper's inner
    # routine is not given, so only a one-sided band is asserted: not worse on
    # average than ten times the table's means
    table = {(int(a), int(b)): (float(c), float(e)) for a, b, c, _, e, _ in read_golden("table_ranrc_tests34.txt")}
    n = 256
    for r in (8, 16):
        errs = {0: [], 1: []}
        for t in range(30):
            g = np.random.default_rng(20_000 * r + t)
            W = g.standard_normal((n, r)) @ g.standard_normal((r, n)) + 1e-10 * g.standard_normal((n, n))
            for loops in (0, 1):
                res = oracle.cynical(W, r, 4 * r, loops, 5, t)
                assert res.status == 0
                E = W - W[:, res.J] @ res.U @ W[res.I]
                errs[loops].append(np.linalg.norm(E, 2) / np.linalg.norm(W, 2))
        assert np.mean(errs[0]) <= 10 * table[(n, r)][0]
        assert np.mean(errs[1]) <= 10 * table[(n, r)][1]
