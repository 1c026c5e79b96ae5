"""Pins of the oracle's whole C-A CUR path (sweeps, nucleus, pre-processing, errors)."""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from paper_1710_07946_amd import workloads


def test_exact_rank_reproduces_input(orc):
    # Theorem thdcmp: a CUR built on a nonsingular r x r generator of a rank-r
    # matrix is a CUR decomposition (W = C U R); only round-off remains.
    A = workloads.orthogonal_lowrank(512, 512, 10, noise=0.0)
    res = orc.ca_cur(A, 10, 3, 2001)
    assert res.status == 0
    assert orc.rel_fro(A, res.I, res.J, res.U) <= 1e-12


def test_outputs_sorted_and_nucleus_is_inverse(orc):
    A = workloads.orthogonal_lowrank()
    res = orc.ca_cur(A, 10, 3, 2001)
    assert res.status == 0
    assert (np.diff(res.I) > 0).all() and (np.diff(res.J) > 0).all()
    G = A[np.ix_(res.I, res.J)]
    assert np.allclose(res.U, np.linalg.inv(G), rtol=1e-10, atol=0)
    assert np.isclose(res.det_log_abs, np.linalg.slogdet(G)[1], rtol=1e-12)
    # reconstruction error is at the noise level (noise std 1e-10 per entry)
    assert orc.rel_fro(A, res.I, res.J, res.U) < 1e-6


def test_converged_sets_are_dominant_both_ways(orc):
    A = workloads.orthogonal_lowrank()
    res = orc.ca_cur(A, 10, 3, 2001)
    delta = 0.01
    # last row step: J is dominant in R = A[I, :]
    R = A[res.I]
    Bc = np.linalg.solve(R[:, res.J], R)
    assert np.abs(Bc).max() <= 1 + delta + 1e-9


def test_rank_one_is_argmax_chain(orc):
    g = np.random.default_rng(3)
    c = g.standard_normal(40)
    rr = g.standard_normal(30)
    A = np.outer(c, rr)
    res = orc.ca_cur(A, 1, 2, 77)
    j0 = orc.draw_distinct(77, 0, 30, 1)[0]
    i1 = np.argmax(np.abs(A[:, j0]))
    j1 = np.argmax(np.abs(A[i1]))
    assert res.I.tolist() == [i1] and res.J.tolist() == [j1]
    assert np.isclose(res.U[0, 0], 1.0 / A[i1, j1])
    assert orc.rel_fro(A, res.I, res.J, res.U) < 1e-15


def test_pm_delta_matrices_fail_where_unread(orc):
    # Example exdlt: with r = 1 the method reads one column first; if the
    # nonzero entry is elsewhere the panel is zero and the method must report
    # a rank-deficient panel; if it is there, the CUR is exact.
    mats = [np.array([float(x) for x in row]).reshape(2, 2) for row in read_golden("pm_delta_2x2.txt")]
    assert len(mats) == 8
    seed = 5
    j0 = orc.draw_distinct(seed, 0, 2, 1)[0]
    fails = 0
    for M in mats:
        res = orc.ca_cur(M, 1, 1, seed)
        if M[:, j0].any():
            assert res.status == 0 and orc.rel_fro(M, res.I, res.J, res.U) == 0.0
        else:
            assert res.status == 2 and res.rank_found == 0
            fails += 1
    assert fails == 4  # half of them, as the example states


def _vol(A, I, J):
    return abs(np.linalg.det(A[np.ix_(I, J)]))


@pytest.mark.parametrize("seed", range(6))
def test_two_step_loop_global_volume_bound(orc, seed):
    # Theorem coc-avlm with k = l = r (p = r): after a column step and a row
    # step on a rank-r matrix the generator is ((1+delta)^2 r)^r-maximal.
    g = np.random.default_rng(300 + seed)
    m, n = int(g.integers(5, 9)), int(g.integers(5, 9))
    r = int(g.integers(1, 3))
    A = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    res = orc.ca_cur(A, r, 1, seed)
    assert res.status == 0
    best = max(_vol(A, list(I), list(J)) for I in itertools.combinations(range(m), r)
               for J in itertools.combinations(range(n), r))
    delta = 0.01
    assert best <= ((1 + delta) ** 2 * r) ** r * _vol(A, res.I, res.J) * (1 + 1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_chebyshev_error_bound(orc, seed):
    # Theorem th12 with k = l = r: ||E||_C <= h (r+1) sigma_{r+1}(W) where
    # h = (max volume) / (volume of the generator), found by brute force.
    g = np.random.default_rng(400 + seed)
    m, n, r = 8, 7, 2
    A = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 1e-3 * g.standard_normal((m, n))
    res = orc.ca_cur(A, r, 3, seed)
    assert res.status == 0
    best = max(_vol(A, list(I), list(J)) for I in itertools.combinations(range(m), r)
               for J in itertools.combinations(range(n), r))
    h = best / _vol(A, res.I, res.J)
    E = A - A[:, res.J] @ res.U @ A[res.I]
    s = np.linalg.svd(A, compute_uv=False)
    assert np.abs(E).max() <= h * (r + 1) * s[r] * (1 + 1e-9)


def _scaled_lowrank(m=300, n=200, r=6, seed=0):
    # rows and columns with log-normal scales: few dominant entries, so C-A
    # settles on a fixed point after two sweeps
    g = np.random.default_rng(seed)
    A = (np.exp(g.standard_normal(m))[:, None] * g.standard_normal((m, r))) @ \
        (g.standard_normal((r, n)) * np.exp(g.standard_normal(n))[None, :])
    return A + 1e-8 * g.standard_normal((m, n))


def test_fixed_point_early_stop(orc):
    A = _scaled_lowrank()
    a = orc.ca_cur(A, 6, 20, 7)
    b = orc.ca_cur(A, 6, a.sweeps_run, 7)
    assert a.sweeps_run < 20
    assert a.I.tolist() == b.I.tolist() and a.J.tolist() == b.J.tolist()
    assert np.array_equal(a.U, b.U)


def test_warm_start_columns(orc):
    A = workloads.orthogonal_lowrank()
    cold = orc.ca_cur(A, 10, 3, 2001)
    j0 = np.sort(orc.draw_distinct(2001, 0, 512, 10))
    warm = orc.ca_cur(A, 10, 3, 999, init_cols=j0[::-1].copy())
    assert warm.I.tolist() == cold.I.tolist() and warm.J.tolist() == cold.J.tolist()


def test_float32_input_is_exact_upcast(orc):
    A = workloads.orthogonal_lowrank(200, 150, 6, noise=1e-6).astype(np.float32)
    a = orc.ca_cur(A, 6, 3, 5)
    b = orc.ca_cur(A.astype(np.float64), 6, 3, 5)
    assert a.I.tolist() == b.I.tolist() and a.J.tolist() == b.J.tolist() and np.array_equal(a.U, b.U)


def test_bf16_bits_input(orc):
    A = workloads.orthogonal_lowrank(128, 96, 4, noise=1e-4).astype(np.float32)
    bits = (A.view(np.uint32) >> 16).astype(np.uint16)      # truncate to bf16
    back = (bits.astype(np.uint32) << 16).view(np.float32)
    a = orc.ca_cur(bits, 4, 3, 8)
    b = orc.ca_cur(back.astype(np.float64), 4, 3, 8)
    assert a.status == 0 and a.I.tolist() == b.I.tolist() and a.J.tolist() == b.J.tolist()


@pytest.mark.parametrize("m,n", [(300, 260), (260, 300), (256, 256)])
def test_preprocessed_start(orc, m, n):
    # Algorithm algrhtcur with the abridged SRHT multiplier: the start set
    # comes from greedy QRP on the sketch; the result is accurate.
    A = workloads.factor_gaussian(m, n, 12, 1e-9, seeds=(1, 2, 3), dtype=np.float64)
    res = orc.ca_cur(A, 12, 3, 2011, preprocess=1, ah_depth=2, ah_samples=24)
    assert res.status == 0
    assert orc.rel_fro(A, res.I, res.J, res.U) < 1e-6
    # the start set is the greedy QRP choice on the sketch
    side = 1 if m >= n else 0
    Y, _ = orc.sketch(A, side, 2, 24, 2011)
    st, piv, _, _ = orc.qrp(Y, 12)
    assert st == 0


def test_invalid_arguments(orc):
    A = np.ones((10, 8))
    assert orc.ca_cur(A, 9, 1, 0).status == 1     # r > min(m, n)
    assert orc.ca_cur(A, 0, 1, 0).status == 1     # r < 1
    assert orc.ca_cur(A, 2, 0, 0).status == 1     # sweeps < 1
    B = workloads.orthogonal_lowrank(20, 20, 3, noise=1e-3)
    B[:, :] = np.where(np.arange(20)[None, :] == 5, np.nan, B)
    res = orc.ca_cur(B, 3, 2, 0, init_cols=np.array([5, 6, 7]))
    assert res.status == 1                        # non-finite entry in a gathered panel


def test_error_statistics_sanity_band(orc):
    # Table tb_ranrc, Tests 2 (n = 256): mean relative spectral error of C-A on
    # perturbed factor-Gaussian inputs.  The paper used another subalgorithm,
    # so only a one-sided band is asserted: maxvol C-A is not worse on average.
    table = {(int(a), int(b)): float(c) for a, b, c, _ in read_golden("table_ranrc_tests2.txt")}
    n = 256
    for r in (8, 16):
        errs = []
        for t in range(30):
            g = np.random.default_rng(10_000 * r + t)
            W = g.standard_normal((n, r)) @ g.standard_normal((r, n)) + 1e-10 * g.standard_normal((n, n))
            res = orc.ca_cur(W, r, 5, t)
            assert res.status == 0
            E = W - W[:, res.J] @ res.U @ W[res.I]
            errs.append(np.linalg.norm(E, 2) / np.linalg.norm(W, 2))
        assert np.mean(errs) <= 10 * table[(n, r)]
