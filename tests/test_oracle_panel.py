"""Pins of the oracle's panel LU and maxvol (App. D: alggos start, algdomin swaps)."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla


def _lapack_pivot_rows(P):
    """Original row ids chosen by LAPACK getrf, in pivot order."""
    lu, piv = sla.lu_factor(P)
    perm = np.arange(P.shape[0])
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    return perm[: P.shape[1]]


@pytest.mark.parametrize("m,r,seed", [(40, 5, 0), (300, 10, 1), (64, 16, 2), (17, 17, 3), (1000, 3, 4)])
def test_panel_lu_pivots_match_lapack(orc, m, r, seed):
    P = np.random.default_rng(seed).standard_normal((m, r))
    st, piv, LU, rank, mm = orc.panel_lu(P)
    assert st == 0 and rank == r
    assert piv.tolist() == _lapack_pivot_rows(P).tolist()
    # factors: P[piv] = L11 U and the other rows = L21 U
    U = np.triu(LU[piv])
    L11 = np.tril(LU[piv], -1) + np.eye(r)
    assert np.allclose(L11 @ U, P[piv], atol=1e-12)
    rest = np.setdiff1d(np.arange(m), piv)
    assert np.allclose(LU[rest] @ U, P[rest], atol=1e-12)


def test_panel_lu_ties_go_to_lowest_row(orc):
    P = np.array([[1.0, 2.0], [-3.0, 1.0], [3.0, 5.0], [0.5, 0.25]])
    st, piv, LU, rank, mm = orc.panel_lu(P)
    assert piv[0] == 1  # |-3| == |3|: lowest row wins
    assert mm == 0.0


def test_panel_lu_rank_deficient(orc):
    # column 1 = 2 x column 0 and the first pivot is a power of two, so the
    # elimination of column 1 is exact and leaves zeros: rank 1 is reported
    g = np.random.default_rng(7)
    P = g.uniform(-1, 1, size=(30, 3))
    P[5, 0] = 4.0
    P[:, 1] = 2.0 * P[:, 0]
    st, piv, LU, rank, mm = orc.panel_lu(P)
    assert st == 2 and rank == 1
    st, piv, LU, rank, mm = orc.panel_lu(np.zeros((5, 2)))
    assert st == 2 and rank == 0


def _vol(P, rows):
    return abs(np.linalg.det(P[list(rows)]))


@pytest.mark.parametrize("m,r,seed", [(50, 4, 0), (200, 10, 1), (120, 16, 2), (33, 7, 3)])
def test_maxvol_dominance_and_local_maximality(orc, m, r, seed):
    g = np.random.default_rng(seed)
    P = g.standard_normal((m, r)) * np.exp(0.5 * g.standard_normal(m))[:, None]
    delta = 0.01
    res = orc.maxvol(P, delta)
    assert res.status == 0 and res.converged == 1
    I = res.slots
    # (i) stop rule recomputed from scratch: every entry of P P[I]^-1 is <= 1 + delta
    Bfull = np.linalg.solve(P[I].T, P.T).T
    assert np.abs(Bfull).max() <= 1 + delta + 1e-12
    # (v) the rank-one updated B equals the recomputation
    assert np.allclose(res.B, Bfull, atol=1e-10)
    # (ii) no single swap increases the volume by more than 1 + delta (Lemma lelcliden)
    v0 = _vol(P, I)
    for i in range(m):
        if i in I:
            continue
        for j in range(r):
            J = I.copy()
            J[j] = i
            assert _vol(P, J) <= (1 + delta) * v0 * (1 + 1e-10)


def test_maxvol_each_swap_multiplies_det_by_b(orc):
    g = np.random.default_rng(11)
    P = g.standard_normal((150, 8))
    res = orc.maxvol(P, 0.0)
    assert res.swaps > 0
    st, piv, _, _, _ = orc.panel_lu(P)
    cur = piv.copy()
    for (i, j), b in zip(res.trace_idx, res.trace_val):
        before = _vol(P, cur)
        cur[j] = i
        assert np.isclose(_vol(P, cur) / before, abs(b), rtol=1e-9)
        assert abs(b) > 1.0
    assert cur.tolist() == res.slots.tolist()


@pytest.mark.parametrize("seed", range(8))
def test_maxvol_global_bound_brute_force(orc, seed):
    # Theorem thlclglb: a column-wise locally (1+delta)-maximal submatrix is
    # (1+delta)^r r^(r/2)-maximal among all r-subsets.
    g = np.random.default_rng(200 + seed)
    m = int(g.integers(6, 13))
    r = int(g.integers(1, 4))
    P = g.standard_normal((m, r))
    delta = 0.01
    res = orc.maxvol(P, delta)
    best = max(_vol(P, s) for s in itertools.combinations(range(m), r))
    assert best <= (1 + delta) ** r * r ** (r / 2) * _vol(P, res.slots) * (1 + 1e-12)


def test_maxvol_r1_is_argmax(orc):
    g = np.random.default_rng(12)
    P = g.standard_normal((99, 1))
    res = orc.maxvol(P, 0.01)
    assert res.slots[0] == np.argmax(np.abs(P[:, 0])) and res.swaps == 0


def test_maxvol_swap_cap(orc):
    g = np.random.default_rng(13)
    P = g.standard_normal((400, 12))
    full = orc.maxvol(P, 0.0)
    assert full.swaps >= 1
    capped = orc.maxvol(P, 0.0, max_swaps=0)
    assert capped.converged == 0 and capped.swaps == 0
    st, piv, _, _, _ = orc.panel_lu(P)
    assert capped.slots.tolist() == piv.tolist()


def test_maxvol_square_panel_needs_no_swap(orc):
    P = np.random.default_rng(14).standard_normal((6, 6))
    res = orc.maxvol(P, 0.01)
    assert res.status == 0 and res.swaps == 0 and sorted(res.slots.tolist()) == list(range(6))
