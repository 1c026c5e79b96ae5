"""Pins of the oracle's k x l generators of large r-projective volume
(Algorithm algprjvlm with Algorithms alg1tor and algrup as its black box;
Theorem th2 for the expansion factor; Algorithm algcnnncl for the canonical
nucleus; Theorems thcandec and th3 for what the resulting CUR guarantees).

The greedy stages are checked against an independent route (LAPACK's
pivoted QR for the two QRP stages, explicit determinants for every
expansion), against closed forms (r = 1) and against their invariance under
an orthogonal change of the panel's coordinates (Lemma leprwnmp); the
expansion-contraction exchanges against brute-force local maximality and the
product of eqs. (eqb) and (eqa); the whole loop against exact recovery and
the brute-force Chebyshev bound of Theorem th3."""
import itertools

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1710_07946_amd import workloads


def trunc_pinv(G, r):
    u, s, vt = np.linalg.svd(G, full_matrices=False)
    return vt[:r].T @ np.diag(1.0 / s[:r]) @ u[:, :r].T, np.sum(np.log(s[:r]))


@pytest.mark.parametrize("k,l,r", [(7, 7, 3), (9, 5, 2), (5, 9, 4), (12, 12, 12), (6, 4, 4), (1, 1, 1)])
def test_pinv_trunc_matches_lapack_svd(k, l, r):
    g = np.random.default_rng(k * 100 + l * 10 + r)
    G = g.standard_normal((k, l))
    st, X, rk, lv = oracle.pinv_trunc(G, r)
    ref, ref_lv = trunc_pinv(G, r)
    assert st == 0 and rk == r
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)
    assert abs(lv - ref_lv) <= 1e-12 * max(1.0, abs(ref_lv))
    if r == min(k, l):  # the truncation is G itself (Remark reklr_kl)
        assert np.linalg.norm(X - np.linalg.pinv(G)) <= 1e-12 * np.linalg.norm(X)


def test_pinv_trunc_of_an_exact_rank_r_generator_is_its_pseudo_inverse():
    g = np.random.default_rng(3)
    G = g.standard_normal((10, 3)) @ g.standard_normal((3, 8))
    st, X, rk, _ = oracle.pinv_trunc(G, 3)
    assert st == 0 and rk == 3
    assert np.linalg.norm(G @ X @ G - G) <= 1e-12 * np.linalg.norm(G)
    assert np.linalg.norm(X @ G @ X - X) <= 1e-12 * np.linalg.norm(X)


def test_pinv_trunc_drops_null_directions():
    # rank 2 with r = 4: only the two nonzero singular values are kept
    G = np.zeros((5, 6))
    G[0, 0], G[1, 3] = 2.0, -0.5
    st, X, rk, _ = oracle.pinv_trunc(G, 4)
    assert st == 0 and rk == 2
    assert np.allclose(X, np.linalg.pinv(G), atol=1e-15)


def test_pinv_trunc_rejects_bad_ranks():
    G = np.ones((3, 4))
    assert oracle.pinv_trunc(G, 0)[0] == oracle.EINVAL
    assert oracle.pinv_trunc(G, 4)[0] == oracle.EINVAL


def test_r1_selection_is_the_order_of_projections_on_the_largest_item():
    # r = 1: R' is q^T P^T with q along the largest item; alg1tor takes the
    # largest |R'_i| and algrup adds items by y^2 / sum of chosen y^2, i.e. in
    # decreasing |R'_i| (ties to the lower item)
    g = np.random.default_rng(21)
    P = g.standard_normal((60, 7))
    st, out, _, mm = oracle.projective_select(P, 1, 12)
    assert st == 0 and mm > 1e-9
    p0 = int(np.argmax(np.sum(P * P, axis=1)))
    y = np.abs(P @ P[p0]) / np.linalg.norm(P[p0])
    want = sorted(range(60), key=lambda i: (-y[i], i))[:12]
    assert out.tolist() == want


def independent_selection(P, r, k):
    """The same three stages by another route: LAPACK's pivoted QR for the
    two QRP stages, then every expansion by explicit determinants."""
    piv1 = scipy.linalg.qr(P.T, pivoting=True, mode="r")[1][:r]
    Q, _ = np.linalg.qr(P[piv1].T)            # orthonormal basis of the first r pivots
    Rp = Q.T @ P.T                             # r x items, equal to R' up to an r x r rotation
    piv2 = scipy.linalg.qr(Rp, pivoting=True, mode="r")[1][:r]
    chosen = list(piv2)
    for _ in range(r, k):
        S = Rp[:, chosen]
        best, bv = -1, -np.inf
        for i in range(P.shape[0]):
            if i in chosen:
                continue
            T = np.hstack([S, Rp[:, i:i + 1]])
            v = np.linalg.slogdet(T @ T.T)[1]
            if v > bv:
                best, bv = i, v
        chosen.append(best)
    return chosen


@pytest.mark.parametrize("items,w,r,k,seed", [(50, 8, 3, 8, 1), (70, 12, 5, 12, 2), (40, 6, 6, 10, 3),
                                              (33, 9, 2, 9, 4)])
def test_selection_matches_lapack_qrp_and_determinants(items, w, r, k, seed):
    P = np.random.default_rng(seed).standard_normal((items, w))
    st, out, _, mm = oracle.projective_select(P, r, k)
    assert st == 0
    assert mm > 1e-8  # margins wide enough for LAPACK's downdated norms to agree
    assert out.tolist() == independent_selection(P, r, k)


def test_each_expansion_maximises_the_volume_factor_of_eq_b():
    # v_2(S + y)^2 / v_2(S)^2 = 1 + y^T (S S^T)^{-1} y (Theorem th2): the item
    # chosen at each expansion step gives the largest volume of all candidates
    P = np.random.default_rng(8).standard_normal((45, 10))
    r, k = 4, 11
    st, out, _, _ = oracle.projective_select(P, r, k)
    assert st == 0
    piv1 = scipy.linalg.qr(P.T, pivoting=True, mode="r")[1][:r]
    Q, _ = np.linalg.qr(P[piv1].T)
    Rp = Q.T @ P.T
    for g in range(r, k):
        S = Rp[:, out[:g]]
        base = np.linalg.det(S @ S.T)
        vols = {}
        for i in range(45):
            if i in out[:g]:
                continue
            T = np.hstack([S, Rp[:, i:i + 1]])
            vols[i] = np.linalg.det(T @ T.T)
            y = Rp[:, i]
            assert vols[i] / base == pytest.approx(1.0 + y @ np.linalg.solve(S @ S.T, y), rel=1e-9)
        assert max(vols, key=vols.get) == out[g]


def test_selection_is_invariant_under_orthogonal_mixing_of_coordinates():
    # Lemma leprwnmp: volumes (and r-projective volumes) are unchanged by a
    # unitary factor, so P and P Q lead to the same items
    g = np.random.default_rng(5)
    P = g.standard_normal((80, 9))
    Q, _ = np.linalg.qr(g.standard_normal((9, 9)))
    a = oracle.projective_select(P, 4, 13)
    b = oracle.projective_select(P @ Q, 4, 13)
    assert a[0] == 0 and b[0] == 0 and min(a[3], b[3]) > 1e-8
    assert a[1].tolist() == b[1].tolist()


def test_k_equal_r_stops_after_alg1tor():
    P = np.random.default_rng(6).standard_normal((30, 5))
    st, out, _, _ = oracle.projective_select(P, 3, 3)
    piv1 = scipy.linalg.qr(P.T, pivoting=True, mode="r")[1][:3]
    Q, _ = np.linalg.qr(P[piv1].T)
    piv2 = scipy.linalg.qr(Q.T @ P.T, pivoting=True, mode="r")[1][:3]
    assert st == 0 and out.tolist() == list(piv2)


def test_rank_deficient_panel_is_singular():
    P = np.zeros((20, 4))
    P[3, 1] = 1.0  # rank 1
    st, _, rank, _ = oracle.projective_select(P, 2, 4)
    assert st == oracle.ESINGULAR and rank == 1


@pytest.mark.parametrize("k,l", [(10, 10), (14, 9), (8, 16)])
def test_exact_rank_r_inputs_are_reproduced(k, l):
    # a canonical CUR whose generator has the rank of W is exact (Theorem thcandec)
    g = np.random.default_rng(k + l)
    W = g.standard_normal((150, 5)) @ g.standard_normal((5, 120))
    c = oracle.projective_cur(W, 5, k, l, 3, 17)
    assert c.status == 0 and len(c.I) == k and len(c.J) == l and c.U.shape == (l, k)
    assert np.all(np.diff(c.I) > 0) and np.all(np.diff(c.J) > 0)
    E = W - W[:, c.J] @ c.U @ W[c.I]
    assert np.linalg.norm(E) <= 1e-12 * np.linalg.norm(W)
    assert c.nucleus_rank == 5


def test_start_set_is_the_seeded_draw_and_loops_reach_a_fixed_point():
    W = workloads.orthogonal_lowrank(120, 100, 4, noise=1e-5, seeds=(1, 2, 3))
    one = oracle.projective_cur(W, 4, 8, 8, 1, 99)
    many = oracle.projective_cur(W, 4, 8, 8, 12, 99)
    assert one.status == 0 and many.status == 0
    assert many.sweeps_run < 12  # stopped at a repeated pair of sets
    # the one-sweep result is what a column step from the seeded columns and a
    # row step give
    J0 = np.sort(oracle.draw_distinct(99, 0, 100, 8))
    st, I, _, _ = oracle.projective_select(W[:, J0], 4, 8, max_swaps=64)
    I = np.sort(I)
    st2, J, _, _ = oracle.projective_select(W[I].T, 4, 8, max_swaps=64)
    assert st == 0 and st2 == 0
    assert one.I.tolist() == I.tolist() and one.J.tolist() == sorted(J.tolist())


def test_theorem_th3_chebyshev_bound_by_brute_force():
    # ||W - C U R||_C <= h f(k, l, r) sigma_{r+1}(W), h = the largest
    # r-projective volume over all k x l submatrices / the chosen one's
    m = n = 7
    k = l = 3
    r = 2
    g = np.random.default_rng(12)
    W = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 1e-2 * g.standard_normal((m, n))
    c = oracle.projective_cur(W, r, k, l, 4, 5)
    assert c.status == 0

    def pv(B):
        return np.prod(np.linalg.svd(B, compute_uv=False)[:r])

    best = max(pv(W[np.ix_(I, J)]) for I in itertools.combinations(range(m), k)
               for J in itertools.combinations(range(n), l))
    h = best / pv(W[np.ix_(c.I, c.J)])
    assert np.exp(c.det_log_abs) == pytest.approx(pv(W[np.ix_(c.I, c.J)]), rel=1e-12)
    f = np.sqrt((k + 1) * (l + 1) / ((k - r + 1) * (l - r + 1)))
    sig = np.linalg.svd(W, compute_uv=False)
    E = W - W[:, c.J] @ c.U @ W[c.I]
    assert np.abs(E).max() <= h * f * sig[r] * (1 + 1e-12)


def r_prime(P, r):
    """R' by another route (LAPACK's pivoted QR of P^T), up to a rotation."""
    piv1 = scipy.linalg.qr(P.T, pivoting=True, mode="r")[1][:r]
    Q, _ = np.linalg.qr(P[piv1].T)
    return Q.T @ P.T


def gram_det(Rp, S):
    return np.linalg.det(Rp[:, S] @ Rp[:, S].T)


@pytest.mark.parametrize("items,w,r,k,seed,delta", [(200, 20, 8, 12, 30, 0.0), (70, 10, 4, 8, 20, 0.0),
                                                    (60, 9, 3, 7, 11, 0.01), (80, 8, 4, 12, 58, 0.0)])
def test_refinement_ends_locally_maximal(items, w, r, k, seed, delta):
    # no single exchange (add a candidate, drop a member) multiplies v_2^2 by
    # more than 1 + delta (the stop rule), by brute force over all pairs
    P = np.random.default_rng(seed).standard_normal((items, w))
    st, out, _, mm, sw, cv = oracle.projective_select(P, r, k, delta=delta, max_swaps=100, full=True)
    assert st == 0 and cv == 1 and mm > 1e-8
    Rp = r_prime(P, r)
    S = list(out)
    base = gram_det(Rp, S)
    for c in range(items):
        if c in S:
            continue
        for q in range(k):
            T = S[:q] + [c] + S[q + 1:]
            assert gram_det(Rp, T) <= (1 + delta) * base * (1 + 1e-9)
    # and the exchanges only ever raised the volume of the greedy choice
    g = oracle.projective_select(P, r, k, max_swaps=0)[1]
    assert base >= gram_det(Rp, list(g)) * (1 - 1e-12)
    print("exchanges", sw)


def test_exchange_gain_is_the_product_of_eq_b_and_eq_a():
    # the volume after one exchange equals the greedy set's volume times
    # (1 + y_b^T (S S^T)^{-1} y_b) (1 - y_s^T (S' S'^T)^{-1} y_s)
    P = np.random.default_rng(20).standard_normal((70, 10))
    r, k = 4, 8
    g = list(oracle.projective_select(P, r, k, max_swaps=0)[1])
    st, one, _, _, sw, cv = oracle.projective_select(P, r, k, delta=0.0, max_swaps=1, full=True)
    assert st == 0 and sw == 1
    Rp = r_prime(P, r)
    b = [i for i in one if i not in g]
    s_ = [i for i in g if i not in one]
    assert len(b) == 1 and len(s_) == 1
    M = Rp[:, g] @ Rp[:, g].T
    yb = Rp[:, b[0]]
    grow = 1 + yb @ np.linalg.solve(M, yb)
    M2 = M + np.outer(yb, yb)
    ys = Rp[:, s_[0]]
    shrink = 1 - ys @ np.linalg.solve(M2, ys)
    assert gram_det(Rp, list(one)) == pytest.approx(gram_det(Rp, g) * grow * shrink, rel=1e-9)
    assert grow * shrink > 1.0


def test_refinement_caps_and_thresholds():
    P = np.random.default_rng(30).standard_normal((200, 20))
    full = oracle.projective_select(P, 8, 12, delta=0.0, max_swaps=100, full=True)
    assert full[4] == 2 and full[5] == 1
    capped = oracle.projective_select(P, 8, 12, delta=0.0, max_swaps=1, full=True)
    assert capped[4] == 1 and capped[5] == 0          # stopped by the cap with gain left
    none = oracle.projective_select(P, 8, 12, delta=1e9, max_swaps=100, full=True)
    greedy = oracle.projective_select(P, 8, 12, max_swaps=0)
    assert none[4] == 0 and none[5] == 1 and none[1].tolist() == greedy[1].tolist()
    # r = 1: the greedy order of |R'_i| is already locally maximal
    r1 = oracle.projective_select(P, 1, 6, delta=0.0, max_swaps=100, full=True)
    assert r1[4] == 0 and r1[5] == 1


def test_bigger_generators_do_not_lose_accuracy():
    # Theorem th3 with k = l = 4r bounds the error by a smaller multiple of
    # sigma_{r+1} than k = l = r; on a noisy rank-r input the larger
    # generator's error stays within a small factor of the noise level
    W = workloads.orthogonal_lowrank(200, 180, 6, noise=1e-6, seeds=(31, 32, 33))
    c4 = oracle.projective_cur(W, 6, 24, 24, 3, 41)
    assert c4.status == 0
    e4 = np.linalg.norm(W - W[:, c4.J] @ c4.U @ W[c4.I]) / np.linalg.norm(W)
    noise = 1e-6 * np.sqrt(200 * 180) / np.linalg.norm(W)
    assert e4 < 3.0 * noise


def test_invalid_arguments():
    W = np.ones((10, 8))
    assert oracle.projective_cur(W, 3, 2, 4, 1, 0).status == oracle.EINVAL   # k < r
    assert oracle.projective_cur(W, 3, 4, 9, 1, 0).status == oracle.EINVAL   # l > n
    assert oracle.projective_cur(W, 3, 4, 4, 0, 0).status == oracle.EINVAL   # no sweep


@pytest.mark.parametrize("k,l,distinct,seed", [(56, 63, 50, 1), (63, 56, 50, 2), (64, 64, 40, 3), (60, 48, 45, 4)])
def test_pinv_trunc_of_repeated_rows_keeps_the_exact_rank(k, l, distinct, seed):
    # a generator drawn with repetition (as by sampling): k rows of which only
    # `distinct` differ, each rescaled, so its exact rank is `distinct`.  The
    # columns the rotations leave at rounding level must not count: the kept
    # rank is LAPACK's numerical rank and X its pseudo-inverse
    g = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(g.standard_normal((distinct, distinct)))
    Q2, _ = np.linalg.qr(g.standard_normal((l, l)))
    s = np.geomspace(1.0, 7e-4, distinct)
    base = (Q1 * s) @ Q2[:distinct]
    pick = np.sort(np.concatenate([np.arange(distinct), g.integers(0, distinct, k - distinct)]))
    G = base[pick] * g.uniform(0.5, 2.0, k)[:, None]
    r = min(k, l) - 1
    st, X, rk, _ = oracle.pinv_trunc(G, r)
    assert st == 0 and rk == np.linalg.matrix_rank(G) == distinct
    ref, _ = trunc_pinv(G, distinct)
    assert np.linalg.norm(X - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.linalg.norm(G @ X @ G - G) <= 1e-10 * np.linalg.norm(G)
