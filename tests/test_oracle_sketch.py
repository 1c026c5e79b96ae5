"""Pins of the oracle's abridged SRHT sketch (App. B) and greedy QRP (App. D, alg1tor)."""
import numpy as np
import pytest
import scipy.linalg as sla

from conftest import read_golden


def _recover_multiplier(orc, n, d, seed):
    """Sketch the identity with every column sampled and undo the sampling,
    the sign diagonal and the scale: returns H_{N,d} as the oracle applies it."""
    Y, smp = orc.sketch(np.eye(n), 0, d, n, seed)
    H = np.zeros((n, n))
    H[:, smp] = Y
    scale = 2.0 ** (-d / 2)  # sqrt(N/l) = 1 when l = N
    D = np.array([orc.sign(seed, c) for c in range(n)])
    return (H / scale) * D[:, None]


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_full_depth_is_walsh_hadamard(orc, k):
    # d = log2 n: the recursion (eqrfd) runs to the end and gives H_n.
    n = 2 ** k
    H = _recover_multiplier(orc, n, k, seed=17)
    assert np.array_equal(np.rint(H), sla.hadamard(n))


@pytest.mark.parametrize("d,s", [(1, 3), (2, 5), (3, 4), (3, 2500 // 100)])
def test_abridged_is_kron_hadamard_identity(orc, d, s):
    n = (2 ** d) * s
    H = _recover_multiplier(orc, n, d, seed=3)
    assert np.array_equal(np.rint(H), np.kron(sla.hadamard(2 ** d), np.eye(s)))


def test_printed_h_n1_h_n2(orc):
    rows = read_golden("abridged_hadamard_blocks.txt")
    blocks = {}
    i = 0
    while i < len(rows):
        name, r, c = rows[i][0], int(rows[i][1]), int(rows[i][2])
        blocks[name] = np.array([[int(x) for x in rows[i + 1 + a]] for a in range(r)])
        i += 1 + r
    s = 3
    for name, d in (("H_n1", 1), ("H_n2", 2)):
        H = _recover_multiplier(orc, (2 ** d) * s, d, seed=5)
        assert np.array_equal(np.rint(H), np.kron(blocks[name], np.eye(s)))


def test_orthogonal_up_to_scaling_and_sparsity(orc):
    d, s = 3, 6
    H = _recover_multiplier(orc, (2 ** d) * s, d, seed=9)
    assert np.allclose(H.T @ H, (2 ** d) * np.eye(H.shape[0]))
    assert (np.count_nonzero(H, axis=0) == 2 ** d).all()
    assert (np.count_nonzero(H, axis=1) == 2 ** d).all()


def test_zero_padding_and_linearity(orc):
    g = np.random.default_rng(0)
    A = g.standard_normal((7, 21))           # 21 is not a multiple of 8
    Ap = np.zeros((7, 24))
    Ap[:, :21] = A
    Y, smp = orc.sketch(A, 0, 3, 6, 11)
    Yp, smpp = orc.sketch(Ap, 0, 3, 6, 11)
    assert np.array_equal(smp, smpp)
    assert np.allclose(Y, Yp, rtol=0, atol=1e-14)
    B = g.standard_normal((7, 21))
    Y2, _ = orc.sketch(A + 2 * B, 0, 3, 6, 11)
    YB, _ = orc.sketch(B, 0, 3, 6, 11)
    assert np.allclose(Y2, Y + 2 * YB, atol=1e-12)


def test_left_form_is_right_form_of_transpose(orc):
    g = np.random.default_rng(1)
    A = g.standard_normal((40, 9))
    YL, sl = orc.sketch(A, 1, 2, 7, 23)
    YR, sr = orc.sketch(np.ascontiguousarray(A.T), 0, 2, 7, 23)
    assert np.array_equal(sl, sr)
    assert np.array_equal(YL, YR)


def test_sketch_matches_dense_product(orc):
    g = np.random.default_rng(2)
    m, n, d, l, seed = 11, 40, 3, 9, 77
    A = g.standard_normal((m, n))
    Y, smp = orc.sketch(A, 0, d, l, seed)
    s = n // 2 ** d
    D = np.diag([orc.sign(seed, c) for c in range(n)])
    M = D @ np.kron(sla.hadamard(2 ** d), np.eye(s)) * 2.0 ** (-d / 2) * np.sqrt(n / l)
    assert np.allclose(Y, A @ M[:, smp], atol=1e-12)


def test_sketch_float32_is_exact_upcast(orc):
    g = np.random.default_rng(3)
    A = g.standard_normal((16, 32)).astype(np.float32)
    Y32, _ = orc.sketch(A, 0, 2, 5, 1)
    Y64, _ = orc.sketch(A.astype(np.float64), 0, 2, 5, 1)
    assert np.array_equal(Y32, Y64)


# ---------------------------------------------------------------- greedy QRP
def test_qrp_first_pivot_is_max_norm(orc):
    g = np.random.default_rng(4)
    Z = g.standard_normal((300, 12))
    st, piv, rank, mm = orc.qrp(Z, 5)
    assert st == 0 and rank == 5
    assert piv[0] == np.argmax((Z ** 2).sum(1))


@pytest.mark.parametrize("seed", range(6))
def test_qrp_matches_lapack_geqp3(orc, seed):
    # greedy column pivoting is what LAPACK geqp3 computes; it downdates the
    # norms instead of recomputing them, so only compare when the decisions
    # are well separated.
    g = np.random.default_rng(100 + seed)
    items, w, k = 200, 16, 10
    Z = g.standard_normal((items, w)) * np.exp(g.standard_normal(items))[:, None]
    st, piv, rank, mm = orc.qrp(Z, k)
    assert st == 0
    if mm < 1e-6:
        pytest.skip("near tie")
    _, _, P = sla.qr(Z.T, pivoting=True, mode="economic")
    assert piv.tolist() == P[:k].tolist()


def test_qrp_volume_increase_matches_distance(orc):
    # each new item multiplies the volume of the chosen set by its distance
    # to the span of the items chosen before (the residual norm it was chosen by)
    g = np.random.default_rng(5)
    Z = g.standard_normal((60, 8))
    st, piv, rank, mm = orc.qrp(Z, 6)
    for t in range(1, 6):
        S = Z[piv[:t]]
        prev = Z[piv[:t - 1]]
        vol = np.sqrt(np.linalg.det(S @ S.T))
        vol_prev = np.sqrt(np.linalg.det(prev @ prev.T)) if t > 1 else 1.0
        # best achievable distance among the remaining items
        Q, _ = np.linalg.qr(prev.T) if t > 1 else (np.zeros((8, 0)), None)
        res = Z - (Z @ Q) @ Q.T
        dist = np.linalg.norm(res, axis=1)
        dist[piv[:t - 1]] = -1
        assert np.isclose(vol / vol_prev, dist.max(), rtol=1e-10)
        assert piv[t - 1] == np.argmax(dist)


def test_qrp_rank_deficient(orc):
    # items spanning only the first two coordinates: the third pick finds a
    # zero residual and reports rank 2 (reflections keep exact zeros)
    g = np.random.default_rng(6)
    Z = np.zeros((50, 4))
    Z[:, :2] = g.standard_normal((50, 2))
    st, piv, rank, mm = orc.qrp(Z, 3)
    assert st == 2 and rank == 2
    st, piv, rank, mm = orc.qrp(np.zeros((10, 4)), 2)
    assert st == 2 and rank == 0
