"""Pins of the oracle's quasi-Gaussian multiplier G_q = B_1 P_1 ... B_q P_q
(random cyclic bidiagonal factors times random permutations, eq. (def11) in
the section on pre-processing with quasi Gaussian matrices): the permutation
is a bijection, the sparse column expansion equals the dense product of the
explicit factors, the product's entries approach a Gaussian distribution as
the number of factors grows (Theorem thm1), the sketch equals the dense
product, and C-A started from it recovers rank-r inputs."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


@pytest.mark.parametrize("N", [2, 3, 5, 64, 100, 1000, 4097])
def test_feistel_is_a_bijection(N):
    for factor in (1, 2, 5):
        img = [oracle.feistel(17, factor, N, x) for x in range(N)]
        assert sorted(img) == list(range(N))
    if N >= 64:  # not the identity, and the factors differ
        assert [oracle.feistel(17, 1, N, x) for x in range(N)] != list(range(N))
        assert [oracle.feistel(17, 1, N, x) for x in range(N)] != [oracle.feistel(17, 2, N, x) for x in range(N)]


def dense_factor(seed, i, N):
    """B_i P_i from the definitions: P_i e_c = e_{pi_i(c)}; B_i has ones on the
    diagonal and s_{i,j} at (j, (j - 1) mod N), the sign from SplitMix64
    stream 7 at (i - 1) N + j."""
    P = np.zeros((N, N))
    for c in range(N):
        P[oracle.feistel(seed, i, N, c), c] = 1.0
    B = np.eye(N)
    for j in range(N):
        s = -1.0 if oracle.rng_u64(seed, 7, (i - 1) * N + j) >> 63 else 1.0
        B[j, (j - 1) % N] += s
    return B @ P


@pytest.mark.parametrize("q", [0, 1, 2, 3, 5])
def test_column_expansion_equals_the_dense_product(q):
    N, seed = 50, 23
    G = np.eye(N)
    for i in range(1, q + 1):
        G = G @ dense_factor(seed, i, N)
    for c in range(N):
        pos, coef = oracle.bidiag_column(seed, N, q, c)
        col = np.zeros(N)
        col[pos] = coef
        assert np.array_equal(col, G[:, c]), c
        assert list(pos) == sorted(pos) and (coef != 0).all() and len(pos) <= 2 ** q


def test_products_fill_in_and_look_gaussian():
    # Theorem thm1: products of many random bidiagonal-times-permutation
    # factors tend to a Gaussian matrix.  Sanity band at order 32 with 16
    # factors: every entry filled in, mean near 0, skewness near 0, and a
    # kurtosis in the range of a Gaussian's (3) for each realization
    N = 32
    for seed in range(4):
        G = np.eye(N)
        for i in range(1, 17):
            G = G @ dense_factor(1000 + seed, i, N)
        x = G.ravel()
        z = (x - x.mean()) / x.std()
        assert (x != 0).mean() > 0.95
        assert abs(x.mean()) < 0.15 * x.std()
        assert abs((z ** 3).mean()) < 0.3
        assert 2.5 < (z ** 4).mean() < 6.0


@pytest.mark.parametrize("side", [0, 1])
def test_sketch_equals_the_dense_product(side):
    g = np.random.default_rng(3)
    m, n, q, l, seed = 70, 60, 3, 12, 41
    A = g.standard_normal((m, n))
    Y, smp = oracle.sketch_bidiag(A, side, q, l, seed)
    dim = m if side else n
    assert np.array_equal(smp, oracle.draw_distinct(seed, 2, dim, l))
    G = np.eye(dim)
    for i in range(1, q + 1):
        G = G @ dense_factor(seed, i, dim)
    GS = G[:, smp]
    ref = (GS.T @ A).T if side else A @ GS
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(300, 200), (200, 300)])
def test_ca_from_the_bidiagonal_sketch_recovers_rank_r(shape):
    m, n = shape
    g = np.random.default_rng(8)
    W = g.standard_normal((m, 6)) @ g.standard_normal((6, n))
    res = oracle.ca_cur(W, 6, 2, 19, preprocess=2, ah_depth=3, ah_samples=16)
    assert res.status == 0
    assert oracle.rel_fro(W, res.I, res.J, res.U) < 1e-12


def test_bidiagonal_start_on_the_512_workload():
    # the first workload with the bidiagonal start (q = 3, l = 2r): as accurate
    # as the random start to within the noise level
    A = workloads.orthogonal_lowrank()
    res = oracle.ca_cur(A, 10, 3, 2001, preprocess=2, ah_depth=3, ah_samples=20)
    ref = oracle.ca_cur(A, 10, 3, 2001)
    assert res.status == 0
    assert oracle.rel_fro(A, res.I, res.J, res.U) < 10 * oracle.rel_fro(A, ref.I, ref.J, ref.U) + 1e-9
