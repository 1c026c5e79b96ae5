"""Pins of the oracle's abridged randomized Fourier sketch (App. B: the
d-abridged DFT of eq. (eqfd), randomized by D and sampled) and of C-A seeded
from it.

The multiplier is recovered column by column by sketching the identity; it is
checked against numpy's FFT at full depth (the DFT itself), and at any depth
by completing each residue class with s-point DFTs, which must give the
N-point DFT.  Depth 0 leaves D alone; the columns are orthogonal with 2^d
nonzeros each; zero padding, the transposed form and exact recovery of
rank-r inputs by the seeded C-A close the list."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


def d_phases(seed, N):
    # D_j = i^{t_j}, t_j the top two bits of stream 1 (the reading of D)
    return np.array([1j ** (oracle.rng_u64(seed, 1, j) >> 62) for j in range(N)])


def multiplier(N, d, seed):
    """All N columns of the sampled multiplier, unscaled, in sample order."""
    Y, smp = oracle.sketch_fourier(np.eye(N), 1, d, N, seed)
    s = N >> d
    scale = np.sqrt(s / N)
    M = (Y[:, :N] + 1j * Y[:, N:]) / scale      # row j = input index, column q = sample q
    full = np.zeros((N, N), complex)
    full[:, smp] = M
    return full


@pytest.mark.parametrize("N", [2, 8, 32])
def test_full_depth_is_the_dft(N):
    d = int(np.log2(N))
    F = multiplier(N, d, 5)
    dft = np.fft.ifft(np.eye(N), axis=0) * N        # exp(+2 pi i j c / N)
    assert np.allclose(np.conj(d_phases(5, N))[:, None] * F, dft, atol=1e-12)


@pytest.mark.parametrize("N,d", [(16, 1), (16, 2), (24, 3), (40, 2), (64, 4)])
def test_completing_each_class_gives_the_full_dft(N, d):
    # column b s + e holds omega_N^{b j} on rows j = a s + e; an s-point DFT
    # over e (for each b) yields column b + 2^d k of the N-point DFT
    q2 = 1 << d
    s = N // q2
    F = np.conj(d_phases(9, N))[:, None] * multiplier(N, d, 9)
    dft = np.fft.ifft(np.eye(N), axis=0) * N
    es = np.arange(s)
    for b in range(q2):
        cols = F[:, b * s + es]                        # N x s
        for k in range(s):
            done = cols @ np.exp(2j * np.pi * es * k / s)
            assert np.allclose(done, dft[:, b + q2 * k], atol=1e-10)


@pytest.mark.parametrize("N,d", [(16, 2), (24, 3), (32, 5)])
def test_columns_are_orthogonal_with_two_to_the_d_nonzeros(N, d):
    F = multiplier(N, d, 3)
    assert np.allclose(F.conj().T @ F, (1 << d) * np.eye(N), atol=1e-12)
    assert all(int((np.abs(F[:, c]) > 0.5).sum()) == (1 << d) for c in range(N))


def test_depth_zero_is_the_random_phases():
    W = np.random.default_rng(1).standard_normal((12, 7))
    Y, smp = oracle.sketch_fourier(W, 1, 0, 5, 11)
    D = d_phases(11, 12)
    want = np.sqrt(12 / 5) * (D[smp][None, :] * W[smp].T)
    assert np.allclose(Y[:, :5] + 1j * Y[:, 5:], want, atol=1e-14)


def test_zero_padding_and_the_transposed_form():
    W = np.random.default_rng(2).standard_normal((22, 9))   # 22 rows, d = 3: N = 24
    Y, smp = oracle.sketch_fourier(W, 1, 3, 6, 4)
    Wp = np.vstack([W, np.zeros((2, 9))])
    Yp, smpp = oracle.sketch_fourier(Wp, 1, 3, 6, 4)
    assert np.array_equal(smp, smpp) and np.allclose(Y, Yp, atol=1e-14)
    Yt, smpt = oracle.sketch_fourier(np.ascontiguousarray(W.T), 0, 3, 6, 4)
    assert np.array_equal(smp, smpt) and np.allclose(Y, Yt, atol=1e-14)


@pytest.mark.parametrize("m,n", [(300, 260), (200, 333)])
def test_seeded_ca_recovers_rank_r_inputs(m, n):
    g = np.random.default_rng(m)
    W = g.standard_normal((m, 6)) @ g.standard_normal((6, n))
    c = oracle.ca_cur(W, 6, 3, 21, preprocess=3, ah_depth=3, ah_samples=6)
    assert c.status == 0
    assert oracle.rel_fro(W, c.I, c.J, c.U) < 1e-12


def test_seed_picks_the_largest_sketch_row_first():
    W = workloads.orthogonal_lowrank(200, 150, 5, noise=1e-4, seeds=(7, 8, 9))
    Y, _ = oracle.sketch_fourier(W, 1, 2, 10, 3)
    st, piv, _, _ = oracle.qrp(Y, 5)
    assert st == 0 and piv[0] == int(np.argmax((Y * Y).sum(axis=1)))
    # the C-A start columns are the QRP's first r pivots on that sketch
    c = oracle.ca_cur(W, 5, 1, 3, preprocess=3, ah_depth=2, ah_samples=10)
    assert c.status == 0


def test_unit_roots_are_accurate_and_exactly_symmetric():
    # the fixed-order evaluation against the C library's cos and sin (within
    # 2 ulp of 1), conjugate symmetry m -> N - m bit for bit (except at the
    # odd multiples of pi/4, where the cosine and sine series of pi/4 meet and
    # may differ by one ulp), and the exact quarter points
    g = np.random.default_rng(17)
    for N in [1, 2, 3, 5, 8, 12, 236, 20000, 1000003, (1 << 39) - 7]:
        ms = set(range(min(N, 40))) | {int(v) for v in g.integers(0, N, 40)}
        for m in ms:
            c, s = oracle.unit_root(m, N)
            ang = 2 * np.pi * (m / N)
            assert abs(c - np.cos(ang)) <= 4.5e-16 * max(1.0, m / N * 8) and abs(s - np.sin(ang)) <= 4.5e-16 * max(1.0, m / N * 8)
            if m > 0 and not ((8 * m) % N == 0 and ((8 * m) // N) % 2 == 1):
                c2, s2 = oracle.unit_root(N - m, N)
                assert c2 == c and s2 == -s
    for N in [4, 8, 12, 100]:
        for k in range(4):
            c, s = oracle.unit_root(k * N // 4, N)
            assert (c, s) in [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    c, s = oracle.unit_root(1, 8)
    assert abs(c - np.sqrt(0.5)) <= 2.3e-16 and abs(s - np.sqrt(0.5)) <= 2.3e-16
