"""The Laplacian single-layer input (the integral-equation matrices (i) of
the tests of the pre-processors) and the oracle's C-A on it with each start.

The generator is pinned to closed forms: log|2 - z| is harmonic in |z| < 2,
so its integral over the whole unit circle is 2 pi log 2 (mean value
property), and its Fourier series log 2 - sum_k cos(k phi) / (k 2^k) gives
every arc integral exactly; the matrix is circulant with unit spectral
norm and singular values falling by about half per Fourier mode.  The C-A
runs are checked against the SVD's optimal error."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads


def arc_integral_series(n, terms=60):
    # integral of log|2 - e^{i phi}| over [2 pi d / n, 2 pi (d + 1) / n]
    h = 2 * np.pi / n
    d = np.arange(n)
    k = np.arange(1, terms + 1)[:, None]
    a, b = h * d[None, :], h * (d[None, :] + 1)
    return h * np.log(2.0) - ((np.sin(k * b) - np.sin(k * a)) / (k * k * 2.0 ** k)).sum(axis=0)


@pytest.mark.parametrize("n,quad", [(7, 24), (64, 8), (300, 8)])
def test_entries_match_the_fourier_series(n, quad):
    W = workloads.laplacian_single_layer(n, quad=quad)
    c = arc_integral_series(n)
    psi = 1.0 / np.abs(np.fft.fft(c)).max()
    assert np.allclose(W[0], psi * c, rtol=0, atol=1e-14)
    # the whole circle: mean value property
    assert abs(W[0].sum() / psi - 2 * np.pi * np.log(2.0)) <= 1e-13


def test_circulant_with_unit_norm_and_halving_spectrum():
    n = 200
    W = workloads.laplacian_single_layer(n)
    for i in (1, 57, 199):
        assert np.array_equal(W[i], np.roll(W[0], i))
    s = np.linalg.svd(W, compute_uv=False)
    assert abs(s[0] - 1.0) <= 1e-13
    # modes +-k share a singular value, proportional to 1 / (k 2^k) up to
    # the arc average sin(k h / 2) / (k h / 2), h = 2 pi / n
    pairs = s[1:21:2]
    assert np.allclose(s[1:21:2], s[2:22:2], rtol=1e-10)
    k = np.arange(1, 11)
    x = k * np.pi / n
    model = np.sin(x) / x / (k * 2.0 ** k)
    assert np.allclose(pairs / pairs[0], model / model[0], rtol=1e-6)


@pytest.mark.parametrize("pre,depth,samples", [(0, 0, 0), (1, 3, 24), (2, 3, 24), (3, 3, 12)])
def test_ca_with_each_start_is_near_optimal(pre, depth, samples):
    n, r = 256, 11
    W = workloads.laplacian_single_layer(n)
    kw = {} if pre == 0 else dict(preprocess=pre, ah_depth=depth, ah_samples=samples)
    c = oracle.ca_cur(W, r, 4, 5, **kw)
    assert c.status == 0
    s = np.linalg.svd(W, compute_uv=False)
    opt = np.sqrt((s[r:] ** 2).sum()) / np.linalg.norm(W)
    assert oracle.rel_fro(W, c.I, c.J, c.U) <= 20 * opt
