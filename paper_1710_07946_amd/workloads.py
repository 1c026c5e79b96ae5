"""Seeded synthetic inputs for the C-A CUR path.

This module only *makes inputs*: it holds none of the method's arithmetic and
is shared by the tests, the benchmark and the smoke check, so that the GPU
library and the CPU oracle always see identical matrices.  Every generator is
a pure function of its seeds (NumPy ``default_rng``), so the same call gives
the same bytes on any machine.

Workloads (shapes and value distributions of the paper's experiments, which
used factor-Gaussian matrices plus small Gaussian noise, and FMM far-field
blocks; see the experiments section and the FMM section of the paper):

* ``orthogonal_lowrank``  A = U diag(sigma) V^T + noise, U, V from QR of
  Gaussian matrices (512 x 512, rank 10, sigma_i = 2^-i, noise std 1e-10).
* ``factor_gaussian``     A = X Y / ||X Y||_F + noise (20000 x 20000, rank 50,
  noise std 1e-6), the perturbed factor-Gaussian family of the experiments.
* ``fmm_blocks``          off-diagonal interaction blocks 1/|x - y| between
  well separated 2-D point clusters.
* ``laplacian_single_layer``  the discretized single-layer potential of the
  Laplacian from the unit circle to the circle of radius 2 (the integral-
  equation input of the tests of the pre-processors), normalized to unit
  spectral norm; deterministic.
* ``graded_lowrank``      X diag(s) Y + noise with Gaussian factors and the
  column scales s_a = 10^(-2 a / (r - 1)) (numerical rank r, singular values
  spread over two decades), FP32, the stand-in for the integral-equation
  inputs of the tests of C-A with DMM08 sampling (1000 x 1000, numerical
  rank up to 25, Tables 7 and 8).
* ``decaying_spectrum``   tall matrix with 64 unit singular values followed by
  an i^-2 decay floored at 1e-7 (generated on the device: its 8.8 TFLOP
  construction is out of reach of a host).

The ``*_device`` variants build the same families with torch on a GPU (the
large batched and tall workloads), seeded by the same integers; the
benchmark uses them to avoid minutes of host-side generation.

The noise parameter is a standard deviation.
"""
from __future__ import annotations

import numpy as np


def orthogonal_lowrank(m: int = 512, n: int = 512, r: int = 10, noise: float = 1e-10,
                       seeds=(1001, 1002, 1003), sigma=None, dtype=np.float64) -> np.ndarray:
    """U diag(sigma) V^T + noise * N(0,1); sigma defaults to 2^-i, i = 0..r-1."""
    U, _ = np.linalg.qr(np.random.default_rng(seeds[0]).standard_normal((m, r)))
    V, _ = np.linalg.qr(np.random.default_rng(seeds[1]).standard_normal((n, r)))
    if sigma is None:
        sigma = 2.0 ** -np.arange(r)
    A = (U * np.asarray(sigma, np.float64)) @ V.T
    if noise:
        A = A + noise * np.random.default_rng(seeds[2]).standard_normal((m, n))
    return np.ascontiguousarray(A.astype(dtype))


def factor_gaussian(m: int, n: int, r: int, noise: float, seeds=(1011, 1012, 1013),
                    dtype=np.float32, chunk_rows: int = 2048) -> np.ndarray:
    """X Y scaled to unit Frobenius norm, plus i.i.d. N(0, noise^2), rows made in chunks."""
    X = np.random.default_rng(seeds[0]).standard_normal((m, r))
    Y = np.random.default_rng(seeds[1]).standard_normal((r, n))
    # ||X Y||_F^2 = trace(X^T X Y Y^T)
    fro = float(np.sqrt(np.trace((X.T @ X) @ (Y @ Y.T))))
    g = np.random.default_rng(seeds[2])
    A = np.empty((m, n), dtype)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = (X[r0:r1] @ Y) / fro
        if noise:
            blk += noise * g.standard_normal((r1 - r0, n))
        A[r0:r1] = blk.astype(dtype)
    return A


def fmm_block_shapes(count: int, lo: int = 64, hi: int = 1024, seed: int = 1021):
    """Independent uniform row / column counts in [lo, hi] for each block."""
    g = np.random.default_rng(seed)
    ms = g.integers(lo, hi + 1, size=count)
    ns = g.integers(lo, hi + 1, size=count)
    return ms.astype(np.int64), ns.astype(np.int64)


def fmm_block(m: int, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """K_ij = 1/|x_i - y_j| for x uniform in [0,1]^2 and y uniform in the unit
    box [1+g, 2+g] x [0,1], g ~ U[2,3] (separation at least two box widths)."""
    gen = np.random.default_rng(seed)
    gap = gen.uniform(2.0, 3.0)
    x = gen.uniform(0.0, 1.0, size=(m, 2))
    y = gen.uniform(0.0, 1.0, size=(n, 2))
    y[:, 0] += 1.0 + gap
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    return (1.0 / d).astype(dtype)


def fmm_batch(count: int, shape_seed: int = 1021, block_seed0: int = 1022000, align_elems: int = 64,
              dtype=np.float32):
    """All blocks stored row-major one after another in one flat buffer.

    Returns (flat buffer, descriptors int64[count, 4] = (offset, m, n, lda)).
    Each block starts at a multiple of ``align_elems`` elements (256 B for FP32).
    """
    ms, ns = fmm_block_shapes(count, seed=shape_seed)
    desc = np.zeros((count, 4), np.int64)
    off = 0
    for b in range(count):
        desc[b] = (off, ms[b], ns[b], ns[b])
        off += int(ms[b] * ns[b])
        off = (off + align_elems - 1) // align_elems * align_elems
    flat = np.zeros(off, dtype)
    for b in range(count):
        o, m, n, _ = desc[b]
        flat[o:o + m * n] = fmm_block(int(m), int(n), block_seed0 + b, dtype).ravel()
    return flat, desc


def fmm_points(count: int, shape_seed: int = 1021, block_seed0: int = 1022000):
    """The point sets behind ``fmm_batch``'s blocks (same shapes and streams),
    all in one float64 array of shape (P, 2): block b's m row points, then its
    n column points.  Returns (points, descriptors int64[count, 4] =
    (x_off, y_off, m, n))."""
    ms, ns = fmm_block_shapes(count, seed=shape_seed)
    desc = np.zeros((count, 4), np.int64)
    parts = []
    off = 0
    for b in range(count):
        m, n = int(ms[b]), int(ns[b])
        gen = np.random.default_rng(block_seed0 + b)
        gap = gen.uniform(2.0, 3.0)
        x = gen.uniform(0.0, 1.0, size=(m, 2))
        y = gen.uniform(0.0, 1.0, size=(n, 2))
        y[:, 0] += 1.0 + gap
        desc[b] = (off, off + m, m, n)
        parts += [x, y]
        off += m + n
    return np.ascontiguousarray(np.concatenate(parts, axis=0)), desc


def laplacian_single_layer(n: int, quad: int = 8, dtype=np.float64) -> np.ndarray:
    """n x n matrix w_ij = psi * integral of log|2 omega^i - y| over the arc of
    the unit circle between the angles 2 pi j / n and 2 pi (j + 1) / n,
    omega = exp(2 pi i / n), psi such that ||W||_2 = 1 (the input matrices
    (i) of the tests of the pre-processors).

    The distance from 2 omega^i to a point of the arc depends only on the
    angle between them, so w_ij = c[(j - i) mod n] with c[d] the integral
    of log|2 - e^{i phi}| over [2 pi d / n, 2 pi (d + 1) / n], evaluated by
    `quad`-point Gauss-Legendre on each arc (the integrand is analytic
    there: |2 - e^{i phi}| >= 1).  W is circulant, so its singular values
    are |DFT(c)| and psi = 1 / max |DFT(c)|."""
    h = 2.0 * np.pi / n
    x, w = np.polynomial.legendre.leggauss(quad)
    d = np.arange(n, dtype=np.float64)
    phi = h * (d[:, None] + 0.5 * (x[None, :] + 1.0))
    c = 0.5 * h * (np.log(np.abs(2.0 - np.exp(1j * phi))) * w[None, :]).sum(axis=1)
    c /= np.abs(np.fft.fft(c)).max()
    idx = (np.arange(n)[None, :] - np.arange(n)[:, None]) % n
    return np.ascontiguousarray(c[idx].astype(dtype))


def graded_lowrank(m: int, n: int, r: int, noise: float, seed: int, dtype=np.float32) -> np.ndarray:
    """X diag(s) Y / ||X diag(s) Y||_F + N(0, noise^2), X (m x r), Y (r x n)
    standard Gaussian, s_a = 10^(-2 a / (r - 1)) (s = 1 for r = 1)."""
    g = np.random.default_rng(seed)
    s = 10.0 ** (-2.0 * np.arange(r) / max(r - 1, 1))
    A = (g.standard_normal((m, r)) * s) @ g.standard_normal((r, n))
    A /= np.linalg.norm(A)
    A += noise * g.standard_normal((m, n))
    return np.ascontiguousarray(A.astype(dtype))


def graded_lowrank_batch_device(count: int, m: int, n: int, r: int, noise: float, seed0: int, device):
    """`count` ``graded_lowrank`` blocks (FP32) generated on a GPU by torch's
    device generator (block b seeded with seed0 + b), stored back to back in a
    flat tensor.  Returns (flat device tensor, descriptors int64[count, 4])."""
    import torch
    desc = np.array([(b * m * n, m, n, n) for b in range(count)], np.int64)
    flat = torch.empty(count * m * n, dtype=torch.float32, device=device)
    s = torch.tensor(10.0 ** (-2.0 * np.arange(r) / max(r - 1, 1)), dtype=torch.float64, device=device)
    g = torch.Generator(device=device)
    for b in range(count):
        g.manual_seed(seed0 + b)
        X = torch.randn(m, r, generator=g, device=device, dtype=torch.float64) * s
        Y = torch.randn(r, n, generator=g, device=device, dtype=torch.float64)
        A = X @ Y
        A /= torch.linalg.norm(A)
        A += noise * torch.randn(m, n, generator=g, device=device, dtype=torch.float64)
        flat[b * m * n:(b + 1) * m * n] = A.to(torch.float32).reshape(-1)
    return flat, desc


def decaying_spectrum_sigma(n: int, lead: int = 64, floor: float = 1e-7) -> np.ndarray:
    """sigma_i = 1 for i <= lead, max(i^-2, floor) after (1-based i)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    s = np.maximum(i ** -2.0, floor)
    s[:lead] = 1.0
    return s


def sample_omega(m: int, n: int, count: int, seed: int):
    """`count` distinct entries drawn uniformly, returned as (rows, cols) sorted by row then column."""
    g = np.random.default_rng(seed)
    flat = g.choice(m * n, size=count, replace=False)
    flat.sort()
    return (flat // n).astype(np.int64), (flat % n).astype(np.int64)


# ---------------------------------------------------------------- device-side generators
def fmm_batch_device(count: int, device, shape_seed: int = 1021, block_seed0: int = 1022000,
                     align_elems: int = 64, shapes=None):
    """``fmm_batch`` evaluated on a GPU: the same shapes, points and layout (points
    from the same NumPy streams), kernel values computed in FP64 and rounded
    to FP32.  ``shapes`` = (ms, ns) replaces the seeded shapes.  Returns (flat
    device tensor, descriptors int64[count, 4])."""
    import torch
    ms, ns = fmm_block_shapes(count, seed=shape_seed) if shapes is None else shapes
    desc = np.zeros((count, 4), np.int64)
    off = 0
    for b in range(count):
        desc[b] = (off, ms[b], ns[b], ns[b])
        off += int(ms[b] * ns[b])
        off = (off + align_elems - 1) // align_elems * align_elems
    flat = torch.zeros(off, dtype=torch.float32, device=device)
    for b in range(count):
        o, m, n, _ = (int(v) for v in desc[b])
        gen = np.random.default_rng(block_seed0 + b)
        gap = gen.uniform(2.0, 3.0)
        x = gen.uniform(0.0, 1.0, size=(m, 2))
        y = gen.uniform(0.0, 1.0, size=(n, 2))
        y[:, 0] += 1.0 + gap
        xd = torch.from_numpy(x).to(device)
        yd = torch.from_numpy(y).to(device)
        dx = xd[:, None, 0] - yd[None, :, 0]
        dy = xd[:, None, 1] - yd[None, :, 1]
        d = torch.sqrt(dx * dx + dy * dy)
        flat[o:o + m * n] = (1.0 / d).to(torch.float32).reshape(-1)
    return flat, desc


def factor_gaussian_device(m: int, n: int, r: int, noise: float, seed: int, device, dtype=None):
    """X Y / ||X Y||_F + N(0, noise^2) with X, Y standard Gaussian (rank r),
    drawn by torch's device generator seeded with ``seed``; FP32 by default."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    X = torch.randn(m, r, generator=g, device=device, dtype=torch.float64)
    Y = torch.randn(r, n, generator=g, device=device, dtype=torch.float64)
    fro = torch.sqrt(torch.trace((X.T @ X) @ (Y @ Y.T)))
    A = (X @ Y) / fro
    if noise:
        A += noise * torch.randn(m, n, generator=g, device=device, dtype=torch.float64)
    return A.to(dtype)


def decaying_spectrum_device(m: int = 65536, n: int = 8192, lead: int = 64, floor: float = 1e-7,
                             seed: int = 1031, device="cuda", dtype=None, chunk_rows: int = 8192):
    """X diag(sigma) Y^T / sqrt(n) with X (m x n), Y (n x n) standard Gaussian and
    sigma from ``decaying_spectrum_sigma`` (numerical rank ``lead``), built in
    row chunks in FP64 on the device and rounded to ``dtype`` (FP32 default)."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sig = torch.from_numpy(decaying_spectrum_sigma(n, lead, floor)).to(device)
    Y = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    SY = (sig[:, None] * Y.T) / float(np.sqrt(n))   # diag(sigma) Y^T / sqrt(n)
    del Y
    A = torch.empty(m, n, dtype=dtype, device=device)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        X = torch.randn(r1 - r0, n, generator=g, device=device, dtype=torch.float64)
        A[r0:r1] = (X @ SY).to(dtype)
    return A
