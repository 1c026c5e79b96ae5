"""GPU parity of C-A on the pre-processed matrix W' = W D (H_{2^d} (x) I_s)
(Tests 2 with abridged randomized Hadamard pre-processing, Section 13),
whose entries the kernel forms on the fly, against the oracle's C-A on the
oracle's W'; bar as in test_gpu_parity."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


def gpu_hadamard(lra, A_np, r, sweeps, seed, d, **kw):
    print("gpu_hadamard", A_np.shape, A_np.dtype, "r=%d sweeps=%d seed=%d d=%d" % (r, sweeps, seed, d), kw,
          flush=True)
    out = lra.lra_cur_hadamard(torch.from_numpy(A_np).cuda(), r, sweeps, seed, d, track_margin=True, **kw)
    torch.cuda.synchronize()
    return out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()


@pytest.mark.parametrize("d", [0, 1, 3, 6])
def test_preprocessed_512_fp64(lra, d):
    A = workloads.orthogonal_lowrank()
    Wp = oracle.hadamard_apply(A, d, 2001)
    o = oracle.ca_cur(Wp, 10, 3, 2001)
    g = gpu_hadamard(lra, A, 10, 3, 2001, d)
    assert_parity(Wp, g, o, 1e-6)


@pytest.mark.parametrize("m,n,r,d,team", [(1000, 999, 20, 3, 0), (300, 700, 8, 2, 5), (700, 300, 8, 3, 1)])
def test_preprocessed_ragged_fp32(lra, m, n, r, d, team):
    # n not a multiple of 2^d: W is zero-padded to N columns
    A = workloads.factor_gaussian(m, n, r, 1e-6, seeds=(m, n, d)).astype(np.float32)
    Wp = oracle.hadamard_apply(A, d, 17)
    o = oracle.ca_cur(Wp, r, 3, 17)
    g = gpu_hadamard(lra, A, r, 3, 17, d, team_size=team)
    assert_parity(Wp, g, o, 1e-4)


def test_lra_of_w_from_the_preprocessed_cur(lra):
    # W ~ W'[:, J] U W'[I, :] M^T / 2^d with the GPU's sets and nucleus
    A = workloads.orthogonal_lowrank(400, 300, 7, noise=1e-9, seeds=(2, 3, 4))
    d = 3
    I, J, U, info = gpu_hadamard(lra, A, 7, 3, 5, d)
    assert info["status"] == 0
    Wp = oracle.hadamard_apply(A, d, 5)
    N = Wp.shape[1]
    # rows of M^T / 2^d applied through the oracle's transform of the identity
    Mt = oracle.hadamard_apply(np.eye(300), d, 5)  # = M restricted to the first 300 rows
    approx = Wp[:, J] @ U @ Wp[I, :] @ Mt.T / (1 << d)
    assert approx.shape == A.shape and N >= 300
    assert np.linalg.norm(approx - A) <= 1e-6 * np.linalg.norm(A)
