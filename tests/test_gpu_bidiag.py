"""GPU parity of the C-A path started from the quasi-Gaussian multiplier of
random bidiagonal factors (eq. (def11), section on pre-processing with quasi
Gaussian matrices) against the oracle; bar as in test_gpu_parity."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads
from test_gpu_parity import assert_parity, gpu_cur

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


@pytest.mark.parametrize("q,l", [(0, 20), (1, 20), (3, 20), (6, 30)])
def test_bidiag_start_512_fp64(lra, q, l):
    A = workloads.orthogonal_lowrank()
    kw = dict(preprocess=2, ah_depth=q, ah_samples=l)
    o = oracle.ca_cur(A, 10, 3, 2001, **kw)
    g = gpu_cur(lra, A, 10, 3, 2001, **kw)
    assert_parity(A, g, o, 1e-6)


def test_bidiag_start_wide_fp64(lra):
    # m < n: the multiplier acts on the columns; its QRP picks rows and one row
    # step turns them into the start columns
    A = workloads.orthogonal_lowrank(300, 700, 8, noise=1e-7, seeds=(11, 12, 13))
    kw = dict(preprocess=2, ah_depth=3, ah_samples=24)
    o = oracle.ca_cur(A, 8, 3, 5, **kw)
    g = gpu_cur(lra, A, 8, 3, 5, **kw)
    assert_parity(A, g, o, 1e-6)


def test_bidiag_start_fp32_team(lra):
    A = workloads.factor_gaussian(3000, 2000, 16, 1e-6, seeds=(61, 62, 63))
    kw = dict(preprocess=2, ah_depth=3, ah_samples=64)
    o = oracle.ca_cur(A, 16, 3, 9, **kw)
    g = gpu_cur(lra, A, 16, 3, 9, **kw)
    assert g[3]["team_size"] > 1
    assert_parity(A, g, o, 1e-4)


def test_bidiag_invalid_options(lra):
    A = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(lra.LraError):
        lra.lra_cur(A, 4, 1, 0, preprocess=2, ah_depth=7, ah_samples=8)   # 2^7 terms
    with pytest.raises(lra.LraError):
        lra.lra_cur(A, 4, 1, 0, preprocess=2, ah_depth=3, ah_samples=3)   # l < r
