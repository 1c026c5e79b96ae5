"""GPU parity of the cynical CUR (Section 1.3, Fig. 3; Tests 3 and Tests 4 of
Section 13) against the oracle on the same seeded inputs; bar as in
test_gpu_parity."""
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


def gpu_cynical(lra, A_np, r, k, loops, sweeps, seed, **kw):
    print("gpu_cynical", A_np.shape, A_np.dtype, "r=%d k=%d loops=%d sweeps=%d seed=%d" % (r, k, loops, sweeps, seed),
          kw, flush=True)
    out = lra.lra_cur_cynical(torch.from_numpy(A_np).cuda(), r, k, loops, sweeps, seed, **kw)
    torch.cuda.synchronize()
    return out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()


@pytest.mark.parametrize("loops", [0, 1, 2])
def test_cynical_512_fp64(lra, loops):
    A = workloads.orthogonal_lowrank()
    o = oracle.cynical(A, 10, 40, loops, 3, 2001)
    g = gpu_cynical(lra, A, 10, 40, loops, 3, 2001)
    assert_parity(A, g, o, 1e-6, margin=False)
    assert g[3]["team_size"] == (1 if loops == 0 else 4)


def test_cynical_fp32_rank16_k64_team(lra):
    # Tests 4 with k = 4r = 64 on a 3000 x 2000 FP32 factor-Gaussian rank-16
    # input; the rank-64 loop runs over a team of 19 workgroups
    A = workloads.factor_gaussian(3000, 2000, 16, 1e-6, seeds=(61, 62, 63))
    o = oracle.cynical(A, 16, 64, 1, 3, 9)
    g = gpu_cynical(lra, A, 16, 64, 1, 3, 9)
    assert g[3]["team_size"] > 1
    assert_parity(A, g, o, 1e-4, margin=False)


def test_cynical_team_size_does_not_change_results(lra):
    # (team 3 is the smallest whose 700 / 3-row slices of 36 doubles fit LDS)
    A = workloads.orthogonal_lowrank(700, 530, 9, noise=1e-8, seeds=(5, 6, 7))
    ref = gpu_cynical(lra, A, 9, 36, 1, 3, 77, team_size=3)
    for team in (4, 7):
        g = gpu_cynical(lra, A, 9, 36, 1, 3, 77, team_size=team)
        assert g[3]["team_size"] == team
        assert g[0].tolist() == ref[0].tolist() and g[1].tolist() == ref[1].tolist()
        assert np.array_equal(g[2], ref[2])


@pytest.mark.parametrize("loops", [0, 1])
def test_cynical_non_finite_entry(lra, loops):
    # a NaN in the first drawn column: the rank-k column step (loops = 1) or
    # the sketch W[K, L] (loops = 0) reads it; both sides report LRA_EINVAL
    A = workloads.orthogonal_lowrank(300, 200, 5, noise=1e-6, seeds=(1, 2, 3))
    j0 = int(np.sort(oracle.draw_distinct(4, 0, 200, 20))[0])
    A[:, j0] = np.nan
    o = oracle.cynical(A, 5, 20, loops, 2, 4)
    g = gpu_cynical(lra, A, 5, 20, loops, 2, 4)
    assert o.status == lra.LRA_EINVAL
    assert g[3]["status"] == lra.LRA_EINVAL
    assert (g[0] == -1).all() and np.isnan(g[2]).all()
