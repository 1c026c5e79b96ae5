"""C-A with each start (random, abridged SRHT, bidiagonal product, abridged
Fourier) on the Laplacian single-layer input of the tests of the
pre-processors, on the GPU beside the oracle.

Every run must reach the oracle's status and an error within 20 times the
SVD's optimal rank-r error.  The parity bar of the other C-A paths applies
where the oracle's smallest decision margin is at least 1e-6: equal index
sets, and reconstructions agreeing to 1e-6 (FP64 input) or 1e-4 (FP32).
This input is circulant and symmetric, so its pivot searches meet exact
ties in value.  The oracle reports margin 0 and the comparison rests on the
error bar: both sides break an exact tie toward the lower index, but
rounding in the updates decides which candidates stay tied."""
import numpy as np
import pytest

import oracle
from paper_1710_07946_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lra():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07946_amd as lra
    lra.load()
    return lra


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("pre,depth,samples", [(0, 0, 0), (1, 3, 24), (2, 3, 24), (3, 3, 12)])
@pytest.mark.parametrize("n,r", [(512, 11), (1000, 21)])
def test_ca_on_the_laplacian(lra, n, r, pre, depth, samples, dt):
    W = workloads.laplacian_single_layer(n)
    if dt == "f32":
        W = W.astype(np.float32)
    kw = {} if pre == 0 else dict(preprocess=pre, ah_depth=depth, ah_samples=samples)
    print("laplacian n=%d r=%d %s %s" % (n, r, dt, kw), flush=True)
    o = oracle.ca_cur(W, r, 4, 17, **kw)
    out = lra.lra_cur(torch.from_numpy(W).cuda(), r, 4, 17, **kw)
    torch.cuda.synchronize()
    I, J, U, info = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy(), out.info()
    assert info["status"] == o.status == 0
    W64 = W.astype(np.float64)
    err = np.linalg.norm(W64 - W64[:, J] @ U @ W64[I]) / np.linalg.norm(W64)
    s = np.linalg.svd(W64, compute_uv=False)
    assert err <= 20 * np.sqrt((s[r:] ** 2).sum()) / np.linalg.norm(W64) + (1e-6 if dt == "f32" else 0)
    if o.min_margin >= 1e-6:
        assert I.tolist() == o.I.tolist() and J.tolist() == o.J.tolist()
        Xo, Xg = W64[:, o.J] @ o.U @ W64[o.I], W64[:, J] @ U @ W64[I]
        assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) <= (1e-6 if dt == "f64" else 1e-4)
