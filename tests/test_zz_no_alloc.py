"""The allocation-free gradient entry point (rbdi_mlp_grad_noalloc, through the
C ABI) against rbdi_mlp_grad on the same network and samples: two calls in a
row, the second with fewer samples, each bitwise equal (same kernels, same
summation order); the size limit is enforced."""
import numpy as np
import pytest

from oracle import mlp as omlp
from parity_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbdi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_11806_amd import rbdi as r
    r.load()
    return r


def test_grad_noalloc_equals_grad(rbdi):
    import torch
    rng = np.random.default_rng(17)
    p = omlp.init_params(seed=19).astype(np.float32)
    net = rbdi.Mlp(p, 0.05)
    stream = torch.cuda.current_stream()
    for n in (rbdi.MLP_GRAD_NOALLOC_MAX, 1000):
        announce(f"mlp_grad_noalloc n={n}")
        z = rng.normal(size=(n, 6)).astype(np.float32)
        t = rng.normal(size=(n, 6)).astype(np.float32)
        g_ref, loss_ref = net.grad(z, t)
        zd = torch.from_numpy(z).cuda()
        td = torch.from_numpy(t).cuda()
        gd = torch.full((rbdi.N_MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        ld = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.grad_noalloc(zd, td, gd, ld, stream=stream)
        stream.synchronize()
        g, loss = gd.cpu().numpy(), float(ld.cpu().numpy()[0])
        assert np.array_equal(g, g_ref), np.abs(g - g_ref).max()
        assert loss == loss_ref
    # beyond the fixed array: a clear error, nothing launched
    n = rbdi.MLP_GRAD_NOALLOC_MAX + 1
    zd = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(rbdi.RbdiError, match="outside"):
        net.grad_noalloc(zd, zd, gd, ld, stream=stream)
