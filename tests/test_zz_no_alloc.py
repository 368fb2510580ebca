"""The no-allocation variant of the network's loss gradient
(ep_mlp_loss_grad_noalloc, static device scratch) against ep_mlp_loss_grad on
the same parameters and batches, through the C ABI: equal bit for bit on two
calls in a row, the second with a smaller batch, for FP32 and BF16 products;
batches beyond the stated maximum are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from paper_1805_04155_amd import _ep  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402


def _batch(rng, n):
    X = np.zeros((n, _ep.MLP_XS), np.float32)
    X[:, :_ep.MLP_IN] = rng.standard_normal((n, _ep.MLP_IN)).astype(np.float32)
    T = np.zeros((n, _ep.MLP_YS), np.float32)
    T[:, :6] = 0.1 * rng.standard_normal((n, 6)).astype(np.float32)
    T[:, 6] = (rng.random(n) < 0.4).astype(np.float32)
    return (torch.as_tensor(X, device="cuda").contiguous(),
            torch.as_tensor(T, device="cuda").contiguous())


@pytest.mark.parametrize("prec", [_ep.EP_FP32, _ep.EP_BF16])
def test_noalloc_loss_grad_equals_the_allocating_entry_point(prec):
    rng = np.random.default_rng(21)
    params = torch.as_tensor(W.mlp_he_uniform(3).astype(np.float32), device="cuda").contiguous()
    m = _ep.Mlp(prec, _ep.MLP_NOALLOC_MAX_BATCH)
    try:
        _ep.ep_mlp_set_params(m.h, params)
        for n in (_ep.MLP_NOALLOC_MAX_BATCH, 333):
            X, T = _batch(rng, n)
            g_ref = torch.zeros(_ep.MLP_NPARAM, dtype=torch.float32, device="cuda")
            l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
            _ep.ep_mlp_loss_grad(m.h, X, T, n, g_ref, l_ref)
            g = torch.full((_ep.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
            loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
            _ep.ep_mlp_loss_grad_noalloc(prec, params, X, T, n, g, loss)
            torch.cuda.synchronize()
            assert torch.equal(g, g_ref), n
            assert torch.equal(loss, l_ref), n
            assert torch.isfinite(g).all() and float(g.abs().max()) > 0.0
    finally:
        m.close()


def test_noalloc_loss_grad_refuses_oversized_batches():
    params = torch.zeros(_ep.MLP_NPARAM, dtype=torch.float32, device="cuda")
    n = _ep.MLP_NOALLOC_MAX_BATCH + 1
    X = torch.zeros((n, _ep.MLP_XS), dtype=torch.float32, device="cuda")
    T = torch.zeros((n, _ep.MLP_YS), dtype=torch.float32, device="cuda")
    with pytest.raises(_ep.EpError) as ei:
        _ep.ep_mlp_loss_grad_noalloc(_ep.EP_FP32, params, X, T, n)
    assert ei.value.status == _ep.EP_EINVAL
    assert "EP_MLP_NOALLOC_MAX_BATCH" in str(ei.value)
