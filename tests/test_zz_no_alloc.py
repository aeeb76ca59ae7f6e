"""The no-allocation loss-and-gradient entry point (static device staging)
against the allocating one on the same data: bit-identical loss and
gradient, on two calls in a row, the second with a smaller batch, and the
size limit and pointer checks."""
import numpy as np
import pytest

from paper_1612_01501_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def infoli():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1612_01501_amd import infoli as mod
    mod.lib()
    return mod


def _params(seed):
    w = I.mlp_init_params(seed).astype(np.float64)
    w += I.rng(seed + 1).normal(0.0, 0.02, w.shape)
    return w.astype(np.float32)


def _noalloc(infoli, torch, w, x, t):
    dev = torch.device("cuda", 0)
    dw = torch.from_numpy(w).to(dev)
    dx = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
    dt = torch.from_numpy(np.ascontiguousarray(t, np.float32)).to(dev)
    dl = torch.full((1,), float("nan"), device=dev)
    dg = torch.full((infoli.MLP_PARAMS,), float("nan"), device=dev)
    stream = torch.cuda.current_stream(dev)
    infoli.mlp_loss_grad_noalloc(dw.data_ptr(), dx.data_ptr(), dt.data_ptr(), x.shape[0], dl.data_ptr(),
                                 dg.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return float(dl.cpu().numpy()[0]), dg.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(infoli):
    import torch
    w = _params(21)
    for batch, seed in ((8192, 31), (1040, 32)):          # the limit, then a smaller batch
        print(f"no-alloc loss/grad: batch {batch}, seed {seed}", flush=True)
        x, t = I.mlp_batch(batch, seed)
        loss_a, g_a = infoli.mlp_loss_grad(w, x, t)
        loss_b, g_b = _noalloc(infoli, torch, w, x, t)
        assert np.isfinite(loss_a) and np.all(np.isfinite(g_a))
        assert loss_b == loss_a, (loss_b, loss_a)
        np.testing.assert_array_equal(g_b, g_a)


def test_noalloc_rejects_oversize_and_host_pointers(infoli):
    import torch
    dev = torch.device("cuda", 0)
    big = 8192 + 16
    dw = torch.zeros(infoli.MLP_PARAMS, device=dev)
    dx = torch.zeros((big, 16), device=dev)
    dg = torch.zeros(infoli.MLP_PARAMS, device=dev)
    with pytest.raises(infoli.InfoliError) as e:
        infoli.mlp_loss_grad_noalloc(dw.data_ptr(), dx.data_ptr(), dx.data_ptr(), big, 0, dg.data_ptr())
    assert e.value.status == 1 and "8192" in str(e.value)
    with pytest.raises(infoli.InfoliError) as e:
        infoli.mlp_loss_grad_noalloc(dw.data_ptr(), dx.data_ptr(), dx.data_ptr(), 24, 0, dg.data_ptr())
    assert e.value.status == 1
    host = np.zeros((64, 16), np.float32)
    with pytest.raises(infoli.InfoliError) as e:
        infoli.mlp_loss_grad_noalloc(dw.data_ptr(), host.ctypes.data, dx.data_ptr(), 64, 0, dg.data_ptr())
    assert e.value.status == 1 and "device memory" in str(e.value)
    torch.cuda.synchronize()
    # the device is still usable afterwards
    w = _params(4)
    x, t = I.mlp_batch(64, 5)
    la, ga = infoli.mlp_loss_grad(w, x, t)
    lb, gb = _noalloc(infoli, torch, w, x, t)
    assert la == lb
    np.testing.assert_array_equal(ga, gb)
