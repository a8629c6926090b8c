"""The closure network's MFMA kernels against the FP64 oracle (oracle/mlp.py)
at the same FP16 rounding points.

What may differ: the kernels sum in FP32 (products of FP16 values are exact
in FP32) and take tanh as 1 - 2/(exp(2z)+1) in FP32, so a hidden activation
now and then lands on the other side of an FP16 rounding boundary (one FP16
ulp, 2^-11 relative).  Gates: outputs within 2e-3 of max|y| (mean 1e-4), the
loss within 1e-4 relative, the gradient within 2e-3 relative in L2 norm (per
parameter block) -- two orders of magnitude above the FP32 sums, two below
the FP16-versus-FP64 gap of the network itself.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1105_2904_amd import lbm
from paper_1105_2904_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.lib()


def _t(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def _params(seed):
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    theta = wl.mlp_init(seed)
    b = omlp.unpack(theta)
    b["b1"] = rng.uniform(-0.3, 0.3, 64)
    b["b2"] = rng.uniform(-0.3, 0.3, 64)
    b["b3"] = rng.uniform(-0.1, 0.1, 2)
    return omlp.pack(b).astype(np.float32).astype(np.float64)


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(-1.5, 1.5, size=(n, 8)).astype(np.float32).astype(np.float64)
    T = np.stack([np.sin(X[:, 0] * X[:, 1]) + 0.3 * X[:, 2], np.tanh(X[:, 3] - X[:, 4] * X[:, 5])], axis=1)
    return X, T.astype(np.float32).astype(np.float64)


def test_param_count():
    assert lbm.mlp_param_count() == omlp.N_PARAMS == 4866


@pytest.mark.parametrize("n", [1, 17, 1000, 65537])
def test_forward_matches_oracle(n):
    theta = _params(1)
    X, _ = _data(n, 2)
    y = lbm.mlp_forward(_t(theta), _t(X)).cpu().numpy().astype(np.float64)
    yo, _ = omlp.forward(theta, X, quantize=True)
    scale = np.abs(yo).max()
    err = np.abs(y - yo)
    print("forward n=%d max err %.2e mean %.2e (scale %.3f)" % (n, err.max() / scale, err.mean() / scale, scale),
          flush=True)
    assert err.max() <= 2e-3 * scale and err.mean() <= 1e-4 * scale


@pytest.mark.parametrize("n", [64, 777])
def test_gradient_matches_oracle(n):
    theta = _params(3)
    X, T = _data(n, 4)
    loss, g = lbm.mlp_gradient(_t(theta), _t(X), _t(T), loss_scale=1024.0)
    g = g.cpu().numpy().astype(np.float64)
    lo, go = omlp.loss_and_grad(theta, X, T, quantize=True, scale=1024.0)
    assert abs(float(loss.item()) - lo) <= 1e-4 * lo
    k = 0
    for name, shp in omlp.SHAPES:
        m = int(np.prod(shp))
        e = np.linalg.norm(g[k:k + m] - go[k:k + m]) / np.linalg.norm(go[k:k + m])
        print("grad %s rel err %.2e" % (name, e), flush=True)
        assert e <= 2e-3, (name, e)
        k += m
    # and the FP16 gradient is the FP64 gradient to FP16 accuracy
    _, g64 = omlp.loss_and_grad(theta, X, T)
    assert np.linalg.norm(g - g64) <= 3e-2 * np.linalg.norm(g64)


def test_training_on_gpu_fits_a_smooth_target():
    """Adam on the GPU drives the loss of a smooth target down by an order of
    magnitude, and the oracle's forward pass on the trained parameters agrees
    with the loss the kernel reported."""
    import torch
    X, T = _data(4096, 5)
    theta = _t(wl.mlp_init(7))
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    x, t = _t(X), _t(T)
    l0 = float(lbm.mlp_gradient(theta, x, t)[0].item())
    losses = lbm.mlp_train(theta, m, v, x, t, batch=256, steps=3000, lr=3e-3)
    l1 = float(lbm.mlp_gradient(theta, x, t)[0].item())
    lo, _ = omlp.loss_and_grad(theta.cpu().numpy().astype(np.float64), X, T, quantize=True)
    print("training loss %.4e -> %.4e (oracle %.4e), last steps %s" % (l0, l1, lo, losses[-3:].cpu().numpy()),
          flush=True)
    assert l1 < 0.1 * l0
    assert abs(lo - l1) <= 1e-3 * lo
