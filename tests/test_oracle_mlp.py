"""Pins of the oracle's closure network (oracle/mlp.py) against the
mathematics: a one-path network with a closed-form output, central finite
differences of the loss, the FP16-rounded variant against the exact one
within FP16 error, and Adam's first step."""
import numpy as np
import pytest

from oracle import mlp
from paper_1105_2904_amd import workloads as wl


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1, 1, size=(n, 8)), rng.uniform(-0.5, 0.5, size=(n, 2))


def test_parameter_count_and_packing():
    theta = wl.mlp_init(3)
    assert theta.size == mlp.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
    assert np.array_equal(mlp.pack(mlp.unpack(theta)), theta)


def test_single_path_closed_form():
    """Only W1[0,0] = a, W2[0,0] = b, W3[0,:] = (c, d) and b3 = (e, f) are
    non-zero: y = (c tanh(b tanh(a x0)) + e, d tanh(b tanh(a x0)) + f)."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    a, b, c, d, e, f = 0.7, -1.3, 2.0, -0.5, 0.25, 0.125
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][0, 0], p["W3"][0, 1] = a, b, c, d
    p["b3"][:] = (e, f)
    X, _ = _data(50, 1)
    y, _ = mlp.forward(mlp.pack(p), X)
    s = np.tanh(b * np.tanh(a * X[:, 0]))
    assert np.abs(y[:, 0] - (c * s + e)).max() < 1e-15
    assert np.abs(y[:, 1] - (d * s + f)).max() < 1e-15
    # the remaining inputs do not enter
    X2 = X.copy()
    X2[:, 1:] = 0.0
    assert np.array_equal(mlp.forward(mlp.pack(p), X2)[0], y)


def test_gradient_matches_central_differences():
    theta = wl.mlp_init(5) * 1.5
    theta[8 * 64:8 * 64 + 64] = 0.1  # non-zero b1
    X, T = _data(37, 2)
    _, g = mlp.loss_and_grad(theta, X, T)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1, mlp.N_PARAMS - 3]])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss_and_grad(tp, X, T)[0] - mlp.loss_and_grad(tm, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_fp16_rounding_points_stay_within_fp16_error():
    """The FP16-rounded forward and backward (loss scale 1024) agree with the
    FP64 ones to the size FP16 rounding allows (unit roundoff 2^-11 per
    rounding, a few roundings deep)."""
    theta = wl.mlp_init(7)
    X, T = _data(256, 3)
    y, _ = mlp.forward(theta, X)
    yq, _ = mlp.forward(theta, X, quantize=True)
    assert np.abs(yq - y).max() <= 2e-2 * np.abs(y).max()
    assert np.abs(yq - y).max() > 0  # the rounding is really applied
    _, g = mlp.loss_and_grad(theta, X, T)
    _, gq = mlp.loss_and_grad(theta, X, T, quantize=True)
    assert np.linalg.norm(gq - g) <= 2e-2 * np.linalg.norm(g)


def test_adam_first_step_moves_by_lr():
    """After bias correction the first Adam step is -lr * g / (|g| + eps)."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 0.0])
    t1, m, v = mlp.adam(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(t1 - theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_the_loss():
    """Plain Adam on a smooth target lowers the loss: the update direction is
    a descent direction (sign errors in the gradient would raise it)."""
    X, _ = _data(128, 4)
    T = np.stack([np.sin(X[:, 0] + X[:, 1]), X[:, 2] * X[:, 3]], axis=1) * 0.5
    theta = wl.mlp_init(11)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, T)[0]
    for t in range(1, 201):
        _, g = mlp.loss_and_grad(theta, X, T)
        theta, m, v = mlp.adam(theta, m, v, g, t, lr=3e-3)
    assert mlp.loss_and_grad(theta, X, T)[0] < 0.2 * l0
