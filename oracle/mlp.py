"""FP64 reference of the near-contact closure network.

TEST INFRASTRUCTURE ONLY: imported by the tests and nothing else.  Plain
numpy, written from the definition of a two-hidden-layer perceptron and the
chain rule; it shares nothing with the GPU kernels.

Network (8 -> 64 -> 64 -> 2, tanh hidden units):
    z1 = x W1 + b1,  h1 = tanh(z1)
    z2 = h1 W2 + b2, h2 = tanh(z2)
    y  = h2 W3 + b3
Loss over a batch of B rows: L = (1/B) sum_rows sum_o (y - t)^2.

Parameters travel as one flat vector in the order W1 (8x64, row-major),
b1 (64), W2 (64x64), b2 (64), W3 (64x2), b3 (2): 4866 values.

quantize=True rounds to FP16 (nearest even) at the points a network with
FP16 weights on FP16 matrix-core operands has: the inputs, every weight
matrix, the hidden activations h1 and h2, and the backward signals (dL/dy,
dL/dz2, dL/dz1), the latter after multiplication by a loss scale S (a choice
of the mixed-precision kernels, not of the problem); biases, sums and the
scale removal are exact here (FP64).  With quantize=False everything is FP64.
"""
import numpy as np

SHAPES = [("W1", (8, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 2)), ("b3", (2,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def _h(a, quantize):
    return np.asarray(a, dtype=np.float16).astype(np.float64) if quantize else np.asarray(a, dtype=np.float64)


def forward(theta, X, quantize=False):
    """Outputs y [B, 2] and the intermediate values the backward pass needs."""
    p = unpack(theta)
    x = _h(X, quantize)
    W1, W2, W3 = (_h(p[k], quantize) for k in ("W1", "W2", "W3"))
    z1 = x @ W1 + p["b1"]
    h1 = _h(np.tanh(z1), quantize)
    z2 = h1 @ W2 + p["b2"]
    h2 = _h(np.tanh(z2), quantize)
    y = h2 @ W3 + p["b3"]
    return y, {"x": x, "h1": h1, "h2": h2, "W1": W1, "W2": W2, "W3": W3}


def loss_and_grad(theta, X, T, quantize=False, scale=1024.0):
    """Loss and its gradient with respect to the flat parameters.  With
    quantize=True the backward signals are multiplied by `scale` before their
    FP16 rounding and divided by it again in the weight gradients."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    y, c = forward(theta, X, quantize)
    r = y - T
    loss = float((r * r).sum() / B)
    S = scale if quantize else 1.0
    gy = _h(S * 2.0 * r / B, quantize)                 # dL/dy, scaled
    dW3 = c["h2"].T @ gy / S
    db3 = gy.sum(axis=0) / S
    gz2 = _h((gy @ c["W3"].T) * (1.0 - c["h2"] ** 2), quantize)  # tanh' = 1 - tanh^2
    dW2 = c["h1"].T @ gz2 / S
    db2 = gz2.sum(axis=0) / S
    gz1 = _h((gz2 @ c["W2"].T) * (1.0 - c["h1"] ** 2), quantize)
    dW1 = c["x"].T @ gz1 / S
    db1 = gz1.sum(axis=0) / S
    return loss, pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3})


def adam(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015, algorithm 1) at step t >= 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
