"""The edge-wise warm-start network of the learned BP warm start, in plain
float64 NumPy (oracle; test infrastructure only).

The paper leaves the BP initialisation open beyond uniform messages and its
trap analysis (Sec. "BP Fixed-Point Multiplicity"): a BP started elsewhere may
land on another fixed point or need fewer sweeps.  The learned warm start
proposes the measurement-BP messages of a layer from local information; the
network is a two-layer perceptron applied to every component of every directed
edge message independently:

    z = W1 x + b1            (hidden width H = 128, x: F features)
    a = tanh(z)
    y = w2 . a + b2          (one output: the correction to the base message)

with BF16 weights and inputs and float32 accumulation on the device.  This
module computes the same function and its gradients in float64 from the
BF16-rounded weights and inputs, so that the device's forward and backward
kernels can be compared with it, and it is itself pinned by finite differences.

Loss: mean squared error over the rows, L = sum_r (y_r - t_r)^2 / n.
"""

import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64: keep the top 16 bits of the float32 pattern after adding
    0x7FFF plus the lowest kept bit (non-finite values are not expected)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta, F, H):
    """Flat parameter vector -> (W1 [H x F], b1 [H], w2 [H], b2 scalar)."""
    theta = np.asarray(theta, dtype=np.float64)
    W1 = theta[: H * F].reshape(H, F)
    b1 = theta[H * F: H * F + H]
    w2 = theta[H * F + H: H * F + 2 * H]
    b2 = theta[H * F + 2 * H]
    return W1, b1, w2, b2


def n_params(F, H):
    return H * F + 2 * H + 1


def forward(theta, X, F, H, bf16=True):
    """y (n) and the hidden activations a (n x H) for rows X (n x F)."""
    W1, b1, w2, b2 = unpack(theta, F, H)
    if bf16:
        W1, w2, X = bf16_round(W1), bf16_round(w2), bf16_round(X)
    Z = np.asarray(X, dtype=np.float64) @ W1.T + b1[None, :]
    A = np.tanh(Z)
    y = A @ w2 + b2
    return y, A


def loss_and_grad(theta, X, t, F, H, bf16=True):
    """Mean squared error and its gradient with respect to the flat parameters
    (through the BF16-rounded weights: the rounding is taken as the identity
    in the backward pass, as the device does)."""
    W1, b1, w2, b2 = unpack(theta, F, H)
    Xr = bf16_round(X) if bf16 else np.asarray(X, dtype=np.float64)
    W1r = bf16_round(W1) if bf16 else W1
    w2r = bf16_round(w2) if bf16 else w2
    n = Xr.shape[0]
    Z = Xr @ W1r.T + b1[None, :]
    A = np.tanh(Z)
    y = A @ w2r + b2
    r = y - np.asarray(t, dtype=np.float64)
    L = float(np.sum(r * r) / n)
    dy = 2.0 * r / n                      # dL/dy
    g_w2 = A.T @ dy
    g_b2 = float(np.sum(dy))
    dA = dy[:, None] * w2r[None, :]
    dZ = dA * (1.0 - A * A)
    g_W1 = dZ.T @ Xr
    g_b1 = dZ.sum(axis=0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_w2, [g_b2]])
    return L, grad


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1) in float64; returns new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
