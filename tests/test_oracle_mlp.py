"""Pins of the warm-start network's oracle (oracle/mlp.py): the BF16 rounding
against values fixed by the format, and the analytic gradient against central
finite differences of the float64 loss."""

import numpy as np

from oracle import mlp


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.140625, 2 ** -130, 65504.0],
                 dtype=np.float32)
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even pattern (1.0);
    # 1 + 3 * 2^-8 ties between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert list(r[:4]) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6]
    assert r[4] == -3.140625          # exactly representable (8 significant bits)
    assert r[5] == 2.0 ** -130        # subnormal in float32, kept
    assert r[6] == 65536.0            # 65504 rounds up to 2^16 at 8 significant bits


def test_gradient_matches_central_differences():
    F, H = 6, 9
    g = np.random.Generator(np.random.PCG64(5))
    theta = g.standard_normal(mlp.n_params(F, H)) * 0.5
    X = g.standard_normal((23, F))
    t = g.standard_normal(23)
    L, grad = mlp.loss_and_grad(theta, X, t, F, H, bf16=False)
    eps = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = eps
        num[i] = (mlp.loss_and_grad(theta + e, X, t, F, H, bf16=False)[0] -
                  mlp.loss_and_grad(theta - e, X, t, F, H, bf16=False)[0]) / (2 * eps)
    assert np.max(np.abs(num - grad)) <= 1e-8 * max(1.0, np.max(np.abs(grad)))
    y, _ = mlp.forward(theta, X, F, H, bf16=False)
    assert abs(L - np.mean((y - t) ** 2)) <= 1e-14 * L


def test_forward_of_a_hand_computed_case():
    # F = 2, H = 1: y = w2 tanh(w11 x1 + w12 x2 + b1) + b2
    theta = np.array([0.5, -0.25, 0.125, 2.0, -1.0])
    X = np.array([[1.0, 2.0], [0.0, -4.0]])
    y, _ = mlp.forward(theta, X, 2, 1)
    ref = 2.0 * np.tanh(np.array([0.5 - 0.5 + 0.125, 1.0 + 0.125])) - 1.0
    assert np.max(np.abs(y - ref)) <= 1e-15


def test_adam_first_step_moves_every_weight_by_lr():
    # at step 1 the bias-corrected moments are g and g^2, so each weight moves
    # by lr * g / (|g| + eps), i.e. by lr in the direction of -g
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
