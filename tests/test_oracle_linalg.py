"""Pins of oracle.linalg.gram (the Gram matrix of Eq. cholqr) against
brute force and against an independent route (Householder R^T R)."""

import numpy as np

from oracle.linalg import gram


def test_gram_equals_brute_force_on_integers():
    X = np.arange(15, dtype=np.float64).reshape(5, 3) - 7.0
    G = gram(X)
    for i in range(3):
        for j in range(3):
            assert G[i, j] == sum(X[k, i] * X[k, j] for k in range(5))


def test_gram_equals_rtr_of_householder_qr():
    g = np.random.Generator(np.random.PCG64(3))
    X = g.standard_normal((200, 17))
    R = np.linalg.qr(X, mode="r")
    assert np.max(np.abs(gram(X) - R.T @ R)) <= 1e-12 * np.max(np.abs(gram(X)))


def test_gram_of_float32_widens_exactly():
    g = np.random.Generator(np.random.PCG64(4))
    X = g.standard_normal((64, 5)).astype(np.float32)
    G = gram(X)
    # products of two float32 values are exact in float64; one column with itself
    # summed in a fixed order by hand gives the same value to the last rounding
    x = X[:, 2].astype(np.float64)
    s = 0.0
    for v in x:
        s += v * v
    assert abs(G[2, 2] - s) <= 1e-14 * s
    assert G.dtype == np.float64 and np.array_equal(G, G.T)
