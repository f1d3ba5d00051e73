"""Dense linear-algebra definitions used by the gate update's QR step
(oracle; test infrastructure only).

Sec. "Adaptive QR Decomposition", Eq. cholqr: the CholeskyQR path forms the
Gram matrix G = X^T X of the (absorbed, permuted) tall site matrix X and
factors it by Cholesky, R = chol(G), Q = X R^-1; the paper recommends float64
for the Gram.  ``gram`` is that definition written out in float64.
"""

import numpy as np


def gram(X):
    """G = X^T X with float64 products and sums (Eq. cholqr), for any real X
    (m x n); float32 inputs are widened exactly before the products."""
    X = np.asarray(X, dtype=np.float64)
    return X.T @ X
