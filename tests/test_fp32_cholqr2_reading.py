"""How good is the FP32 form's CholeskyQR2 basis?  (Sec. "Adaptive QR
Decomposition", Eq. cholqr; the FP32 form's reading of it.)

The FP32 form factors the float32 site matrix X through a float64 Gram
G1 = X^T X (exact products, float64 sums), a diagonally pivoted Cholesky
that deflates pivots below tol * max G1_jj, and an algebraic second pass
G2 = W1^T G1 W1 with W1 = E_sel R1^-1; the basis Q = X W1 R2^-1 is never
formed.  Written out here with numpy from that description (not from the
kernels), this checks on the CPU what the reading claims: the implicit
basis is orthonormal to about eps64 kappa(X)^2 (the second pass cannot
remove the rounding of G1), and the singular values of the triangular
factor T = R2 R1 -- what the R-core sees -- match those of X to about
eps64 (s_0 / s)^2, on synthetic blocks of chosen condition and on the
absorbed blocks of a real network state."""

import numpy as np

from oracle.network import Config, OperatorNetwork, mode_product, pseudo_sqrt
from oracle.run import layer

EPS64 = 2.0 ** -52


def _fp32_form_cholqr2(X32, tol):
    X = X32.astype(np.float64)
    G1 = X.T @ X
    n = G1.shape[0]
    A = G1.copy()
    dmax = np.max(np.diag(G1))
    sel, rem = [], list(range(n))
    for _ in range(n):
        p = max(rem, key=lambda i: A[i, i])
        if A[p, p] <= tol * dmax:
            break
        sel.append(p)
        rem.remove(p)
        col = A[:, p] / np.sqrt(A[p, p])
        A = A - np.outer(col, col)
    R1 = np.linalg.cholesky(G1[np.ix_(sel, sel)]).T
    W1 = np.zeros((n, len(sel)))
    W1[sel, :] = np.linalg.inv(R1)
    R2 = np.linalg.cholesky(W1.T @ G1 @ W1).T
    Q = X @ W1 @ np.linalg.inv(R2)
    return Q, R2 @ R1, sel


def test_orthogonality_scales_as_eps64_kappa_squared():
    rng = np.random.default_rng(3)
    m, n = 6000, 48
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    for p in range(0, 6):
        X32 = ((U * np.logspace(0, -p, n)) @ V.T).astype(np.float32)
        kappa = np.linalg.cond(X32.astype(np.float64))
        Q, _, sel = _fp32_form_cholqr2(X32, 1e-14)
        assert len(sel) == n
        e = np.max(np.abs(Q.T @ Q - np.eye(n)))
        assert e <= 2 * EPS64 * kappa ** 2 + 16 * n * EPS64, (p, e, kappa)
        if p <= 2:
            assert e < 1e-11


def test_real_blocks_keep_their_spectrum():
    # absorbed, permuted site matrices of a truncating 4x4 run (chi_max 12,
    # five layers): the triangular factor's singular values against X's own
    net = OperatorNetwork(Config(Lx=4, Ly=4, chi_max=12, dt=0.1, J=1.0, h=1.0, bp_tol=1e-11))
    for _ in range(5):
        layer(net)
    lat = net.lat
    worst = 0.0
    blocks = 0
    for v in range(lat.n_sites):
        for (_, _, b) in lat.legs[v]:
            T = net.psi[v]
            env = []
            for pos, (_, _, be) in enumerate(lat.legs[v]):
                if be != b:
                    T = mode_product(T, pseudo_sqrt(net.incoming(be, v), 1e-12)[0], pos)
                    env.append(pos)
            X = np.transpose(T, env + [lat.leg_position(v, b), T.ndim - 1])
            m, n = int(np.prod(X.shape[:-2])), X.shape[-2] * 4
            if m < 2 * n:
                continue
            X32 = X.reshape((m, n), order="F").astype(np.float32)
            _, Tf, sel = _fp32_form_cholqr2(X32, 1e-14)
            sx = np.linalg.svd(X32.astype(np.float64)[:, sel], compute_uv=False)
            st = np.linalg.svd(Tf, compute_uv=False)
            rel = np.abs(st - sx) / sx
            # error relative to each value grows as (s_0 / s)^2 times eps64
            worst = max(worst, float(np.max(rel * (sx / sx[0]) ** 2)))
            keep = sx >= 1e-3 * sx[0]
            assert np.max(rel[keep]) < 1e-10
            blocks += 1
    assert blocks >= 8
    assert worst < 100 * EPS64, worst
