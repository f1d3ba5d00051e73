"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers
with a fixed seed and shapes them like the paper's workloads (saturated site
tensors at bond dimension chi, positive semidefinite environment messages
with a decaying spectrum, lattice/parameter draws for batched runs).
"""

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def site_tensor(seed, dims):
    """Gaussian site tensor with leg dimensions ``dims`` (last = Pauli, 4),
    returned as a Fortran-ordered float64 array (first index fastest)."""
    g = rng(seed)
    return np.asfortranarray(g.standard_normal(size=tuple(dims)))


def haar_orthogonal(seed, n):
    g = rng(seed)
    A = g.standard_normal(size=(n, n))
    Q, R = np.linalg.qr(A)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def env_message(seed, chi, decay=20.0):
    """Symmetric PSD chi x chi message R diag(l) R^T, l_k ~ exp(-k/decay),
    Frobenius norm 1, R Haar-orthogonal."""
    lam = np.exp(-np.arange(chi) / decay)
    lam /= np.linalg.norm(lam)
    R = haar_orthogonal(seed, chi)
    M = (R * lam[None, :]) @ R.T
    return 0.5 * (M + M.T)


def batched_runs(seed=20261202, n=64):
    """Independent runs of the batched form: grid in {3x3,4x4,5x5,6x6},
    h ~ U[0.5, 3.0], J = 1, dt in {0.025, 0.05, 0.1, 0.2}, total time 2.0."""
    g = rng(seed)
    grids = [3, 4, 5, 6]
    dts = [0.025, 0.05, 0.1, 0.2]
    out = []
    for _ in range(n):
        L = int(g.choice(grids))
        dt = float(g.choice(dts))
        h = float(g.uniform(0.5, 3.0))
        out.append(dict(Lx=L, Ly=L, J=1.0, h=h, dt=dt, nsteps=int(round(2.0 / dt))))
    return out
