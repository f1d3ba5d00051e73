"""Exact 2^N operator evolution: the plain definition of C(t) (oracle; test
infrastructure only).

Paper, Sec. "Heisenberg Picture and Spin Autocorrelation": with rho_0
proportional to the identity, C(t) = Tr[Z_c(t) Z_c] / 2^N, where
Z_c(t) = exp(iHt) Z_c exp(-iHt) (Eqs. heisenberg, autocorr).
Sec. "Trotter Decomposition": one step conjugates by
U(dt) = F B F with F the field half-step on every site and B the product of
all bond couplings (Eq. trotter; the XX couplings commute, so their order in
B is immaterial).  Reading of angles and signs: see ``oracle.ptm``.

Qubit v is the v-th tensor factor (site 0 leftmost in every Kronecker
product).  Only for small N (<= 12).
"""

import numpy as np

from .lattice import Lattice
from .ptm import pauli_matrices


def _zvals(N):
    """z_v(s) = +1 / -1 for bit v of basis state s (site 0 = most significant)."""
    s = np.arange(2 ** N)
    return np.array([1 - 2 * ((s >> (N - 1 - v)) & 1) for v in range(N)])


def _hadamard_all(N):
    Hd = np.array([[1, 1], [1, -1]]) / np.sqrt(2.0)
    out = np.array([[1.0]])
    for _ in range(N):
        out = np.kron(out, Hd)
    return out


def trotter_step_unitary(lat: Lattice, J, h, dt):
    """U(dt) = F B F with F = prod_v exp(+i h dt/2 Z_v), B = prod_<ij> exp(+i J dt X_i X_j)."""
    N = lat.n_sites
    z = _zvals(N)
    F = np.exp(1j * (h * dt / 2.0) * z.sum(axis=0))
    zz = np.zeros(2 ** N)
    for v1, v2, _ in lat.bonds:
        zz += z[v1] * z[v2]
    Hd = _hadamard_all(N)
    B = Hd @ np.diag(np.exp(1j * J * dt * zz)) @ Hd
    return (F[:, None] * B) * F[None, :]


def hamiltonian(lat: Lattice, J, h):
    """H = -J sum_<ij> X_i X_j - h sum_i Z_i (paper Eq. hamiltonian), dense real."""
    N = lat.n_sites
    z = _zvals(N)
    Hd = _hadamard_all(N)
    zz = np.zeros(2 ** N)
    for v1, v2, _ in lat.bonds:
        zz += z[v1] * z[v2]
    return -J * (Hd @ np.diag(zz) @ Hd) - h * np.diag(z.sum(axis=0).astype(float))


def site_pauli(N, v, p):
    P = pauli_matrices()
    out = np.array([[1.0 + 0j]])
    for w in range(N):
        out = np.kron(out, P[p] if w == v else P[0])
    return out


def trotter_trajectory(lat: Lattice, J, h, dt, nsteps, centre=None):
    """C(n dt) for n = 0..nsteps under exact Trotter evolution; also returns O."""
    N = lat.n_sites
    c = lat.centre() if centre is None else centre
    Zc = site_pauli(N, c, 3)
    U = trotter_step_unitary(lat, J, h, dt)
    Ud = U.conj().T
    O = Zc.copy()
    Cs = [np.real(np.trace(O @ Zc)) / 2 ** N]
    for _ in range(nsteps):
        O = Ud @ O @ U
        Cs.append(np.real(np.trace(O @ Zc)) / 2 ** N)
    return np.array(Cs), O


def trotter_operators(lat: Lattice, J, h, dt, nsteps, centre=None):
    """List of evolved operators O_n, n = 0..nsteps."""
    N = lat.n_sites
    c = lat.centre() if centre is None else centre
    O = site_pauli(N, c, 3)
    U = trotter_step_unitary(lat, J, h, dt)
    Ud = U.conj().T
    out = [O]
    for _ in range(nsteps):
        O = Ud @ O @ U
        out.append(O)
    return out


def exact_trajectory(lat: Lattice, J, h, times, centre=None):
    """C(t) under exp(-iHt) without Trotter splitting."""
    N = lat.n_sites
    c = lat.centre() if centre is None else centre
    Zc = site_pauli(N, c, 3)
    E, V = np.linalg.eigh(hamiltonian(lat, J, h))
    out = []
    for t in times:
        Ut = (V * np.exp(-1j * E * t)[None, :]) @ V.T
        O = Ut.conj().T @ Zc @ Ut
        out.append(np.real(np.trace(O @ Zc)) / 2 ** N)
    return np.array(out)


def pauli_coefficients(O, N):
    """a[p_0, ..., p_{N-1}] = Tr[(P_p0 x ... x P_p(N-1)) O] / 2^N, real array of shape (4,)*N."""
    P = pauli_matrices()
    Pt = np.stack(P)                           # Pt[p, c, r] = P_p[c, r]
    T = O.reshape((2,) * (2 * N))
    # Tr[P O] = sum_{r,c} O[r, c] P[c, r]; contract site by site, after step v
    # the first v axes are Pauli indices
    for v in range(N):
        # axes now: p_0..p_{v-1}, i_v..i_{N-1}, j_v..j_{N-1}
        nrest = N - v
        i_ax = v
        j_ax = v + nrest
        T = np.tensordot(T, Pt, axes=([i_ax, j_ax], [2, 1]))
        # new p axis is last; move it to position v
        T = np.moveaxis(T, -1, v)
    a = T / 2 ** N
    if np.max(np.abs(a.imag)) > 1e-10:
        raise AssertionError("Hermitian operator must have real Pauli coefficients")
    return a.real.copy()


def pauli_weights(O, N):
    """n(r) = (sum of a_s^2 over the Pauli strings s with a non-identity letter
    at site r) / (sum of all a_s^2): the per-site non-identity Pauli weight of
    Sec. "Operator Spreading and Lightcone Saturation", from the Pauli
    coefficients of the dense operator."""
    a = pauli_coefficients(O, N)
    w = a * a
    tot = w.sum()
    return np.array([1.0 - np.take(w, 0, axis=r).sum() / tot for r in range(N)])


def zzx_trotter_trajectory(lat: Lattice, J, h, dt, nsteps, centre=None):
    """C(n dt) = Tr[Z_c(n dt) Z_c]/2^N for the ZZ-coupling, X-field model
    H = -J sum ZZ - h sum X with the same symmetric splitting, built literally
    from its own factors (no Hadamard): U(dt) = F B F with
    F = prod_v exp(+i h dt/2 X_v) (Kronecker products of the one-site
    rotation cos + i sin X) and B = prod_<ij> exp(+i J dt Z_i Z_j) (diagonal)."""
    N = lat.n_sites
    c = lat.centre() if centre is None else centre
    P = pauli_matrices()
    th = h * dt / 2.0
    f1 = np.cos(th) * P[0] + 1j * np.sin(th) * P[1]
    F = np.array([[1.0 + 0j]])
    for _ in range(N):
        F = np.kron(F, f1)
    z = _zvals(N)
    zz = np.zeros(2 ** N)
    for v1, v2, _ in lat.bonds:
        zz += z[v1] * z[v2]
    U = F @ (np.exp(1j * J * dt * zz)[:, None] * F)
    Ud = U.conj().T
    Zc = site_pauli(N, c, 3)
    O = Zc.copy()
    Cs = [np.real(np.trace(O @ Zc)) / 2 ** N]
    for _ in range(nsteps):
        O = Ud @ O @ U
        Cs.append(np.real(np.trace(O @ Zc)) / 2 ** N)
    return np.array(Cs)
