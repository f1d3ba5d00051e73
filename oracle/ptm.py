"""Pauli transfer matrices of the Trotter gates (oracle; test infrastructure only).

Paper, Sec. "Trotter Decomposition": conjugating by a gate whose generator
is a real Pauli coupling maps Pauli strings to real combinations of Pauli
strings, so in the Pauli basis each gate is a real orthogonal matrix.  The
step is U(dt) ~ R_z(h dt) R_xx(2 J dt) R_z(h dt) (Eq. trotter).

Reading: R_P(theta) = exp(-i theta P / 2), and the
signs follow the Hamiltonian of Eq. hamiltonian, H = -J sum XX - h sum Z, so
that the three factors are the symmetric splitting of exp(-i H dt):
    field half-step   exp(+i (h dt / 2) Z)   on every site
    coupling          exp(+i  J dt  X X)     on every bond
C(t) is invariant under J -> -J, h -> -h and dt -> -dt separately, so this
sign choice does not change any reported value; tests check that invariance.

Definition used here (Heisenberg picture, O -> U^dagger O U, coefficients
c_a of O = sum_a c_a P_a):
    G[a', a] = Tr[P_a' U^dagger P_a U] / 2^k,   c' = G c.
Pauli order p = 0 I, 1 X, 2 Y, 3 Z (Sec. "Pauli Basis Tensor Network");
two-site index 4 * d1 + d2 with d1 on the lower-numbered site.
Tables are built numerically from this trace formula, not from closed forms.
"""

import numpy as np
from scipy.linalg import expm


def pauli_matrices():
    I = np.eye(2, dtype=complex)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    Z = np.array([[1, 0], [0, -1]], dtype=complex)
    return [I, X, Y, Z]


def ptm_of_unitary(U, k):
    """Real PTM of O -> U^dagger O U on k qubits (k = 1 or 2)."""
    P = pauli_matrices()
    if k == 1:
        basis = P
    elif k == 2:
        basis = [np.kron(P[a], P[b]) for a in range(4) for b in range(4)]
    else:
        raise ValueError("k must be 1 or 2")
    n = len(basis)
    G = np.zeros((n, n), dtype=complex)
    Ud = U.conj().T
    for a in range(n):
        img = Ud @ basis[a] @ U
        for ap in range(n):
            G[ap, a] = np.trace(basis[ap] @ img) / 2 ** k
    if np.max(np.abs(G.imag)) > 1e-13:
        raise AssertionError("PTM of a real Pauli coupling must be real")
    return G.real.copy()


def field_unitary(h, dt):
    """Half-step of the transverse field: exp(-i (dt/2) (-h Z))."""
    Z = pauli_matrices()[3]
    return expm(-1j * (dt / 2.0) * (-h) * Z)


def coupling_unitary(J, dt):
    """Full step of one Ising bond: exp(-i dt (-J X X))."""
    X = pauli_matrices()[1]
    return expm(-1j * dt * (-J) * np.kron(X, X))


def field_ptm(h, dt):
    return ptm_of_unitary(field_unitary(h, dt), 1)


def coupling_ptm(J, dt):
    return ptm_of_unitary(coupling_unitary(J, dt), 2)
