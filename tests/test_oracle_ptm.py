"""Pins for the oracle's Pauli transfer matrices (paper Sec. "Trotter
Decomposition": the gates are real orthogonal maps in the Pauli basis)."""

import math

import numpy as np
import pytest

from oracle.ptm import field_ptm, coupling_ptm, pauli_matrices
from oracle.lattice import Lattice
from oracle import dense

I, X, Y, Z = 0, 1, 2, 3


@pytest.mark.parametrize("h,dt", [(1.0, 0.05), (-1.0, 0.1), (2.3, 0.2)])
def test_field_ptm_orthogonal_and_fixes_I_Z(h, dt):
    G = field_ptm(h, dt)
    assert np.allclose(G @ G.T, np.eye(4), atol=1e-15)
    for p in (I, Z):
        e = np.zeros(4); e[p] = 1
        assert np.allclose(G @ e, e, atol=1e-15)


def test_field_ptm_rotates_X_into_Y_by_h_dt():
    # exp(+i a Z) X exp(-i a Z) = cos(2a) X - sin(2a) Y with a = h dt / 2
    # (X Z = -i Y; worked by hand), i.e. U^dagger X U for U = exp(-i a Z).
    h, dt = 0.7, 0.3
    G = field_ptm(h, dt)
    a = -h * dt / 2          # U = exp(+i h dt/2 Z) = exp(-i a Z)
    assert math.isclose(G[X, X], math.cos(2 * a), abs_tol=1e-15)
    assert math.isclose(G[Y, X], -math.sin(2 * a), abs_tol=1e-15)


@pytest.mark.parametrize("J,dt", [(1.0, 0.05), (-1.0, 0.1), (0.4, 0.7)])
def test_coupling_ptm_structure(J, dt):
    G = coupling_ptm(J, dt)
    assert np.allclose(G @ G.T, np.eye(16), atol=1e-14)
    # identity on the 8 Pauli strings that commute with X x X
    commuting = [(I, I), (I, X), (X, I), (X, X), (Y, Y), (Y, Z), (Z, Y), (Z, Z)]
    for (a, b) in commuting:
        e = np.zeros(16); e[4 * a + b] = 1
        assert np.allclose(G @ e, e, atol=1e-14)
    # operator-Schmidt rank 4 across the two sites
    Gr = G.reshape(4, 4, 4, 4).transpose(0, 2, 1, 3).reshape(16, 16)
    sv = np.linalg.svd(Gr, compute_uv=False)
    assert np.sum(sv > 1e-12 * sv[0]) == 4


def test_coupling_ptm_ZI_image_by_hand():
    # U = exp(-i phi XX), phi = -J dt: U^dagger (Z x I) U = (Z x I) exp(-2 i phi XX)
    # = cos(2 phi) Z I - i sin(2 phi) (Z X) x X = cos(2 phi) ZI + sin(2 phi) YX
    J, dt = 1.3, 0.11
    phi = -J * dt
    G = coupling_ptm(J, dt)
    col = G[:, 4 * Z + I]
    exp = np.zeros(16)
    exp[4 * Z + I] = math.cos(2 * phi)
    exp[4 * Y + X] = math.sin(2 * phi)
    assert np.allclose(col, exp, atol=1e-15)


def test_ptm_agrees_with_dense_conjugation_on_a_chain():
    # one Trotter step of the 1x2 chain applied as PTMs (G1, G2, G1 on the
    # coefficient vector) equals the dense route's Pauli decomposition of
    # U^dagger O U for a random Hermitian O
    lat = Lattice(2, 1)
    J, h, dt = 0.9, -1.7, 0.23
    rng = np.random.default_rng(5)
    c = rng.standard_normal(16)
    P = pauli_matrices()
    O = sum(c[4 * a + b] * np.kron(P[a], P[b]) for a in range(4) for b in range(4))
    U = dense.trotter_step_unitary(lat, J, h, dt)
    a_dense = dense.pauli_coefficients(U.conj().T @ O @ U, 2).reshape(16)
    G1 = field_ptm(h, dt)
    G11 = np.kron(G1, G1)
    a_ptm = G11 @ coupling_ptm(J, dt) @ G11 @ c
    assert np.allclose(a_ptm, a_dense, atol=1e-13)
