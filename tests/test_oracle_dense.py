"""Pins for the dense 2^N route (paper Eqs. heisenberg, autocorr, trotter)."""

import math

import numpy as np
import pytest

from oracle.lattice import Lattice
from oracle import dense


def test_C0_is_one_and_norm_preserved():
    lat = Lattice(3, 3)
    C, O = dense.trotter_trajectory(lat, 1.0, 1.0, 0.05, 12)
    assert C[0] == 1.0
    assert abs(np.real(np.trace(O @ O)) / 2 ** 9 - 1.0) < 1e-12


@pytest.mark.parametrize("Lx,Ly,J,dt", [(3, 3, 1.0, 0.05), (4, 2, -0.7, 0.1), (5, 1, 1.0, 0.05)])
def test_zero_field_closed_form(Lx, Ly, J, dt):
    # h = 0: all XX terms commute and Z_c anticommutes exactly with the deg(c)
    # terms touching c, so C(t) = prod_j cos(2 J t) = cos(2 J t)^deg(c)
    lat = Lattice(Lx, Ly)
    C, _ = dense.trotter_trajectory(lat, J, 0.0, dt, 15)
    deg = lat.degree(lat.centre())
    t = dt * np.arange(16)
    assert np.allclose(C, np.cos(2 * J * t) ** deg, atol=1e-12)


def test_zero_coupling_is_constant():
    lat = Lattice(3, 2)
    C, _ = dense.trotter_trajectory(lat, 0.0, 1.3, 0.1, 10)
    assert np.allclose(C, 1.0, atol=1e-13)


def test_sign_invariances():
    lat = Lattice(3, 3)
    base, _ = dense.trotter_trajectory(lat, 1.0, 1.0, 0.05, 20)
    for J, h, dt in [(-1.0, 1.0, 0.05), (1.0, -1.0, 0.05), (1.0, 1.0, -0.05), (-1.0, -1.0, 0.05)]:
        other, _ = dense.trotter_trajectory(lat, J, h, dt, 20)
        assert np.max(np.abs(other - base)) < 1e-12


def test_trotter_converges_to_exact_evolution_second_order():
    # the symmetric splitting has O(dt^2) global error: halving dt quarters it
    lat = Lattice(3, 2)
    T = 1.2
    exact = dense.exact_trajectory(lat, 1.0, 1.0, [T])[0]
    errs = []
    for n in (12, 24, 48):
        C, _ = dense.trotter_trajectory(lat, 1.0, 1.0, T / n, n)
        errs.append(abs(C[-1] - exact))
    assert errs[0] < 5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


def test_pauli_coefficients_of_single_site_paulis():
    for p in range(4):
        a = dense.pauli_coefficients(dense.site_pauli(3, 1, p), 3)
        exp = np.zeros((4, 4, 4)); exp[0, p, 0] = 1.0
        assert np.allclose(a, exp, atol=1e-15)
