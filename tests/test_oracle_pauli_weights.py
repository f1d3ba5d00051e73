"""Pins for the oracle's per-site non-identity Pauli weight n(r, t) and the
spreading measures built on it (paper Sec. "Operator Spreading and Lightcone
Saturation", Sec. "Spatial operator spreading", Eq. sfrac).

n(r) is checked against its plain definition on the dense operator (on a
tree, where the gauge BP environment is exact), against the t = 0 state
(a single non-identity letter at the centre), and against the lattice's C4
symmetry about the centre of an odd grid while nothing is truncated; the
spreading measures against hand-computed values."""

import math

import numpy as np
import pytest

from oracle import dense
from oracle.lattice import Lattice
from oracle.network import Config, OperatorNetwork, mode_product, spreading_stats
from oracle.run import layer


def test_t0_weight_sits_on_the_centre():
    net = OperatorNetwork(Config(Lx=3, Ly=3, chi_max=4))
    n = net.pauli_weights()
    ref = np.zeros(9)
    ref[net.centre] = 1.0
    assert np.array_equal(n, ref)
    assert spreading_stats(n, net.lat, net.centre) == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("Lx,Ly,dt", [(5, 1, 0.1), (1, 4, 0.17), (6, 1, 0.05)])
def test_tree_weights_equal_dense_definition(Lx, Ly, dt):
    # a chain is a tree: the converged gauge messages are the exact
    # environments, so the BP estimate is the dense n(r) itself
    cfg = Config(Lx=Lx, Ly=Ly, chi_max=64, dt=dt, J=1.0, h=0.9, bp_tol=1e-13, bp_max_sweeps=200)
    net = OperatorNetwork(cfg)
    nsteps = 8
    ops = dense.trotter_operators(net.lat, cfg.J, cfg.h, cfg.dt, nsteps, centre=net.centre)
    for k in range(1, nsteps + 1):
        layer(net)
        assert net.layer_gate_err < 1e-18
        n_bp = net.pauli_weights()
        n_dense = dense.pauli_weights(ops[k], net.lat.n_sites)
        assert np.max(np.abs(n_bp - n_dense)) < 1e-9, (k, n_bp, n_dense)
    # the same operator in another gauge (a random invertible G and G^-1 on
    # every bond) has direction-dependent messages; from a uniform start the
    # gauge BP finds the new environments and n(r) is unchanged
    rng = np.random.default_rng(Lx + 10 * Ly)
    for b, (v1, v2, _) in enumerate(net.lat.bonds):
        c = net.chi[b]
        G = np.eye(c) + 0.3 * rng.standard_normal((c, c))
        net.psi[v1] = mode_product(net.psi[v1], G.T, net.lat.leg_position(v1, b))
        net.psi[v2] = mode_product(net.psi[v2], np.linalg.inv(G), net.lat.leg_position(v2, b))
    net.cfg.bp_init = "uniform"
    net.gauge_bp()
    assert np.max(np.abs(net.pauli_weights() - n_dense)) < 1e-9


def test_dense_weights_of_a_known_operator():
    # O = (X_0 + Z_0 Z_1) / sqrt(2) on two qubits: strings X I and Z Z with
    # weight 1/2 each; n(0) = 1, n(1) = 1/2
    from oracle.dense import site_pauli
    O = (site_pauli(2, 0, 1) + site_pauli(2, 0, 3) @ site_pauli(2, 1, 3)) / math.sqrt(2.0)
    assert np.allclose(dense.pauli_weights(O, 2), [1.0, 0.5], atol=1e-15)


def test_c4_symmetry_on_odd_grid_while_untruncated():
    cfg = Config(Lx=3, Ly=3, chi_max=64, dt=0.1, J=1.0, h=1.0, bp_tol=1e-13, bp_max_sweeps=400)
    net = OperatorNetwork(cfg)
    lat = net.lat
    rot = [lat.site(2 - lat.coords(v)[1], lat.coords(v)[0]) for v in range(9)]   # 90 degrees about (1, 1)
    assert sorted(rot) == list(range(9)) and rot[net.centre] == net.centre
    for _ in range(3):
        layer(net)
        assert net.layer_gate_err < 1e-18
        n = net.pauli_weights()
        assert np.max(np.abs(n - n[rot])) < 1e-12
        assert np.all((n >= -1e-15) & (n <= 1 + 1e-15))


def test_spreading_stats_hand_values():
    lat = Lattice(3, 3)
    c = lat.centre()
    # uniform weight: mean Manhattan radius (0 + 4 * 1 + 4 * 2) / 9, RMS radius
    # sqrt((0 + 4 * 1 + 4 * 2) / 9) (corners at squared distance 2), S_frac = 1
    r1, r2, sf = spreading_stats(np.full(9, 0.3), lat, c)
    assert abs(r1 - 12.0 / 9.0) < 1e-15 and abs(r2 - math.sqrt(12.0 / 9.0)) < 1e-15 and abs(sf - 1.0) < 1e-15
    # weight on one corner only
    n = np.zeros(9)
    n[lat.site(2, 2)] = 0.7
    assert spreading_stats(n, lat, c) == (2.0, math.sqrt(2.0), 0.0)
    # two sites, equal weight: S_frac = ln 2 / ln 9
    n = np.zeros(9)
    n[c] = n[lat.site(0, 1)] = 1.0
    r1, r2, sf = spreading_stats(n, lat, c)
    assert abs(r1 - 0.5) < 1e-15 and abs(r2 - math.sqrt(0.5)) < 1e-15 and abs(sf - math.log(2) / math.log(9)) < 1e-15
