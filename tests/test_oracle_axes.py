"""Pins of the ZZ-coupling / X-field reading (model_axes "zzx"): the literal
dense evolution of H = -J sum ZZ - h sum X with observable Z_c, built from its
own factors, equals the paper-frame dense evolution of X_c (the global Hadamard
mapping), and the method with model_axes "zzx" reproduces the literal dense
C(t) while no truncation occurs."""

import numpy as np

from oracle import dense
from oracle.lattice import Lattice
from oracle.network import Config
from oracle.run import trajectory


def test_literal_zzx_equals_paper_frame_x_observable():
    lat = Lattice(3, 2)
    lit = dense.zzx_trotter_trajectory(lat, 1.0, 1.3, 0.07, 12)
    # paper frame, observable X at the centre
    N = lat.n_sites
    c = lat.centre()
    Xc = dense.site_pauli(N, c, 1)
    U = dense.trotter_step_unitary(lat, 1.0, 1.3, 0.07)
    O = Xc.copy()
    ref = [1.0]
    for _ in range(12):
        O = U.conj().T @ O @ U
        ref.append(np.real(np.trace(O @ Xc)) / 2 ** N)
    assert np.max(np.abs(lit - np.array(ref))) <= 1e-12
    # and it is a different function from the paper's own C(t)
    paper, _ = dense.trotter_trajectory(lat, 1.0, 1.3, 0.07, 12)
    assert np.max(np.abs(lit - paper)) > 1e-2


def test_method_zzx_matches_literal_dense_while_untruncated():
    lat = Lattice(3, 3)
    lit = dense.zzx_trotter_trajectory(lat, 1.0, 1.0, 0.05, 4)
    C = trajectory(Config(Lx=3, Ly=3, chi_max=64, dt=0.05, model_axes="zzx"), 4)
    # step 1: the chi > 1 bonds form a star (a tree), Bethe is exact
    assert abs(C[0] - 1.0) <= 1e-14
    assert abs(C[1] - lit[1]) <= 1e-12
    # later steps on the loopy 3x3 lattice are the method's Bethe estimate
    assert np.max(np.abs(np.array(C[:5]) - lit)) <= 5e-3


def test_zzx_network_contracts_to_literal_dense_exactly():
    # untruncated layers represent the Trotter operator exactly: the exact
    # contraction of the pinned network equals the literal dense C(t)
    from oracle.contract import pinned_contraction
    from oracle.network import OperatorNetwork
    from oracle.run import layer
    lat = Lattice(2, 3)
    lit = dense.zzx_trotter_trajectory(lat, 0.8, 1.4, 0.06, 4)
    net = OperatorNetwork(Config(Lx=2, Ly=3, J=0.8, h=1.4, dt=0.06, chi_max=256, model_axes="zzx"))
    assert abs(pinned_contraction(net) - 1.0) <= 1e-14
    for n in range(1, 5):
        layer(net)
        assert net.layer_gate_err <= 1e-20
        assert abs(pinned_contraction(net) - lit[n]) <= 1e-12, n
