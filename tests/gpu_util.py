"""Helpers shared by the GPU parity tests (no method arithmetic)."""

import numpy as np
import pytest


def load_hpt():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_30985_amd import hpt as h
    return h


def copy_state(net, sim):
    """Load the oracle network's site tensors and gauge messages into the GPU handle."""
    for v in range(net.lat.n_sites):
        sim.set_site(v, net.psi[v])
    for b in range(net.lat.n_bonds):
        for d in range(2):
            sim.set_message(b, d, net.M[b][d])


def max_rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)
