"""Exact contraction of tiny operator networks, without BP (oracle; test
infrastructure only).

Paper, Sec. "Correlation Function via Belief Propagation", step 1: by Pauli
orthogonality, C(t) is the coefficient of the configuration (Z at c, I
elsewhere) of the network, i.e. the full contraction of all shared bond legs
with every Pauli leg pinned.  With the Pauli legs left open the same
contraction yields every Pauli coefficient a_P of the represented operator;
sum_P a_P^2 = Tr[O^2] / 2^N.
"""

import numpy as np

_LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


def _subscripts(net, pauli_open):
    lat = net.lat
    nb = lat.n_bonds
    if nb + lat.n_sites > len(_LETTERS):
        raise ValueError("network too large for exact contraction")
    terms = []
    for v in range(lat.n_sites):
        s = "".join(_LETTERS[b] for (_, _, b) in lat.legs[v])
        if pauli_open:
            s += _LETTERS[nb + v]
        terms.append(s)
    out = "".join(_LETTERS[nb + v] for v in range(lat.n_sites)) if pauli_open else ""
    return ",".join(terms) + "->" + out


def all_coefficients(net):
    """a[p_0, ..., p_{N-1}] of the operator the network represents."""
    sub = _subscripts(net, True)
    return np.einsum(sub, *net.psi, optimize="greedy")


def pinned_contraction(net, centre=None):
    """Exact C = coefficient of (the observable's Pauli at centre, I elsewhere)."""
    c = net.centre if centre is None else centre
    T = [net.psi[v][..., net.obs_p if v == c else 0] for v in range(net.lat.n_sites)]
    sub = _subscripts(net, False)
    return float(np.einsum(sub, *T, optimize="greedy"))
