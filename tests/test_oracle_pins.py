"""Pins of oracle parts that the trajectory tests reach only indirectly.

* SplitMix64, the generator behind the sign-gauge weights, against its
  published output sequence for seed 0.
* pseudo_sqrt (Algorithm "Gate update", first step: sqrt(mu) and mu^{-1/2})
  against the properties that define it, on a message whose eigenvalues
  straddle the cutoff.
* The dense 2^N route against C(t) values computed by an independent dense
  evolution (first-order-in-name symmetric splitting, H = -J sum XX - h sum Z,
  observable Z at the centre), printed to 10 decimals.
"""

import numpy as np
import pytest

from oracle import dense
from oracle.lattice import Lattice
from oracle.network import splitmix64, gauge_sign_weights, pseudo_sqrt

# published SplitMix64 outputs for seed 0 (the reference generator's first five)
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                    0xF88BB8A8724C81EC, 0x1B39896A51A8749B]


def test_splitmix64_known_answers():
    got = [int(x) for x in splitmix64(5)]
    assert got == SPLITMIX64_SEED0


def test_gauge_sign_weights_from_known_answers():
    w = gauge_sign_weights(5)
    exp = [(x >> 11) * 2.0 ** -53 - 0.5 for x in SPLITMIX64_SEED0]
    assert list(w) == exp                       # exact: 53-bit integers scale exactly
    assert np.all(np.abs(w) <= 0.5)


def _message(rng, w):
    n = len(w)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return V, (V * np.asarray(w)[None, :]) @ V.T


def test_pseudo_sqrt_defining_properties():
    # eigenvalues on both sides of the relative cutoff 1e-12: kept 1, 0.3,
    # 1e-4, 5e-12; dropped 5e-13, 0 and negative rounding noise
    rng = np.random.default_rng(7)
    w = [1.0, 0.3, 1e-4, 5e-12, 5e-13, 0.0, -1e-17]
    V, M = _message(rng, w)
    S, Sinv, ncut = pseudo_sqrt(M, 1e-12)
    assert ncut == 3
    keep = np.array([x > 1e-12 for x in w])
    P = V[:, keep] @ V[:, keep].T                      # projector on the kept eigenspace
    # sqrt(M): symmetric, squares to M on the kept space (dropped part <= 5e-13)
    assert np.max(np.abs(S - S.T)) < 1e-15
    assert np.max(np.abs(S @ S - P @ M @ P)) < 1e-14
    assert np.max(np.abs(S @ S - M)) < 1e-12
    # its eigenvalues are the square roots of the kept ones, zero elsewhere
    ev = np.sort(np.linalg.eigvalsh(S))[::-1]
    # (eigh resolves the small eigenvalues to ~1e-16 absolute: sqrt(w) to ~1e-11)
    assert np.allclose(ev[:4], np.sqrt([1.0, 0.3, 1e-4, 5e-12]), rtol=1e-12, atol=1e-10)
    assert np.max(np.abs(ev[4:])) < 1e-12
    # M^{-1/2}: Pi = S Sinv is the orthogonal projector on the kept
    # eigenspace (symmetric, idempotent, rank 4), Sinv S = Pi, Sinv M Sinv = Pi
    Pi = S @ Sinv
    assert np.max(np.abs(Pi - Pi.T)) < 1e-9
    assert np.max(np.abs(Pi @ Pi - Pi)) < 1e-9
    assert abs(np.trace(Pi) - 4.0) < 1e-9
    assert np.max(np.abs(Sinv @ S - Pi)) < 1e-9
    # (amplifies the rounding of M by |Sinv|^2 = 1 / 5e-12: ~1e-16 * 2e11)
    assert np.max(np.abs(Sinv @ M @ Sinv - Pi)) < 1e-4
    # the kept eigenspace is the constructed one up to the rounding of the
    # eigenvectors: ~1e-16 / (gap 4.5e-12) for the 5e-12 direction
    assert np.max(np.abs(Pi - P)) < 1e-4
    # the well-separated directions are reproduced and the null direction removed
    for j in (0, 1, 2):
        assert np.max(np.abs(Pi @ V[:, j] - V[:, j])) < 1e-10
    assert np.max(np.abs(Pi @ V[:, 5])) < 1e-4
    # absorbing M itself instead of sqrt(M) is caught
    assert np.max(np.abs(S - M)) > 0.1


def test_pseudo_sqrt_full_rank_is_matrix_square_root():
    rng = np.random.default_rng(8)
    V, M = _message(rng, [2.0, 1.0, 0.5, 0.25])
    S, Sinv, ncut = pseudo_sqrt(M, 1e-12)
    assert ncut == 0
    assert np.max(np.abs(S @ S - M)) < 1e-14
    assert np.max(np.abs(Sinv @ M @ Sinv - np.eye(4))) < 1e-13
    # an asymmetric rounding error in the input is symmetrised away
    E = 1e-9 * rng.standard_normal((4, 4))
    S2, _, _ = pseudo_sqrt(M + E - E.T, 1e-12)
    assert np.max(np.abs(S2 - S)) < 1e-14


# independent dense probe, dt = 0.05, J = h = 1, C(n dt) for n = 1..20
DENSE_PROBE = {
    (3, 3): [0.9801659132, 0.9229986696, 0.8350997336, 0.7262148092, 0.6076354203, 0.4904579044,
             0.3840413542, 0.2949340787, 0.2264112208, 0.1786215926, 0.1492172895, 0.1342626063,
             0.1292000698, 0.1296850394, 0.1321681338, 0.1341836049, 0.1343709056, 0.1323025095,
             0.1282090527, 0.1226864571],
    (5, 1): [0.9900332889, 0.9607261975, 0.9138089391, 0.8520069009, 0.7788192746, 0.6982395386,
             0.6144442863, 0.5314793717, 0.4529718277, 0.3818925980, 0.3203892529, 0.2697002152,
             0.2301534884, 0.2012443932, 0.1817792999, 0.1700665648, 0.1641323995, 0.1619384772,
             0.1615796999, 0.1614443782],
    (2, 2): [0.9900332889, 0.9607261975, 0.9138089391, 0.8520069009, 0.7788192745, 0.6982395378,
             0.6144442817, 0.5314793547, 0.4529717805, 0.3818925004, 0.3203891223, 0.2697002321,
             0.2301543000, 0.2012477428, 0.1817891973, 0.1700912894, 0.1641876962, 0.1620523592,
             0.1617992951, 0.1618452267],
}


@pytest.mark.parametrize("geom", sorted(DENSE_PROBE))
def test_dense_route_matches_independent_probe(geom):
    lat = Lattice(*geom)
    C, O = dense.trotter_trajectory(lat, 1.0, 1.0, 0.05, 20)
    assert C[0] == 1.0
    assert np.max(np.abs(np.asarray(C[1:]) - np.asarray(DENSE_PROBE[geom]))) <= 1e-10
    # unitary conjugation keeps Tr[O^2]/2^N = 1
    assert abs(np.real(np.trace(O @ O)) / 2 ** lat.n_sites - 1.0) < 1e-12
