"""hpt_gram64 (the float64 Gram of float32 data, Eq. cholqr) against the
oracle's definition, through the C ABI: ragged sizes that span several 64 x 64
tiles and 16-row chunks, a padded leading dimension (scalar loads), the empty
reduction, and the full-size 10^6 x 400 block of an interior site at chi = 100
on sampled entries; repeated calls give the same G bit for bit."""

import numpy as np
import pytest

from oracle.linalg import gram
from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu


def _run(hpt, Xcm, ldx=None):
    """Xcm: float32 numpy array m x n (column-major semantics); returns G."""
    import torch
    m, n = Xcm.shape
    ldx = m if ldx is None else ldx
    host = np.zeros((n, ldx), dtype=np.float32)
    host[:, :m] = Xcm.T
    X = torch.from_numpy(host).cuda()
    G = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(hpt.gram64_workspace_bytes(m, n), 1), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    import ctypes
    hpt.check(hpt.lib.hpt_gram64(ctypes.c_void_p(X.data_ptr()), m, n, ldx, ctypes.c_void_p(G.data_ptr()), n,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st)), "hpt_gram64")
    torch.cuda.synchronize()
    return G.cpu().numpy()


@pytest.mark.parametrize("m,n,pad", [(1000, 37, 0), (4099, 130, 0), (777, 65, 3), (17, 1, 0), (0, 5, 0),
                                     (100000, 200, 0)])
def test_gram64_matches_oracle(m, n, pad):
    hpt = load_hpt()
    X = inputs.rng(100 + m + n).standard_normal((m, n)).astype(np.float32)
    G = _run(hpt, X, m + pad)
    ref = gram(X)
    scale = gram(np.abs(X)) if m else np.ones((n, n))
    # float64 sums of exact products: error <= m eps64 sum |x_i x_j|
    assert np.all(np.abs(G - ref) <= max(m, 1) * 2.3e-16 * scale + 1e-300)
    assert np.array_equal(G, G.T)
    G2 = _run(hpt, X, m + pad)
    assert np.array_equal(G, G2)


def test_gram64_full_size_block_sampled():
    hpt = load_hpt()
    import torch
    m, n = 10 ** 6, 400
    g = torch.Generator(device="cuda").manual_seed(7)
    X = torch.randn((n, m), generator=g, dtype=torch.float32, device="cuda")
    G = torch.empty((n, n), dtype=torch.float64, device="cuda")
    hpt.gram64(X, G)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy()
    idx = inputs.rng(11).integers(0, n, size=(40, 2))
    cols = sorted(set(idx.ravel().tolist()))
    Xc = {c: X[c].double().cpu().numpy() for c in cols}
    for i, j in idx:
        ref = gram(np.stack([Xc[i], Xc[j]], axis=1))[0, 1]
        bound = m * 2.3e-16 * float(np.dot(np.abs(Xc[i]), np.abs(Xc[j])))
        assert abs(Gh[i, j] - ref) <= bound, (i, j, Gh[i, j], ref)
    assert np.array_equal(Gh, Gh.T)


def test_gram64_argument_errors():
    hpt = load_hpt()
    import ctypes
    P = ctypes.c_void_p
    assert hpt.lib.hpt_gram64(P(16), -1, 3, 4, P(16), 3, P(16), 1 << 20, None) == -1
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 4, P(16), 3, P(16), 1 << 20, None) == -1   # ldx < m
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 8, P(16), 2, P(16), 1 << 20, None) == -1   # ldg < n
    assert hpt.lib.hpt_gram64(P(16), 8, 3, 8, P(16), 3, P(16), 8, None) == -2          # short workspace
