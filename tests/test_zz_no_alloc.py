"""hpt_gram64_noalloc (the float64 Gram of Eq. cholqr with its partials in the
library's static device scratch) against hpt_gram64 (caller workspace) and the
oracle, through the C ABI: two calls in a row, the second smaller, each equal
bit for bit to the workspace entry point on the same input; sizes past the
scratch limit are refused before any launch."""

import ctypes

import numpy as np
import pytest

from oracle.linalg import gram
from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu


def _pair(hpt, m, n, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((n, m), generator=g, dtype=torch.float32, device="cuda")
    Gw = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    Gn = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(hpt.gram64_workspace_bytes(m, n), 1), dtype=torch.uint8, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    hpt.check(hpt.lib.hpt_gram64(P(X.data_ptr()), m, n, m, P(Gw.data_ptr()), n, P(ws.data_ptr()), ws.numel(), st),
              "hpt_gram64")
    hpt.check(hpt.lib.hpt_gram64_noalloc(P(X.data_ptr()), m, n, m, P(Gn.data_ptr()), n, st), "hpt_gram64_noalloc")
    torch.cuda.synchronize()
    return X, Gw.cpu().numpy(), Gn.cpu().numpy()


def test_noalloc_gram_matches_workspace_entry_point_twice():
    hpt = load_hpt()
    for m, n, seed in ((200000, 300, 1), (5003, 70, 2)):
        X, Gw, Gn = _pair(hpt, m, n, seed)
        assert np.array_equal(Gw, Gn), (m, n)
        Xh = X.double().cpu().numpy().T
        ref = gram(Xh)
        bound = m * 2.3e-16 * gram(np.abs(Xh))
        assert np.all(np.abs(Gn - ref) <= bound), (m, n)


def test_noalloc_gram_refuses_sizes_past_the_scratch():
    hpt = load_hpt()
    P = ctypes.c_void_p
    n = hpt_max_n = 2897
    assert hpt.lib.hpt_gram64_noalloc(P(256), 16, n, 16, P(256), n, None) == -1
    assert hpt.lib.hpt_gram64_noalloc(P(256), -1, 4, 16, P(256), 4, None) == -1
    assert hpt.lib.hpt_gram64_noalloc(P(256), 16, 0, 16, None, 0, None) == 0
    assert hpt_max_n == 2897
