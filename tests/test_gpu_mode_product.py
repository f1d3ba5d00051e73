"""hpt_mode_product_f32 (the float32 mode product of the absorb step and the
gauge-BP environment products, Sec. "Gate Update" item 1) against the
oracle's float64 mode product, through the C ABI.  The shapes reach every
kernel form: the leading leg (inner == 1, with and without 16-byte loads),
16-row strips (odd or short inner), 32-row strips (even inner >= 32), each
with ragged strip and block tails and every factor width 16 .. 128 (the
chi = 100 instantiation with 25 k-steps, and n = 112 with 28); then the
full-size legs of an interior site at chi = 100 on sampled outputs.  Float32
MFMA products summed in float32: |error| <= 2 (n + 2) eps32 sum_k |S_jk x_k|.
Repeated calls give the same output bit for bit."""

import numpy as np
import pytest

from oracle.network import mode_product
from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _case(hpt, n, inner, outer, seed):
    import torch
    r = inputs.rng(seed)
    A = r.standard_normal((outer, n, inner)).astype(np.float32)   # column-major inner x n x outer
    S = r.standard_normal((n, n)).astype(np.float32)              # S[j, k]
    src = torch.from_numpy(A).cuda()
    Sd = torch.from_numpy(np.ascontiguousarray(S.T)).cuda()       # column-major S
    dst = hpt.mode_product_f32(src, Sd, inner, outer)
    dst2 = hpt.mode_product_f32(src, Sd, inner, outer)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert np.array_equal(out, dst2.cpu().numpy())
    T = A.astype(np.float64).transpose(2, 1, 0)                     # (inner, n, outer)
    ref = mode_product(T, S.astype(np.float64), 1).transpose(2, 1, 0)
    bound = mode_product(np.abs(T), np.abs(S.astype(np.float64)), 1).transpose(2, 1, 0)
    err = np.abs(out.astype(np.float64) - ref)
    assert np.all(err <= 2 * (n + 2) * EPS32 * bound + 1e-30), float((err / (bound + 1e-30)).max())


@pytest.mark.parametrize("n,outer", [(100, 1007), (17, 16), (128, 333), (64, 50), (99, 21), (112, 40)])
def test_leading_leg(n, outer):
    _case(load_hpt(), n, 1, outer, 1000 + n + outer)


@pytest.mark.parametrize("n,inner,outer", [(100, 33, 9), (45, 17, 5), (100, 16, 4), (80, 30, 3), (128, 19, 2)])
def test_16_row_strips(n, inner, outer):
    _case(load_hpt(), n, inner, outer, 2000 + n + inner)


@pytest.mark.parametrize("n,inner,outer", [(100, 250, 7), (96, 64, 3), (112, 96, 2), (128, 40, 3), (3, 32, 1),
                                           (50, 1000, 4), (100, 10000, 4), (64, 34, 5)])
def test_32_row_strips(n, inner, outer):
    _case(load_hpt(), n, inner, outer, 3000 + n + inner)


def test_shapes_not_served_are_rejected():
    import torch
    hpt = load_hpt()
    x = torch.zeros(4096, dtype=torch.float32, device="cuda")
    S = torch.zeros(16 * 16, dtype=torch.float32, device="cuda").view(16, 16)
    for inner, outer in [(8, 32), (1, 8)]:
        with pytest.raises(hpt.HptError):
            hpt.mode_product_f32(x[:inner * 16 * outer], S, inner, outer)
    S2 = torch.zeros(129 * 129, dtype=torch.float32, device="cuda").view(129, 129)
    y = torch.zeros(129 * 16, dtype=torch.float32, device="cuda")
    with pytest.raises(hpt.HptError):
        hpt.mode_product_f32(y, S2, 1, 16)


@pytest.mark.parametrize("inner,outer", [(1, 4 * 10 ** 6), (10 ** 4, 400), (10 ** 6, 4)])
def test_full_size_interior_legs_sampled(inner, outer):
    """chi = 100, an interior site's 4 chi^4 = 4e8 entries, the mode on leg
    0 (leading), 2 and 3 (the last before the Pauli leg)."""
    import torch
    hpt = load_hpt()
    n = 100
    g = torch.Generator(device="cuda").manual_seed(inner + outer)
    src = torch.randn(inner * n * outer, generator=g, dtype=torch.float32, device="cuda")
    S = torch.randn((n, n), generator=g, dtype=torch.float32, device="cuda")   # column-major: S[j, k] = S_t[k, j]
    dst = hpt.mode_product_f32(src, S, inner, outer)
    torch.cuda.synchronize()
    r = inputs.rng(inner + 17)
    a = torch.from_numpy(r.integers(0, inner, size=300)).cuda()
    b = torch.from_numpy(r.integers(0, outer, size=300)).cuda()
    x = src.view(outer, n, inner)[b, :, a].double().cpu().numpy()            # (300, n): x[s, k]
    y = dst.view(outer, n, inner)[b, :, a].double().cpu().numpy()
    St = S.double().cpu().numpy()                                            # St[k, j] = S[j, k]
    ref = x @ St
    bound = np.abs(x) @ np.abs(St)
    assert np.all(np.abs(y - ref) <= 2 * (n + 2) * EPS32 * bound)
    # the last strip of the slab and the last column block
    tail = dst.view(outer, n, inner)[outer - 1, :, inner - 1].double().cpu().numpy()
    xt = src.view(outer, n, inner)[outer - 1, :, inner - 1].double().cpu().numpy()
    assert np.all(np.abs(tail - xt @ St) <= 2 * (n + 2) * EPS32 * (np.abs(xt) @ np.abs(St)))
