"""How the gfx950 bf16 MFMA (v_mfma_f32_16x16x32_bf16, the instruction of the
split-bf16 products of HPT_FP32_BF16X6) rounds the float32 sum of its 32
products, through hpt_bf16_mfma_sum.  All inputs are exact in bf16 and the
exact sums are known; every output lane must agree.

Measured behaviour pinned here: the 8 products of one lane group (k in
[8g, 8g + 8)) are aligned to the largest of them and kept to one bit below its
float32 ulp, lower bits truncated (toward zero in magnitude); the group sums
and the accumulator then add with round-to-nearest.  So a product far below
the largest one of its group loses its low bits toward zero: a magnitude
bias, the cause of the one-signed drift of the split-bf16 form."""

import numpy as np
import pytest

from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu
U = 2.0 ** -23   # float32 ulp at 1


def _sum(hpt, a, c):
    import ctypes
    import torch
    x = torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    hpt.check(hpt.lib.hpt_bf16_mfma_sum(ctypes.c_void_p(x.data_ptr()), float(c), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "hpt_bf16_mfma_sum")
    o = out.cpu().numpy().astype(np.float64)
    assert np.all(o == o[0])
    return o[0]


def test_small_products_beside_a_large_one_are_truncated():
    hpt = load_hpt()
    # 1 + 31 * 2^-25 = 1 + 7.75 ulp: the 7 quarter-ulp products of the first
    # group vanish beside the 1 (truncated), the other 24 add exactly: 1 + 6 ulp
    # (round-to-nearest of the exact sum would give 1 + 8 ulp)
    a = [1.0] + [2.0 ** -25] * 31
    assert (_sum(hpt, a, 0.0) - 1.0) / U == 6.0
    # the same with every sign flipped: the loss is toward zero in magnitude
    assert (_sum(hpt, [-x for x in a], 0.0) + 1.0) / U == -6.0
    # half-ulp products keep their one bit: 1 + 3.5 ulp -> 1 + 4 (nearest),
    # then + 3 x 4 ulp: 1 + 16 ulp, as the exact 15.5 ulp rounds
    assert (_sum(hpt, [1.0] + [2.0 ** -24] * 31, 0.0) - 1.0) / U == 16.0


def test_products_of_one_size_and_the_accumulator_round_to_nearest():
    hpt = load_hpt()
    # 31 quarter-ulp products alone (exact 7.75 ulp), then onto c = 1: 1 + 8 ulp
    assert (_sum(hpt, [0.0] + [2.0 ** -25] * 31, 1.0) - 1.0) / U == 8.0
