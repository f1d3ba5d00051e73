"""The arithmetic behind the split-bf16 products (precision HPT_FP32_BF16X6),
checked on the host with an exact emulation of round-to-nearest-even bf16.

Every float32 x is written as h + m + l with h = bf16(x), m = bf16(x - h),
l = bf16(x - h - m); the GPU product keeps the six terms hh, hm, mh, mm, hl,
lh of (ha + ma + la)(hb + mb + lb).  Both facts used by the kernel are pinned
here: the split is exact, and the dropped terms stay below 2^-22 |a b| (the
float32 unit roundoff is 2^-24)."""

import numpy as np


def bf16(x):
    """float32 -> nearest bf16 (ties to even), returned as float32."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split3(x):
    x = np.asarray(x, dtype=np.float32)
    h = bf16(x)
    r = (x - h).astype(np.float32)      # exact: x and h share the leading bits
    m = bf16(r)
    l = bf16((r - m).astype(np.float32))
    return h, m, l


def _samples(n=200000, seed=5):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(1.0, 2.0, n)
    expo = rng.integers(-60, 60, n)
    sign = rng.choice([-1.0, 1.0], n)
    return (sign * mant * 2.0 ** expo).astype(np.float32)


def test_three_way_split_is_exact():
    x = _samples()
    h, m, l = split3(x)
    assert np.array_equal(h.astype(np.float64) + m.astype(np.float64) + l.astype(np.float64), x.astype(np.float64))
    # every part is a bf16 value (low 16 bits clear)
    for p in (h, m, l):
        assert not np.any(p.view(np.uint32) & 0xFFFF)


def test_six_products_are_float32_accurate():
    a, b = _samples(seed=1), _samples(seed=2)
    ha, ma, la = (p.astype(np.float64) for p in split3(a))
    hb, mb, lb = (p.astype(np.float64) for p in split3(b))
    six = ha * hb + ha * mb + ma * hb + ma * mb + ha * lb + la * hb
    exact = a.astype(np.float64) * b.astype(np.float64)
    rel = np.abs(six - exact) / np.abs(exact)
    assert rel.max() <= 2.0 ** -22
    # three products (the common bf16x3 scheme) would not be: ~2^-16
    three = ha * hb + ha * mb + ma * hb
    assert (np.abs(three - exact) / np.abs(exact)).max() > 2.0 ** -20
