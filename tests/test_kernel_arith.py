"""Host checks of the integer-division shortcut the per-pixel kernels rely on
(no GPU): for the hue, saturation and colour-stretch quotients the kernels
compute floor(n / d) as the truncation of one float fma, (n + 1/2) * rd with
rd = a hardware reciprocal of d (accurate to an ulp).  The float arithmetic is
emulated exactly: (n + 1/2) * r is exact in float64 (at most 43 significant
bits) and rounding it once to float32 is what an fma does.  Every float32 r
within two ulps of 1/d is tried, which also covers the exact halvings the
kernels apply to a reciprocal."""
import numpy as np
import pytest


def _near(x, k=2):
    """float32 values within k ulps of the float32 nearest x."""
    c = np.float32(x)
    out = [c]
    lo = hi = c
    for _ in range(k):
        lo = np.nextafter(lo, np.float32(0))
        hi = np.nextafter(hi, np.float32(np.inf))
        out += [lo, hi]
    return out


def _check(d, nmax):
    n = np.arange(nmax, dtype=np.float64)
    want = np.arange(nmax, dtype=np.int64) // d
    for r in _near(1.0 / d):
        got = np.floor(((n + 0.5) * np.float64(r)).astype(np.float32)).astype(np.int64)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (d, float(r), int(bad[0]))


def test_fma_division_all_divisors_reached():
    # divisors: 2V and 2d (saturation and hue, up to 510), V (colour, up to 255);
    # numerators below 2^18 (hue: 661 d + ... < 168 556; saturation < 130 306)
    for d in range(1, 511):
        _check(d, 1 << 18)


@pytest.mark.parametrize("d", [1, 2, 3, 7, 127, 255, 256, 257, 509, 510, 4093, 65535])
def test_fma_division_bound_stated(d):
    # the stated domain, n < 2^20, holds with room to spare
    _check(d, 1 << 20)


def test_fma_division_fails_without_half():
    # the 1/2 offset is what makes truncation exact: without it an exact
    # multiple whose reciprocal rounds down truncates one low
    fails = 0
    for d in range(1, 511):
        n = np.arange(0, 1 << 12, dtype=np.float64)
        r = np.nextafter(np.float32(1.0 / d), np.float32(0))
        got = np.floor((n * np.float64(r)).astype(np.float32)).astype(np.int64)
        fails += int(np.count_nonzero(got != np.arange(1 << 12) // d))
    assert fails > 0
