"""Pins of the oracle's general labeller (the method's variants): full-HSV
inRange masks, a filter unit as large as the scene, and the filtered colour
image.  Each is held against something other than the oracle itself: the
standard library's colorsys, hand-worked HSV cases, exact-rational Otsu by a
different formula, the brute-force composition in tests/brute.py, and
closed-form properties."""
import colorsys
import os

import numpy as np
import pytest

from oracle import sil_ref as R
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hsv8_cases.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(v) for v in line.split()[:6]])
    return np.array(rows, dtype=np.int64)


def test_hsv8_hand_worked_cases():
    rows = _golden_rows()
    got = R.hsv8(rows[:, :3].astype(np.uint8)).astype(np.int64)
    np.testing.assert_array_equal(got, rows[:, 3:6])


def test_hsv8_agrees_with_colorsys():
    # every 5th level on each axis plus random triples; the library's float
    # hue and saturation, scaled to the 8-bit convention, lie within half a
    # unit of the oracle's rounded values (hue compared on the circle)
    lv = np.arange(0, 256, 5)
    grid = np.stack(np.meshgrid(lv, lv, lv, indexing="ij"), -1).reshape(-1, 3)
    rnd = np.random.default_rng(11).integers(0, 256, size=(60000, 3))
    rgb = np.concatenate([grid, rnd]).astype(np.uint8)
    hsv = R.hsv8(rgb).astype(np.float64)
    for (r, g, b), (H, S, V) in zip(rgb.tolist(), hsv.tolist()):
        h, s, v = colorsys.rgb_to_hsv(r / 255.0, g / 255.0, b / 255.0)
        assert V == max(r, g, b)
        assert abs(S - s * 255.0) <= 0.5 + 1e-9, (r, g, b, S, s * 255)
        dh = abs(H - h * 180.0) % 180.0
        assert min(dh, 180.0 - dh) <= 0.5 + 1e-9, (r, g, b, H, h * 180)


def test_hsv8_is_scale_free_and_in_range():
    rgb = np.random.default_rng(12).integers(0, 128, size=(20000, 3)).astype(np.uint8)
    a = R.hsv8(rgb).astype(np.int64)
    b = R.hsv8((rgb * 2).astype(np.uint8)).astype(np.int64)
    assert a[:, 0].max() <= 179
    # doubling a colour keeps its hue and saturation up to one rounding step
    assert np.abs(a[:, 1] - b[:, 1]).max() <= 1
    dh = np.abs(a[:, 0] - b[:, 0]) % 180
    assert np.minimum(dh, 180 - dh).max() <= 1
    np.testing.assert_array_equal(b[:, 2], 2 * a[:, 2])


def test_filtered_band_closed_forms():
    for v in range(1, 256, 17):
        for vc in range(0, 256, 15):
            assert R.filtered_band(v, v, vc) == vc      # the brightest band becomes vc
            assert R.filtered_band(0, v, vc) == 0
            assert R.filtered_band(v // 2, v, v) == v // 2  # vc == v leaves the colour
    assert R.filtered_band(0, 0, 200) == 0
    assert R.filtered_band(1, 2, 1) == 1  # 0.5 rounds up
    assert R.filtered_band(1, 4, 2) == 1  # 0.5 rounds up


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_vacuous_limits_equal_the_fused_labeller(dtype):
    rng = np.random.default_rng(21 if dtype == "u8" else 22)
    for trial in range(6):
        H, W = int(rng.integers(20, 90)), int(rng.integers(20, 90))
        if dtype == "u8":
            scene = rng.integers(0, 256, size=(3, H, W)).astype(np.uint8)
            p = R.make_params(chip=int(rng.choice([8, 16, 33, 256])), patch_h=13, patch_w=21)
        else:
            scene = rng.integers(0, 11000, size=(3, H, W)).astype(np.uint16)
            p = R.make_params(dtype=R.U16, chip=int(rng.choice([8, 16, 33, 256])),
                              patch_h=13, patch_w=21)
        lab, hist, chips = R.label(scene, p, want_chips=True)
        ex = R.label_ex(scene, p, want_chips=True)
        np.testing.assert_array_equal(ex["masks"], (1 << lab.astype(np.uint32)).astype(np.uint8))
        np.testing.assert_array_equal(ex["counts"], hist)
        np.testing.assert_array_equal(ex["chips"], chips)


def _masks_from(Hc, Sc, Vc, lo, hi):
    bits = np.zeros(Vc.shape, dtype=np.uint8)
    for c in range(3):
        m = ((Hc >= lo[c][0]) & (Hc <= hi[c][0]) & (Sc >= lo[c][1]) & (Sc <= hi[c][1])
             & (Vc >= lo[c][2]) & (Vc <= hi[c][2]))
        bits |= (m.astype(np.uint8) << c)
    return bits


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_full_hsv_masks_match_brute_force(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(12, 30)), int(rng.integers(12, 30))
    scene = rng.integers(0, 256, size=(3, H, W)).astype(np.uint8)
    # overlapping, gappy, hue- and saturation-bounded ranges
    lo = [[0, 40, 0], [20, 0, 60], [100, 10, 150]]
    hi = [[90, 255, 120], [179, 200, 220], [170, 255, 255]]
    chip = int(rng.choice([7, 16, 64]))
    p = R.make_params(lo=lo, hi=hi, chip=chip, patch_h=9, patch_w=11)
    ex = R.label_ex(scene, p, sel=(2, 0, 1), want_rgb=True)
    Vc, planes = brute.filtered_v(scene, chip=chip, sel=(2, 0, 1))
    blue, green, red = planes
    hsv = R.hsv8(np.stack([red, green, blue], -1).astype(np.uint8)).astype(np.int64)
    want = _masks_from(hsv[..., 0], hsv[..., 1], Vc, lo, hi)
    np.testing.assert_array_equal(ex["masks"], want)
    ny, nx = -(-H // 9), -(-W // 11)
    counts = np.zeros((ny, nx, 3), dtype=np.int64)
    for c in range(3):
        bit = (want >> c) & 1
        for py in range(ny):
            for px in range(nx):
                counts[py, px, c] = bit[py * 9:(py + 1) * 9, px * 11:(px + 1) * 11].sum()
    np.testing.assert_array_equal(ex["counts"], counts)
    # the filtered colour image: its brightest band is exactly Vc
    np.testing.assert_array_equal(ex["rgb"].max(axis=0), Vc)


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_scene_level_filter_unit_matches_brute_force(dtype):
    rng = np.random.default_rng(41 if dtype == "u8" else 42)
    H, W = 30, 37
    if dtype == "u8":
        scene = rng.integers(0, 256, size=(3, H, W)).astype(np.uint8)
        p = R.make_params(chip=1 << 20)
    else:
        scene = rng.integers(0, 11000, size=(3, H, W)).astype(np.uint16)
        p = R.make_params(dtype=R.U16, chip=1 << 20)
    # the fused labeller stops at 256 x 256 chips; the general one takes the scene
    assert R.validate(3, (0, 1, 2), H, W, W, W, p) == R.EUNSUPPORTED
    ex = R.label_ex(scene, p, want_rgb=True, want_chips=True)
    labels, hist, infos = brute.label_scene(scene, dtype=dtype, chip=1 << 20)
    np.testing.assert_array_equal(ex["masks"], (1 << labels.astype(np.uint32)).astype(np.uint8))
    np.testing.assert_array_equal(ex["counts"], hist)
    ci = ex["chips"][0, 0]
    for k in ("t", "lo", "hi", "gate", "stretch"):
        assert int(ci[k]) == infos[(0, 0)][k], k
    Vc, _ = brute.filtered_v(scene, dtype=dtype, chip=1 << 20)
    np.testing.assert_array_equal(ex["rgb"].max(axis=0), Vc)


def test_filter_off_rgb_is_the_8bit_colour():
    rng = np.random.default_rng(43)
    scene = rng.integers(0, 11000, size=(3, 17, 19)).astype(np.uint16)
    p = R.make_params(dtype=R.U16, filter=0)
    ex = R.label_ex(scene, p, want_rgb=True)
    want = np.vectorize(lambda v: brute.rescale_decimal(int(v)))(scene)
    np.testing.assert_array_equal(ex["rgb"], want)


def test_large_chip_statistics_are_exact():
    # chips of up to 2^27 pixels: the between-class comparisons exceed 128 bits
    uni = np.full(256, 1 << 19, dtype=np.uint32)  # N = 2^27
    st = R.chip_stats(uni)
    assert st["t"] == 127 and st["gate"] == 1  # eta = 16384/21845 > 3/4
    k = (1 << 27) >> 8
    assert st["lo"] == k // (1 << 19) and st["hi"] == 255 - k // (1 << 19)
    two = np.zeros(256, dtype=np.uint32)
    two[40], two[200] = 3 << 24, 5 << 24
    st = R.chip_stats(two)
    assert st["t"] == 40 and st["gate"] == 1
    rng = np.random.default_rng(44)
    for trial in range(12):
        h = np.zeros(256, dtype=np.int64)
        nz = rng.choice(256, size=int(rng.integers(2, 40)), replace=False)
        h[nz] = rng.integers(1, 1 << 22, size=nz.size)
        while h.sum() > (1 << 27):
            h //= 2
        if (h > 0).sum() < 2:
            continue
        t, eta = brute.otsu_hist_within(h)
        st = R.chip_stats(h.astype(np.uint32))
        assert st["t"] == t
        assert st["gate"] == int(eta >= brute.Fraction(3, 4))


def test_validate_ex():
    p = R.make_params(lo=[[0, 40, 0], [20, 0, 60], [100, 10, 150]],
                      hi=[[90, 255, 120], [179, 200, 220], [170, 255, 255]])
    assert R.validate_ex(3, (0, 1, 2), 100, 100, 100, 100, p) == R.OK
    assert R.validate(3, (0, 1, 2), 100, 100, 100, 100, p) != R.OK
    big = R.make_params(chip=1 << 20)
    assert R.validate_ex(3, (0, 1, 2), 11585, 11585, 11585, 11585, big) == R.OK   # < 2^27 px
    assert R.validate_ex(3, (0, 1, 2), 11586, 11586, 11586, 11586, big) == R.EUNSUPPORTED
    assert R.validate_ex(3, (0, 1, 2), 11586, 11586, 11586, 11586,
                         R.make_params(chip=1 << 20, filter=0)) == R.OK
    assert R.validate_ex(3, (0, 1, 3), 10, 10, 10, 10, p) == R.EINVAL
    assert R.validate_ex(3, (0, 1, 2), 10, 10, 10, 9, p) == R.EINVAL
    assert R.validate_ex(3, (0, 1, 2), 10, 10, 10, 10,
                         R.make_params(dtype=R.U16, refl_max=70000)) == R.EUNSUPPORTED
