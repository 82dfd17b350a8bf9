"""Pins of the CPU oracle's individual steps (no GPU).

Every expected value comes from the paper's printed limits (tests/golden),
from closed forms, or from the brute-force checkers in tests/brute.py, which
take a different route (library routines, pixel lists, within-class variance,
exact fractions) than the oracle's integer histogram formulas.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import sil_ref as R
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---- paper constants ----------------------------------------------------------

def test_default_limits_are_the_papers():
    """Section III-B limits (golden file) are the oracle's defaults."""
    p = R.make_params()
    for cid, _name, *vals in _read_table("paper_hsv_limits.txt"):
        c = int(cid)
        lo, hi = [int(v) for v in vals[:3]], [int(v) for v in vals[3:]]
        assert [p.lo[c][j] for j in range(3)] == lo
        assert [p.hi[c][j] for j in range(3)] == hi


def test_v_boundaries_u8():
    """Inclusive limits: 30 water / 31 thin / 204 thin / 205 thick (filter off)."""
    rows = _read_table("v_boundaries.txt")
    v = np.array([int(r[0]) for r in rows], dtype=np.uint8)
    want = np.array([int(r[1]) for r in rows], dtype=np.uint8)
    scene = np.stack([v, v // 2, v // 3])[:, None, :]  # V = max = v
    labels, hist = R.label(scene, R.make_params(filter=0, patch_h=1, patch_w=len(v)))
    assert (labels[0] == want).all()
    assert hist.sum() == len(v)
    for c in range(3):
        assert hist[0, 0, c] == (want == c).sum()


def test_v_boundaries_u16():
    """Reflectance cut-offs follow from round-half-up rescaling to 8 bits:
    1196 -> 30, 1197 -> 31, 8019 -> 204, 8020 -> 205 (refl_max 10000)."""
    xs = np.array([0, 1196, 1197, 8019, 8020, 10000, 65535], dtype=np.uint16)
    want = [0, 0, 1, 1, 2, 2, 2]
    assert [brute.rescale_decimal(int(x)) for x in xs] == [0, 30, 31, 204, 205, 255, 255]
    scene = np.stack([xs, xs, xs])[:, None, :]
    labels, _ = R.label(scene, R.make_params(dtype=R.U16, filter=0))
    assert labels[0].tolist() == want


@pytest.mark.parametrize("refl_max", [10000, 1, 2, 255, 256, 4095, 65535, 12345])
def test_rescale_matches_decimal(refl_max):
    xs = list(range(0, 65536, 1 if refl_max == 10000 else 37)) + [65535]
    got = [R.rescale(x, refl_max) for x in xs]
    want = [brute.rescale_decimal(x, refl_max) for x in xs]
    assert got == want


def test_value_plane_is_band_max():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 256, (4, 9, 11)).astype(np.uint8)
    V = R.value_plane(s, sel=(3, 0, 2))
    assert (V == np.maximum(np.maximum(s[3], s[0]), s[2])).all()


def test_class_of_each_value():
    p = R.make_params()
    rows = {int(a): int(b) for a, b in _read_table("v_boundaries.txt")}
    for v in range(256):
        c = R.class_of(v, p)
        H, S, V = 0, 0, v
        want, n = brute.in_range_class(np.array(H), np.array(S), np.array(V))
        assert n == 1 and c == int(want)
        if v in rows:
            assert c == rows[v]


# ---- median -------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (2, 2), (3, 3), (13, 17), (64, 65)])
def test_median_matches_scipy(shape):
    rng = np.random.default_rng(sum(shape))
    for spread in (3, 256):
        V = rng.integers(0, spread, shape).astype(np.uint8)
        assert (R.median3x3(V) == brute.median3x3(V)).all()


def test_median_of_binary_image_is_majority():
    rng = np.random.default_rng(11)
    B = (rng.random((20, 23)) < 0.5).astype(np.uint8)
    P = np.pad(B, 1, mode="edge").astype(np.int32)
    votes = sum(P[1 + dy:1 + dy + 20, 1 + dx:1 + dx + 23] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    assert (R.median3x3(B * 255) == np.where(votes >= 5, 255, 0)).all()


# ---- Otsu, gate, ranks -----------------------------------------------------------

def _hist(px):
    return np.bincount(np.asarray(px, dtype=np.int64), minlength=256)


def test_otsu_uniform_closed_form():
    """Uniform 0..255: the class means always differ by 128, so t* maximises
    w0*w1 -> t* = 127; eta = 16384/21845, just above 3/4."""
    h = np.ones(256)
    info = R.chip_stats(h)
    assert info["t"] == 127 and info["gate"] == 1
    px = list(range(256))
    assert brute.eta(px, 127) == Fraction(16384, 21845)
    assert R.chip_stats(h, R.make_params(eta_num=16384, eta_den=21845))["gate"] == 1
    assert R.chip_stats(h, R.make_params(eta_num=16385, eta_den=21845))["gate"] == 0


@pytest.mark.parametrize("a,b", [(0, 255), (10, 200), (100, 101), (3, 90)])
def test_otsu_two_spikes(a, b):
    """Two values a < b: every t in [a, b-1] is a perfect split (eta = 1);
    the smallest, t = a, wins."""
    h = np.zeros(256)
    h[a] = 7
    h[b] = 3
    info = R.chip_stats(h, R.make_params(eta_num=1, eta_den=1))
    assert info["t"] == a and info["gate"] == 1


def test_otsu_constant_chip_has_no_split():
    for v in (0, 77, 255):
        h = np.zeros(256)
        h[v] = 100
        info = R.chip_stats(h)
        assert info["t"] == -1 and info["gate"] == 0 and info["stretch"] == 0
        assert info["lo"] == v and info["hi"] == v


def test_otsu_matches_within_class_brute_force():
    rng = np.random.default_rng(123)
    for trial in range(60):
        n = int(rng.integers(2, 90))
        kind = trial % 3
        if kind == 0:
            px = rng.integers(0, 256, n)
        elif kind == 1:
            px = rng.integers(100, 110, n)  # narrow: many ties between splits
        else:
            px = np.concatenate([rng.normal(40, 5, n // 2), rng.normal(200, 20, n - n // 2)])
            px = np.clip(np.round(px), 0, 255).astype(np.int64)
        info = R.chip_stats(_hist(px))
        t = brute.otsu_within(px)
        assert info["t"] == (-1 if t is None else t), (trial, px)
        if t is not None:
            e = brute.eta(px, t)
            assert info["gate"] == int(e >= Fraction(3, 4))


def test_gate_edge_cases():
    # eta exactly at the gate passes (>=)
    px = [0, 0, 0, 255]  # t* = 0, eta = 1
    assert R.chip_stats(_hist(px), R.make_params(eta_num=1, eta_den=1))["gate"] == 1
    px = [10, 20, 30]  # three equally spaced values
    t = brute.otsu_within(px)
    e = brute.eta(px, t)
    assert e == Fraction(3, 4)
    assert R.chip_stats(_hist(px))["gate"] == 1
    assert R.chip_stats(_hist(px), R.make_params(eta_num=751, eta_den=1000))["gate"] == 0


def test_ranks_match_sort():
    rng = np.random.default_rng(9)
    for n in (1, 2, 255, 256, 257, 511, 512, 1000, 65536):
        px = rng.integers(0, 256, n)
        for cs in (1, 4, 8, 31):
            info = R.chip_stats(_hist(px), R.make_params(clip_shift=cs))
            assert (info["lo"], info["hi"]) == brute.ranks(px, cs), (n, cs)


# ---- stretch ------------------------------------------------------------------

def test_stretch_closed_forms():
    for lo, hi in [(0, 255), (10, 20), (31, 204), (100, 101)]:
        assert R.stretch(lo, lo, hi) == 0 and R.stretch(hi, lo, hi) == 255
        assert R.stretch(max(lo - 1, 0), lo, hi) == 0 and R.stretch(min(hi + 1, 255), lo, hi) == 255
    assert all(R.stretch(m, 0, 255) == m for m in range(256))  # identity range
    # half-up: (m - lo)*255/(hi - lo) = 127.5 -> 128
    assert R.stretch(1, 0, 2) == 128


def test_stretch_matches_fractions():
    rng = np.random.default_rng(17)
    cases = [(int(m), int(lo), int(hi)) for m, lo, hi in rng.integers(0, 256, (20000, 3))]
    cases += [(m, lo, lo + 1) for lo in range(0, 255, 7) for m in range(0, 256, 5)]
    for m, lo, hi in cases:
        if hi <= lo:
            continue
        assert R.stretch(m, lo, hi) == brute.stretch(m, lo, hi), (m, lo, hi)


# ---- colour rendering ---------------------------------------------------------

def _palette():
    pal = np.zeros((256, 3), dtype=np.uint8)  # ids the paper does not name: black
    for cid, _name, r, g, b in _read_table("paper_class_colours.txt"):
        pal[int(cid)] = (int(r), int(g), int(b))
    return pal


def test_render_rgb_uses_the_papers_colours():
    """Every id 0..255 once, in a row of odd length: the three classes get
    the colours the paper names (golden file), every other id black."""
    ids = np.arange(256, dtype=np.uint8)[::-1].reshape(1, 256)
    lab = np.zeros((2, 257), dtype=np.uint8)
    lab[0, :256] = ids
    lab[1, :] = 1
    out = R.render_rgb(lab)
    pal = _palette()
    assert (out[0, :256] == pal[ids[0]]).all()
    assert (out[1] == pal[1]).all()
    assert tuple(out[0, 256]) == tuple(pal[0])


def test_render_rgb_of_labelled_scene():
    """End to end: a scene with one V per class (filter off) renders as the
    paper's colours of those classes."""
    v = np.array([10, 100, 230, 30, 31, 204, 205], dtype=np.uint8)
    scene = np.stack([v, v // 2, v // 3])[:, None, :]
    labels, _ = R.label(scene, R.make_params(filter=0, patch_h=1, patch_w=len(v)))
    out = R.render_rgb(labels)
    want = _palette()[[0, 1, 2, 0, 1, 1, 2]]
    assert (out[0] == want).all()


def test_render_rgb_leaves_row_padding():
    """rgb rows longer than 3 W keep their bytes past 3 W."""
    lib = R.lib()
    lab = np.array([[0, 1, 2], [2, 1, 0]], dtype=np.uint8)
    rgb = np.full((2, 11), 7, dtype=np.uint8)
    lib.sil_ref_render_rgb(lab.ctypes.data, 2, 3, 3, rgb.ctypes.data, 11)
    assert (rgb[:, 9:] == 7).all()
    pal = _palette()
    assert (rgb[:, :9].reshape(2, 3, 3) == pal[lab]).all()
