"""End-to-end pins of the oracle (no GPU): brute-force composition on tiny
scenes, the exhaustive HSV check, invariants and metamorphic relations."""
import numpy as np
import pytest

from oracle import sil_ref as R
from tests import brute
import synth


def _scene(rng, H, W, dtype, nb=3):
    kind = rng.integers(0, 3)
    if kind == 0:
        s = rng.integers(0, 256, (nb, H, W))
    elif kind == 1:  # two populations with noise: Otsu-gated chips
        base = np.where(rng.random((H, W)) < 0.5, 40, 200)
        s = np.clip(base[None] + rng.normal(0, 12, (nb, H, W)), 0, 255)
    else:  # narrow band: gate mostly fails
        s = rng.integers(120, 135, (nb, H, W))
    s = s.astype(np.uint8)
    if dtype == "u16":
        s = synth.to_u16(s[:3], seed=int(rng.integers(1 << 30)))
    return s


@pytest.mark.parametrize("seed", range(24))
def test_oracle_matches_brute_force_composition(seed):
    rng = np.random.default_rng(1000 + seed)
    H, W = int(rng.integers(1, 23)), int(rng.integers(1, 23))
    dtype = "u16" if seed % 3 == 0 else "u8"
    chip = int(rng.choice([1, 2, 3, 5, 7, 16]))
    ph, pw = int(rng.choice([1, 3, 4, 7, 64])), int(rng.choice([1, 2, 5, 9, 64]))
    filt = 0 if seed % 5 == 4 else 1
    cs = int(rng.choice([1, 2, 8]))
    s = _scene(rng, H, W, dtype)
    kw = dict(filter=filt, chip=chip, clip_shift=cs, patch_h=ph, patch_w=pw)
    p = R.make_params(dtype=R.U16 if dtype == "u16" else R.U8, **kw)
    labels, hist, chips = R.label(s, p, want_chips=True)
    bl, bh, binfo = brute.label_scene(s, dtype=dtype, **kw)
    assert (labels == bl).all()
    assert (hist == bh).all()
    if filt:
        for (cy, cx), d in binfo.items():
            c = chips[cy, cx]
            assert (c["t"], c["lo"], c["hi"], c["gate"], c["stretch"]) == \
                (d["t"], d["lo"], d["hi"], d["gate"], d["stretch"])


def test_hsv_limits_reduce_to_v_exhaustive():
    """All 2^24 8-bit colours: the paper's three 3-D inRange masks on the
    hexcone HSV (hue/saturation limits included) give exactly one mask per
    colour, and it is the class the oracle assigns from V alone."""
    v = np.arange(1 << 24, dtype=np.uint32)
    R8 = (v >> 16).astype(np.uint8)
    G8 = ((v >> 8) & 255).astype(np.uint8)
    B8 = (v & 255).astype(np.uint8)
    scene = np.stack([B8, G8, R8]).reshape(3, 4096, 4096)
    labels, hist = R.label(scene, R.make_params(filter=0, patch_h=4096, patch_w=4096))
    Hh, S, V = brute.hsv_opencv8(R8, G8, B8)
    assert Hh.max() <= 180 and S.max() <= 255
    cls, n = brute.in_range_class(Hh, S, V)
    assert (n == 1).all()
    assert (labels.ravel() == cls).all()
    # V = max(R,G,B): class counts follow from the count of colours per max value
    counts = np.array([(m + 1) ** 3 - m ** 3 for m in range(256)])
    assert hist[0, 0, 0] == counts[:31].sum()
    assert hist[0, 0, 1] == counts[31:205].sum()
    assert hist[0, 0, 2] == counts[205:].sum()


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_invariants_on_generated_scene(dtype):
    spec = synth.config_small()
    spec.dtype = dtype
    s = synth.generate(spec)
    for ph, pw in [(64, 64), (256, 256), (100, 37), (512, 512)]:
        p = R.make_params(dtype=R.U16 if dtype == "u16" else R.U8, patch_h=ph, patch_w=pw)
        labels, hist = R.label(s, p)
        assert labels.max() <= 2
        ny, nx = hist.shape[:2]
        # counts = recount of the label plane; each patch holds its pixel count
        for py in range(ny):
            for px in range(nx):
                blk = labels[py * ph:(py + 1) * ph, px * pw:(px + 1) * pw]
                assert hist[py, px].tolist() == np.bincount(blk.ravel(), minlength=3).tolist()
        assert hist.sum() == labels.size


def test_band_permutation_invariance():
    rng = np.random.default_rng(3)
    s = rng.integers(0, 256, (5, 40, 33)).astype(np.uint8)
    p = R.make_params(chip=16, patch_h=8, patch_w=8)
    l0, h0 = R.label(s, p, sel=(0, 1, 2))
    for sel in [(2, 1, 0), (1, 0, 2)]:
        l1, h1 = R.label(s, p, sel=sel)
        assert (l0 == l1).all() and (h0 == h1).all()
    l2, _ = R.label(s, p, sel=(3, 1, 2))
    assert l2.shape == l0.shape


def test_u16_scene_agrees_with_its_8bit_rescale():
    """Labelling a reflectance scene equals labelling its 8-bit rescale
    (the rescale is monotone, so it commutes with max and median)."""
    spec = synth.config_small()
    s8 = synth.generate_u8(spec)
    s16 = synth.to_u16(s8, seed=9)
    lut = np.array([brute.rescale_decimal(x) for x in range(65536)], dtype=np.uint8)
    r8 = lut[s16]
    for filt in (0, 1):
        la, ha = R.label(s16, R.make_params(dtype=R.U16, filter=filt, patch_h=64, patch_w=64))
        lb, hb = R.label(r8, R.make_params(dtype=R.U8, filter=filt, patch_h=64, patch_w=64))
        assert (la == lb).all() and (ha == hb).all()


def test_class_is_monotone_in_median_within_chip():
    spec = synth.config_small()
    s = synth.generate_u8(spec)
    p = R.make_params(chip=128)
    labels, _, chips = R.label(s, p, want_chips=True)
    Vm = R.median3x3(R.value_plane(s))
    for cy in range(4):
        for cx in range(4):
            lab = labels[cy * 128:(cy + 1) * 128, cx * 128:(cx + 1) * 128].ravel()
            vm = Vm[cy * 128:(cy + 1) * 128, cx * 128:(cx + 1) * 128].ravel()
            order = np.argsort(vm, kind="stable")
            assert (np.diff(lab[order].astype(int)) >= 0).all()
            # a1/a2 are the class boundaries along Vm
            a1, a2 = chips[cy, cx]["a1"], chips[cy, cx]["a2"]
            assert ((vm >= a1).astype(int) + (vm >= a2) == lab).all()


def test_filter_only_relabels_within_chip_stats():
    """With a gate no chip can pass (eta >= 1 only for two-valued chips),
    the filter reduces to the 3x3 median followed by the thresholds."""
    rng = np.random.default_rng(8)
    s = np.clip(rng.normal(130, 40, (3, 50, 61)), 0, 255).astype(np.uint8)
    labels, _ = R.label(s, R.make_params(eta_num=1, eta_den=1, chip=25))
    Vm = brute.median3x3(np.max(s, axis=0))
    want, _ = brute.in_range_class(0 * Vm, 0 * Vm, Vm)
    assert (labels == want).all()
