"""GPU parity of the general labeller (sil_label_ex) against the oracle's
sil_ref_label_ex, bit for bit: full-HSV masks, per-patch mask counts, the
filtered colour image and per-chip statistics, for filter units from one
pixel to the whole scene.  Every call goes through the C ABI."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import sil_ref as R
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sil():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13135_amd import sil as S
    S.lib()
    return S


def _dev(scene_np):
    t = torch.from_numpy(scene_np.view(np.int16) if scene_np.dtype == np.uint16 else scene_np)
    return t.cuda()


def run_gpu(S, scene_np, fields, sel=(0, 1, 2), W=None, rgb=True, pad=0):
    nb, H, pitch = scene_np.shape
    W = pitch if W is None else W
    p = S.Params(**fields)
    dev = _dev(scene_np)
    mbuf = torch.full((H, W + pad), 0xEE, dtype=torch.uint8, device="cuda")
    out = {"masks": mbuf}
    if rgb:
        out["rgb"] = torch.full((3, H, W + pad), 0xEE, dtype=torch.uint8, device="cuda")
    ny, nx = S.hist_dims(H, W, p)
    out["counts"] = torch.full((ny, nx, 3), -5, dtype=torch.int32, device="cuda")
    res = S.label_ex(dev, p, sel=sel, W=W, rgb=rgb, chips=p.filter == 1, out=out)
    torch.cuda.synchronize()
    m = res["masks"].cpu().numpy()
    if pad:
        assert (m[:, W:] == 0xEE).all(), "mask bytes beyond W were written"
    g = {"masks": m[:, :W], "counts": res["counts"].cpu().numpy().astype(np.uint32)}
    if rgb:
        c = res["rgb"].cpu().numpy()
        if pad:
            assert (c[:, :, W:] == 0xEE).all(), "colour bytes beyond W were written"
        g["rgb"] = c[:, :, :W]
    if p.filter == 1:
        g["chips"] = S.decode_chip_info(res["chips"].cpu().numpy())
    return g


def run_oracle(scene_np, fields, sel=(0, 1, 2), W=None, rgb=True):
    p = R.make_params(**fields)
    return R.label_ex(scene_np, p, sel=sel, W=W, want_rgb=rgb,
                      want_chips=fields.get("filter", 1) == 1)


def assert_same(g, o, what):
    for k in ("masks", "counts", "rgb", "chips"):
        if k not in o:
            continue
        a, b = g[k], o[k]
        if k == "chips":
            for f in ("t", "lo", "hi", "gate", "stretch", "a1", "a2"):
                assert (a[f] == b[f]).all(), f"{what}: chip field {f} differs"
            continue
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            idx = tuple(bad[0])
            raise AssertionError(f"{what}: {k} has {len(bad)} mismatches, first at {idx}: "
                                 f"gpu {a[idx]} oracle {b[idx]}")


LIMITS = [
    # the paper's (vacuous H/S)
    (R.make_params().lo, None),
    # hue/saturation-bounded, overlapping and gappy
    ([[0, 40, 0], [20, 0, 60], [100, 10, 150]], [[90, 255, 120], [179, 200, 220], [170, 255, 255]]),
    ([[10, 0, 0], [0, 128, 31], [60, 0, 100]], [[30, 127, 255], [179, 255, 204], [61, 90, 255]]),
]


def _limits(i):
    lo, hi = LIMITS[i]
    if hi is None:
        d = R.make_params()
        return dict(lo=[[d.lo[c][j] for j in range(3)] for c in range(3)],
                    hi=[[d.hi[c][j] for j in range(3)] for c in range(3)])
    return dict(lo=lo, hi=hi)


CASES = []
_rng = np.random.default_rng(2024)
for _i in range(14):
    CASES.append(dict(
        H=int(_rng.integers(1, 300)), W=int(_rng.integers(1, 300)),
        dtype=["u8", "u16"][_i % 2],
        chip=int(_rng.choice([1, 7, 16, 64, 100, 256, 300, 1 << 20])),
        filter=int(_rng.random() < 0.8),
        patch=(int(_rng.choice([1, 5, 16, 64, 256, 4096])), int(_rng.choice([3, 17, 100, 256]))),
        limits=_i % 3, sel=tuple(int(v) for v in _rng.permutation(3)), seed=_i))


@pytest.mark.parametrize("case", CASES, ids=[f"c{i}" for i in range(len(CASES))])
def test_random_cases_bitexact(sil, case):
    _say(f"case {case}")
    rng = np.random.default_rng(case["seed"])
    H, W = case["H"], case["W"]
    if case["dtype"] == "u8":
        s = rng.integers(0, 256, size=(3, H, W)).astype(np.uint8)
        fields = dict(dtype=R.U8)
    else:
        s = rng.integers(0, 11000, size=(3, H, W)).astype(np.uint16)
        fields = dict(dtype=R.U16)
    fields.update(chip=case["chip"], filter=case["filter"], patch_h=case["patch"][0],
                  patch_w=case["patch"][1], **_limits(case["limits"]))
    g = run_gpu(sil, s, fields, sel=case["sel"], pad=3)
    o = run_oracle(s, fields, sel=case["sel"])
    assert_same(g, o, str(case))


@pytest.mark.parametrize("refl_max", [40000, 65535, 12345])
def test_general_rescale_with_hue_saturation(sil, refl_max):
    """Full scales whose rescale constants need more than 24 bits (40000,
    65535) take the per-pixel pass's 32-bit rescale, 12345 its 24-bit one;
    each with hue/saturation-bounded limits, filter on and off, colour output."""
    rng = np.random.default_rng(refl_max)
    s = rng.integers(0, 65536, size=(3, 300, 1100)).astype(np.uint16)
    for flt in (1, 0):
        fields = dict(dtype=R.U16, refl_max=refl_max, chip=128, filter=flt, patch_h=50,
                      patch_w=70, **_limits(2))
        _say(f"case general rescale refl_max {refl_max} filter {flt}")
        assert_same(run_gpu(sil, s, fields, pad=5), run_oracle(s, fields),
                    f"refl_max {refl_max} filter {flt}")


@pytest.mark.parametrize("chip", [64, 256, 1 << 20])
def test_generated_scene_bitexact(sil, chip):
    """A seeded synthetic u16 scene (Voronoi ice field, haze and shadow), filter
    units from 64 pixels to the whole scene, all three limit sets."""
    spec = synth.SceneSpec(700, 900, 77, "u16",
                           synth.blobs_for_coverage(700, 900, 77, 1, 2, 0.10),
                           synth.blobs_for_coverage(700, 900, 77, 2, 1, 0.05))
    s = synth.generate(spec)
    for i in range(3):
        fields = dict(dtype=R.U16, chip=chip, **_limits(i))
        _say(f"case generated chip {chip} limits {i}")
        assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), f"chip {chip} limits {i}")


def test_vacuous_limits_match_the_fused_labeller(sil):
    """With the paper's limits the general path's masks are the fused path's
    labels as one-hot bits, on the GPU, for chips the fused path takes."""
    spec = synth.SceneSpec(1000, 1300, 5, "u16",
                           synth.blobs_for_coverage(1000, 1300, 5, 1, 2, 0.10),
                           synth.blobs_for_coverage(1000, 1300, 5, 2, 1, 0.05))
    s = synth.generate(spec)
    dev = _dev(s)
    for chip in (64, 200, 256):
        p = sil.Params(dtype=sil.U16, chip=chip, patch_h=100, patch_w=130)
        lab, hist = sil.label(dev, p)
        ex = sil.label_ex(dev, p)
        torch.cuda.synchronize()
        want = (torch.ones_like(lab) << lab.to(torch.int32)).to(torch.uint8)
        assert torch.equal(ex["masks"], want), chip
        assert torch.equal(ex["counts"], hist), chip


def test_rescale_every_16bit_value(sil):
    """All 65536 reflectance values through the 8-bit rescale (filter off, so
    the colour output is the rescaled band), for several full scales."""
    v = np.arange(65536, dtype=np.uint16).reshape(256, 256)
    s = np.stack([v, v[::-1], np.zeros_like(v)])
    for refl_max in (1, 3, 255, 10000, 40000, 65535):
        fields = dict(dtype=R.U16, refl_max=refl_max, filter=0)
        _say(f"case rescale refl_max {refl_max}")
        assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), f"refl_max {refl_max}")


def test_every_8bit_colour(sil):
    """All 2^24 colours in one 4096 x 4096 scene: the hue and saturation behind
    each mask boundary, for two hue/saturation-bounded limit sets, with the
    filter off and on."""
    r = np.arange(1 << 24, dtype=np.uint32)
    s = np.stack([(r & 255), (r >> 8) & 255, (r >> 16) & 255]).astype(np.uint8).reshape(3, 4096, 4096)
    for i in (1, 2):
        for flt in (0, 1):
            fields = dict(dtype=R.U8, filter=flt, **_limits(i))
            _say(f"case all colours limits {i} filter {flt}")
            assert_same(run_gpu(sil, s, fields, rgb=flt == 1),
                        run_oracle(s, fields, rgb=flt == 1), f"all colours {i} {flt}")


def test_full_tile_scene_level_bitexact(sil):
    """The 10980x10980 uint16 tile with the whole scene as one filter unit (one
    histogram of 120.6 M pixels) and with 256 x 256 chips, full-HSV limits,
    colour output: everything against the oracle."""
    spec = synth.config_tile()
    _say("case full tile: generating")
    s = synth.generate(spec)
    for chip in (1 << 20, 256):
        fields = dict(dtype=R.U16, chip=chip, **_limits(1))
        _say(f"case full tile chip {chip}: gpu")
        g = run_gpu(sil, s, fields)
        _say(f"case full tile chip {chip}: oracle")
        o = run_oracle(s, fields)
        assert_same(g, o, f"full tile chip {chip}")
        del g, o


def test_workspace_and_errors(sil):
    S = sil
    s = _dev(np.zeros((3, 40, 50), dtype=np.uint16))
    p = S.Params(dtype=S.U16)
    need = S.workspace_bytes(40, 50, p)
    assert need > 0 and S.workspace_bytes(40, 50, S.Params(dtype=S.U16, filter=0)) == 0
    with pytest.raises(ValueError):
        S.label_ex(s, p, workspace=torch.empty((need - 1,), dtype=torch.uint8, device="cuda"))
    # a misaligned 16-bit scene is refused before anything is enqueued
    flat = torch.zeros((3 * 40 * 50 * 2 + 2,), dtype=torch.uint8, device="cuda")
    masks = torch.zeros((40, 50), dtype=torch.uint8, device="cuda")
    ws0 = torch.empty((need,), dtype=torch.uint8, device="cuda")
    pc = p.to_c()
    rc = S.lib().sil_label_ex(ctypes.c_void_p(flat.data_ptr() + 1), 3,
                              (ctypes.c_int32 * 3)(0, 1, 2), 40, 50, 50, ctypes.byref(pc),
                              ctypes.c_void_p(masks.data_ptr()), 50, None, None, 0, None,
                              ctypes.c_void_p(ws0.data_ptr()), need, None)
    assert rc == S.EINVAL
    rc = S.lib().sil_label_ex(ctypes.c_void_p(flat.data_ptr()), 3,
                              (ctypes.c_int32 * 3)(0, 1, 2), 40, 50, 50, ctypes.byref(pc),
                              ctypes.c_void_p(masks.data_ptr()), 50, None, None, 0, None,
                              ctypes.c_void_p(ws0.data_ptr()), need - 1, None)
    assert rc == S.EINVAL
    assert (masks == 0).all()
    assert S.validate_ex(3, (0, 1, 2), 11586, 11586, 11586, 11586,
                         S.Params(chip=1 << 20)) == S.EUNSUPPORTED
    assert S.validate_ex(3, (0, 1, 3), 40, 50, 50, 50, p) == S.EINVAL
    # a second call on the same workspace gives the same bytes (nothing kept)
    ws = torch.empty((need,), dtype=torch.uint8, device="cuda")
    g = torch.Generator().manual_seed(3)
    sc = _dev((torch.randint(0, 11000, (3, 40, 50), generator=g).numpy()).astype(np.uint16))
    a = S.label_ex(sc, p, workspace=ws, rgb=True)
    b = S.label_ex(sc, p, workspace=ws, rgb=True)
    torch.cuda.synchronize()
    for k in ("masks", "counts", "rgb"):
        assert torch.equal(a[k], b[k]), k
