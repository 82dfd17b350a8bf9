"""GPU parity: libsil's kernels against the CPU oracle, bit for bit.

Labels and per-patch counts are integer results, so the bar is exact
equality; per-chip statistics (Otsu split, gate, truncation levels, class
boundaries) are compared too.  Every call goes through the C ABI via the
ctypes binding.
"""
import hashlib
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


def _to_dev(scene_np, offset=0):
    """Upload [nb, H, pitch]; with offset > 0 the tensor starts `offset`
    elements into a larger buffer (misaligned base)."""
    t = torch.from_numpy(scene_np.view(np.int16) if scene_np.dtype == np.uint16 else scene_np)
    if offset:
        flat = torch.empty(scene_np.size + offset, dtype=t.dtype)
        flat[offset:] = t.reshape(-1)
        dev = flat.cuda()[offset:].view(scene_np.shape)
    else:
        dev = t.cuda()
    return dev


def run_gpu(S, scene_np, fields, W=None, sel=(0, 1, 2), offset=0, label_pad=0, label_off=0):
    H = scene_np.shape[1]
    W = scene_np.shape[2] if W is None else W
    dev = _to_dev(scene_np, offset)
    p = S.Params(**fields)
    lp = W + label_pad
    lbuf = torch.full((H * lp + label_off,), 0xEE, dtype=torch.uint8, device="cuda")
    labels = lbuf[label_off:].view(H, lp)
    ny, nx = S.hist_dims(H, W, p)
    hist = torch.full((ny, nx, 3), -7, dtype=torch.int32, device="cuda")
    out = S.label(dev, p, sel=sel, W=W, labels=labels, hist=hist, chips=fields.get("filter", 1) == 1)
    torch.cuda.synchronize()
    lab = labels.cpu().numpy()
    if label_pad:
        assert (lab[:, W:] == 0xEE).all(), "bytes beyond W were written"
    chips = S.decode_chip_info(out[2].cpu().numpy()) if len(out) == 3 else None
    return lab[:, :W], hist.cpu().numpy().astype(np.uint32), chips


def run_oracle(scene_np, fields, W=None, sel=(0, 1, 2)):
    p = R.make_params(**fields)
    return R.label(scene_np, p, sel=sel, W=W, want_chips=fields.get("filter", 1) == 1)


def assert_same(g, o, what=""):
    gl, gh, gc = g
    ol, oh = o[0], o[1]
    if not (gl == ol).all():
        bad = np.argwhere(gl != ol)
        y, x = bad[0]
        raise AssertionError(f"{what}: {len(bad)} label mismatches, first at {(y, x)}: "
                             f"gpu {gl[y, x]} oracle {ol[y, x]}")
    assert (gh == oh).all(), f"{what}: hist mismatch"
    if gc is not None and len(o) == 3:
        oc = o[2]
        for f in ("t", "lo", "hi", "gate", "stretch", "a1", "a2"):
            assert (gc[f] == oc[f]).all(), f"{what}: chip field {f} differs"


def test_small_scene_bitexact(sil):
    """512x512 uint8 scene, one haze and one shadow blob, chip 256, patch 64."""
    spec = synth.config_small()
    s = synth.generate(spec)
    fields = dict(dtype=R.U8, patch_h=64, patch_w=64)
    _say("case small u8 512x512")
    assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), "small")
    f0 = dict(fields, filter=0)
    assert_same(run_gpu(sil, s, f0), run_oracle(s, f0), "small filter0")


RNG_CASES = [
    # H, W, dtype, chip, ph, pw, filter, pitch_pad, offset, label_pad, label_off
    (1, 1, "u8", 256, 256, 256, 1, 0, 0, 0, 0),
    (1, 1, "u16", 1, 1, 1, 1, 0, 0, 0, 0),
    (2, 3, "u8", 256, 1, 1, 1, 0, 0, 3, 1),
    (3, 300, "u16", 256, 3, 300, 1, 1, 1, 0, 0),
    (300, 3, "u8", 7, 300, 3, 1, 0, 0, 1, 0),
    (37, 53, "u8", 1, 3, 3, 1, 0, 0, 0, 0),
    (37, 53, "u16", 7, 64, 64, 1, 0, 0, 0, 0),
    (255, 257, "u8", 256, 256, 256, 1, 0, 0, 0, 0),
    (256, 256, "u16", 256, 256, 256, 1, 0, 0, 0, 0),
    (257, 255, "u16", 256, 64, 64, 1, 0, 0, 0, 0),
    (513, 1000, "u8", 64, 64, 64, 1, 0, 0, 0, 0),
    (513, 1000, "u16", 64, 256, 256, 1, 4, 0, 5, 2),
    (700, 901, "u16", 256, 300, 300, 1, 0, 0, 0, 0),
    (700, 901, "u16", 256, 512, 256, 1, 0, 0, 0, 0),
    (700, 901, "u8", 256, 1, 1, 1, 0, 0, 0, 0),
    (700, 901, "u8", 256, 3, 3, 1, 0, 1, 0, 0),
    (1000, 1300, "u16", 256, 256, 256, 1, 0, 0, 0, 0),
    (1000, 1300, "u16", 256, 256, 256, 1, 3, 1, 0, 0),
    (1000, 1300, "u16", 256, 100, 37, 0, 0, 0, 0, 0),
    (1000, 1300, "u8", 256, 64, 64, 0, 1, 3, 2, 1),
    (1000, 1300, "u16", 256, 256, 256, 0, 0, 0, 0, 0),
    (999, 1001, "u16", 64, 128, 192, 1, 0, 0, 0, 0),
    (1031, 517, "u8", 128, 256, 256, 1, 0, 0, 0, 0),
    (260, 4100, "u16", 256, 256, 256, 1, 0, 0, 0, 0),
    # aligned rows (vector loads) with widths that end inside a lane's 4
    # columns: the right-edge chips clamp the loaded columns to W-1
    (300, 901, "u16", 256, 256, 256, 1, 3, 0, 0, 0),
    (513, 1003, "u16", 256, 256, 256, 1, 1, 0, 0, 0),
    (257, 1022, "u8", 256, 256, 256, 1, 2, 0, 0, 0),
    (100, 130, "u16", 256, 256, 256, 1, 2, 0, 0, 0),
    (37, 53, "u8", 256, 7, 9, 1, 3, 0, 0, 0),
    (333, 777, "u16", 64, 64, 64, 1, 3, 0, 0, 0),
    (70, 4, "u16", 256, 256, 256, 1, 0, 0, 0, 0),
    (90, 5, "u8", 3, 256, 256, 1, 3, 0, 0, 0),
    # filter off with patches that tile-align: tile totals, stored or added
    (700, 1300, "u16", 256, 512, 768, 0, 3, 0, 0, 0),
    (600, 1100, "u8", 256, 256, 512, 0, 0, 0, 0, 0),
    (513, 1001, "u16", 256, 256, 256, 0, 3, 0, 0, 0),
    (300, 299, "u16", 256, 256, 256, 0, 1, 0, 3, 1),
]


def _rand_scene(rng, H, W, dtype, pitch):
    kind = int(rng.integers(0, 3))
    if kind == 0:
        s8 = rng.integers(0, 256, (3, H, W)).astype(np.uint8)
    elif kind == 1:
        base = np.where(rng.random((H, W)) < 0.4, 45, np.where(rng.random((H, W)) < 0.5, 140, 215))
        s8 = np.clip(base[None] + rng.normal(0, 10, (3, H, W)), 0, 255).astype(np.uint8)
    else:
        spec = synth.SceneSpec(H, W, int(rng.integers(1 << 30)), "u8",
                               [synth.Blob(H // 3, W // 2, max(H, W) / 4)],
                               [synth.Blob(2 * H // 3, W // 3, max(H, W) / 5)])
        s8 = synth.generate_u8(spec)
    if dtype == "u16":
        s = synth.to_u16(s8, seed=int(rng.integers(1 << 30)), pitch=pitch)
        if rng.random() < 0.3:  # saturated reflectance above full scale
            s[0, : H // 2, : W // 3] = 65535
    else:
        s = np.zeros((3, H, pitch), dtype=np.uint8)
        s[:, :, :W] = s8
    return s


@pytest.mark.parametrize("case", RNG_CASES, ids=[f"c{i}" for i in range(len(RNG_CASES))])
def test_random_shapes_bitexact(sil, case):
    H, W, dtype, chip, ph, pw, filt, pitch_pad, off, lpad, loff = case
    rng = np.random.default_rng(hash(case) & 0xFFFFFFFF)
    s = _rand_scene(rng, H, W, dtype, W + pitch_pad)
    fields = dict(dtype=R.U16 if dtype == "u16" else R.U8, chip=chip, patch_h=ph, patch_w=pw,
                  filter=filt)
    _say(f"case {case}")
    g = run_gpu(sil, s, fields, W=W, offset=off, label_pad=lpad, label_off=loff)
    o = run_oracle(s, fields, W=W)
    assert_same(g, o, str(case))


def _adversarial():
    out = []
    H, W = 300, 520
    out.append(("zeros", np.zeros((3, H, W), np.uint8)))
    out.append(("max", np.full((3, H, W), 255, np.uint8)))
    yy, xx = np.mgrid[0:H, 0:W]
    for a, b in [(30, 31), (204, 205), (0, 255), (31, 204)]:
        cb = np.where((yy + xx) % 2 == 0, a, b).astype(np.uint8)
        out.append((f"checker{a}-{b}", np.stack([cb, cb, cb])))
    blocks = np.where(((yy // 7) + (xx // 5)) % 2 == 0, 100, 101).astype(np.uint8)
    out.append(("otsu-tie spikes", np.stack([blocks, blocks // 2, blocks // 3])))
    const_chips = ((yy // 64) * 37 + (xx // 64) * 11) % 256
    out.append(("constant chips", np.stack([const_chips.astype(np.uint8)] * 3)))
    ramp = (xx % 256).astype(np.uint8)
    out.append(("uniform ramp", np.stack([ramp, ramp, ramp])))
    # three horizontal bands per 64-row period with counts n, 2n, n: Otsu's
    # ratio ties exactly between a split below and above the middle band (the
    # smallest t wins), and the bands survive the median
    band = yy % 64
    lvl = ((yy // 64) * 29 + (xx // 64) * 7) % 150
    spikes = np.where(band < 16, lvl, np.where(band < 48, lvl + 40, lvl + 80)).astype(np.uint8)
    out.append(("symmetric three spikes", np.stack([spikes, spikes // 2, spikes // 3])))
    return out


@pytest.mark.parametrize("chip", [64, 256])
def test_adversarial_scenes(sil, chip):
    for name, s in _adversarial():
        for fields in (dict(chip=chip, patch_h=64, patch_w=64), dict(chip=chip, filter=0),
                       dict(chip=chip, patch_h=chip, patch_w=chip)):
            _say(f"case adversarial {name} {fields}")
            assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), f"{name} {fields}")


def test_permuted_and_extra_bands(sil):
    rng = np.random.default_rng(4)
    s = rng.integers(0, 256, (5, 301, 299)).astype(np.uint8)
    fields = dict(chip=128, patch_h=50, patch_w=50)
    for sel in [(4, 2, 0), (1, 3, 2)]:
        _say(f"case bands {sel}")
        assert_same(run_gpu(sil, s, fields, sel=sel), run_oracle(s, fields, sel=sel), str(sel))


def test_refl_max_variants(sil):
    rng = np.random.default_rng(12)
    s = rng.integers(0, 65536, (3, 200, 333)).astype(np.uint16)
    for rm in (1, 255, 4095, 10000, 16384, 40000, 65535):
        fields = dict(dtype=R.U16, refl_max=rm, chip=128, patch_h=128, patch_w=128)
        _say(f"case refl_max {rm}")
        assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), f"refl_max {rm}")
        f0 = dict(fields, filter=0)
        assert_same(run_gpu(sil, s, f0), run_oracle(s, f0), f"refl_max {rm} filter0")


def test_param_variants(sil):
    spec = synth.config_small()
    s = synth.generate(spec)
    for fields in (dict(clip_shift=1), dict(clip_shift=31), dict(eta_num=0, eta_den=1),
                   dict(eta_num=1, eta_den=1), dict(eta_num=9, eta_den=10),
                   dict(lo=[[0, 0, 0], [0, 0, 100], [0, 0, 101]],
                        hi=[[185, 255, 99], [185, 255, 100], [185, 255, 255]]),
                   dict(lo=[[0, 0, 0], [0, 0, 1], [0, 0, 150]],
                        hi=[[185, 255, 149], [185, 255, 0], [185, 255, 255]])):
        _say(f"case params {fields}")
        assert_same(run_gpu(sil, s, fields), run_oracle(s, fields), str(fields))


def test_full_tile_bitexact(sil):
    """The 10980x10980 uint16 tile (3 bands, 10 % haze / 5 % shadow), chip and
    patch 256, in the launch configuration the benchmark times; every label,
    count and chip statistic against the oracle, with the filter and without
    it (thresholds only)."""
    spec = synth.config_tile()
    _say("case full tile: generating")
    s = synth.generate(spec)
    fields = dict(dtype=R.U16)
    # label rows 11008 bytes apart (128-byte aligned), as the benchmark allocates them
    _say("case full tile: gpu pitch 10980, label pitch 11008")
    g = run_gpu(sil, s, fields, label_pad=11008 - 10980)
    _say("case full tile: oracle")
    o = run_oracle(s, fields)
    assert_same(g, o, "full tile")
    del o
    # thresholds only (filter 0), as the benchmark's thresholds-only mode runs it
    f0 = dict(fields, filter=0)
    _say("case full tile: filter 0, gpu and oracle")
    assert_same(run_gpu(sil, s, f0, label_pad=11008 - 10980), run_oracle(s, f0), "full tile filter0")
    # the same scene with padded (16-byte aligned) rows and unpadded label rows
    # gives the same result
    spec.pitch = 10984
    sp = synth.generate(spec)
    _say("case full tile: gpu pitch 10984, label pitch 10980")
    g2 = run_gpu(sil, sp, fields, W=10980)
    assert (g2[0] == g[0]).all() and (g2[1] == g[1]).all()


def test_repeatable_and_stream_ordered(sil):
    """Repeated launches on a side stream give identical bytes (no races)."""
    spec = synth.config_small()
    s = synth.generate(spec)
    dev = _to_dev(np.tile(s, (1, 4, 4)))
    p = sil.Params(patch_h=100, patch_w=100)
    side = torch.cuda.Stream()
    digests = set()
    with torch.cuda.stream(side):
        for _ in range(8):
            lab, hist = sil.label(dev, p, stream=side)
            side.synchronize()
            digests.add(hashlib.sha256(lab.cpu().numpy().tobytes()
                                       + hist.cpu().numpy().tobytes()).hexdigest())
    assert len(digests) == 1


def test_errors_raise_before_launch(sil):
    s = torch.zeros((3, 10, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(sil.SilError) as e:
        sil.label(s, sil.Params(chip=0))
    assert e.value.code == sil.EINVAL
    with pytest.raises(sil.SilError) as e:
        sil.label(s, sil.Params(chip=300))
    assert e.value.code == sil.EUNSUPPORTED
    with pytest.raises(ValueError):
        sil.label(s, sil.Params(dtype=sil.U16))


def test_batched_launches_equal_single_scene(sil):
    """Chip ranges of several scenes labelled by sil_label_batch, split at
    arbitrary chip boundaries over several launches, give exactly the
    single-scene result (and so the oracle's)."""
    rng = np.random.default_rng(21)
    p = sil.Params(dtype=sil.U16)
    scenes, refs, outs = [], [], []
    for (H, W) in [(512, 512), (300, 1100), (1031, 777), (2048, 2048), (64, 64), (257, 513)]:
        s16 = _rand_scene(rng, H, W, "u16", W)
        dev = _to_dev(s16)
        lab, hist = sil.label(dev, p)
        ny, nx = hist.shape[:2]
        refs.append((lab.clone(), hist.clone()))
        outs.append((torch.full((H, W), 0xEE, dtype=torch.uint8, device="cuda"),
                     torch.full((ny, nx, 3), -1, dtype=torch.int32, device="cuda")))
        scenes.append(dev)
    torch.cuda.synchronize()
    # label every scene's chips in uneven pieces, interleaving scenes per launch
    pending = [[0, sil.chip_count(s.shape[1], s.shape[2], p)] for s in scenes]
    launches = 0
    while any(b < n for b, n in pending):
        jobs = []
        for i, (b, n) in enumerate(pending):
            if b < n and rng.random() < 0.8:
                cnt = int(min(n - b, rng.integers(1, 40)))
                jobs.append(sil.Job(scenes[i], outs[i][0], outs[i][1], b, cnt))
                pending[i][0] += cnt
        if jobs:
            _say(f"case batch launch {launches}: {[(j.chip_begin, j.chip_count) for j in jobs]}")
            sil.label_batch(jobs, p)
            launches += 1
    torch.cuda.synchronize()
    assert launches > 3
    for (rl, rh), (ol, oh) in zip(refs, outs):
        assert torch.equal(rl, ol) and torch.equal(rh, oh)
    # and the scenes agree with the oracle
    s_np = scenes[2].cpu().numpy().view(np.uint16)
    ol, oh = R.label(s_np, R.make_params(dtype=R.U16))
    assert (outs[2][0].cpu().numpy() == ol).all() and (outs[2][1].cpu().numpy() == oh).all()


def test_batch_rejects_bad_jobs(sil):
    s = torch.zeros((3, 300, 300), dtype=torch.int16, device="cuda")
    lab = torch.empty((300, 300), dtype=torch.uint8, device="cuda")
    hist = torch.empty((2, 2, 3), dtype=torch.int32, device="cuda")
    p = sil.Params(dtype=sil.U16)
    with pytest.raises(sil.SilError) as e:
        sil.label_batch([sil.Job(s, lab, hist, 3, 2)], p)  # chips 3..4 of 4
    assert e.value.code == sil.EINVAL
    with pytest.raises(sil.SilError) as e:
        sil.label_batch([sil.Job(s, lab, hist, 0, 1)], sil.Params(dtype=sil.U16, patch_h=64,
                                                                   patch_w=64))
    assert e.value.code == sil.EUNSUPPORTED
