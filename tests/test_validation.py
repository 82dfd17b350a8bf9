"""Argument validation of the C ABI (no GPU): the GPU library's host-side
validator and the oracle's, written separately, follow one contract."""
import ctypes
import os
import re
import subprocess

import pytest

from oracle import sil_ref as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GPU_LIB = os.path.join(ROOT, "paper_2403_13135_amd", "libsil.so")

needs_lib = pytest.mark.skipif(not os.path.exists(GPU_LIB),
                               reason="libsil.so not built (run __graft_entry__.build())")

PAPER = dict(lo=[[0, 0, 0], [0, 0, 31], [0, 0, 205]], hi=[[185, 255, 30], [185, 255, 204],
                                                         [185, 255, 255]])

# (description, field overrides, call overrides, expected code)
CASES = [
    ("defaults", {}, {}, 0),
    ("u16 defaults", dict(dtype=2), {}, 0),
    ("filter off, huge chip", dict(filter=0, chip=100000), {}, 0),
    ("bad abi", dict(abi=2), {}, -1),
    ("bad dtype", dict(dtype=3), {}, -1),
    ("refl_max 0", dict(dtype=2, refl_max=0), {}, -1),
    ("filter 2", dict(filter=2), {}, -1),
    ("chip 0", dict(chip=0), {}, -1),
    ("clip_shift 0", dict(clip_shift=0), {}, -1),
    ("clip_shift 32", dict(clip_shift=32), {}, -1),
    ("eta den 0", dict(eta_den=0), {}, -1),
    ("eta num > den", dict(eta_num=5, eta_den=4), {}, -1),
    ("patch_h 0", dict(patch_h=0), {}, -1),
    ("patch_w 0", dict(patch_w=0), {}, -1),
    ("H 0", {}, dict(H=0), -1),
    ("W 0", {}, dict(W=0), -1),
    ("pitch < W", {}, dict(pitch=9), -1),
    ("label pitch < W", {}, dict(label_pitch=9), -1),
    ("nbands 0", {}, dict(nbands=0), -1),
    ("sel out of range", {}, dict(sel=(0, 1, 3)), -1),
    ("sel negative", {}, dict(sel=(-1, 1, 2)), -1),
    ("overlapping V ranges", dict(lo=[[0, 0, 0], [0, 0, 30], [0, 0, 205]], hi=PAPER["hi"]), {}, -1),
    ("gap in V ranges", dict(lo=[[0, 0, 0], [0, 0, 32], [0, 0, 205]], hi=PAPER["hi"]), {}, -2),
    ("hue limit below 179", dict(lo=PAPER["lo"], hi=[[170, 255, 30], [185, 255, 204],
                                                      [185, 255, 255]]), {}, -2),
    ("saturation limit", dict(lo=[[0, 5, 0], [0, 0, 31], [0, 0, 205]], hi=PAPER["hi"]), {}, -2),
    ("chip 257 with filter", dict(chip=257), {}, -2),
    ("empty thin range ok", dict(lo=[[0, 0, 0], [0, 0, 1], [0, 0, 101]],
                                 hi=[[185, 255, 100], [185, 255, 0], [185, 255, 255]]), {}, 0),
]

GPU_ONLY = [
    ("V order not water<=thin<=thick", dict(lo=[[0, 0, 205], [0, 0, 31], [0, 0, 0]],
                                            hi=[[185, 255, 255], [185, 255, 204],
                                                [185, 255, 30]]), {}, -2, 0),
    # the chip walk's 34 rows are addressed with 32-bit offsets
    ("u16 rows of 2^32/34 bytes", dict(dtype=2), dict(H=1, W=10, pitch=(1 << 32) // 68 + 1,
                                                       label_pitch=10), -2, 0),
    ("u16 rows just below", dict(dtype=2), dict(H=1, W=10, pitch=(1 << 32) // 68 - 1,
                                                 label_pitch=10), 0, 0),
    ("filter off, long rows", dict(dtype=2, filter=0), dict(H=1, W=10, pitch=(1 << 32) // 68 + 1,
                                                             label_pitch=10), 0, 0),
]


def _call(validate, params, call):
    c = dict(nbands=3, sel=(0, 1, 2), H=10, W=10, pitch=10, label_pitch=10)
    c.update(call)
    return validate(c["nbands"], c["sel"], c["H"], c["W"], c["pitch"], c["label_pitch"], params)


@pytest.mark.parametrize("name,fields,call,code", CASES, ids=[c[0] for c in CASES])
def test_oracle_validation(name, fields, call, code):
    assert _call(R.validate, R.make_params(**fields), call) == code


@needs_lib
@pytest.mark.parametrize("name,fields,call,code", CASES, ids=[c[0] for c in CASES])
def test_gpu_lib_validation(name, fields, call, code):
    from paper_2403_13135_amd import sil
    p = sil.Params()
    raw_abi = fields.pop("abi", None) if "abi" in fields else None
    for k, v in fields.items():
        setattr(p, k, v)
    if raw_abi is None:
        assert _call(sil.validate, p, call) == code
    else:
        cp = p.to_c()
        cp.abi = raw_abi
        s = (ctypes.c_int32 * 3)(0, 1, 2)
        assert sil.lib().sil_validate(3, s, 10, 10, 10, 10, ctypes.byref(cp)) == code


@needs_lib
@pytest.mark.parametrize("name,fields,call,gpu_code,oracle_code", GPU_ONLY,
                         ids=[c[0] for c in GPU_ONLY])
def test_gpu_only_restrictions(name, fields, call, gpu_code, oracle_code):
    from paper_2403_13135_amd import sil
    p = sil.Params()
    for k, v in fields.items():
        setattr(p, k, v)
    assert _call(sil.validate, p, call) == gpu_code
    assert _call(R.validate, R.make_params(**fields), call) == oracle_code


@needs_lib
def test_library_exports_every_declared_symbol():
    """Every function declared in include/*.h is exported by libsil.so."""
    decls = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            decls |= set(re.findall(r"\b(sil_[a-z0-9_]+)\s*\(", text))
    assert decls, "no declarations found"
    out = subprocess.run(["nm", "-D", "--defined-only", GPU_LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    assert decls <= exported, decls - exported
    lib = ctypes.CDLL(GPU_LIB)
    for d in decls:
        assert hasattr(lib, d)


@needs_lib
def test_hist_dims_and_defaults():
    from paper_2403_13135_amd import sil
    assert sil.hist_dims(10980, 10980, sil.Params()) == (43, 43)
    assert sil.hist_dims(512, 512, sil.Params(patch_h=64, patch_w=64)) == (8, 8)
    assert sil.hist_dims(7, 300, sil.Params(patch_h=3, patch_w=300)) == (3, 1)
    cp = sil.Params().to_c()
    op = R.make_params()
    assert bytes(cp) == bytes(op)  # same defaults, same layout
    assert sil.strerror(-2) and sil.strerror(0)


# The general labeller's contract: any H/S/V limits and any chip side, up to
# chips of 2^27 pixels; every other check as the fused labeller's.
EX_CASES = [
    ("defaults", {}, {}, 0),
    ("overlapping V ranges", dict(lo=[[0, 0, 0], [0, 0, 30], [0, 0, 205]], hi=PAPER["hi"]), {}, 0),
    ("gap in V ranges", dict(lo=[[0, 0, 0], [0, 0, 32], [0, 0, 205]], hi=PAPER["hi"]), {}, 0),
    ("hue and saturation limits", dict(lo=[[0, 40, 0], [20, 0, 60], [100, 10, 150]],
                                       hi=[[90, 255, 120], [179, 200, 220], [170, 255, 255]]),
     {}, 0),
    ("lo above hi", dict(lo=[[200, 0, 0], [0, 0, 31], [0, 0, 205]], hi=PAPER["hi"]), {}, 0),
    ("chip 257 with filter", dict(chip=257), {}, 0),
    ("scene-level chip", dict(chip=1 << 30), dict(H=11585, W=11585, pitch=11585,
                                                  label_pitch=11585), 0),
    ("chip beyond 2^27 px", dict(chip=1 << 30), dict(H=11586, W=11586, pitch=11586,
                                                     label_pitch=11586), -2),
    ("tall chip beyond 2^27 px", dict(chip=20000), dict(H=20000, W=7000, pitch=7000,
                                                        label_pitch=7000), -2),
    ("filter off, any chip", dict(filter=0, chip=1 << 30), dict(H=11586, W=11586, pitch=11586,
                                                                label_pitch=11586), 0),
    ("refl_max above 16 bits", dict(dtype=2, refl_max=70000), {}, -2),
    ("bad dtype", dict(dtype=3), {}, -1),
    ("chip 0", dict(chip=0), {}, -1),
    ("clip_shift 32", dict(clip_shift=32), {}, -1),
    ("eta num > den", dict(eta_num=5, eta_den=4), {}, -1),
    ("patch_w 0", dict(patch_w=0), {}, -1),
    ("mask pitch < W", {}, dict(label_pitch=9), -1),
    ("pitch < W", {}, dict(pitch=9), -1),
    ("sel out of range", {}, dict(sel=(0, 1, 3)), -1),
]


@pytest.mark.parametrize("name,fields,call,code", EX_CASES, ids=[c[0] for c in EX_CASES])
def test_oracle_validation_ex(name, fields, call, code):
    assert _call(R.validate_ex, R.make_params(**fields), call) == code


@needs_lib
@pytest.mark.parametrize("name,fields,call,code", EX_CASES, ids=[c[0] for c in EX_CASES])
def test_gpu_lib_validation_ex(name, fields, call, code):
    from paper_2403_13135_amd import sil
    p = sil.Params()
    for k, v in fields.items():
        setattr(p, k, v)
    assert _call(sil.validate_ex, p, call) == code


@needs_lib
def test_workspace_sizes():
    from paper_2403_13135_amd import sil
    assert sil.workspace_bytes(10980, 10980, sil.Params(filter=0)) == 0
    n = sil.workspace_bytes(10980, 10980, sil.Params(chip=1 << 20))
    assert n >= 10980 * 10980 + 256 * 4 + 256
    m = sil.workspace_bytes(10980, 10980, sil.Params())
    assert m >= 10980 * 10980 + 43 * 43 * 256 * 5



@needs_lib
def test_unet_bn_channel_rule():
    """Batch-norm entry points take channel counts that divide 256 and refuse
    others before touching any buffer (the element-wise kernels keep one
    group of 8 channels per thread across their grid stride)."""
    lib = ctypes.CDLL(GPU_LIB)
    vp, f32, i64, i32 = ctypes.c_void_p, ctypes.c_float, ctypes.c_int64, ctypes.c_int32
    lib.sil_unet_bn_relu.argtypes = [vp, vp, vp, vp, f32, i64, vp, vp, i64, i32, vp]
    lib.sil_unet_affine_relu.argtypes = [vp, vp, vp, vp, i64, i32, vp]
    dummy = ctypes.c_void_p(16)
    for C in (24, 40, 512, 4, 0):
        assert lib.sil_unet_bn_relu(dummy, dummy, dummy, dummy, 1e-5, 10, dummy, dummy, 10, C,
                                    None) == -1, C
        assert lib.sil_unet_affine_relu(dummy, dummy, dummy, dummy, 10, C, None) == -1, C
