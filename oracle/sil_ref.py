"""ctypes wrapper of the CPU oracle ``libsil_ref.so`` (test infrastructure only).

Parameters are given as a plain dict of field values (the same field names as
the GPU library's parameter block), so that tests can hand one description of
a run to both sides without sharing code.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, EINVAL, EUNSUPPORTED = 0, -1, -2
U8, U16 = 1, 2
ABI_VERSION = 1


class Params(ctypes.Structure):
    _fields_ = [
        ("abi", ctypes.c_uint32),
        ("dtype", ctypes.c_uint32),
        ("refl_max", ctypes.c_uint32),
        ("lo", (ctypes.c_uint8 * 3) * 3),
        ("hi", (ctypes.c_uint8 * 3) * 3),
        ("pad", ctypes.c_uint8 * 2),
        ("filter", ctypes.c_uint32),
        ("chip", ctypes.c_uint32),
        ("clip_shift", ctypes.c_uint32),
        ("eta_num", ctypes.c_uint32),
        ("eta_den", ctypes.c_uint32),
        ("patch_h", ctypes.c_uint32),
        ("patch_w", ctypes.c_uint32),
    ]


class ChipInfo(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int32),
        ("lo", ctypes.c_uint8),
        ("hi", ctypes.c_uint8),
        ("gate", ctypes.c_uint8),
        ("stretch", ctypes.c_uint8),
        ("a1", ctypes.c_uint16),
        ("a2", ctypes.c_uint16),
    ]


CHIP_DTYPE = np.dtype([("t", "<i4"), ("lo", "u1"), ("hi", "u1"), ("gate", "u1"),
                       ("stretch", "u1"), ("a1", "<u2"), ("a2", "<u2")])
assert CHIP_DTYPE.itemsize == ctypes.sizeof(ChipInfo)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER
        L.sil_ref_params_default.argtypes = [P(Params)]
        L.sil_ref_label.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32),
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    P(Params), ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p]
        L.sil_ref_label.restype = ctypes.c_int
        L.sil_ref_validate.argtypes = [ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       P(Params)]
        L.sil_ref_validate.restype = ctypes.c_int
        L.sil_ref_hist_dims.argtypes = [ctypes.c_int32, ctypes.c_int32, P(Params),
                                        P(ctypes.c_int32), P(ctypes.c_int32)]
        L.sil_ref_hist_dims.restype = ctypes.c_int
        L.sil_ref_value_plane.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                          P(ctypes.c_int32), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_void_p]
        L.sil_ref_rescale.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.sil_ref_rescale.restype = ctypes.c_uint8
        L.sil_ref_median3x3.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p]
        L.sil_ref_chip_stats.argtypes = [ctypes.c_void_p, P(Params), P(ChipInfo)]
        L.sil_ref_stretch.argtypes = [ctypes.c_uint8, ctypes.c_uint8, ctypes.c_uint8]
        L.sil_ref_stretch.restype = ctypes.c_uint8
        L.sil_ref_class_of.argtypes = [ctypes.c_uint8, P(Params)]
        L.sil_ref_class_of.restype = ctypes.c_int
        L.sil_ref_validate_ex.argtypes = L.sil_ref_validate.argtypes
        L.sil_ref_validate_ex.restype = ctypes.c_int
        L.sil_ref_label_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32),
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       P(Params), ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p]
        L.sil_ref_label_ex.restype = ctypes.c_int
        L.sil_ref_hsv8_many.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.sil_ref_filtered_band.argtypes = [ctypes.c_uint8, ctypes.c_uint8, ctypes.c_uint8]
        L.sil_ref_filtered_band.restype = ctypes.c_uint8
        L.sil_ref_render_rgb.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
        L.sil_ref_render_rgb.restype = None
        L.sil_ref_strerror.argtypes = [ctypes.c_int]
        L.sil_ref_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"sil_ref error {code}: {lib().sil_ref_strerror(code).decode()}")
        self.code = code


def make_params(**fields) -> Params:
    """Paper defaults, overridden by ``fields`` (``lo``/``hi`` as 3x3 nested lists)."""
    p = Params()
    lib().sil_ref_params_default(ctypes.byref(p))
    for k, v in fields.items():
        if k in ("lo", "hi"):
            arr = getattr(p, k)
            for c in range(3):
                for j in range(3):
                    arr[c][j] = int(v[c][j])
        else:
            setattr(p, k, int(v))
    return p


def _sel_array(sel):
    return (ctypes.c_int32 * 3)(*[int(s) for s in sel])


def hist_dims(H, W, params):
    ny, nx = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().sil_ref_hist_dims(H, W, ctypes.byref(params), ctypes.byref(ny),
                                 ctypes.byref(nx))
    if rc:
        raise OracleError(rc)
    return ny.value, nx.value


def validate(nbands, sel, H, W, pitch, label_pitch, params):
    return lib().sil_ref_validate(nbands, _sel_array(sel), H, W, pitch, label_pitch,
                                  ctypes.byref(params))


def label(scene: np.ndarray, params: Params = None, sel=(0, 1, 2), W: int = None,
          want_chips: bool = False):
    """Run the oracle on ``scene`` of shape [nbands, H, pitch] (uint8/uint16).

    ``W`` defaults to the pitch.  Returns (labels [H, W] uint8, hist [ny, nx, 3]
    uint32[, chips [ncy, ncx] structured]).
    """
    if params is None:
        params = make_params()
    scene = np.ascontiguousarray(scene)
    nb, H, pitch = scene.shape
    W = pitch if W is None else W
    want = U8 if scene.dtype == np.uint8 else U16
    if scene.dtype not in (np.uint8, np.uint16) or params.dtype != want:
        raise ValueError("scene dtype does not match params.dtype")
    ny, nx = hist_dims(H, W, params)
    labels = np.full((H, W), 0xEE, dtype=np.uint8)
    hist = np.zeros((ny, nx, 3), dtype=np.uint32)
    chips = None
    chips_ptr = None
    if want_chips:
        C = params.chip
        chips = np.zeros(((H + C - 1) // C, (W + C - 1) // C), dtype=CHIP_DTYPE)
        chips_ptr = chips.ctypes.data
    rc = lib().sil_ref_label(scene.ctypes.data, nb, _sel_array(sel), H, W, pitch,
                             ctypes.byref(params), labels.ctypes.data, W,
                             hist.ctypes.data, chips_ptr)
    if rc:
        raise OracleError(rc)
    return (labels, hist, chips) if want_chips else (labels, hist)


# ---- single steps (unit pins) ------------------------------------------------

def value_plane(scene: np.ndarray, dtype=None, refl_max=10000, sel=(0, 1, 2)):
    scene = np.ascontiguousarray(scene)
    nb, H, W = scene.shape
    dt = U8 if scene.dtype == np.uint8 else U16
    V = np.zeros((H, W), dtype=np.uint8)
    lib().sil_ref_value_plane(scene.ctypes.data, nb, _sel_array(sel), H, W, W, dt,
                              refl_max, V.ctypes.data)
    return V


def rescale(x: int, refl_max: int = 10000) -> int:
    return int(lib().sil_ref_rescale(x, refl_max))


def median3x3(V: np.ndarray) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.uint8)
    H, W = V.shape
    out = np.zeros_like(V)
    lib().sil_ref_median3x3(V.ctypes.data, H, W, out.ctypes.data)
    return out


def chip_stats(h, params: Params = None) -> dict:
    if params is None:
        params = make_params()
    h = np.ascontiguousarray(h, dtype=np.uint32)
    assert h.shape == (256,)
    info = ChipInfo()
    lib().sil_ref_chip_stats(h.ctypes.data, ctypes.byref(params), ctypes.byref(info))
    return {f: getattr(info, f) for f, _ in ChipInfo._fields_}


def stretch(m: int, lo: int, hi: int) -> int:
    return int(lib().sil_ref_stretch(m, lo, hi))


def class_of(vc: int, params: Params = None) -> int:
    if params is None:
        params = make_params()
    return int(lib().sil_ref_class_of(vc, ctypes.byref(params)))


# ---- the general labeller (variants) -----------------------------------------

def validate_ex(nbands, sel, H, W, pitch, mask_pitch, params):
    return lib().sil_ref_validate_ex(nbands, _sel_array(sel), H, W, pitch, mask_pitch,
                                     ctypes.byref(params))


def label_ex(scene: np.ndarray, params: Params = None, sel=(0, 1, 2), W: int = None,
             want_rgb: bool = False, want_chips: bool = False):
    """General labeller on ``scene`` [nbands, H, pitch]: returns a dict with
    ``masks`` [H, W] (bit c = mask c), ``counts`` [ny, nx, 3], and, when asked,
    ``rgb`` [3, H, W] (the filtered bands in ``sel`` order) and ``chips``."""
    if params is None:
        params = make_params()
    scene = np.ascontiguousarray(scene)
    nb, H, pitch = scene.shape
    W = pitch if W is None else W
    want = U8 if scene.dtype == np.uint8 else U16
    if scene.dtype not in (np.uint8, np.uint16) or params.dtype != want:
        raise ValueError("scene dtype does not match params.dtype")
    ny, nx = hist_dims(H, W, params)
    masks = np.full((H, W), 0xEE, dtype=np.uint8)
    counts = np.zeros((ny, nx, 3), dtype=np.uint32)
    rgb = np.full((3, H, W), 0xEE, dtype=np.uint8) if want_rgb else None
    chips = None
    if want_chips:
        C = params.chip
        chips = np.zeros(((H + C - 1) // C, (W + C - 1) // C), dtype=CHIP_DTYPE)
    rc = lib().sil_ref_label_ex(scene.ctypes.data, nb, _sel_array(sel), H, W, pitch,
                                ctypes.byref(params), masks.ctypes.data, W, counts.ctypes.data,
                                rgb.ctypes.data if want_rgb else None, W,
                                chips.ctypes.data if want_chips else None)
    if rc:
        raise OracleError(rc)
    out = {"masks": masks, "counts": counts}
    if want_rgb:
        out["rgb"] = rgb
    if want_chips:
        out["chips"] = chips
    return out


def hsv8(rgb: np.ndarray) -> np.ndarray:
    """OpenCV-convention 8-bit HSV of [..., 3] (r, g, b) uint8 triples."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    out = np.zeros_like(rgb)
    lib().sil_ref_hsv8_many(rgb.ctypes.data, rgb.size // 3, out.ctypes.data)
    return out


def filtered_band(c: int, v: int, vc: int) -> int:
    return int(lib().sil_ref_filtered_band(c, v, vc))


def render_rgb(labels: np.ndarray, W: int = None) -> np.ndarray:
    """Colour image [H, W, 3] (R, G, B) of a class-id plane [H, >=W] u8
    (sections III-A/III-B colours: water green, thin ice blue, thick ice red,
    other ids black)."""
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    H, pitch = lab.shape
    W = pitch if W is None else W
    out = np.zeros((H, W, 3), dtype=np.uint8)
    lib().sil_ref_render_rgb(lab.ctypes.data, H, W, pitch, out.ctypes.data, 3 * W)
    return out
