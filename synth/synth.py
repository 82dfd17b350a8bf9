"""ctypes driver of ``synth.c`` plus the host-built tables it needs."""
import ctypes
import math
import os
import statistics
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsynth.so")

CLASS_MEANS = (40, 140, 220)  # open water, thin ice, thick ice (8-bit brightness)
NOISE_SIGMA = 8
CELL = 64


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
           os.path.join(HERE, "synth.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Blob(ctypes.Structure):
    _fields_ = [("cy", ctypes.c_int64), ("cx", ctypes.c_int64), ("s2", ctypes.c_int64)]


class _Cfg(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("cell", ctypes.c_int32),
                ("mean", ctypes.c_int32 * 3), ("noise", ctypes.POINTER(ctypes.c_int8)),
                ("gtab", ctypes.POINTER(ctypes.c_uint32)), ("gtab_len", ctypes.c_int32),
                ("haze", ctypes.POINTER(_Blob)), ("n_haze", ctypes.c_int32),
                ("shadow", ctypes.POINTER(_Blob)), ("n_shadow", ctypes.c_int32)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.synth_scene_u8.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.synth_u8_to_u16.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.synth_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.synth_hash.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _noise_table() -> np.ndarray:
    """round(sigma * Phi^-1((i + 0.5) / 4096)), i.e. N(0, sigma^2) by inversion."""
    nd = statistics.NormalDist()
    return np.array([round(NOISE_SIGMA * nd.inv_cdf((i + 0.5) / 4096)) for i in range(4096)],
                    dtype=np.int8)


def _gauss_table() -> np.ndarray:
    """Q16 exp(-i/128) for i = floor(64 d^2 / sigma^2), until it rounds to 0."""
    n = int(math.ceil(128 * math.log(2 * 65536))) + 1
    return np.array([round(65536 * math.exp(-i / 128.0)) for i in range(n)], dtype=np.uint32)


_TABLES = {}


def _tables():
    if not _TABLES:
        _TABLES["noise"] = _noise_table()
        _TABLES["gtab"] = _gauss_table()
    return _TABLES["noise"], _TABLES["gtab"]


@dataclass
class Blob:
    cy: int
    cx: int
    sigma: float


@dataclass
class SceneSpec:
    H: int
    W: int
    seed: int
    dtype: str = "u8"  # "u8" or "u16"
    haze: List[Blob] = field(default_factory=list)
    shadow: List[Blob] = field(default_factory=list)
    pitch: Optional[int] = None  # u16 row pitch in elements (default W)


def blobs_for_coverage(H, W, seed, stream, k, frac) -> List[Blob]:
    """k blobs whose g >= 1/2 discs cover about ``frac`` of the scene in total:
    sigma = sqrt(frac*H*W / (k * 2*pi*ln 2)); centres uniform, seeded."""
    sigma = math.sqrt(frac * H * W / (k * 2 * math.pi * math.log(2)))
    rng = np.random.default_rng([seed, stream])
    return [Blob(int(rng.integers(0, H)), int(rng.integers(0, W)), sigma) for _ in range(k)]


def config_small(seed: int = 1) -> SceneSpec:
    rng = np.random.default_rng([seed, 7])
    H = W = 512
    haze = [Blob(int(rng.integers(96, H - 96)), int(rng.integers(96, W - 96)), 96.0)]
    shadow = [Blob(int(rng.integers(96, H - 96)), int(rng.integers(96, W - 96)), 96.0)]
    return SceneSpec(H, W, seed, "u8", haze, shadow)


def config_tile(seed: int = 2, pitch: Optional[int] = None) -> SceneSpec:
    H = W = 10980
    return SceneSpec(H, W, seed, "u16", blobs_for_coverage(H, W, seed, 1, 4, 0.10),
                     blobs_for_coverage(H, W, seed, 2, 2, 0.05), pitch)


def _blob_array(blobs):
    arr = (_Blob * max(1, len(blobs)))()
    for i, b in enumerate(blobs):
        arr[i].cy, arr[i].cx = int(b.cy), int(b.cx)
        arr[i].s2 = max(1, int(round(b.sigma * b.sigma)))
    return arr


def generate_u8(spec: SceneSpec, want_truth: bool = False):
    """[3, H, W] uint8 scene (B2, B3, B4 order) and optionally the class truth."""
    noise, gtab = _tables()
    haze, shadow = _blob_array(spec.haze), _blob_array(spec.shadow)
    cfg = _Cfg()
    cfg.seed = spec.seed
    cfg.cell = CELL
    for i in range(3):
        cfg.mean[i] = CLASS_MEANS[i]
    cfg.noise = noise.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
    cfg.gtab = gtab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    cfg.gtab_len = len(gtab)
    cfg.haze, cfg.n_haze = haze, len(spec.haze)
    cfg.shadow, cfg.n_shadow = shadow, len(spec.shadow)
    out = np.empty((3, spec.H, spec.W), dtype=np.uint8)
    truth = np.empty((spec.H, spec.W), dtype=np.uint8) if want_truth else None
    _L().synth_scene_u8(ctypes.byref(cfg), spec.H, spec.W, out.ctypes.data,
                        truth.ctypes.data if want_truth else None)
    return (out, truth) if want_truth else out


def to_u16(scene8: np.ndarray, seed: int, pitch: Optional[int] = None) -> np.ndarray:
    """[3, H, pitch] uint16 reflectance drawn from the 8-bit scene's bins."""
    scene8 = np.ascontiguousarray(scene8, dtype=np.uint8)
    _, H, W = scene8.shape
    pitch = W if pitch is None else pitch
    out = np.zeros((3, H, pitch), dtype=np.uint16)
    _L().synth_u8_to_u16(seed, H, W, scene8.ctypes.data, pitch, out.ctypes.data)
    return out


def generate(spec: SceneSpec, want_truth: bool = False):
    """The scene in ``spec.dtype`` ([3, H, pitch]) and optionally the truth."""
    s8, truth = generate_u8(spec, want_truth=True)
    if spec.dtype == "u16":
        s = to_u16(s8, spec.seed, spec.pitch)
    else:
        s = s8
    return (s, truth) if want_truth else s


def coverage(spec: SceneSpec, which: str = "haze") -> float:
    """Fraction of pixels with blob strength g >= 1/2 (measured, for reports)."""
    blobs = spec.haze if which == "haze" else spec.shadow
    if not blobs:
        return 0.0
    step = max(1, min(spec.H, spec.W) // 512)
    ys = np.arange(0, spec.H, step)[:, None]
    xs = np.arange(0, spec.W, step)[None, :]
    hit = np.zeros((len(ys), xs.shape[1]), dtype=bool)
    for b in blobs:
        d2 = (ys - b.cy) ** 2 + (xs - b.cx) ** 2
        hit |= d2 <= 2 * math.log(2) * b.sigma ** 2
    return float(hit.mean())
