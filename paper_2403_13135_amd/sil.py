"""Python binding of libsil (argument marshalling only).

Every step of the labelling runs in the gfx950 kernels of ``libsil.so``; this
module only checks tensor shapes, picks the current HIP stream and forwards
raw device pointers through the C ABI declared in ``include/sil.h``.  There
is no CPU path: if the library is missing, importing the binding's entry
points raises.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsil.so")

OK, EINVAL, EUNSUPPORTED, EDEVICE = 0, -1, -2, -3
U8, U16 = 1, 2
ABI_VERSION = 1


class SilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sil error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
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


CHIP_INFO_BYTES = 12  # sil_chip_info: int32 t; u8 lo, hi, gate, stretch; u16 a1, a2
BATCH_MAX_JOBS = 24


class _Job(ctypes.Structure):
    _fields_ = [
        ("scene", ctypes.c_void_p),
        ("nbands", ctypes.c_int32),
        ("sel", ctypes.c_int32 * 3),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("pitch", ctypes.c_int64),
        ("labels", ctypes.c_void_p),
        ("label_pitch", ctypes.c_int64),
        ("hist", ctypes.c_void_p),
        ("chips", ctypes.c_void_p),
        ("chip_begin", ctypes.c_int32),
        ("chip_count", ctypes.c_int32),
    ]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded ``libsil.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it first (python -m paper_2403_13135_amd._build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.sil_params_default.argtypes = [P(_Params)]
        L.sil_params_default.restype = None
        L.sil_abi_version.argtypes = []
        L.sil_abi_version.restype = ctypes.c_uint32
        L.sil_hist_dims.argtypes = [ctypes.c_int32, ctypes.c_int32, P(_Params),
                                    P(ctypes.c_int32), P(ctypes.c_int32)]
        L.sil_hist_dims.restype = ctypes.c_int
        L.sil_validate.argtypes = [ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, P(_Params)]
        L.sil_validate.restype = ctypes.c_int
        L.sil_label.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32),
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P(_Params),
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
        L.sil_label.restype = ctypes.c_int
        L.sil_chip_count.argtypes = [ctypes.c_int32, ctypes.c_int32, P(_Params),
                                     P(ctypes.c_int32)]
        L.sil_chip_count.restype = ctypes.c_int
        L.sil_label_batch.argtypes = [P(_Job), ctypes.c_int32, P(_Params), ctypes.c_void_p]
        L.sil_label_batch.restype = ctypes.c_int
        L.sil_label_ex_validate.argtypes = L.sil_validate.argtypes
        L.sil_label_ex_validate.restype = ctypes.c_int
        L.sil_label_ex_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, P(_Params),
                                             P(ctypes.c_uint64)]
        L.sil_label_ex_workspace.restype = ctypes.c_int
        L.sil_label_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_int32),
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P(_Params),
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.sil_label_ex.restype = ctypes.c_int
        L.sil_label_ex_noalloc.argtypes = L.sil_label_ex.argtypes[:-3] + [ctypes.c_void_p]
        L.sil_render_rgb.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p]
        L.sil_render_rgb.restype = ctypes.c_int
        L.sil_label_ex_noalloc.restype = ctypes.c_int
        L.sil_strerror.argtypes = [ctypes.c_int]
        L.sil_strerror.restype = ctypes.c_char_p
        if L.sil_abi_version() != ABI_VERSION:
            raise RuntimeError("libsil ABI version mismatch")
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().sil_strerror(code).decode()


def _check(code: int):
    if code != OK:
        raise SilError(code, strerror(code))


@dataclass
class Params:
    """Labelling parameters (``sil_params``).  Defaults are the paper's HSV
    limits (section III-B) and the filter constants of include/sil.h."""
    dtype: int = U8
    refl_max: int = 10000
    lo: Sequence[Sequence[int]] = field(
        default_factory=lambda: [[0, 0, 0], [0, 0, 31], [0, 0, 205]])
    hi: Sequence[Sequence[int]] = field(
        default_factory=lambda: [[185, 255, 30], [185, 255, 204], [185, 255, 255]])
    filter: int = 1
    chip: int = 256
    clip_shift: int = 8
    eta_num: int = 3
    eta_den: int = 4
    patch_h: int = 256
    patch_w: int = 256

    def to_c(self) -> _Params:
        p = _Params()
        lib().sil_params_default(ctypes.byref(p))
        for name in ("dtype", "refl_max", "filter", "chip", "clip_shift", "eta_num",
                     "eta_den", "patch_h", "patch_w"):
            setattr(p, name, int(getattr(self, name)))
        for c in range(3):
            for j in range(3):
                p.lo[c][j] = int(self.lo[c][j])
                p.hi[c][j] = int(self.hi[c][j])
        return p

    def fields(self) -> dict:
        """Plain field dict (for handing the same run to another implementation)."""
        return {k: getattr(self, k) for k in self.__dataclass_fields__}


def hist_dims(H: int, W: int, params: Params) -> Tuple[int, int]:
    ny, nx = ctypes.c_int32(), ctypes.c_int32()
    p = params.to_c()
    _check(lib().sil_hist_dims(H, W, ctypes.byref(p), ctypes.byref(ny), ctypes.byref(nx)))
    return ny.value, nx.value


def validate(nbands: int, sel, H: int, W: int, pitch: int, label_pitch: int,
             params: Params) -> int:
    s = (ctypes.c_int32 * 3)(*[int(v) for v in sel])
    p = params.to_c()
    return lib().sil_validate(nbands, s, H, W, pitch, label_pitch, ctypes.byref(p))


_SCENE_DTYPES = {U8: (torch.uint8,), U16: (torch.uint16, torch.int16)}


def label_pitch_for(W: int) -> int:
    """Row pitch (bytes) for a label plane of width W: W rounded up to a
    multiple of 128, so every row starts on a cache-line boundary and the
    labeller writes whole lines."""
    return (int(W) + 127) // 128 * 128


def alloc_labels(H: int, W: int, device) -> torch.Tensor:
    """An [H, W] uint8 label plane whose rows are ``label_pitch_for(W)`` bytes
    apart (a view of an [H, pitch] allocation)."""
    return torch.empty((H, label_pitch_for(W)), dtype=torch.uint8, device=device)[:, :W]


def label(scene: torch.Tensor, params: Optional[Params] = None, sel=(0, 1, 2),
          W: Optional[int] = None, labels: Optional[torch.Tensor] = None,
          hist: Optional[torch.Tensor] = None, chips: bool = False,
          stream: Optional[torch.cuda.Stream] = None):
    """Label ``scene`` ([nbands, H, pitch] on the GPU) with ``sil_label``.

    ``W`` defaults to the pitch (the last dimension).  ``labels`` ([H, >=W]
    uint8, any row stride) and ``hist`` ([ny, nx, 3] int32/uint32) may be given
    to reuse buffers; by default labels come from ``alloc_labels``.  Returns (labels, hist) or (labels, hist, chip_info_bytes) with
    ``chips=True`` (a uint8 tensor of ``[ncy, ncx, 12]`` raw sil_chip_info).
    Enqueued on ``stream`` (default: the current stream); not synchronised.
    """
    if params is None:
        params = Params(dtype=U16 if scene.dtype in _SCENE_DTYPES[U16] else U8)
    if scene.dim() != 3 or not scene.is_cuda:
        raise ValueError("scene must be a [nbands, H, pitch] GPU tensor")
    if scene.dtype not in _SCENE_DTYPES[params.dtype]:
        raise ValueError(f"scene dtype {scene.dtype} does not match params.dtype")
    if not scene.is_contiguous():
        raise ValueError("scene must be contiguous (planar, rows of `pitch` elements)")
    nb, H, pitch = scene.shape
    W = pitch if W is None else int(W)
    dev = scene.device
    ny, nx = hist_dims(H, W, params)
    if labels is None:
        labels = alloc_labels(H, W, dev)
    if labels.dtype != torch.uint8 or labels.dim() != 2 or labels.shape[0] != H \
            or labels.shape[1] < W or labels.stride(1) != 1:
        raise ValueError("labels must be uint8 [H, >=W] with unit column stride")
    if hist is None:
        hist = torch.empty((ny, nx, 3), dtype=torch.int32, device=dev)
    if hist.shape != (ny, nx, 3) or hist.dtype not in (torch.int32, torch.uint32) \
            or not hist.is_contiguous():
        raise ValueError(f"hist must be contiguous int32 [{ny}, {nx}, 3]")
    chip_t = None
    if chips:
        C = params.chip
        chip_t = torch.zeros(((H + C - 1) // C, (W + C - 1) // C, CHIP_INFO_BYTES),
                             dtype=torch.uint8, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    sel_c = (ctypes.c_int32 * 3)(*[int(v) for v in sel])
    p = params.to_c()
    rc = lib().sil_label(ctypes.c_void_p(scene.data_ptr()), nb, sel_c, H, W, pitch,
                         ctypes.byref(p), ctypes.c_void_p(labels.data_ptr()),
                         labels.stride(0), ctypes.c_void_p(hist.data_ptr()),
                         ctypes.c_void_p(chip_t.data_ptr()) if chips else None,
                         ctypes.c_void_p(s.cuda_stream))
    _check(rc)
    return (labels, hist, chip_t) if chips else (labels, hist)


def render_rgb(labels: torch.Tensor, W: Optional[int] = None, out: Optional[torch.Tensor] = None,
               stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Colour image of a class-id plane with ``sil_render_rgb``: labels
    [H, >=W] uint8 on the GPU (any row stride) -> [H, W, 3] uint8 (R, G, B):
    water green, thin ice blue, thick ice red, other ids black.  ``out`` may be
    a uint8 [H, W, 3] tensor with unit strides in its last two dimensions."""
    if labels.dtype != torch.uint8 or labels.dim() != 2 or not labels.is_cuda \
            or labels.stride(1) != 1:
        raise ValueError("labels must be a uint8 [H, >=W] GPU tensor with unit column stride")
    H = labels.shape[0]
    W = labels.shape[1] if W is None else int(W)
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.uint8, device=labels.device)
    if out.dtype != torch.uint8 or out.shape != (H, W, 3) or out.stride(2) != 1 \
            or out.stride(1) != 3:
        raise ValueError(f"out must be uint8 [{H}, {W}, 3] with interleaved pixels")
    s = stream if stream is not None else torch.cuda.current_stream(labels.device)
    _check(lib().sil_render_rgb(ctypes.c_void_p(labels.data_ptr()), H, W, labels.stride(0),
                                ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                ctypes.c_void_p(s.cuda_stream)))
    return out


def decode_chip_info(raw) -> list:
    """Decode a [..., 12] uint8 array of sil_chip_info into dicts (host side)."""
    import numpy as np
    dt = np.dtype([("t", "<i4"), ("lo", "u1"), ("hi", "u1"), ("gate", "u1"),
                   ("stretch", "u1"), ("a1", "<u2"), ("a2", "<u2")])
    arr = np.ascontiguousarray(np.asarray(raw, dtype=np.uint8))
    return arr.reshape(-1).view(dt).reshape(arr.shape[:-1])


def chip_count(H: int, W: int, params: Params) -> int:
    n = ctypes.c_int32()
    p = params.to_c()
    _check(lib().sil_chip_count(H, W, ctypes.byref(p), ctypes.byref(n)))
    return n.value


@dataclass
class Job:
    """One scene's share of a batched launch (``sil_job``).  ``scene`` is a
    [nbands, H, pitch] GPU tensor; ``labels`` [H, >=W] uint8 and ``hist``
    [ny, nx, 3] int32 are the scene's full output buffers; chips
    [chip_begin, chip_begin + chip_count) are labelled by the call."""
    scene: torch.Tensor
    labels: torch.Tensor
    hist: torch.Tensor
    chip_begin: int
    chip_count: int
    W: Optional[int] = None
    sel: Tuple[int, int, int] = (0, 1, 2)
    chips: Optional[torch.Tensor] = None


def make_job_struct(job: Job) -> _Job:
    nb, H, pitch = job.scene.shape
    j = _Job()
    j.scene = job.scene.data_ptr()
    j.nbands = nb
    for i in range(3):
        j.sel[i] = int(job.sel[i])
    j.H = H
    j.W = pitch if job.W is None else int(job.W)
    j.pitch = pitch
    j.labels = job.labels.data_ptr()
    j.label_pitch = job.labels.stride(0)
    j.hist = job.hist.data_ptr()
    j.chips = job.chips.data_ptr() if job.chips is not None else None
    j.chip_begin = int(job.chip_begin)
    j.chip_count = int(job.chip_count)
    return j


def label_batch(jobs: Sequence[Job], params: Params,
                stream: Optional[torch.cuda.Stream] = None) -> None:
    """One ``sil_label_batch`` launch over the jobs' chip ranges (asynchronous)."""
    if not jobs or len(jobs) > BATCH_MAX_JOBS:
        raise ValueError(f"1..{BATCH_MAX_JOBS} jobs per batch")
    arr = (_Job * len(jobs))(*[make_job_struct(j) for j in jobs])
    s = stream if stream is not None else torch.cuda.current_stream(jobs[0].scene.device)
    p = params.to_c()
    _check(lib().sil_label_batch(arr, len(jobs), ctypes.byref(p), ctypes.c_void_p(s.cuda_stream)))


# ---- the general labeller (variants) -----------------------------------------

def validate_ex(nbands: int, sel, H: int, W: int, pitch: int, mask_pitch: int,
                params: Params) -> int:
    s = (ctypes.c_int32 * 3)(*[int(v) for v in sel])
    p = params.to_c()
    return lib().sil_label_ex_validate(nbands, s, H, W, pitch, mask_pitch, ctypes.byref(p))


def workspace_bytes(H: int, W: int, params: Params) -> int:
    n = ctypes.c_uint64()
    p = params.to_c()
    _check(lib().sil_label_ex_workspace(H, W, ctypes.byref(p), ctypes.byref(n)))
    return n.value


def label_ex(scene: torch.Tensor, params: Optional[Params] = None, sel=(0, 1, 2),
             W: Optional[int] = None, counts: bool = True, rgb: bool = False,
             chips: bool = False, workspace: Optional[torch.Tensor] = None,
             out: Optional[dict] = None, stream: Optional[torch.cuda.Stream] = None,
             noalloc: bool = False) -> dict:
    """The general labeller ``sil_label_ex`` on ``scene`` ([nbands, H, pitch]
    on the GPU): full-HSV masks, any filter unit, optional filtered colour.

    Returns a dict with ``masks`` [H, W] uint8 (bit c = mask c), ``counts``
    [ny, nx, 3] int32 (if asked), ``rgb`` [3, H, W] uint8 (if asked; masks and
    colour rows are ``label_pitch_for(W)`` bytes apart unless given) and
    ``chips`` (raw [ncy, ncx, 12] sil_chip_info bytes, if asked).  ``out`` may
    hold preallocated tensors under the same keys; ``workspace`` a uint8 GPU
    tensor of at least ``workspace_bytes`` bytes (allocated here if omitted).
    ``noalloc`` calls ``sil_label_ex_noalloc`` instead, whose workspace is the
    library's own per-device array (no workspace argument).  Enqueued on
    ``stream`` (default: the current stream); not synchronised.
    """
    if params is None:
        params = Params(dtype=U16 if scene.dtype in _SCENE_DTYPES[U16] else U8)
    if scene.dim() != 3 or not scene.is_cuda or not scene.is_contiguous():
        raise ValueError("scene must be a contiguous [nbands, H, pitch] GPU tensor")
    if scene.dtype not in _SCENE_DTYPES[params.dtype]:
        raise ValueError(f"scene dtype {scene.dtype} does not match params.dtype")
    nb, H, pitch = scene.shape
    W = pitch if W is None else int(W)
    dev = scene.device
    out = dict(out or {})
    masks = out.get("masks")
    if masks is None:
        masks = out["masks"] = alloc_labels(H, W, dev)
    if masks.dtype != torch.uint8 or masks.dim() != 2 or masks.shape[0] != H \
            or masks.shape[1] < W or masks.stride(1) != 1:
        raise ValueError("masks must be uint8 [H, >=W] with unit column stride")
    cnt = None
    if counts:
        ny, nx = hist_dims(H, W, params)
        cnt = out.get("counts")
        if cnt is None:
            cnt = out["counts"] = torch.empty((ny, nx, 3), dtype=torch.int32, device=dev)
        if cnt.shape != (ny, nx, 3) or cnt.dtype not in (torch.int32, torch.uint32) \
                or not cnt.is_contiguous():
            raise ValueError(f"counts must be contiguous int32 [{ny}, {nx}, 3]")
    col = None
    if rgb:
        col = out.get("rgb")
        if col is None:
            col = out["rgb"] = torch.empty((3, H, label_pitch_for(W)), dtype=torch.uint8,
                                           device=dev)[:, :, :W]
        if col.dtype != torch.uint8 or col.dim() != 3 or col.shape[0] != 3 \
                or col.shape[1] != H or col.shape[2] < W or col.stride(2) != 1 \
                or col.stride(0) != H * col.stride(1):
            raise ValueError("rgb must be planar uint8 [3, H, >=W]")
    chip_t = None
    if chips:
        C = params.chip
        chip_t = out.get("chips")
        if chip_t is None:
            chip_t = out["chips"] = torch.zeros(
                ((H + C - 1) // C, (W + C - 1) // C, CHIP_INFO_BYTES), dtype=torch.uint8,
                device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    sel_c = (ctypes.c_int32 * 3)(*[int(v) for v in sel])
    p = params.to_c()
    args = [ctypes.c_void_p(scene.data_ptr()), nb, sel_c, H, W, pitch, ctypes.byref(p),
            ctypes.c_void_p(masks.data_ptr()), masks.stride(0),
            ctypes.c_void_p(cnt.data_ptr()) if cnt is not None else None,
            ctypes.c_void_p(col.data_ptr()) if col is not None else None,
            col.stride(1) if col is not None else 0,
            ctypes.c_void_p(chip_t.data_ptr()) if chip_t is not None else None]
    if noalloc:
        _check(lib().sil_label_ex_noalloc(*args, ctypes.c_void_p(s.cuda_stream)))
        return out
    need = workspace_bytes(H, W, params)
    if need and workspace is None:
        workspace = torch.empty((need,), dtype=torch.uint8, device=dev)
    if need and (workspace.dtype != torch.uint8 or workspace.numel() < need
                 or not workspace.is_cuda):
        raise ValueError(f"workspace must be a uint8 GPU tensor of >= {need} bytes")
    _check(lib().sil_label_ex(*args, ctypes.c_void_p(workspace.data_ptr()) if need else None,
                              need, ctypes.c_void_p(s.cuda_stream)))
    return out
