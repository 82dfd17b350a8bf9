"""Python binding of the continuous-batching server (``include/sil_server.h``).

Argument marshalling only: admission, batching, launches and completion
tracking run in the native runtime (``csrc/server.cpp``) and the gfx950
kernels of ``libsil.so``.
"""
import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import sil


class _Config(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_chips_per_launch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("nstreams", ctypes.c_int32),
                ("max_queue", ctypes.c_int32)]


HOST_SCENE = 1  # SIL_REQ_HOST_SCENE


class _Request(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("nbands", ctypes.c_int32),
                ("sel", ctypes.c_int32 * 3), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("pitch", ctypes.c_int64), ("tag", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class _Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("labels", ctypes.c_void_p), ("hist", ctypes.c_void_p),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("label_pitch", ctypes.c_int32), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("chips", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("active", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("pad", ctypes.c_int32)]


_bound = False


def _lib():
    global _bound
    L = sil.lib()
    if not _bound:
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.sil_server_config_default.argtypes = [P(_Config)]
        L.sil_server_config_default.restype = None
        L.sil_server_create.argtypes = [P(sil._Params), P(_Config), P(vp)]
        L.sil_server_submit.argtypes = [vp, P(_Request)]
        L.sil_server_pump.argtypes = [vp, P(ctypes.c_int32)]
        L.sil_server_poll.argtypes = [vp, P(_Completion), ctypes.c_int32, P(ctypes.c_int32)]
        L.sil_server_release.argtypes = [vp, ctypes.c_uint64]
        L.sil_server_drain.argtypes = [vp]
        L.sil_server_cancel.argtypes = [vp, ctypes.c_uint64]
        L.sil_server_expire.argtypes = [vp, ctypes.c_double, P(ctypes.c_uint64), ctypes.c_int32,
                                        P(ctypes.c_int32)]
        L.sil_server_get_stats.argtypes = [vp, P(_Stats)]
        L.sil_server_clock_ms.argtypes = [vp]
        L.sil_server_clock_ms.restype = ctypes.c_double
        L.sil_server_run.argtypes = [vp, P(_Request), P(ctypes.c_double), ctypes.c_int32,
                                     ctypes.c_int32, P(_Completion), P(ctypes.c_double)]
        L.sil_server_destroy.argtypes = [vp]
        for f in ("sil_server_create", "sil_server_submit", "sil_server_pump", "sil_server_poll",
                  "sil_server_release", "sil_server_drain", "sil_server_get_stats",
                  "sil_server_cancel", "sil_server_expire",
                  "sil_server_run", "sil_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        _bound = True
    return L


def _check(rc):
    if rc != sil.OK:
        raise sil.SilError(rc, sil.strerror(rc))


class _DevView:
    """Zero-copy view of device memory for torch.as_tensor."""

    def __init__(self, ptr, shape, typestr, strides=None):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2,
                                         "strides": strides}


@dataclass
class Completion:
    tag: int
    H: int
    W: int
    launches: int
    t_submit_ms: float
    t_admit_ms: float
    t_done_ms: float
    labels_ptr: int
    hist_ptr: int
    chip: int
    label_pitch: int

    def labels(self) -> torch.Tensor:
        """[H, W] uint8 view of the arena (rows `label_pitch` bytes apart; valid
        until release)."""
        return torch.as_tensor(_DevView(self.labels_ptr, (self.H, self.W), "|u1",
                                        (self.label_pitch, 1)), device="cuda")

    def hist(self) -> torch.Tensor:
        c = self.chip
        shape = ((self.H + c - 1) // c, (self.W + c - 1) // c, 3)
        return torch.as_tensor(_DevView(self.hist_ptr, shape, "<i4"), device="cuda")


def _completion(c: _Completion, chip: int) -> Completion:
    return Completion(c.tag, c.H, c.W, c.launches, c.t_submit_ms, c.t_admit_ms, c.t_done_ms,
                      c.labels or 0, c.hist or 0, chip, c.label_pitch)


def _request(scene: torch.Tensor, tag: int, W: Optional[int] = None, sel=(0, 1, 2)) -> _Request:
    """A request for a device scene, or for a host scene (copied into the
    server's arena at admission; page-locked memory lets the copy overlap)."""
    nb, H, pitch = scene.shape
    if not scene.is_contiguous():
        raise ValueError("scene must be contiguous")
    r = _Request()
    r.scene = scene.data_ptr()
    r.flags = 0 if scene.is_cuda else HOST_SCENE
    r.nbands = nb
    for i in range(3):
        r.sel[i] = int(sel[i])
    r.H, r.W, r.pitch, r.tag = H, pitch if W is None else int(W), pitch, int(tag)
    return r


class Server:
    """Continuous-batching labelling server on the current GPU."""

    def __init__(self, params: sil.Params, arena_bytes: int = 4 << 30,
                 max_chips_per_launch: int = 4096, max_inflight: int = 4, nstreams: int = 2,
                 max_queue: int = 65536):
        L = _lib()
        cfg = _Config()
        L.sil_server_config_default(ctypes.byref(cfg))
        cfg.arena_bytes, cfg.max_chips_per_launch = int(arena_bytes), int(max_chips_per_launch)
        cfg.max_inflight, cfg.nstreams, cfg.max_queue = int(max_inflight), int(nstreams), \
            int(max_queue)
        self.params = params
        self._p = params.to_c()
        self._h = ctypes.c_void_p()
        _check(L.sil_server_create(ctypes.byref(self._p), ctypes.byref(cfg),
                                   ctypes.byref(self._h)))
        self._scenes = {}

    def close(self):
        if self._h:
            _check(_lib().sil_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, scene: torch.Tensor, tag: int, W: Optional[int] = None, sel=(0, 1, 2)):
        """Queue a request; a GPU ``scene`` must be resident (its writes
        completed); a host ``scene`` is copied into the arena at admission."""
        r = _request(scene, tag, W, sel)
        _check(_lib().sil_server_submit(self._h, ctypes.byref(r)))
        self._scenes[int(tag)] = scene  # keep it alive until released

    def pump(self) -> int:
        n = ctypes.c_int32()
        _check(_lib().sil_server_pump(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, max_n: int = 256) -> List[Completion]:
        buf = (_Completion * max_n)()
        n = ctypes.c_int32()
        _check(_lib().sil_server_poll(self._h, buf, max_n, ctypes.byref(n)))
        return [_completion(buf[i], self.params.chip) for i in range(n.value)]

    def release(self, tag: int):
        _check(_lib().sil_server_release(self._h, int(tag)))
        self._scenes.pop(int(tag), None)

    def cancel(self, tag: int):
        """Withdraw a request that is still queued (raises if it was admitted)."""
        _check(_lib().sil_server_cancel(self._h, int(tag)))
        self._scenes.pop(int(tag), None)

    def expire(self, max_wait_ms: float, max_n: int = 4096) -> List[int]:
        """Withdraw queued requests that waited longer than max_wait_ms; their tags."""
        buf = (ctypes.c_uint64 * max_n)()
        n = ctypes.c_int32()
        _check(_lib().sil_server_expire(self._h, float(max_wait_ms), buf, max_n,
                                        ctypes.byref(n)))
        tags = [int(buf[i]) for i in range(n.value)]
        for t in tags:
            self._scenes.pop(t, None)
        return tags

    def drain(self):
        _check(_lib().sil_server_drain(self._h))

    def clock_ms(self) -> float:
        return _lib().sil_server_clock_ms(self._h)

    def stats(self) -> dict:
        st = _Stats()
        _check(_lib().sil_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _Stats._fields_ if f != "pad"}

    def run(self, scenes: Sequence[torch.Tensor], arrival_ms: Sequence[float], release: bool,
            tags: Optional[Sequence[int]] = None):
        """Play a trace natively (``sil_server_run``); returns (completions, start_ms)."""
        n = len(scenes)
        tags = list(range(n)) if tags is None else list(tags)
        reqs = (_Request * n)(*[_request(s, t) for s, t in zip(scenes, tags)])
        arr = (ctypes.c_double * n)(*[float(a) for a in arrival_ms])
        out = (_Completion * n)()
        start = ctypes.c_double()
        _check(_lib().sil_server_run(self._h, reqs, arr, n, 1 if release else 0, out,
                                     ctypes.byref(start)))
        return [_completion(out[i], self.params.chip) for i in range(n)], start.value


# ---- the serving workload ----------------------------------------------------

SIZES = (512, 2048, 4096, 10980)


def make_pool(seeds_per_size: int = 2, base_seed: int = 1000, device="cuda"):
    """uint16 scenes {size: [(seed, tensor)]} from the seeded generator (one
    haze and one shadow blob each; seeds base_seed + i), on the GPU, or in
    page-locked host memory with device="pinned"."""
    import synth
    pool = {}
    k = 0
    for n in SIZES:
        pool[n] = []
        for _ in range(seeds_per_size):
            seed = base_seed + k
            k += 1
            spec = synth.SceneSpec(n, n, seed, "u16",
                                   synth.blobs_for_coverage(n, n, seed, 1, 1, 0.10),
                                   synth.blobs_for_coverage(n, n, seed, 2, 1, 0.05))
            t = torch.from_numpy(synth.generate(spec).view(np.int16))
            t = t.pin_memory() if device == "pinned" else t.to(device)
            pool[n].append((seed, t))
    torch.cuda.synchronize()
    return pool


def make_trace(n_requests: int, rate_per_ms: float, pool, seed: int = 7):
    """Poisson arrivals at `rate_per_ms`; sizes uniform over SIZES, scene
    uniform over that size's pool.  Returns (arrival_ms, [(size, idx)])."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_ms, n_requests) if rate_per_ms > 0 else \
        np.zeros(n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    picks = []
    for _ in range(n_requests):
        size = SIZES[int(rng.integers(0, len(SIZES)))]
        picks.append((size, int(rng.integers(0, len(pool[size])))))
    return arrivals.tolist(), picks
