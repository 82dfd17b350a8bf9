"""Brute-force checkers used to pin the oracle (tests only).

Each function computes its quantity from the textbook definition with a
different route than the oracle: library routines (scipy's median filter,
numpy sorting and bincount, the decimal and fractions modules, statistics'
population variance), pixel lists instead of histograms, and the
within-class-variance form of Otsu's criterion instead of the between-class
form.  They are slow and meant for tiny inputs.
"""
from decimal import Decimal, ROUND_HALF_UP
from fractions import Fraction
import statistics

import numpy as np
import scipy.ndimage

PAPER_LO = [[0, 0, 0], [0, 0, 31], [0, 0, 205]]
PAPER_HI = [[185, 255, 30], [185, 255, 204], [185, 255, 255]]


def rescale_decimal(x: int, refl_max: int = 10000) -> int:
    """8-bit value of a reflectance: round-half-up of x*255/refl_max, capped at 255."""
    q = (Decimal(x) * 255 / Decimal(refl_max)).quantize(Decimal(1), rounding=ROUND_HALF_UP)
    return min(255, int(q))


def hsv_opencv8(R, G, B):
    """OpenCV 8-bit RGB->HSV from the hexcone definition: V = max, S = 255*(V-min)/V,
    H = hue in degrees / 2 in [0, 180).  Vectorised, float64, rounded."""
    R = np.asarray(R, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    V = np.maximum(np.maximum(R, G), B)
    mn = np.minimum(np.minimum(R, G), B)
    delta = V - mn
    with np.errstate(divide="ignore", invalid="ignore"):
        S = np.where(V > 0, 255.0 * delta / np.where(V > 0, V, 1), 0.0)
        d = np.where(delta > 0, delta, 1)
        h = np.where(V == R, 60.0 * (G - B) / d,
                     np.where(V == G, 120.0 + 60.0 * (B - R) / d, 240.0 + 60.0 * (R - G) / d))
    h = np.where(delta > 0, h, 0.0)
    h = np.where(h < 0, h + 360.0, h)
    H = np.round(h / 2.0)
    return H, np.round(S), V


def in_range_class(H, S, V, lo=PAPER_LO, hi=PAPER_HI):
    """Three 3-D inRange masks; returns (class index or -1, number of masks hit)."""
    hits = []
    for c in range(3):
        m = ((H >= lo[c][0]) & (H <= hi[c][0]) & (S >= lo[c][1]) & (S <= hi[c][1])
             & (V >= lo[c][2]) & (V <= hi[c][2]))
        hits.append(m)
    n = hits[0].astype(np.int32) + hits[1] + hits[2]
    cls = np.where(hits[0], 0, np.where(hits[1], 1, np.where(hits[2], 2, -1)))
    return cls, n


def median3x3(V):
    """3x3 median with replicated borders (scipy 'nearest' mode)."""
    return scipy.ndimage.median_filter(np.asarray(V), size=3, mode="nearest")


def otsu_within(pixels):
    """Otsu's threshold as the minimiser of the within-class variance
    sum_{class} sum_{p in class} (v_p - mean_class)^2 over splits {v <= t}|{v > t},
    t = 0..254, both classes non-empty; smallest t on ties; None if no split."""
    px = sorted(int(v) for v in pixels)
    best_t, best = None, None
    for t in range(255):
        c0 = [v for v in px if v <= t]
        c1 = [v for v in px if v > t]
        if not c0 or not c1:
            continue
        sw = Fraction(0)
        for cl in (c0, c1):
            mu = Fraction(sum(cl), len(cl))
            sw += sum((v - mu) ** 2 for v in cl)
        if best is None or sw < best:
            best, best_t = sw, t
    return best_t


def eta(pixels, t):
    """Separability sigma_B^2 / sigma_T^2 at split t, with sigma_T^2 the population
    variance and sigma_B^2 = sigma_T^2 - within-class variance."""
    px = [Fraction(int(v)) for v in pixels]
    total = statistics.pvariance(px)
    c0 = [v for v in px if v <= t]
    c1 = [v for v in px if v > t]
    within = (len(c0) * statistics.pvariance(c0) + len(c1) * statistics.pvariance(c1)) / len(px)
    return (total - within) / total


def ranks(pixels, clip_shift=8):
    """(k+1)-th smallest and (k+1)-th largest value, k = N >> clip_shift."""
    s = np.sort(np.asarray(pixels).ravel())
    k = s.size >> clip_shift
    return int(s[k]), int(s[s.size - 1 - k])


def stretch(m, lo, hi):
    """Truncate to [lo, hi], map linearly onto [0, 255], round half up."""
    c = min(max(m, lo), hi)
    return int(Fraction(c - lo) * 255 / (hi - lo) + Fraction(1, 2)) if hi > lo else m


def filtered_v(scene, dtype="u8", refl_max=10000, filter=1, chip=256, clip_shift=8,
               eta_num=3, eta_den=4, sel=(0, 1, 2)):
    """The filtered brightness Vc [H, W] (int64) composed from the checkers
    above, and the 8-bit (blue, green, red) planes it came from."""
    s = np.asarray(scene)
    planes = [s[i].astype(np.int64) for i in sel]
    if dtype == "u16":
        lut = {}
        planes = [np.vectorize(lambda v: lut.setdefault(v, rescale_decimal(int(v), refl_max)))(
            pl).astype(np.int64) for pl in planes]
    V = np.maximum(np.maximum(planes[0], planes[1]), planes[2])
    if filter == 0:
        return V, planes
    Hh, W = V.shape
    Vm = median3x3(V)
    Vc = Vm.copy()
    for cy in range((Hh + chip - 1) // chip):
        for cx in range((W + chip - 1) // chip):
            blk = Vm[cy * chip:(cy + 1) * chip, cx * chip:(cx + 1) * chip]
            px = blk.ravel().tolist()
            t = otsu_within(px)
            gate = t is not None and eta(px, t) >= Fraction(eta_num, eta_den)
            rlo, rhi = ranks(px, clip_shift)
            if gate and rhi > rlo:
                Vc[cy * chip:(cy + 1) * chip, cx * chip:(cx + 1) * chip] = np.vectorize(
                    lambda m: stretch(int(m), rlo, rhi))(blk)
    return Vc, planes


def otsu_hist_within(h):
    """Otsu from a histogram with exact rationals, by the within-class form:
    minimise sum over both classes of (sum v^2 h - (sum v h)^2 / weight), t =
    0..254, both classes non-empty, smallest t on ties.  Returns (t or None,
    eta = 1 - within / total as a Fraction or None)."""
    h = [int(x) for x in h]
    N = sum(h)
    S = sum(v * h[v] for v in range(256))
    Q = sum(v * v * h[v] for v in range(256))
    total = Fraction(Q) - Fraction(S * S, N)
    best_t, best = None, None
    w0 = s0 = q0 = 0
    for t in range(255):
        w0 += h[t]
        s0 += t * h[t]
        q0 += t * t * h[t]
        w1, s1, q1 = N - w0, S - s0, Q - q0
        if w0 == 0 or w1 == 0:
            continue
        sw = Fraction(q0) - Fraction(s0 * s0, w0) + Fraction(q1) - Fraction(s1 * s1, w1)
        if best is None or sw < best:
            best, best_t = sw, t
    if best_t is None:
        return None, None
    return best_t, 1 - best / total


def label_scene(scene, dtype="u8", refl_max=10000, filter=1, chip=256, clip_shift=8,
                eta_num=3, eta_den=4, patch_h=256, patch_w=256, sel=(0, 1, 2),
                lo=PAPER_LO, hi=PAPER_HI):
    """The labeller composed from the checkers above (tiny scenes only).

    Returns labels [H, W], hist [ny, nx, 3], chip infos {(cy, cx): dict}."""
    s = np.asarray(scene)
    planes = [s[i].astype(np.int64) for i in sel]
    x = np.maximum(np.maximum(planes[0], planes[1]), planes[2])
    if dtype == "u16":
        lut = {}
        V = np.vectorize(lambda v: lut.setdefault(v, rescale_decimal(int(v), refl_max)))(x)
    else:
        V = x
    V = V.astype(np.int64)
    Hh, W = V.shape
    infos = {}
    if filter == 0:
        Vc = V
    else:
        Vm = median3x3(V)
        Vc = Vm.copy()
        for cy in range((Hh + chip - 1) // chip):
            for cx in range((W + chip - 1) // chip):
                blk = Vm[cy * chip:(cy + 1) * chip, cx * chip:(cx + 1) * chip]
                px = blk.ravel().tolist()
                t = otsu_within(px)
                gate = t is not None and eta(px, t) >= Fraction(eta_num, eta_den)
                rlo, rhi = ranks(px, clip_shift)
                st = gate and rhi > rlo
                infos[(cy, cx)] = dict(t=-1 if t is None else t, lo=rlo, hi=rhi, gate=int(gate),
                                       stretch=int(st))
                if st:
                    Vc[cy * chip:(cy + 1) * chip, cx * chip:(cx + 1) * chip] = np.vectorize(
                        lambda m: stretch(int(m), rlo, rhi))(blk)
    # hue and saturation of the pixel's colour (scale-free, so they apply to
    # reflectance too); the filter changes brightness only
    Hc, Sc, _ = hsv_opencv8(planes[2], planes[1], planes[0])
    cls, n = in_range_class(Hc, Sc, Vc, lo, hi)
    assert (n == 1).all()
    ny, nx = (Hh + patch_h - 1) // patch_h, (W + patch_w - 1) // patch_w
    hist = np.zeros((ny, nx, 3), dtype=np.int64)
    yy, xx = np.mgrid[0:Hh, 0:W]
    np.add.at(hist, (yy // patch_h, xx // patch_w, cls), 1)
    return cls.astype(np.uint8), hist, infos
