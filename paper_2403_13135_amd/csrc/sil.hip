// sil.hip -- gfx950 kernels and C ABI of libsil, the sea-ice auto-labeller
// of arXiv 2403.13135 (section III-A "Filtering Out the Thin Clouds and
// Shadows", section III-B "Auto-labeling Method" and "Scaling
// Auto-labeling").  The operation each entry point computes is stated in
// include/sil.h.
//
// Work decomposition (filter = 1): one 512-thread workgroup per chip
// (<= 256 x 256 pixels).  Wave w owns chip rows [32w, 32w + 32); lane l owns
// columns [4l, 4l + 4).  Each wave walks its 34 input rows (one halo row
// above and below) once, keeping a three-row window of V = max(B,G,R) in
// registers; horizontal neighbours come from the adjacent lanes through DPP
// wave shifts and the two chip-edge halo columns are fetched once per wave.
// Even waves walk down and odd waves walk up, so the halo row two adjacent
// waves share is read by both at about the same time (one HBM fetch).
//   phase 1: 3x3 median (column sort + median of three triples, exact), the
//            16->8-bit rescale (applied after the median: order statistics
//            commute with a non-decreasing map), a 32-copy LDS histogram
//            (copy = lane % 32, so the 64 lanes of an atomic never share a
//            bank except across the two half-waves), and the 8-bit medians
//            kept packed in 32 registers per lane;
//   phase 2: one wave reduces the histogram and runs exact Otsu (128-bit
//            cross-multiplied comparisons), the eta gate, rank-k truncation
//            levels and the stretch, folded with the class limits into a
//            256-entry class table in LDS;
//   phase 3: labels from the table, 4 pixels per 32-bit store, counts.
// Chips are assigned so that each XCD (workgroup id mod 8) receives a
// contiguous run of chips in raster order: horizontally adjacent chips run
// concurrently on one XCD and share their halo cache lines in its L2.
//
// filter = 0 uses a plain streaming kernel over the same tiling.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <mutex>

#include "sil.h"

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kRowsPerWave = 32;
constexpr int kTile = kWaves * kRowsPerWave;  // 256: chip side handled per workgroup
constexpr int kCopies = 32;                   // LDS histogram copies
constexpr int kMaxPatchSlots = 1024;          // LDS per-patch counters per workgroup
constexpr int kPrefetch = 4;                  // rows of loads in flight per wave

enum CountMode : uint32_t {
  CM_HIST_STORE = 0,   // patch == chip: counts from the chip histogram, plain store
  CM_HIST_ATOMIC = 1,  // chip tiles the patch: counts from the histogram, atomic add
  CM_PIX_LDS = 2,      // per-pixel counts in LDS, then store or atomic add
  CM_PIX_GLOBAL = 3    // per-pixel counts straight to global atomics
};

struct KArgs {
  const void* scene;
  int64_t off[3];  // element offsets of the blue, green, red planes
  int64_t pitch;
  int32_t H, W;
  uint8_t* labels;
  int64_t lpitch;
  uint32_t* hist;
  int32_t ny, nx, ph, pw;
  sil_chip_info* chips;
  int32_t chip, ncy, ncx, nchips, per_xcd;
  // 16-bit rescale: V = ((min(x, x_sat) * 255 + half) * magic) >> shift
  uint32_t x_sat, half, magic, shift;
  uint32_t t1, t2;  // first V of class >= 1 and >= 2 (256 if none)
  uint32_t X1, X2;  // the same boundaries on raw input values (filter = 0)
  uint32_t clip_shift, eta_num, eta_den;
  uint32_t count_mode;
  uint32_t pix_store;  // CM_PIX_LDS: 1 plain store (patches nest in chips), 0 atomic
  int32_t npy_l, npx_l;
  uint32_t label_vec;  // 4-byte label stores allowed
};

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
  return min(min(a, b), c);
}
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) {
  return max(max(a, b), c);
}
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// Lane i receives lane i-1's value; lane 0 receives `edge`.
__device__ __forceinline__ uint32_t from_left(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138 /*wave_shr:1*/, 0xF,
                                               0xF, false);
}
// Lane i receives lane i+1's value; lane 63 receives `edge`.
__device__ __forceinline__ uint32_t from_right(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130 /*wave_shl:1*/, 0xF,
                                               0xF, false);
}

template <typename T>
__device__ __forceinline__ uint32_t rescale(uint32_t x, const KArgs& a, bool fast24) {
  if constexpr (sizeof(T) == 1) {
    return x;
  } else {
    uint32_t n = min(x, a.x_sat) * 255u + a.half;
    if (fast24) {
      // n < 2^24 and magic < 2^24 (checked on the host): 24-bit multiplies
      uint64_t p = (uint64_t)(n & 0xFFFFFFu) * (uint64_t)(a.magic & 0xFFFFFFu);
      return (uint32_t)(p >> a.shift);
    }
    return (uint32_t)(((uint64_t)n * a.magic) >> a.shift);
  }
}

// ---- loads ------------------------------------------------------------------

// Raw 4-pixel row segments of the three bands.
template <typename T, bool VEC>
struct Raw {
  uint32_t v[3][4];
};
template <>
struct Raw<uint16_t, true> {
  uint2 v[3];
};
template <>
struct Raw<uint8_t, true> {
  uint32_t v[3];
};

// Load columns [gx, gx+4) of row gy.  VEC: one aligned vector per band (the
// caller guarantees gx + 3 < W and alignment).  Otherwise element loads with
// columns clamped to W - 1.
template <typename T, bool VEC>
__device__ __forceinline__ void load_raw(const KArgs& a, int32_t gy, int32_t gx, Raw<T, VEC>& r) {
  const T* base = (const T*)a.scene + (int64_t)gy * a.pitch;
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int b = 0; b < 3; ++b) r.v[b] = *(const uint2*)(base + a.off[b] + gx);
    } else {
#pragma unroll
      for (int b = 0; b < 3; ++b) r.v[b] = *(const uint32_t*)(base + a.off[b] + gx);
    }
  } else {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) r.v[b][j] = base[a.off[b] + min(gx + j, a.W - 1)];
  }
}

// max over the three bands, 4 pixels
template <typename T, bool VEC>
__device__ __forceinline__ void max_bands(const Raw<T, VEC>& r, uint32_t x[4]) {
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 2) {
      uint32_t lo[3], hi[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        lo[b] = r.v[b].x;
        hi[b] = r.v[b].y;
      }
      x[0] = max3u(lo[0] & 0xFFFFu, lo[1] & 0xFFFFu, lo[2] & 0xFFFFu);
      x[1] = max3u(lo[0] >> 16, lo[1] >> 16, lo[2] >> 16);
      x[2] = max3u(hi[0] & 0xFFFFu, hi[1] & 0xFFFFu, hi[2] & 0xFFFFu);
      x[3] = max3u(hi[0] >> 16, hi[1] >> 16, hi[2] >> 16);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        x[j] = max3u((r.v[0] >> (8 * j)) & 0xFFu, (r.v[1] >> (8 * j)) & 0xFFu,
                     (r.v[2] >> (8 * j)) & 0xFFu);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = max3u(r.v[0][j], r.v[1][j], r.v[2][j]);
  }
}

// One pixel: max over the bands at (gy, gx), gx clamped into [0, W).
template <typename T>
__device__ __forceinline__ uint32_t max_bands_at(const KArgs& a, int32_t gy, int32_t gx) {
  gx = min(max(gx, 0), a.W - 1);
  const T* base = (const T*)a.scene + (int64_t)gy * a.pitch + gx;
  return max3u(base[a.off[0]], base[a.off[1]], base[a.off[2]]);
}

// ---- wave helpers -----------------------------------------------------------

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = min(v, (uint32_t)__shfl_xor(v, d));
  return v;
}
__device__ __forceinline__ int32_t wave_max32(int32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = max(v, (int32_t)__shfl_xor(v, d));
  return v;
}

// ---- per-pixel class counting (patches that do not align with chips) --------

struct PixCount {
  int32_t key;   // current patch key, -1 none
  uint32_t cnt;  // three 10-bit class counters
};

__device__ __forceinline__ void pix_flush(const KArgs& a, uint32_t* s_cnt, bool lds, int32_t key,
                                          uint32_t cnt) {
  if (cnt == 0) return;
  uint32_t c[3] = {cnt & 1023u, (cnt >> 10) & 1023u, cnt >> 20};
  if (lds) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (c[k]) atomicAdd(&s_cnt[key * 3 + k], c[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (c[k]) atomicAdd(&a.hist[(int64_t)key * 3 + k], c[k]);
  }
}

__device__ __forceinline__ void pix_add(const KArgs& a, uint32_t* s_cnt, bool lds, PixCount& pc,
                                        int32_t key, uint32_t cls) {
  if (key != pc.key) {
    pix_flush(a, s_cnt, lds, pc.key, pc.cnt);
    pc.key = key;
    pc.cnt = 0;
  }
  pc.cnt += 1u << (10u * cls);
}

// Copy a workgroup's LDS patch counters to the global counts.
__device__ __forceinline__ void pix_publish(const KArgs& a, const uint32_t* s_cnt, int32_t y0,
                                            int32_t ch, int32_t x0, int32_t cw) {
  const int32_t py0 = y0 / a.ph, px0 = x0 / a.pw;
  const int32_t npy = (y0 + ch - 1) / a.ph - py0 + 1;
  const int32_t npx = (x0 + cw - 1) / a.pw - px0 + 1;
  for (int32_t i = threadIdx.x; i < npy * npx * 3; i += kThreads) {
    int32_t k = i % 3, slot = i / 3;
    int32_t ly = slot / npx, lx = slot - ly * npx;
    uint32_t v = s_cnt[(ly * a.npx_l + lx) * 3 + k];
    uint32_t* dst = &a.hist[((int64_t)(py0 + ly) * a.nx + (px0 + lx)) * 3 + k];
    if (a.pix_store)
      *dst = v;
    else if (v)
      atomicAdd(dst, v);
  }
}

// ---- stores -----------------------------------------------------------------

// Store 4 packed labels of row gy at chip-relative columns [c, c+4); valid_n
// of them (0..4) lie inside the chip.
__device__ __forceinline__ void store_labels(const KArgs& a, int32_t gy, int32_t gx, int valid_n,
                                             uint32_t packed) {
  uint8_t* dst = a.labels + (int64_t)gy * a.lpitch + gx;
  if (valid_n == 4 && a.label_vec) {
    *(uint32_t*)dst = packed;
  } else {
    for (int j = 0; j < valid_n; ++j) dst[j] = (uint8_t)(packed >> (8 * j));
  }
}

// ---- filter = 1 -------------------------------------------------------------

struct FilterLds {
  uint32_t hist[256 * kCopies];
  uint32_t hsum[256];
  uint32_t cnt[kMaxPatchSlots * 3];
  uint8_t lut[256];
};

// Phase 1 for one wave: walk 34 rows, median, rescale, histogram, keep the
// packed 8-bit medians in vm[].
template <typename T, bool VEC, bool FAST24>
__device__ __forceinline__ void filter_phase1(const KArgs& a, FilterLds& s, int32_t y0, int32_t x0,
                                              int32_t ch, int32_t cw, int wave, int lane,
                                              uint32_t vm[kRowsPerWave]) {
  const bool down = (wave & 1) == 0;
  const int32_t wy0 = wave * kRowsPerWave;
  const int32_t gx = x0 + 4 * lane;

  // input row of walk step s (0..33): chip row -1..32 (down) or 32..-1 (up)
  auto row_of = [&](int st) -> int32_t {
    int32_t r = down ? st - 1 : kRowsPerWave - st;
    return min(max(y0 + wy0 + r, 0), a.H - 1);
  };

  // Halo columns of the chip, one value per walk step held by lane `step`.
  int32_t hstep = min(lane, kRowsPerWave + 1);
  uint32_t halo_l = max_bands_at<T>(a, row_of(hstep), x0 - 1);
  uint32_t halo_r = max_bands_at<T>(a, row_of(hstep), x0 + 4 * 64);

  // columns of this lane that lie inside the chip
  const int valid_cols = min(max(cw - 4 * lane, 0), 4);
  const uint32_t copy = (uint32_t)(lane & (kCopies - 1));

  Raw<T, VEC> ring[kPrefetch];
#pragma unroll
  for (int p = 0; p < kPrefetch; ++p) load_raw<T, VEC>(a, row_of(p), gx, ring[p]);

  uint32_t w0[6], w1[6], w2[6];  // rows at steps s-2, s-1, s: [left, 4 own, right]

#pragma unroll
  for (int st = 0; st < kRowsPerWave + 2; ++st) {
    uint32_t x[4];
    max_bands<T, VEC>(ring[st % kPrefetch], x);
    if (st + kPrefetch < kRowsPerWave + 2)
      load_raw<T, VEC>(a, row_of(st + kPrefetch), gx, ring[st % kPrefetch]);

    uint32_t hl = (uint32_t)__builtin_amdgcn_readlane((int)halo_l, st);
    uint32_t hr = (uint32_t)__builtin_amdgcn_readlane((int)halo_r, st);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      w0[c] = w1[c];
      w1[c] = w2[c];
    }
    w2[0] = from_left(x[3], hl);
    w2[1] = x[0];
    w2[2] = x[1];
    w2[3] = x[2];
    w2[4] = x[3];
    w2[5] = from_right(x[0], hr);
    if (st < 2) continue;

    // output row of this step (chip-relative)
    const int k = st - 2;
    const int32_t rout = wy0 + (down ? k : kRowsPerWave - 1 - k);
    const int nvalid = rout < ch ? valid_cols : 0;

    uint32_t lo[6], mi[6], hi[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      lo[c] = min3u(w0[c], w1[c], w2[c]);
      mi[c] = med3u(w0[c], w1[c], w2[c]);
      hi[c] = max3u(w0[c], w1[c], w2[c]);
    }
    uint32_t packed = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t m = med3u(max3u(lo[j], lo[j + 1], lo[j + 2]), med3u(mi[j], mi[j + 1], mi[j + 2]),
                         min3u(hi[j], hi[j + 1], hi[j + 2]));
      uint32_t v = rescale<T>(m, a, FAST24);
      atomicAdd(&s.hist[(v << 5) | copy], j < nvalid ? 1u : 0u);
      packed |= v << (8 * j);
    }
    vm[k] = packed;
  }
}

// Phase 2: exact chip statistics in one wave; writes the class table.
__device__ void filter_phase2(const KArgs& a, FilterLds& s, int chip_id, int32_t y0, int32_t x0,
                              int lane) {
  uint32_t h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) h[i] = s.hsum[4 * lane + i];
  uint32_t cl = h[0] + h[1] + h[2] + h[3];
  uint32_t sl = 0;
  uint64_t ql = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t v = 4 * lane + i;
    sl += v * h[i];
    ql += (uint64_t)(v * v) * h[i];
  }
  const uint32_t c_inc = wave_incl_scan(cl, lane);
  const uint32_t s_inc = wave_incl_scan(sl, lane);
  const uint32_t N = (uint32_t)__builtin_amdgcn_readlane((int)c_inc, 63);
  const uint32_t S = (uint32_t)__builtin_amdgcn_readlane((int)s_inc, 63);
  const uint64_t Q = wave_sum64(ql);

  // Otsu over the lane's four split points t = 4*lane + i (t <= 254)
  typedef unsigned __int128 u128;
  bool have = false;
  u128 bnum = 0;
  uint64_t bden = 1;
  uint32_t bt = 0;
  {
    uint32_t w0 = c_inc - cl, s0 = s_inc - sl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = 4 * lane + i;
      w0 += h[i];
      s0 += t * h[i];
      if (t < 255 && w0 > 0 && w0 < N) {
        // (w1*S0 - w0*S1) = N*S0 - w0*S
        int64_t d = (int64_t)N * s0 - (int64_t)w0 * S;
        uint64_t ad = (uint64_t)(d < 0 ? -d : d);
        u128 num = (u128)ad * ad;
        uint64_t den = (uint64_t)w0 * (N - w0);
        if (!have || num * bden > bnum * den) {
          have = true;
          bnum = num;
          bden = den;
          bt = t;
        }
      }
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t on_lo = __shfl_xor((uint64_t)bnum, d);
    uint64_t on_hi = __shfl_xor((uint64_t)(bnum >> 64), d);
    uint64_t oden = __shfl_xor(bden, d);
    uint32_t ot = __shfl_xor(bt, d);
    int ohave = __shfl_xor((int)have, d);
    u128 onum = ((u128)on_hi << 64) | on_lo;
    bool take = false;
    if (ohave) {
      if (!have) {
        take = true;
      } else {
        u128 l = onum * bden, r = bnum * oden;
        take = l > r || (l == r && ot < bt);
      }
    }
    if (take) {
      have = true;
      bnum = onum;
      bden = oden;
      bt = ot;
    }
  }

  bool gate = false;
  if (have) {
    uint64_t var = (uint64_t)N * Q - (uint64_t)S * S;
    gate = (u128)a.eta_den * bnum >= (u128)((uint64_t)a.eta_num * bden) * var;
  }

  // truncation levels at rank k from each tail
  const uint32_t kk = N >> a.clip_shift;
  uint32_t lo_c = 256;
  int32_t hi_c = -1;
  {
    uint32_t cum = c_inc - cl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t v = 4 * lane + i;
      uint32_t before = cum;  // count of values < v
      cum += h[i];
      if (cum > kk && lo_c == 256) lo_c = v;
      if (N - before > kk) hi_c = (int32_t)v;
    }
  }
  const uint32_t lo = wave_min32(lo_c);
  const uint32_t hi = (uint32_t)wave_max32(hi_c);
  const bool stretch = gate && hi > lo;

  // class table over median values m = 4*lane + i
  uint32_t cc0 = 0, cc1 = 0, cc2 = 0, a1c = 256, a2c = 256;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t m = 4 * lane + i;
    uint32_t vc = m;
    if (stretch) {
      uint32_t c = min(max(m, lo), hi);
      vc = ((c - lo) * 255u + (hi - lo) / 2u) / (hi - lo);
    }
    const uint32_t cls = (vc >= a.t1) + (vc >= a.t2);
    s.lut[m] = (uint8_t)cls;
    cc0 += cls == 0 ? h[i] : 0;
    cc1 += cls == 1 ? h[i] : 0;
    cc2 += cls == 2 ? h[i] : 0;
    if (cls >= 1) a1c = min(a1c, m);
    if (cls >= 2) a2c = min(a2c, m);
  }
  cc0 = wave_sum32(cc0);
  cc1 = wave_sum32(cc1);
  cc2 = wave_sum32(cc2);
  const uint32_t a1 = wave_min32(a1c), a2 = wave_min32(a2c);

  if (lane == 0) {
    if (a.chips) {
      sil_chip_info ci;
      ci.t = have ? (int32_t)bt : -1;
      ci.lo = (uint8_t)lo;
      ci.hi = (uint8_t)hi;
      ci.gate = gate;
      ci.stretch = stretch;
      ci.a1 = (uint16_t)a1;
      ci.a2 = (uint16_t)a2;
      a.chips[chip_id] = ci;
    }
    if (a.count_mode == CM_HIST_STORE || a.count_mode == CM_HIST_ATOMIC) {
      const int64_t pidx = ((int64_t)(y0 / a.ph) * a.nx + (x0 / a.pw)) * 3;
      if (a.count_mode == CM_HIST_STORE) {
        a.hist[pidx + 0] = cc0;
        a.hist[pidx + 1] = cc1;
        a.hist[pidx + 2] = cc2;
      } else {
        atomicAdd(&a.hist[pidx + 0], cc0);
        atomicAdd(&a.hist[pidx + 1], cc1);
        atomicAdd(&a.hist[pidx + 2], cc2);
      }
    }
  }
}

template <typename T, bool VEC, bool FAST24>
__global__ __launch_bounds__(kThreads, 4) void k_filter(KArgs a) {
  __shared__ FilterLds s;
  const int b = blockIdx.x;
  const int chip_id = (b & 7) * a.per_xcd + (b >> 3);
  if (chip_id >= a.nchips) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t cy = chip_id / a.ncx, cx = chip_id - cy * a.ncx;
  const int32_t y0 = cy * a.chip, x0 = cx * a.chip;
  const int32_t ch = min(a.chip, a.H - y0), cw = min(a.chip, a.W - x0);
  const bool active = wave * kRowsPerWave < ch;
  const bool pix = a.count_mode >= CM_PIX_LDS;
  const bool pix_lds = a.count_mode == CM_PIX_LDS;

  for (int i = threadIdx.x; i < 256 * kCopies / 4; i += kThreads)
    ((uint4*)s.hist)[i] = make_uint4(0, 0, 0, 0);
  if (pix_lds)
    for (int i = threadIdx.x; i < a.npy_l * a.npx_l * 3; i += kThreads) s.cnt[i] = 0;
  __syncthreads();

  uint32_t vm[kRowsPerWave];
  if (active) {
    // Whole-vector loads need every lane's 4 columns inside the scene.
    if (VEC && x0 + 4 * 64 <= a.W)
      filter_phase1<T, VEC, FAST24>(a, s, y0, x0, ch, cw, wave, lane, vm);
    else
      filter_phase1<T, false, FAST24>(a, s, y0, x0, ch, cw, wave, lane, vm);
  }
  __syncthreads();

  if (threadIdx.x < 256) {
    const uint32_t bin = threadIdx.x;
    uint32_t sum = 0;
#pragma unroll 8
    for (uint32_t c = 0; c < kCopies; ++c) sum += s.hist[(bin << 5) | ((c + bin) & (kCopies - 1))];
    s.hsum[bin] = sum;
  }
  __syncthreads();
  if (wave == 0) filter_phase2(a, s, chip_id, y0, x0, lane);
  __syncthreads();

  if (active) {
    const bool down = (wave & 1) == 0;
    const int32_t wy0 = wave * kRowsPerWave;
    const int valid_cols = min(max(cw - 4 * lane, 0), 4);
    const int32_t gx = x0 + 4 * lane;
    PixCount pc{-1, 0};
    int32_t colkey[4];
    if (pix) {
      const int32_t px_base = pix_lds ? x0 / a.pw : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) colkey[j] = min(gx + j, a.W - 1) / a.pw - px_base;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int32_t rout = wy0 + (down ? k : kRowsPerWave - 1 - k);
      if (rout >= ch) continue;
      const int32_t gy = y0 + rout;
      const uint32_t v = vm[k];
      uint32_t cls[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) cls[j] = s.lut[(v >> (8 * j)) & 0xFFu];
      const uint32_t packed = cls[0] | (cls[1] << 8) | (cls[2] << 16) | (cls[3] << 24);
      if (valid_cols > 0) store_labels(a, gy, gx, valid_cols, packed);
      if (pix) {
        const int32_t py = gy / a.ph - (pix_lds ? y0 / a.ph : 0);
        const int32_t rowkey = py * (pix_lds ? a.npx_l : a.nx);
        for (int j = 0; j < valid_cols; ++j) pix_add(a, s.cnt, pix_lds, pc, rowkey + colkey[j], cls[j]);
      }
    }
    if (pix) pix_flush(a, s.cnt, pix_lds, pc.key, pc.cnt);
  }
  if (pix_lds) {
    __syncthreads();
    pix_publish(a, s.cnt, y0, ch, x0, cw);
  }
}

// ---- filter = 0: thresholds only ----------------------------------------------

template <typename T, bool VEC>
__global__ __launch_bounds__(kThreads, 4) void k_thresh(KArgs a) {
  __shared__ uint32_t s_cnt[kMaxPatchSlots * 3];
  const int b = blockIdx.x;
  const int tile_id = (b & 7) * a.per_xcd + (b >> 3);
  if (tile_id >= a.nchips) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t ty = tile_id / a.ncx, tx = tile_id - ty * a.ncx;
  const int32_t y0 = ty * kTile, x0 = tx * kTile;
  const int32_t ch = min(kTile, a.H - y0), cw = min(kTile, a.W - x0);
  const bool pix_lds = a.count_mode == CM_PIX_LDS;
  if (pix_lds) {
    for (int i = threadIdx.x; i < a.npy_l * a.npx_l * 3; i += kThreads) s_cnt[i] = 0;
    __syncthreads();
  }
  const int32_t wy0 = wave * kRowsPerWave;
  if (wy0 < ch) {
    const int32_t gx = x0 + 4 * lane;
    const int valid_cols = min(max(cw - 4 * lane, 0), 4);
    PixCount pc{-1, 0};
    int32_t colkey[4];
    const int32_t px_base = pix_lds ? x0 / a.pw : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) colkey[j] = min(gx + j, a.W - 1) / a.pw - px_base;
    const bool vec = VEC && x0 + 4 * 64 <= a.W;
    for (int r = 0; r < kRowsPerWave && wy0 + r < ch; ++r) {
      const int32_t gy = y0 + wy0 + r;
      uint32_t x[4];
      if (vec) {
        Raw<T, VEC> raw;
        load_raw<T, VEC>(a, gy, gx, raw);
        max_bands<T, VEC>(raw, x);
      } else {
        Raw<T, false> raw;
        load_raw<T, false>(a, gy, gx, raw);
        max_bands<T, false>(raw, x);
      }
      uint32_t cls[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) cls[j] = (x[j] >= a.X1) + (x[j] >= a.X2);
      const uint32_t packed = cls[0] | (cls[1] << 8) | (cls[2] << 16) | (cls[3] << 24);
      if (valid_cols > 0) store_labels(a, gy, gx, valid_cols, packed);
      const int32_t py = gy / a.ph - (pix_lds ? y0 / a.ph : 0);
      const int32_t rowkey = py * (pix_lds ? a.npx_l : a.nx);
      for (int j = 0; j < valid_cols; ++j) pix_add(a, s_cnt, pix_lds, pc, rowkey + colkey[j], cls[j]);
    }
    pix_flush(a, s_cnt, pix_lds, pc.key, pc.cnt);
  }
  if (pix_lds) {
    __syncthreads();
    pix_publish(a, s_cnt, y0, ch, x0, cw);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- host side ----------------------------------------------------------------

// Host copy of the 16->8-bit rescale, used only to derive kernel constants.
uint32_t host_rescale(uint32_t x, uint32_t d) {
  uint64_t q = ((uint64_t)x * 255u + d / 2u) / d;
  return q > 255u ? 255u : (uint32_t)q;
}

struct RescaleConst {
  uint32_t d = 0, x_sat = 0, half = 0, magic = 0, shift = 0;
  bool fast24 = false;
};

// Division by refl_max as a multiply-shift (Granlund & Montgomery, "Division
// by invariant integers using multiplication", 1994), verified over every
// reachable numerator.
bool derive_rescale(uint32_t d, RescaleConst* rc) {
  static std::mutex mu;
  static RescaleConst cache;
  std::lock_guard<std::mutex> g(mu);
  if (cache.d == d) {
    *rc = cache;
    return true;
  }
  RescaleConst r;
  r.d = d;
  r.half = d / 2u;
  uint32_t xs = 0;
  while (xs < 65535u && host_rescale(xs, d) < 255u) ++xs;
  r.x_sat = xs;
  const uint64_t nmax = (uint64_t)xs * 255u + r.half;
  int nb = 0;
  while ((nmax >> nb) != 0) ++nb;
  int l = 0;
  while ((1ull << l) < d) ++l;
  auto check = [&](uint64_t m, int s) {
    for (uint32_t x = 0; x <= xs; ++x) {
      uint64_t n = (uint64_t)x * 255u + r.half;
      if (((n * m) >> s) != n / d) return false;
    }
    return true;
  };
  // prefer a 24-bit magic (full-rate 24-bit multiplies on the device)
  for (int s = nb + l; s < 64 && !r.fast24; ++s) {
    uint64_t m = ((1ull << s) + d - 1) / d;
    if (m >= (1ull << 24)) break;
    if (nmax < (1ull << 24) && check(m, s)) {
      r.magic = (uint32_t)m;
      r.shift = (uint32_t)s;
      r.fast24 = true;
    }
  }
  if (!r.fast24) {
    int s = nb + l;
    uint64_t m = ((1ull << s) + d - 1) / d;
    if (m >= (1ull << 32) || !check(m, s)) return false;
    r.magic = (uint32_t)m;
    r.shift = (uint32_t)s;
  }
  cache = r;
  *rc = r;
  return true;
}

int v_class_table(const sil_params* p, int cls[256]) {
  for (int v = 0; v < 256; ++v) {
    int n = 0, c = -1;
    for (int k = 0; k < 3; ++k)
      if (p->lo[k][2] <= v && v <= p->hi[k][2]) {
        ++n;
        c = k;
      }
    if (n > 1) return SIL_EINVAL;
    if (n == 0) return SIL_EUNSUPPORTED;
    cls[v] = c;
  }
  return SIL_OK;
}

int validate(int32_t nbands, const int32_t* sel, int32_t H, int32_t W, int64_t pitch,
             int64_t label_pitch, const sil_params* p) {
  if (!p || !sel) return SIL_EINVAL;
  if (p->abi != SIL_ABI_VERSION) return SIL_EINVAL;
  if (p->dtype != SIL_U8 && p->dtype != SIL_U16) return SIL_EINVAL;
  if (p->dtype == SIL_U16 && p->refl_max < 1) return SIL_EINVAL;
  if (p->filter > 1 || p->chip < 1 || p->clip_shift < 1 || p->clip_shift > 31)
    return SIL_EINVAL;
  if (p->eta_den < 1 || p->eta_num > p->eta_den) return SIL_EINVAL;
  if (p->patch_h < 1 || p->patch_w < 1) return SIL_EINVAL;
  if (H < 1 || W < 1 || nbands < 1 || pitch < W || label_pitch < W) return SIL_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (sel[i] < 0 || sel[i] >= nbands) return SIL_EINVAL;
  int cls[256];
  int rc = v_class_table(p, cls);
  if (rc != SIL_OK) return rc;
  for (int k = 0; k < 3; ++k)
    if (p->lo[k][0] != 0 || p->hi[k][0] < 179 || p->lo[k][1] != 0 || p->hi[k][1] != 255)
      return SIL_EUNSUPPORTED;
  for (int v = 1; v < 256; ++v)
    if (cls[v] < cls[v - 1]) return SIL_EUNSUPPORTED;
  if (p->filter == 1 && p->chip > 256) return SIL_EUNSUPPORTED;
  if (p->dtype == SIL_U16 && p->refl_max > 65535) return SIL_EUNSUPPORTED;
  if ((int64_t)nbands * H > INT64_MAX / pitch) return SIL_EUNSUPPORTED;
  if ((int64_t)H > INT64_MAX / label_pitch) return SIL_EUNSUPPORTED;
  return SIL_OK;
}

template <typename T>
void launch_typed(const KArgs& a, bool vec, bool fast24, int filter, int grid,
                  hipStream_t stream) {
  if (filter == 1) {
    if (vec) {
      if (fast24)
        hipLaunchKernelGGL((k_filter<T, true, true>), dim3(grid), dim3(kThreads), 0, stream, a);
      else
        hipLaunchKernelGGL((k_filter<T, true, false>), dim3(grid), dim3(kThreads), 0, stream, a);
    } else {
      if (fast24)
        hipLaunchKernelGGL((k_filter<T, false, true>), dim3(grid), dim3(kThreads), 0, stream, a);
      else
        hipLaunchKernelGGL((k_filter<T, false, false>), dim3(grid), dim3(kThreads), 0, stream, a);
    }
  } else {
    if (vec)
      hipLaunchKernelGGL((k_thresh<T, true>), dim3(grid), dim3(kThreads), 0, stream, a);
    else
      hipLaunchKernelGGL((k_thresh<T, false>), dim3(grid), dim3(kThreads), 0, stream, a);
  }
}

}  // namespace

extern "C" {

void sil_params_default(sil_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->abi = SIL_ABI_VERSION;
  p->dtype = SIL_U8;
  p->refl_max = 10000;
  // section III-B limits, classes ordered by V: water, thin ice, thick ice
  const uint8_t lo[3][3] = {{0, 0, 0}, {0, 0, 31}, {0, 0, 205}};
  const uint8_t hi[3][3] = {{185, 255, 30}, {185, 255, 204}, {185, 255, 255}};
  memcpy(p->lo, lo, sizeof(lo));
  memcpy(p->hi, hi, sizeof(hi));
  p->filter = 1;
  p->chip = 256;
  p->clip_shift = 8;
  p->eta_num = 3;
  p->eta_den = 4;
  p->patch_h = 256;
  p->patch_w = 256;
}

uint32_t sil_abi_version(void) { return SIL_ABI_VERSION; }

int sil_hist_dims(int32_t H, int32_t W, const sil_params* p, int32_t* ny, int32_t* nx) {
  if (!p || !ny || !nx || H < 1 || W < 1 || p->patch_h < 1 || p->patch_w < 1)
    return SIL_EINVAL;
  *ny = (int32_t)(((int64_t)H + p->patch_h - 1) / p->patch_h);
  *nx = (int32_t)(((int64_t)W + p->patch_w - 1) / p->patch_w);
  return SIL_OK;
}

int sil_validate(int32_t nbands, const int32_t sel[3], int32_t H, int32_t W, int64_t pitch,
                 int64_t label_pitch, const sil_params* p) {
  return validate(nbands, sel, H, W, pitch, label_pitch, p);
}

const char* sil_strerror(int code) {
  switch (code) {
    case SIL_OK: return "success";
    case SIL_EINVAL: return "invalid argument";
    case SIL_EUNSUPPORTED: return "unsupported parameters";
    case SIL_EDEVICE: return "HIP launch failure";
    default: return "unknown error";
  }
}

int sil_label(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
              int64_t pitch, const sil_params* p, uint8_t* labels, int64_t label_pitch,
              uint32_t* hist, sil_chip_info* chips, void* stream) {
  if (!scene || !labels || !hist) return SIL_EINVAL;
  int rc = validate(nbands, sel, H, W, pitch, label_pitch, p);
  if (rc != SIL_OK) return rc;

  KArgs a;
  memset(&a, 0, sizeof(a));
  a.scene = scene;
  for (int b = 0; b < 3; ++b) a.off[b] = (int64_t)sel[b] * H * pitch;
  a.pitch = pitch;
  a.H = H;
  a.W = W;
  a.labels = labels;
  a.lpitch = label_pitch;
  a.hist = hist;
  sil_hist_dims(H, W, p, &a.ny, &a.nx);
  a.ph = (int32_t)p->patch_h;
  a.pw = (int32_t)p->patch_w;
  a.chips = p->filter == 1 ? chips : nullptr;
  a.clip_shift = p->clip_shift;
  a.eta_num = p->eta_num;
  a.eta_den = p->eta_den;

  const int32_t tile = p->filter == 1 ? (int32_t)p->chip : kTile;
  a.chip = tile;
  a.ncy = (H + tile - 1) / tile;
  a.ncx = (W + tile - 1) / tile;
  const int64_t nchips = (int64_t)a.ncy * a.ncx;
  if (nchips > (int64_t)INT32_MAX - 8) return SIL_EUNSUPPORTED;
  a.nchips = (int32_t)nchips;
  a.per_xcd = (int32_t)((nchips + 7) / 8);

  int cls[256];
  v_class_table(p, cls);
  a.t1 = 256;
  a.t2 = 256;
  for (int v = 255; v >= 0; --v) {
    if (cls[v] >= 1) a.t1 = (uint32_t)v;
    if (cls[v] >= 2) a.t2 = (uint32_t)v;
  }

  RescaleConst rcst;
  const size_t esize = p->dtype == SIL_U16 ? 2 : 1;
  if (p->dtype == SIL_U16) {
    if (!derive_rescale(p->refl_max, &rcst)) return SIL_EUNSUPPORTED;
    a.x_sat = rcst.x_sat;
    a.half = rcst.half;
    a.magic = rcst.magic;
    a.shift = rcst.shift;
    // raw-value boundaries for filter = 0
    a.X1 = 65536;
    a.X2 = 65536;
    for (uint32_t x = 65536; x-- > 0;) {
      uint32_t v = host_rescale(x, p->refl_max);
      if (v >= a.t1) a.X1 = x;
      if (v >= a.t2) a.X2 = x;
    }
  } else {
    a.X1 = a.t1;
    a.X2 = a.t2;
  }

  // how the per-patch counts are produced
  bool zero_hist;
  if (p->filter == 1 && a.ph == tile && a.pw == tile) {
    a.count_mode = CM_HIST_STORE;
    zero_hist = false;
  } else if (p->filter == 1 && a.ph % tile == 0 && a.pw % tile == 0) {
    a.count_mode = CM_HIST_ATOMIC;
    zero_hist = true;
  } else {
    a.npy_l = (tile - 1) / a.ph + 2;
    a.npx_l = (tile - 1) / a.pw + 2;
    if ((int64_t)a.npy_l * a.npx_l <= kMaxPatchSlots) {
      a.count_mode = CM_PIX_LDS;
      a.pix_store = (tile % a.ph == 0 && tile % a.pw == 0) ? 1u : 0u;
      zero_hist = a.pix_store == 0;
    } else {
      a.count_mode = CM_PIX_GLOBAL;
      zero_hist = true;
    }
  }

  // vector paths need aligned rows and chip origins
  const uintptr_t vbytes = 4 * esize;
  const bool vec = ((uintptr_t)scene % vbytes == 0) && ((pitch * esize) % vbytes == 0) &&
                   (tile % 4 == 0);
  a.label_vec = ((uintptr_t)labels % 4 == 0) && (label_pitch % 4 == 0) && (tile % 4 == 0);

  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (zero_hist) {
    int64_t n = (int64_t)a.ny * a.nx * 3;
    int g = (int)((n + 255) / 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, hist, n, 0u);
  }
  const int grid = a.per_xcd * 8;
  if (p->dtype == SIL_U16)
    launch_typed<uint16_t>(a, vec, rcst.fast24, (int)p->filter, grid, st);
  else
    launch_typed<uint8_t>(a, vec, false, (int)p->filter, grid, st);
  if (hipGetLastError() != hipSuccess) return SIL_EDEVICE;
  return SIL_OK;
}

}  // extern "C"
