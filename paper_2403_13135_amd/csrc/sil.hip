// sil.hip -- gfx950 kernels and C ABI of libsil, the sea-ice auto-labeller
// of arXiv 2403.13135 (section III-A "Filtering Out the Thin Clouds and
// Shadows", section III-B "Auto-labeling Method" and "Scaling
// Auto-labeling").  The operation each entry point computes is stated in
// include/sil.h.
//
// Work decomposition (filter = 1): one 512-thread workgroup per chip
// (<= 256 x 256 pixels).  Wave w owns chip rows [32w, 32w + 32); lane l owns
// columns [4l, 4l + 4).
//   phase 1: each wave's walk over its 34 input rows (chip_walk.h): V =
//            max(B,G,R), the exact 3x3 median (column sort + median of three
//            triples), the 16->8-bit rescale (rescale.h; after the median:
//            order statistics commute with a non-decreasing map), a 32-copy
//            LDS histogram (copy = lane % 32, so the 64 lanes of an atomic
//            never share a bank except across the two half-waves), and the
//            8-bit medians kept packed in 32 registers per lane;
//   phase 2: one wave reduces the histogram and runs exact Otsu (a double
//            precision pass, 128-bit cross-multiplied comparisons for
//            near-ties), the eta gate, rank-k truncation levels and the
//            stretch, folded with the class limits into two cut-offs on the
//            median (the class is non-decreasing in it);
//   phase 3: labels from the cut-offs, 4 pixels per 32-bit store, counts.
// Workgroup b labels chip b in raster order.  The hardware deals consecutive
// workgroups to the 8 XCDs in turn, so the chips in flight form one band of
// whole chip rows, and at any moment the waves of the chips of a chip row
// read the same scene rows side by side.
//
// filter = 0 uses a plain streaming kernel over the same tiling.  A batched
// launch (sil_label_batch) covers chip ranges of several scenes, each scene's
// descriptor passed by value in the kernel arguments.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "sil.h"

namespace {

#include "chip_walk.h"
#include "rescale.h"

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kRowsPerWave = kWalkRows;
constexpr int kTile = kWaves * kRowsPerWave;  // 256: chip side handled per workgroup
constexpr int kCopies = kWalkCopies;          // LDS histogram copies
constexpr int kMaxPatchSlots = 1024;          // LDS per-patch counters per workgroup
#ifndef SIL_WAVES_PER_EU
#define SIL_WAVES_PER_EU 4
#endif
// Label stores bypass the L2's write-back order (nontemporal): mixed with the
// chip walk's reads, written-back lines reach HBM in scattered order otherwise.
#ifndef SIL_NT_LABELS
#define SIL_NT_LABELS 1
#endif
constexpr int kPrefetch = kWalkPrefetch;      // rows of loads in flight per wave

constexpr int kMaxBatch = SIL_BATCH_MAX_JOBS; // scenes per batched launch

enum CountMode : uint32_t {
  CM_HIST_STORE = 0,   // patch == chip: counts from the chip histogram, plain store
  CM_HIST_ATOMIC = 1,  // chip tiles the patch: counts from the histogram, atomic add
  CM_PIX_LDS = 2,      // per-pixel counts in LDS, then store or atomic add
  CM_PIX_GLOBAL = 3    // per-pixel counts straight to global atomics
};

// Per-scene arguments.
struct Scene {
  const char* scene;     // planar bands, bytes
  uint8_t* labels;
  uint32_t* hist;
  sil_chip_info* chips;  // nullable
  int64_t off[3];        // byte offsets of the blue, green, red planes
  int64_t pitch;         // input row pitch, bytes
  int64_t lpitch;        // label row pitch, bytes
  int32_t H, W;
  int32_t ny, nx;        // count array
  int32_t ncx, nchips;   // chip grid
  int32_t chip_begin;    // first chip (raster order) labelled by this launch
  uint32_t vec;          // aligned rows: vector loads allowed
  uint32_t label_vec;    // 4-byte label stores allowed
  uint32_t pad;
};

// Arguments shared by every scene of a launch.
struct Shared {
  int32_t chip, ph, pw;
  // 16-bit rescale: V = ((min(x, x_sat) * 255 + half) * magic) >> shift
  uint32_t x_sat, half, magic, shift;
  uint32_t t1, t2;  // first V of class >= 1 and >= 2 (256 if none)
  uint32_t X1, X2;  // the same boundaries on raw input values (filter = 0)
  uint32_t clip_shift, eta_num, eta_den;
  uint32_t count_mode;
  uint32_t pix_store;  // CM_PIX_LDS: 1 plain store (patches nest in chips), 0 atomic
  int32_t npy_l, npx_l;
};

struct Batch {
  Scene sc[kMaxBatch];
  int32_t prefix[kMaxBatch + 1];  // chips of scenes [0, j) in this launch
  int32_t n;
};



#ifndef SIL_XCD_GROUP
#define SIL_XCD_GROUP 4
#endif
constexpr int kXcdGroup = SIL_XCD_GROUP;  // horizontally adjacent chips per XCD visit
constexpr int kDeal = 8 * kXcdGroup;      // workgroups of one dealing round

// Workgroup id -> chip (raster order).  The hardware deals consecutive
// workgroup ids to the 8 XCDs in turn; ids b and b + 8 land on the same XCD.
// Each round of kDeal ids covers kDeal consecutive chips, and XCD x takes
// the kXcdGroup neighbours [x * kXcdGroup, (x + 1) * kXcdGroup) of it, so the
// halo columns between them are fetched into one L2, while the chips in
// flight still form one band of whole chip rows.
__device__ __forceinline__ int work_index() {
  const int b = blockIdx.x;
  const int q = b / kDeal, r = b - q * kDeal;
  return q * kDeal + (r & 7) * kXcdGroup + (r >> 3);
}
inline int deal_grid(int64_t n) { return (int)((n + kDeal - 1) / kDeal * kDeal); }

template <typename T>
__device__ __forceinline__ uint32_t rescale(uint32_t x, const Shared& sh, bool fast24) {
  if constexpr (sizeof(T) == 1) {
    return x;
  } else {
    if (fast24) return rescale24(x, sh.x_sat, sh.half, sh.magic, sh.shift);
    const uint32_t n = min(x, sh.x_sat) * 255u + sh.half;
    return (uint32_t)(((uint64_t)n * sh.magic) >> sh.shift);
  }
}

// ---- loads ------------------------------------------------------------------
//
// Row bases are wave-uniform (scalar registers); each lane adds a 32-bit byte
// offset, so every load is a scalar-base + vector-offset global load.

// Row gy (wave-uniform).  VEC: one aligned vector per band at coff[0] (the
// caller guarantees the 4 columns lie inside the scene).  Otherwise element
// loads at the 4 (clamped) column offsets coff[j], packed the same way.
template <typename T, bool VEC>
__device__ __forceinline__ void load_raw(const Scene& sc, int32_t gy, const uint32_t coff[4],
                                         uint32_t hoff, Raw<T>& r) {
  const char* row = sc.scene + (int64_t)gy * sc.pitch;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const char* rb = row + sc.off[b];
    if constexpr (VEC) {
      if constexpr (sizeof(T) == 2)
        r.v[b] = *(const uint2*)(rb + coff[0]);
      else
        r.v[b] = *(const uint32_t*)(rb + coff[0]);
    } else {
      uint32_t e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) e[j] = *(const T*)(rb + coff[j]);
      if constexpr (sizeof(T) == 2)
        r.v[b] = make_uint2(e[0] | (e[1] << 16), e[2] | (e[3] << 16));
      else
        r.v[b] = e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
    }
    r.h[b] = *(const T*)(rb + hoff);
  }
}

// ---- wave helpers -----------------------------------------------------------

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
// ---- per-pixel class counting (patches that do not align with chips) --------

struct PixCount {
  int32_t key;   // current patch key, -1 none
  uint32_t cnt;  // three 10-bit class counters
};

__device__ __forceinline__ void pix_flush(const Scene& sc, uint32_t* s_cnt, bool lds, int32_t key,
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
      if (c[k]) atomicAdd(&sc.hist[(int64_t)key * 3 + k], c[k]);
  }
}

__device__ __forceinline__ void pix_add(const Scene& sc, uint32_t* s_cnt, bool lds, PixCount& pc,
                                        int32_t key, uint32_t cls) {
  if (key != pc.key) {
    pix_flush(sc, s_cnt, lds, pc.key, pc.cnt);
    pc.key = key;
    pc.cnt = 0;
  }
  pc.cnt += 1u << (10u * cls);
}

// Copy a workgroup's LDS patch counters to the global counts.
__device__ __forceinline__ void pix_publish(const Shared& sh, const Scene& sc,
                                            const uint32_t* s_cnt, int32_t y0, int32_t ch,
                                            int32_t x0, int32_t cw) {
  const int32_t py0 = y0 / sh.ph, px0 = x0 / sh.pw;
  const int32_t npy = (y0 + ch - 1) / sh.ph - py0 + 1;
  const int32_t npx = (x0 + cw - 1) / sh.pw - px0 + 1;
  for (int32_t i = threadIdx.x; i < npy * npx * 3; i += kThreads) {
    int32_t k = i % 3, slot = i / 3;
    int32_t ly = slot / npx, lx = slot - ly * npx;
    uint32_t v = s_cnt[(ly * sh.npx_l + lx) * 3 + k];
    uint32_t* dst = &sc.hist[((int64_t)(py0 + ly) * sc.nx + (px0 + lx)) * 3 + k];
    if (sh.pix_store)
      *dst = v;
    else if (v)
      atomicAdd(dst, v);
  }
}

// Store 4 packed labels at byte offset `off` of a label row; valid_n (0..4)
// of them lie inside the chip.
__device__ __forceinline__ void store_labels(uint8_t* row, uint32_t off, int valid_n, bool vec4,
                                             uint32_t packed) {
  if (valid_n == 4 && vec4) {
    if constexpr (SIL_NT_LABELS)
      __builtin_nontemporal_store(packed, (uint32_t*)(row + off));
    else
      *(uint32_t*)(row + off) = packed;
  } else {
    for (int j = 0; j < valid_n; ++j) row[off + j] = (uint8_t)(packed >> (8 * j));
  }
}

// ---- filter = 1 -------------------------------------------------------------

struct FilterLds {
  uint32_t hist[256 * kCopies];
  uint32_t hsum[256];
  uint32_t cut[2];
  uint32_t cnt[kMaxPatchSlots * 3];
};

// ---- wave primitives for phase 2: DPP within rows of 16 lanes, readlane and
// ballot across rows (no LDS crossbar round trips on the chain) -----------

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_or0(uint32_t x) {
  // lanes whose source lies outside their row of 16 receive 0
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_val(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
// Inclusive prefix sum over the wave: Hillis-Steele within each row of 16
// lanes (row_shr 1, 2, 4, 8), then the totals of the earlier rows.
__device__ __forceinline__ uint32_t wave_scan(uint32_t x, int lane) {
  x += dpp_or0<0x111>(x);
  x += dpp_or0<0x112>(x);
  x += dpp_or0<0x114>(x);
  x += dpp_or0<0x118>(x);
  const uint32_t r0 = lane_val(x, 15), r1 = lane_val(x, 31), r2 = lane_val(x, 47);
  return x + (lane >= 16 ? r0 : 0u) + (lane >= 32 ? r1 : 0u) + (lane >= 48 ? r2 : 0u);
}
__device__ __forceinline__ uint32_t wave_total(uint32_t x, int lane) {
  return lane_val(wave_scan(x, lane), 63);
}
// Maximum over the wave of non-negative doubles.
__device__ __forceinline__ double wave_max_nonneg(double v) {
  auto step = [](double a, auto ctrl) {
    const uint64_t b = __builtin_bit_cast(uint64_t, a);
    const uint32_t lo = dpp_or0<decltype(ctrl)::value>((uint32_t)b);
    const uint32_t hi = dpp_or0<decltype(ctrl)::value>((uint32_t)(b >> 32));
    return fmax(a, __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo));
  };
  v = step(v, std::integral_constant<int, 0x111>{});
  v = step(v, std::integral_constant<int, 0x112>{});
  v = step(v, std::integral_constant<int, 0x114>{});
  v = step(v, std::integral_constant<int, 0x118>{});
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  double m = 0.0;
#pragma unroll
  for (int r = 15; r < 64; r += 16) {
    const uint64_t x = ((uint64_t)lane_val((uint32_t)(b >> 32), r) << 32) | lane_val((uint32_t)b, r);
    m = fmax(m, __builtin_bit_cast(double, x));
  }
  return m;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Phase 2: exact chip statistics in one wave from the chip's 256-bin
// histogram (lane l holds bins 4l..4l+3 in h).  Writes the chip's debug
// record and its counts (patch modes that take them from the histogram), and
// returns the first median value of class >= 1 and of class >= 2 (256 if
// none): the class is non-decreasing in the median, so these two cut-offs
// determine it.
//
// Otsu's threshold is the t maximising (w1*S0 - w0*S1)^2 / (w0*w1), smallest
// t on ties, compared exactly.  A double-precision pass finds it first: the
// ratio is d^2 / den with |d| < 2^41 and den < 2^33 exact in doubles, so the
// computed ratio has a relative error below 2^-51, and every t whose exact
// ratio is the maximum lies within a factor (1 - 2^-40) of the largest
// computed ratio.  When exactly one t passes that test it is the answer;
// otherwise the passing t are compared exactly in 128-bit integers.
__device__ uint2 filter_phase2(const Shared& sh, const Scene& sc, const uint32_t h[4],
                               int chip_id, int32_t y0, int32_t x0, int lane) {
  typedef unsigned __int128 u128;
  const uint32_t cl = h[0] + h[1] + h[2] + h[3];
  uint32_t sl = 0;
  uint64_t ql = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t v = 4 * lane + i;
    sl += v * h[i];
    ql += (uint64_t)(v * v) * h[i];
  }
  const uint32_t c_inc = wave_scan(cl, lane);
  const uint32_t s_inc = wave_scan(sl, lane);
  const uint32_t N = lane_val(c_inc, 63);
  const uint32_t S = lane_val(s_inc, 63);
  // sum of squares in two 32-bit parts: Q < 2^32 * 255^2 / 2^16 per part
  const uint64_t Q = ((uint64_t)wave_total((uint32_t)(ql >> 16), lane) << 16) +
                     wave_total((uint32_t)(ql & 0xFFFFu), lane);

  // Otsu candidates t = 4*lane + i (t <= 254, both classes non-empty)
  bool valid[4];
  int64_t dd[4];
  uint64_t den[4];
  double r[4];
  {
    uint32_t w0 = c_inc - cl, s0 = s_inc - sl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = 4 * lane + i;
      w0 += h[i];
      s0 += t * h[i];
      valid[i] = t < 255 && w0 > 0 && w0 < N;
      // (w1*S0 - w0*S1) = N*S0 - w0*S
      dd[i] = (int64_t)N * s0 - (int64_t)w0 * S;
      den[i] = (uint64_t)w0 * (N - w0);
      const double d = (double)dd[i];
      r[i] = valid[i] ? d * d / (double)den[i] : 0.0;
    }
  }
  const bool have = ballot(valid[0] || valid[1] || valid[2] || valid[3]) != 0;
  u128 bnum = 0;
  uint64_t bden = 1;
  uint32_t bt = 0;
  if (have) {
    const double rmax = wave_max_nonneg(fmax(fmax(r[0], r[1]), fmax(r[2], r[3])));
    const double thr = rmax * (1.0 - 0x1p-40);
    bool cand[4];
    uint32_t nc = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cand[i] = valid[i] && r[i] >= thr;
      nc += cand[i];
    }
    if (wave_total(nc, lane) == 1) {
      const int L = (int)__builtin_ctzll(ballot(nc != 0));
      const int i = cand[0] ? 0 : cand[1] ? 1 : cand[2] ? 2 : 3;
      const uint64_t ad = (uint64_t)(dd[i] < 0 ? -dd[i] : dd[i]);
      const u128 num = (u128)ad * ad;
      bt = 4 * L + lane_val((uint32_t)i, L);
      const uint64_t n_lo = (uint64_t)num, n_hi = (uint64_t)(num >> 64);
      bnum = ((u128)(((uint64_t)lane_val((uint32_t)(n_hi >> 32), L) << 32) |
                     lane_val((uint32_t)n_hi, L))
              << 64) |
             (((uint64_t)lane_val((uint32_t)(n_lo >> 32), L) << 32) | lane_val((uint32_t)n_lo, L));
      bden = ((uint64_t)lane_val((uint32_t)(den[i] >> 32), L) << 32) | lane_val((uint32_t)den[i], L);
    } else {
      // several candidates: exact comparison among them, smallest t on ties
      bool lhave = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (!cand[i]) continue;
        const uint64_t ad = (uint64_t)(dd[i] < 0 ? -dd[i] : dd[i]);
        const u128 num = (u128)ad * ad;
        if (!lhave || num * bden > bnum * den[i]) {
          lhave = true;
          bnum = num;
          bden = den[i];
          bt = 4 * lane + i;
        }
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint64_t on_lo = __shfl_xor((uint64_t)bnum, d);
        const uint64_t on_hi = __shfl_xor((uint64_t)(bnum >> 64), d);
        const uint64_t oden = __shfl_xor(bden, d);
        const uint32_t ot = __shfl_xor(bt, d);
        const int ohave = __shfl_xor((int)lhave, d);
        const u128 onum = ((u128)on_hi << 64) | on_lo;
        bool take = false;
        if (ohave) {
          if (!lhave) {
            take = true;
          } else {
            const u128 l = onum * bden, rr = bnum * oden;
            take = l > rr || (l == rr && ot < bt);
          }
        }
        if (take) {
          lhave = true;
          bnum = onum;
          bden = oden;
          bt = ot;
        }
      }
    }
  }

  bool gate = false;
  if (have) {
    const uint64_t var = (uint64_t)N * Q - (uint64_t)S * S;
    gate = (u128)sh.eta_den * bnum >= (u128)((uint64_t)sh.eta_num * bden) * var;
  }

  // truncation levels at rank k from each tail: lo = min{v : #(<= v) > k},
  // hi = max{v : #(>= v) > k}; the lanes holding such v form a suffix and a
  // prefix of the wave respectively
  const uint32_t kk = N >> sh.clip_shift;
  uint32_t lo_c = 256;
  int32_t hi_c = -1;
  uint32_t ex[4];  // number of values below bin 4*lane + i
  {
    uint32_t cum = c_inc - cl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t v = 4 * lane + i;
      ex[i] = cum;
      if (N - cum > kk) hi_c = (int32_t)v;
      cum += h[i];
      if (cum > kk && lo_c == 256) lo_c = v;
    }
  }
  const uint64_t blo = ballot(lo_c < 256), bhi = ballot(hi_c >= 0);
  const uint32_t lo = blo ? lane_val(lo_c, (int)__builtin_ctzll(blo)) : 256u;
  const uint32_t hi = bhi ? lane_val((uint32_t)hi_c, 63 - (int)__builtin_clzll(bhi)) : 0xFFFFFFFFu;
  const bool stretch = gate && hi > lo;

  // class of each median value m = 4*lane + i; the class is non-decreasing in m
  uint32_t a1c = 256, a2c = 256;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t m = 4 * lane + i;
    uint32_t vc = m;
    if (stretch) {
      const uint32_t c = min(max(m, lo), hi);
      vc = ((c - lo) * 255u + (hi - lo) / 2u) / (hi - lo);
    }
    const uint32_t cls = (vc >= sh.t1) + (vc >= sh.t2);
    if (cls >= 1) a1c = min(a1c, m);
    if (cls >= 2) a2c = min(a2c, m);
  }
  const uint64_t b1 = ballot(a1c < 256), b2 = ballot(a2c < 256);
  const uint32_t a1 = b1 ? lane_val(a1c, (int)__builtin_ctzll(b1)) : 256u;
  const uint32_t a2 = b2 ? lane_val(a2c, (int)__builtin_ctzll(b2)) : 256u;
  // pixels below a median value a: the count before its bin plus the bin's
  // lower part
  auto below = [&](uint32_t a) -> uint32_t {
    if (a >= 256) return N;
    const uint32_t j = a & 3u;
    const uint32_t e = j == 0 ? ex[0] : j == 1 ? ex[1] : j == 2 ? ex[2] : ex[3];
    return lane_val(e, (int)(a >> 2));
  };
  const uint32_t n1 = below(a1), n2 = below(a2);
  const uint32_t cc0 = n1, cc1 = n2 - n1, cc2 = N - n2;

  if (lane == 0) {
    if (sc.chips) {
      sil_chip_info ci;
      ci.t = have ? (int32_t)bt : -1;
      ci.lo = (uint8_t)lo;
      ci.hi = (uint8_t)hi;
      ci.gate = gate;
      ci.stretch = stretch;
      ci.a1 = (uint16_t)a1;
      ci.a2 = (uint16_t)a2;
      sc.chips[chip_id] = ci;
    }
    if (sh.count_mode == CM_HIST_STORE || sh.count_mode == CM_HIST_ATOMIC) {
      const int64_t pidx = ((int64_t)(y0 / sh.ph) * sc.nx + (x0 / sh.pw)) * 3;
      if (sh.count_mode == CM_HIST_STORE) {
        sc.hist[pidx + 0] = cc0;
        sc.hist[pidx + 1] = cc1;
        sc.hist[pidx + 2] = cc2;
      } else {
        atomicAdd(&sc.hist[pidx + 0], cc0);
        atomicAdd(&sc.hist[pidx + 1], cc1);
        atomicAdd(&sc.hist[pidx + 2], cc2);
      }
    }
  }
  return make_uint2(a1, a2);
}

// Labels of 4 packed 8-bit medians: per byte (m >= a1) + (m >= a2), with
// k = (256 - a) in both 16-bit halves; even and odd bytes go through the
// 16-bit halves separately (m + 256 - a < 512, so no carry crosses a half).
__device__ __forceinline__ uint32_t labels_of(uint32_t v, uint32_t k1, uint32_t k2) {
  const uint32_t e = v & 0x00FF00FFu, o = (v >> 8) & 0x00FF00FFu;
  const uint32_t le = (((e + k1) >> 8) & 0x00010001u) + (((e + k2) >> 8) & 0x00010001u);
  const uint32_t lo = (((o + k1) >> 8) & 0x00010001u) + (((o + k2) >> 8) & 0x00010001u);
  return le | (lo << 8);
}

// A chip of a launch: its scene, raster id and extent.
struct ChipAt {
  const Scene* sc;
  int32_t chip_id, y0, x0, ch, cw;
};

__device__ __forceinline__ ChipAt chip_at(const Shared& sh, const Scene& sc, int32_t chip_id) {
  ChipAt c;
  c.sc = &sc;
  c.chip_id = chip_id;
  const int32_t cy = chip_id / sc.ncx, cx = chip_id - cy * sc.ncx;
  c.y0 = cy * sh.chip;
  c.x0 = cx * sh.chip;
  c.ch = min(sh.chip, sc.H - c.y0);
  c.cw = min(sh.chip, sc.W - c.x0);
  return c;
}

__device__ __forceinline__ void zero_hist(FilterLds& s, int t0, int nt) {
  for (int i = t0; i < 256 * kCopies / 4; i += nt) ((uint4*)s.hist)[i] = make_uint4(0, 0, 0, 0);
}

// One chip, all three phases, by the whole workgroup.  PIX: patch counts per
// pixel (patches that do not nest with chips); otherwise from the histogram.
template <typename T, bool FAST24, bool PIX>
__device__ __forceinline__ void filter_chip(const Shared& sh, const ChipAt& c, FilterLds& s) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Scene& sc = *c.sc;
  const int32_t y0 = c.y0, x0 = c.x0, ch = c.ch, cw = c.cw;
  const bool active = wave * kRowsPerWave < ch;
  constexpr bool pix = PIX;
  const bool pix_lds = PIX && sh.count_mode == CM_PIX_LDS;
  // whole-vector loads need aligned rows (the walk clamps the right edge)
  const bool vec = sc.vec != 0;

  // the walk's first rows are in flight while the histogram is cleared
  Raw<T> ring[kPrefetch];
  const char* const planes[3] = {sc.scene + sc.off[0], sc.scene + sc.off[1],
                                 sc.scene + sc.off[2]};
  const Walk<T> wk(planes, sc.pitch, sc.H, sc.W, y0, x0, wave, lane);
  if (active && vec) walk_prefetch<T>(wk, ring);
  zero_hist(s, threadIdx.x, kThreads);
  if (pix_lds)
    for (int i = threadIdx.x; i < sh.npy_l * sh.npx_l * 3; i += kThreads) s.cnt[i] = 0;
  __syncthreads();

  uint32_t vm[kRowsPerWave];
  if (active)
    walk_wave<T>(wk, vec, s.hist, ch, cw, wave, lane, vm, ring,
                 [&](uint32_t m) { return rescale<T>(m, sh, FAST24); });
  __syncthreads();

  if (threadIdx.x < 256) {
    const uint32_t bin = threadIdx.x;
    uint32_t sum = 0;
#pragma unroll 8
    for (uint32_t k = 0; k < kCopies; ++k) sum += s.hist[bin * kCopies + ((k + bin) & (kCopies - 1))];
    s.hsum[bin] = sum;
  }
  __syncthreads();
  if (wave == 0) {
    uint32_t h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = s.hsum[4 * lane + i];
    const uint2 a = filter_phase2(sh, sc, h, c.chip_id, y0, x0, lane);
    if (lane == 0) {
      s.cut[0] = a.x;
      s.cut[1] = a.y;
    }
  }
  __syncthreads();
  const uint32_t k1 = (256u - s.cut[0]) * 0x00010001u, k2 = (256u - s.cut[1]) * 0x00010001u;

  if (active) {
    const bool down = (wave & 1) == 0;
    const int32_t wy0 = wave * kRowsPerWave;
    const int valid_cols = min(max(cw - 4 * lane, 0), 4);
    const int32_t gx = x0 + 4 * lane;
    const uint32_t loff = (uint32_t)gx;
    const bool vec4 = sc.label_vec != 0;
    PixCount pc{-1, 0};
    int32_t colkey[4] = {0, 0, 0, 0};
    if constexpr (pix) {
      const int32_t px_base = pix_lds ? x0 / sh.pw : 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) colkey[j] = min(gx + j, sc.W - 1) / sh.pw - px_base;
    }
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int32_t rout = wy0 + (down ? k : kRowsPerWave - 1 - k);
      if (rout >= ch) continue;
      const int32_t gy = y0 + rout;
      const uint32_t packed = labels_of(vm[k], k1, k2);
      if (valid_cols > 0)
        store_labels(sc.labels + (int64_t)gy * sc.lpitch, loff, valid_cols, vec4, packed);
      if constexpr (pix) {
        const int32_t py = gy / sh.ph - (pix_lds ? y0 / sh.ph : 0);
        const int32_t rowkey = py * (pix_lds ? sh.npx_l : sc.nx);
        for (int j = 0; j < valid_cols; ++j)
          pix_add(sc, s.cnt, pix_lds, pc, rowkey + colkey[j], (packed >> (8 * j)) & 0xFFu);
      }
    }
    if constexpr (pix) pix_flush(sc, s.cnt, pix_lds, pc.key, pc.cnt);
  }
  if (pix_lds) {
    __syncthreads();
    pix_publish(sh, sc, s.cnt, y0, ch, x0, cw);
  }
}

template <typename T, bool FAST24, bool PIX>
__global__ __launch_bounds__(kThreads, SIL_WAVES_PER_EU) void k_filter(Shared sh, Scene sc) {
  __shared__ FilterLds s;
  const int chip_id = work_index();
  if (chip_id >= sc.nchips) return;
  filter_chip<T, FAST24, PIX>(sh, chip_at(sh, sc, chip_id), s);
}

// Chips of up to kMaxBatch scenes in one launch: scene j contributes chips
// [chip_begin, chip_begin + prefix[j+1] - prefix[j]).
template <typename T, bool FAST24>
__global__ __launch_bounds__(kThreads, SIL_WAVES_PER_EU) void k_filter_batch(Shared sh, Batch bt) {
  __shared__ FilterLds s;
  const int i = work_index();
  if (i >= bt.prefix[bt.n]) return;
  int j = 0;
  while (j + 1 < bt.n && bt.prefix[j + 1] <= i) ++j;
  const Scene& sc = bt.sc[j];
  filter_chip<T, FAST24, false>(sh, chip_at(sh, sc, sc.chip_begin + (i - bt.prefix[j])), s);
}

// ---- filter = 0: thresholds only ----------------------------------------------

template <typename T, bool VEC>
__device__ __forceinline__ void thresh_rows(const Shared& sh, const Scene& sc, uint32_t* s_cnt,
                                            int32_t y0, int32_t x0, int32_t ch, int32_t cw,
                                            int wave, int lane, bool pix_lds) {
  const int32_t wy0 = wave * kRowsPerWave;
  const int32_t gx = x0 + 4 * lane;
  const int valid_cols = min(max(cw - 4 * lane, 0), 4);
  uint32_t coff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) coff[j] = (uint32_t)(min(gx + j, sc.W - 1) * (int)sizeof(T));
  const bool vec4 = sc.label_vec != 0;
  PixCount pc{-1, 0};
  int32_t colkey[4];
  const int32_t px_base = pix_lds ? x0 / sh.pw : 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) colkey[j] = min(gx + j, sc.W - 1) / sh.pw - px_base;
  for (int r = 0; r < kRowsPerWave && wy0 + r < ch; ++r) {
    const int32_t gy = y0 + wy0 + r;
    Raw<T> raw;
    load_raw<T, VEC>(sc, gy, coff, coff[0], raw);
    uint32_t x[4];
    max_bands<T>(raw, x);
    uint32_t cls[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) cls[j] = (x[j] >= sh.X1) + (x[j] >= sh.X2);
    const uint32_t packed = cls[0] | (cls[1] << 8) | (cls[2] << 16) | (cls[3] << 24);
    if (valid_cols > 0)
      store_labels(sc.labels + (int64_t)gy * sc.lpitch, (uint32_t)gx, valid_cols, vec4, packed);
    const int32_t py = gy / sh.ph - (pix_lds ? y0 / sh.ph : 0);
    const int32_t rowkey = py * (pix_lds ? sh.npx_l : sc.nx);
    for (int j = 0; j < valid_cols; ++j)
      pix_add(sc, s_cnt, pix_lds, pc, rowkey + colkey[j], cls[j]);
  }
  pix_flush(sc, s_cnt, pix_lds, pc.key, pc.cnt);
}

template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_thresh(Shared sh, Scene sc) {
  __shared__ uint32_t s_cnt[kMaxPatchSlots * 3];
  const int tile_id = work_index();
  if (tile_id >= sc.nchips) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t ty = tile_id / sc.ncx, tx = tile_id - ty * sc.ncx;
  const int32_t y0 = ty * kTile, x0 = tx * kTile;
  const int32_t ch = min(kTile, sc.H - y0), cw = min(kTile, sc.W - x0);
  const bool pix_lds = sh.count_mode == CM_PIX_LDS;
  if (pix_lds) {
    for (int i = threadIdx.x; i < sh.npy_l * sh.npx_l * 3; i += kThreads) s_cnt[i] = 0;
    __syncthreads();
  }
  if (wave * kRowsPerWave < ch) {
    if (sc.vec && x0 + 4 * 64 <= sc.W)
      thresh_rows<T, true>(sh, sc, s_cnt, y0, x0, ch, cw, wave, lane, pix_lds);
    else
      thresh_rows<T, false>(sh, sc, s_cnt, y0, x0, ch, cw, wave, lane, pix_lds);
  }
  if (pix_lds) {
    __syncthreads();
    pix_publish(sh, sc, s_cnt, y0, ch, x0, cw);
  }
}

// filter = 0 with patches that tile-align (each 256 x 256 tile lies in one
// patch): the tile's rows through the chip walk's loads (32 rows per wave,
// 3-row prefetch ring, clamped right edge), the class of each pixel from its
// raw V against the two boundaries, nontemporal label stores, and the tile's
// class totals from per-lane counters.  STORE: the patch is the tile (plain
// stores); otherwise atomics into counts the host cleared.
template <typename T, bool STORE>
__global__ __launch_bounds__(kThreads, 4) void k_thresh_walk(Shared sh, Scene sc) {
  __shared__ uint32_t s_tot[3];
  const int tile_id = work_index();
  if (tile_id >= sc.nchips) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t ty = tile_id / sc.ncx, tx = tile_id - ty * sc.ncx;
  const int32_t y0 = ty * kTile, x0 = tx * kTile;
  const int32_t ch = min(kTile, sc.H - y0), cw = min(kTile, sc.W - x0);
  if (threadIdx.x < 3) s_tot[threadIdx.x] = 0;
  __syncthreads();

  const int32_t wy0 = wave * kRowsPerWave;
  if (wy0 < ch) {
    const char* const planes[3] = {sc.scene + sc.off[0], sc.scene + sc.off[1],
                                   sc.scene + sc.off[2]};
    const Walk<T> wk(planes, sc.pitch, sc.H, sc.W, y0, x0, wave, lane);
    const int nv = min(max(cw - 4 * lane, 0), 4);
    const uint32_t loff = (uint32_t)(x0 + 4 * lane);
    const bool vec4 = sc.label_vec != 0;
    uint32_t cnt = 0;  // three 10-bit class counters (at most 128 pixels per lane)
    // walk steps 1..32 are the band's rows 0..31 (down) or 31..0 (up); no
    // median, so no halo column
    auto row_of = [&](int st) { return wy0 + (wk.down ? st - 1 : kRowsPerWave - st); };
    auto classify = [&](const Raw<T>& cur, auto perm) {
      uint32_t x[4];
      max_bands<T, decltype(perm)::value>(cur, x, wk.sel);
      uint32_t packed = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t c = (x[j] >= sh.X1) + (x[j] >= sh.X2);
        packed |= c << (8 * j);
        cnt += j < nv ? 1u << (10 * c) : 0u;
      }
      return packed;
    };
    if (sc.vec) {
      // the rows' labels are held until the walk's loads are done, then stored
      // (the reads then stream without interleaved stores)
      Raw<T> ring[kPrefetch];
      uint32_t held[kRowsPerWave];
#pragma unroll
      for (int p = 0; p < kPrefetch; ++p) load_step<T, true, false>(wk, 1 + p, ring[p]);
#pragma unroll
      for (int st = 1; st <= kRowsPerWave; ++st) {
        const Raw<T> cur = ring[(st - 1) % kPrefetch];
        if (st + kPrefetch <= kRowsPerWave)
          load_step<T, true, false>(wk, st + kPrefetch, ring[(st - 1) % kPrefetch]);
        held[st - 1] = row_of(st) < ch ? classify(cur, std::true_type{}) : 0u;
      }
#pragma unroll
      for (int st = 1; st <= kRowsPerWave; ++st) {
        const int32_t r = row_of(st);
        if (r < ch && nv > 0)  // r: wave-uniform
          store_labels(sc.labels + (int64_t)(y0 + r) * sc.lpitch, loff, nv, vec4, held[st - 1]);
      }
    } else {
#pragma unroll 1
      for (int st = 1; st <= kRowsPerWave; ++st) {
        Raw<T> cur;
        load_step<T, false, false>(wk, st, cur);
        const int32_t r = row_of(st);
        if (r >= ch) continue;  // wave-uniform
        const uint32_t packed = classify(cur, std::false_type{});
        if (nv > 0) store_labels(sc.labels + (int64_t)(y0 + r) * sc.lpitch, loff, nv, vec4, packed);
      }
    }
    const uint32_t c0 = wave_sum32(cnt & 1023u), c1 = wave_sum32((cnt >> 10) & 1023u),
                   c2 = wave_sum32(cnt >> 20);
    if (lane == 0) {
      atomicAdd(&s_tot[0], c0);
      atomicAdd(&s_tot[1], c1);
      atomicAdd(&s_tot[2], c2);
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    uint32_t* dst = &sc.hist[((int64_t)(y0 / sh.ph) * sc.nx + x0 / sh.pw) * 3 + threadIdx.x];
    if (STORE)
      *dst = s_tot[threadIdx.x];
    else
      atomicAdd(dst, s_tot[threadIdx.x]);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- host side ----------------------------------------------------------------

static_assert(sizeof(Batch) + sizeof(Shared) <= 3584, "kernel arguments must stay under 4 KiB");

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

int validate_params(const sil_params* p) {
  if (!p) return SIL_EINVAL;
  if (p->abi != SIL_ABI_VERSION) return SIL_EINVAL;
  if (p->dtype != SIL_U8 && p->dtype != SIL_U16) return SIL_EINVAL;
  if (p->dtype == SIL_U16 && p->refl_max < 1) return SIL_EINVAL;
  if (p->filter > 1 || p->chip < 1 || p->clip_shift < 1 || p->clip_shift > 31)
    return SIL_EINVAL;
  if (p->eta_den < 1 || p->eta_num > p->eta_den) return SIL_EINVAL;
  if (p->patch_h < 1 || p->patch_w < 1) return SIL_EINVAL;
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
  return SIL_OK;
}

int validate(int32_t nbands, const int32_t* sel, int32_t H, int32_t W, int64_t pitch,
             int64_t label_pitch, const sil_params* p) {
  if (!p || !sel) return SIL_EINVAL;
  int rc = validate_params(p);
  if (rc == SIL_EINVAL) return rc;
  if (H < 1 || W < 1 || nbands < 1 || pitch < W || label_pitch < W) return SIL_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (sel[i] < 0 || sel[i] >= nbands) return SIL_EINVAL;
  if (rc != SIL_OK) return rc;
  const int64_t esize = p->dtype == SIL_U16 ? 2 : 1;
  if ((int64_t)nbands * H > INT64_MAX / (pitch * esize)) return SIL_EUNSUPPORTED;
  if ((int64_t)H > INT64_MAX / label_pitch) return SIL_EUNSUPPORTED;
  if ((int64_t)W * esize + 1024 > INT32_MAX) return SIL_EUNSUPPORTED;  // 32-bit lane offsets
  // a chip walk addresses its 34 rows with 32-bit offsets from its first row
  if (p->filter == 1 && pitch * esize * (kRowsPerWave + 2) > (int64_t)UINT32_MAX)
    return SIL_EUNSUPPORTED;
  return SIL_OK;
}

// Launch-wide constants from validated parameters.  `tile` is the chip side
// (filter = 1) or the streaming tile (filter = 0).
bool derive_shared(const sil_params* p, int32_t tile, Shared* sh, bool* fast24) {
  memset(sh, 0, sizeof(*sh));
  sh->chip = tile;
  sh->ph = (int32_t)p->patch_h;
  sh->pw = (int32_t)p->patch_w;
  sh->clip_shift = p->clip_shift;
  sh->eta_num = p->eta_num;
  sh->eta_den = p->eta_den;
  int cls[256];
  v_class_table(p, cls);
  sh->t1 = 256;
  sh->t2 = 256;
  for (int v = 255; v >= 0; --v) {
    if (cls[v] >= 1) sh->t1 = (uint32_t)v;
    if (cls[v] >= 2) sh->t2 = (uint32_t)v;
  }
  *fast24 = false;
  if (p->dtype == SIL_U16) {
    RescaleConst rc;
    if (!derive_rescale(p->refl_max, &rc)) return false;
    sh->x_sat = rc.x_sat;
    sh->half = rc.half;
    sh->magic = rc.magic;
    sh->shift = rc.shift;
    *fast24 = rc.fast24;
    // raw-value boundaries for filter = 0: the first x whose rescaled value
    // reaches t (the rescale is non-decreasing), 65536 if none
    auto first_reaching = [&](uint32_t t) {
      uint32_t lo = 0, hi = 65536;
      while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (host_rescale(mid, p->refl_max) >= t)
          hi = mid;
        else
          lo = mid + 1;
      }
      return lo;
    };
    sh->X1 = first_reaching(sh->t1);
    sh->X2 = first_reaching(sh->t2);
  } else {
    sh->X1 = sh->t1;
    sh->X2 = sh->t2;
  }
  return true;
}

void fill_scene(const void* scene, const int32_t* sel, int32_t H, int32_t W, int64_t pitch,
                const sil_params* p, uint8_t* labels, int64_t label_pitch, uint32_t* hist,
                sil_chip_info* chips, int32_t tile, Scene* sc) {
  memset(sc, 0, sizeof(*sc));
  const int64_t esize = p->dtype == SIL_U16 ? 2 : 1;
  sc->scene = (const char*)scene;
  sc->labels = labels;
  sc->hist = hist;
  sc->chips = p->filter == 1 ? chips : nullptr;
  for (int b = 0; b < 3; ++b) sc->off[b] = (int64_t)sel[b] * H * pitch * esize;
  sc->pitch = pitch * esize;
  sc->lpitch = label_pitch;
  sc->H = H;
  sc->W = W;
  sil_hist_dims(H, W, p, &sc->ny, &sc->nx);
  sc->ncx = (W + tile - 1) / tile;
  sc->nchips = ((H + tile - 1) / tile) * sc->ncx;
  // vector loads need 4-pixel-aligned rows and chip origins
  const uintptr_t vbytes = 4 * (uintptr_t)esize;
  sc->vec = ((uintptr_t)scene % vbytes == 0) && ((pitch * esize) % (int64_t)vbytes == 0) &&
            (tile % 4 == 0);
  sc->label_vec = ((uintptr_t)labels % 4 == 0) && (label_pitch % 4 == 0) && (tile % 4 == 0);
}

template <typename T>
void launch_single(const Shared& sh, const Scene& sc, bool fast24, int filter,
                   hipStream_t stream) {
  const dim3 grid(deal_grid(sc.nchips)), block(kThreads);
  if (filter == 1) {
    const bool pix = sh.count_mode >= CM_PIX_LDS;
    if (fast24 && !pix)
      hipLaunchKernelGGL((k_filter<T, true, false>), grid, block, 0, stream, sh, sc);
    else if (fast24)
      hipLaunchKernelGGL((k_filter<T, true, true>), grid, block, 0, stream, sh, sc);
    else if (!pix)
      hipLaunchKernelGGL((k_filter<T, false, false>), grid, block, 0, stream, sh, sc);
    else
      hipLaunchKernelGGL((k_filter<T, false, true>), grid, block, 0, stream, sh, sc);
  } else if (sh.count_mode == CM_HIST_STORE) {
    hipLaunchKernelGGL((k_thresh_walk<T, true>), grid, block, 0, stream, sh, sc);
  } else if (sh.count_mode == CM_HIST_ATOMIC) {
    hipLaunchKernelGGL((k_thresh_walk<T, false>), grid, block, 0, stream, sh, sc);
  } else {
    hipLaunchKernelGGL((k_thresh<T>), grid, block, 0, stream, sh, sc);
  }
}

// Colour of a class id as a little-endian (R, G, B) triple in the low 24 bits:
// water green, thin ice blue, thick ice red, anything else black.
__device__ __forceinline__ uint32_t class_rgb(uint32_t c) {
  return (c == 0u ? 0x00ff00u : 0u) | (c == 1u ? 0xff0000u : 0u) | (c == 2u ? 0x0000ffu : 0u);
}

// Four pixels per thread: one 4-byte read of class ids and three 4-byte writes
// of their 12 colour bytes when the rows allow (VEC), else byte by byte.
template <bool VEC>
__global__ void k_render_rgb(const uint8_t* labels, int32_t H, int32_t W, int64_t lpitch,
                             uint8_t* rgb, int64_t rgb_pitch) {
  const int32_t nq = (W + 3) / 4;
  const int64_t n = (int64_t)H * nq;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t y = (int32_t)(i / nq), x = 4 * (int32_t)(i - (int64_t)y * nq);
    const uint8_t* lrow = labels + (int64_t)y * lpitch;
    uint8_t* crow = rgb + (int64_t)y * rgb_pitch + 3 * (int64_t)x;
    if (VEC && x + 4 <= W) {
      const uint32_t l4 = *(const uint32_t*)(lrow + x);
      const uint32_t c0 = class_rgb(l4 & 255u), c1 = class_rgb((l4 >> 8) & 255u),
                     c2 = class_rgb((l4 >> 16) & 255u), c3 = class_rgb(l4 >> 24);
      uint32_t* o = (uint32_t*)crow;
      o[0] = c0 | (c1 << 24);
      o[1] = (c1 >> 8) | (c2 << 16);
      o[2] = (c2 >> 16) | (c3 << 8);
    } else {
      for (int32_t j = 0; j < 4 && x + j < W; ++j) {
        const uint32_t c = class_rgb(lrow[x + j]);
        crow[3 * j] = (uint8_t)c;
        crow[3 * j + 1] = (uint8_t)(c >> 8);
        crow[3 * j + 2] = (uint8_t)(c >> 16);
      }
    }
  }
}

template <typename T>
void launch_batch(const Shared& sh, const Batch& bt, bool fast24, hipStream_t stream) {
  const dim3 grid(deal_grid(bt.prefix[bt.n])), block(kThreads);
  if (fast24)
    hipLaunchKernelGGL((k_filter_batch<T, true>), grid, block, 0, stream, sh, bt);
  else
    hipLaunchKernelGGL((k_filter_batch<T, false>), grid, block, 0, stream, sh, bt);
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

int sil_chip_count(int32_t H, int32_t W, const sil_params* p, int32_t* nchips) {
  if (!p || !nchips || H < 1 || W < 1 || p->chip < 1) return SIL_EINVAL;
  const int64_t n = (((int64_t)H + p->chip - 1) / p->chip) * (((int64_t)W + p->chip - 1) / p->chip);
  if (n > INT32_MAX) return SIL_EUNSUPPORTED;
  *nchips = (int32_t)n;
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

  const int32_t tile = p->filter == 1 ? (int32_t)p->chip : kTile;
  const int64_t nchips = (((int64_t)H + tile - 1) / tile) * (((int64_t)W + tile - 1) / tile);
  if (nchips > (int64_t)INT32_MAX - kDeal) return SIL_EUNSUPPORTED;
  Shared sh;
  bool fast24;
  if (!derive_shared(p, tile, &sh, &fast24)) return SIL_EUNSUPPORTED;
  Scene sc;
  fill_scene(scene, sel, H, W, pitch, p, labels, label_pitch, hist, chips, tile, &sc);

  // how the per-patch counts are produced
  bool zero_hist;
  // (filter = 0: the tile's totals when patches tile-align, from k_thresh_walk;
  // its walk addresses 34 rows with 32-bit offsets, checked for filter = 1 by
  // validate and here for filter = 0)
  const bool walk_ok = p->filter == 1 || sc.pitch * (kRowsPerWave + 2) <= (int64_t)UINT32_MAX;
  if (walk_ok && sh.ph == tile && sh.pw == tile) {
    sh.count_mode = CM_HIST_STORE;
    zero_hist = false;
  } else if (walk_ok && sh.ph % tile == 0 && sh.pw % tile == 0) {
    sh.count_mode = CM_HIST_ATOMIC;
    zero_hist = true;
  } else {
    sh.npy_l = (tile - 1) / sh.ph + 2;
    sh.npx_l = (tile - 1) / sh.pw + 2;
    if ((int64_t)sh.npy_l * sh.npx_l <= kMaxPatchSlots) {
      sh.count_mode = CM_PIX_LDS;
      sh.pix_store = (tile % sh.ph == 0 && tile % sh.pw == 0) ? 1u : 0u;
      zero_hist = sh.pix_store == 0;
    } else {
      sh.count_mode = CM_PIX_GLOBAL;
      zero_hist = true;
    }
  }

  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (zero_hist) {
    int64_t n = (int64_t)sc.ny * sc.nx * 3;
    int g = (int)((n + 255) / 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, hist, n, 0u);
  }
  if (p->dtype == SIL_U16)
    launch_single<uint16_t>(sh, sc, fast24, (int)p->filter, st);
  else
    launch_single<uint8_t>(sh, sc, false, (int)p->filter, st);
  if (hipGetLastError() != hipSuccess) return SIL_EDEVICE;
  return SIL_OK;
}

int sil_label_batch(const sil_job* jobs, int32_t njobs, const sil_params* p, void* stream) {
  if (!jobs || njobs < 1 || njobs > SIL_BATCH_MAX_JOBS) return SIL_EINVAL;
  int rc = validate_params(p);
  if (rc != SIL_OK) return rc;
  if (p->filter != 1 || p->patch_h != p->chip || p->patch_w != p->chip) return SIL_EUNSUPPORTED;
  const int32_t tile = (int32_t)p->chip;
  Shared sh;
  bool fast24;
  if (!derive_shared(p, tile, &sh, &fast24)) return SIL_EUNSUPPORTED;
  sh.count_mode = CM_HIST_STORE;

  Batch bt;
  memset(&bt, 0, sizeof(bt));
  int64_t total = 0;
  for (int32_t j = 0; j < njobs; ++j) {
    const sil_job& jb = jobs[j];
    if (!jb.scene || !jb.labels || !jb.hist) return SIL_EINVAL;
    rc = validate(jb.nbands, jb.sel, jb.H, jb.W, jb.pitch, jb.label_pitch, p);
    if (rc != SIL_OK) return rc;
    fill_scene(jb.scene, jb.sel, jb.H, jb.W, jb.pitch, p, jb.labels, jb.label_pitch, jb.hist,
               jb.chips, tile, &bt.sc[j]);
    if (jb.chip_begin < 0 || jb.chip_count < 1 ||
        (int64_t)jb.chip_begin + jb.chip_count > bt.sc[j].nchips)
      return SIL_EINVAL;
    bt.sc[j].chip_begin = jb.chip_begin;
    bt.prefix[j] = (int32_t)total;
    total += jb.chip_count;
    if (total > (int64_t)INT32_MAX - kDeal) return SIL_EUNSUPPORTED;
  }
  bt.prefix[njobs] = (int32_t)total;
  bt.n = njobs;

  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (p->dtype == SIL_U16)
    launch_batch<uint16_t>(sh, bt, fast24, st);
  else
    launch_batch<uint8_t>(sh, bt, false, st);
  if (hipGetLastError() != hipSuccess) return SIL_EDEVICE;
  return SIL_OK;
}

int sil_render_rgb(const uint8_t* labels, int32_t H, int32_t W, int64_t lpitch, uint8_t* rgb,
                   int64_t rgb_pitch, void* stream) {
  if (!labels || !rgb || H < 1 || W < 1 || lpitch < W || rgb_pitch < 3 * (int64_t)W)
    return SIL_EINVAL;
  const int64_t n = (int64_t)H * ((W + 3) / 4);
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  const bool vec = ((uintptr_t)labels % 4 == 0) && lpitch % 4 == 0 &&
                   ((uintptr_t)rgb % 4 == 0) && rgb_pitch % 4 == 0;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (vec)
    hipLaunchKernelGGL(k_render_rgb<true>, dim3(grid), dim3(256), 0, st, labels, H, W, lpitch,
                       rgb, rgb_pitch);
  else
    hipLaunchKernelGGL(k_render_rgb<false>, dim3(grid), dim3(256), 0, st, labels, H, W, lpitch,
                       rgb, rgb_pitch);
  if (hipGetLastError() != hipSuccess) return SIL_EDEVICE;
  return SIL_OK;
}

}  // extern "C"
