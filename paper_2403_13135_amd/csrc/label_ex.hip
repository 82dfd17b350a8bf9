// label_ex.hip -- gfx950 kernels and C ABI of the general labeller: the
// variants of the method of arXiv 2403.13135 that the fused labeller
// (sil.hip) does not take.  The operation is stated in include/sil.h
// (sil_label_ex):
//   * the three inRange masks of section III-B on full hue / saturation /
//     value limits (OpenCV 8-bit HSV), emitted as a per-pixel bit mask;
//   * a filter unit of any size up to the whole scene (section III-A
//     filters whole scenes as well as the 256 x 256 chips of section IV);
//   * the filtered colour image c' = c * Vc / V, the U-Net's input in the
//     inference workflow of section III-C.
//
// Three passes over HBM instead of the fused one, because a chip of
// arbitrary size no longer fits one workgroup:
//   A. k_ex_median (filter = 1): blocks own (chip, part) pairs and walk
//      tiles of their chip (16 x 1024, 32 x 512 or 64 x 256 pixels); V = max(B,G,R) of the tile plus a one-pixel
//      halo (clamped at the scene border) is staged in LDS with 8-byte band
//      loads, each thread slides the 3x3 median down four columns (column
//      sorts + median of three triples), writes the 8-bit median plane to the
//      workspace (one word per four pixels) and counts it in an 8-copy LDS
//      histogram; one global atomic per nonzero bin and block.
//   B. k_ex_stats: one wave per chip: exact Otsu with 192-bit cross-
//      multiplied comparisons (chips up to 2^27 pixels), the eta gate, rank-k
//      truncation levels and the stretch, written as a 256-entry table
//      median -> filtered value.
//   C. k_ex_apply: 8 x 1024 tiles, four pixels per thread, row by row with
//      the next row's loads in flight during the current row's work; per
//      pixel the three 8-bit bands, V, the filtered Vc from the chip tables
//      (staged in LDS), H and S, the masks, the filtered colour and per-patch
//      mask counts (per-thread runs, wave-reduced when
//      the wave shares a patch, LDS counters per tile, one global atomic per
//      nonzero counter and tile).
// Divisions by small run-time divisors are exact in float: the hue,
// saturation and colour quotients truncate one fma, (n + 1/2) * (1/d), whose
// error stays inside the margin of the quotient for numerators below 2^20;
// the general rescale uses a float estimate corrected by one integer step.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "sil.h"

namespace {

#include "chip_walk.h"
#include "rescale.h"

constexpr int kThreads = 256;     // threads per block of passes A and C
constexpr int kTR = 16;           // pass A tile rows
constexpr int kTW = 4 * kThreads; // tile columns: 4 per thread
constexpr int kTRC = 8;           // pass C tile rows
constexpr int kMaxTilePatches = 128;
constexpr int kMaxTileChips = 16; // per-chip tables a pass C tile stages in LDS
constexpr int64_t kMaxChipPixels = int64_t(1) << 27;

struct ExArgs {
  const uint8_t* band[3];  // planes sel[0], sel[1], sel[2] (blue, green, red)
  int64_t pitch_b;         // row pitch in bytes
  int32_t H, W;
  int32_t u16;
  uint32_t refl_max, half, sat_n;  // sat_n = 255 * refl_max: first saturating numerator
  float rd;                // 1 / refl_max
  uint32_t magic, shift;   // floor(n / refl_max) = mulhi(n, magic) >> shift below sat_n
  int32_t use_magic;
  // the chip walk's rescale (rescale.h): valid when fast24 is set
  uint32_t x_sat, magic24, shift24;
  int32_t fast24;
  int32_t filter;
  int32_t chip, ncx, nchips;
  int32_t ph, pw, nx;
  int32_t cnt_lds;         // per-tile LDS counters (else per-pixel global atomics)
  uint8_t lo[3][3], hi[3][3];
  uint32_t clip_shift, eta_num, eta_den;
  int32_t in_vec;          // band rows 8-byte (u16) / 4-byte (u8) aligned
  int32_t out_vec;         // mask and colour rows 4-byte aligned
  int32_t lut_lds;         // pass C tiles stage their chips' tables in LDS
  int32_t hs_all;          // every mask admits every hue and saturation
  int64_t vm_pitch;        // row pitch of the median plane (multiple of 128)
  uint8_t* vm;             // workspace: [H][vm_pitch] median plane
  uint32_t* hist;          // workspace: [nchips][256]
  uint8_t* lut;            // workspace: [nchips][256] median -> filtered value
  uint8_t* masks;
  int64_t mask_pitch;
  uint32_t* counts;
  uint8_t* rgb;
  int64_t rgb_pitch;
  sil_chip_info* chips;
};

// floor(n / d) for n < 2^24 and a quotient below 2^20 (rd ~ 1.0f / d to within
// an ulp): the float estimate is within one of the quotient, and one integer
// step corrects it.
__device__ __forceinline__ uint32_t div_small(uint32_t n, uint32_t d, float rd) {
  uint32_t q = (uint32_t)((float)n * rd);
  const int32_t r = (int32_t)n - (int32_t)(q * d);
  return r < 0 ? q - 1 : (r >= (int32_t)d ? q + 1 : q);
}

// floor(n / d) for n < 2^20, given rd within two ulps of 1/d and hrd = rd / 2
// (exact): (n + 1/2) / d sits at least 1/(2d) from either neighbouring
// integer, and the single-rounding product (n + 1/2) * rd is off from it by a
// relative 2^-21.6 at most, which for n < 2^20 is less than that margin; so
// truncation gives the quotient with no correction step.
__device__ __forceinline__ uint32_t div_fma(uint32_t n, float rd, float hrd) {
  return (uint32_t)__builtin_fmaf((float)n, rd, hrd);
}

// 16-bit reflectance to 8 bit: round-half-up of x * 255 / refl_max,
// saturating.  n < 2^24; below the saturation point the quotient is < 255.
template <bool U16>
__device__ __forceinline__ uint32_t to8(uint32_t x, const ExArgs& a) {
  if (!U16) return x;
  const uint32_t n = x * 255u + a.half;
  if (n >= a.sat_n) return 255u;
  return a.use_magic ? __umulhi(n, a.magic) >> a.shift : div_small(n, a.refl_max, a.rd);
}

template <bool U16>
__device__ __forceinline__ uint32_t raw_at(const ExArgs& a, int i, int32_t y, int32_t x) {
  const uint8_t* row = a.band[i] + (int64_t)y * a.pitch_b;
  return U16 ? (uint32_t)((const uint16_t*)row)[x] : (uint32_t)row[x];
}

// V = max over the bands (max commutes with the non-decreasing rescale)
__device__ __forceinline__ uint32_t value_at(const ExArgs& a, int32_t y, int32_t x) {
  if (a.u16) {
    const uint32_t m =
        max(max(raw_at<true>(a, 0, y, x), raw_at<true>(a, 1, y, x)), raw_at<true>(a, 2, y, x));
    return to8<true>(m, a);
  }
  return max(max(raw_at<false>(a, 0, y, x), raw_at<false>(a, 1, y, x)), raw_at<false>(a, 2, y, x));
}

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
  return min(min(a, b), c);
}
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) {
  return max(max(a, b), c);
}
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// ---- pass A: median plane and per-chip histograms ------------------------------

// V of four consecutive pixels (x .. x+3, all inside the row) with one 8-byte
// (u16) or 4-byte (u8) load per band.
__device__ __forceinline__ void value4(const ExArgs& a, int32_t y, int32_t x, uint32_t v[4]) {
  uint32_t m[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const uint8_t* row = a.band[i] + (int64_t)y * a.pitch_b;
    if (a.u16) {
      const uint2 w = *(const uint2*)(row + 2 * (int64_t)x);
      m[0] = max(m[0], w.x & 0xffffu);
      m[1] = max(m[1], w.x >> 16);
      m[2] = max(m[2], w.y & 0xffffu);
      m[3] = max(m[3], w.y >> 16);
    } else {
      const uint32_t w = *(const uint32_t*)(row + x);
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = max(m[j], (w >> (8 * j)) & 255u);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = a.u16 ? to8<true>(m[j], a) : m[j];
}

// Blocks own (chip, part) pairs and walk tiles of their chip: TW columns
// (256, 512 or 1024, the narrowest that spans the chip) by 16 * (1024 / TW)
// rows, so narrow chips keep every thread busy.  The tile's V plus a one-pixel
// halo is staged in LDS (pixel column c at byte c + 4 of its row, so each
// thread's four columns are one aligned word); thread (g, u) then slides the
// 3x3 median down columns 4u .. 4u+3 of rows 16g .. 16g+15.
template <int TW>
__global__ __launch_bounds__(kThreads) void k_ex_median(ExArgs a, int32_t parts) {
  constexpr int RG = kTW / TW;          // row groups
  constexpr int TH = kTR * RG;          // tile rows
  constexpr int WPR = TW / 4 + 2;       // staged words per row
  __shared__ uint32_t svw[TH + 2][WPR];
  __shared__ uint32_t sh[8][256];
  uint8_t* const svb = (uint8_t*)&svw[0][0];
  const int tid = threadIdx.x;
  const int g = tid / (TW / 4), u = tid % (TW / 4);
  for (int i = tid; i < 8 * 256; i += kThreads) (&sh[0][0])[i] = 0;
  const int32_t chip_id = blockIdx.x / parts, part = blockIdx.x % parts;
  const int32_t cy = chip_id / a.ncx, cx = chip_id - cy * a.ncx;
  const int32_t y0 = (int32_t)((int64_t)cy * a.chip), x0 = (int32_t)((int64_t)cx * a.chip);
  const int32_t ch = min(a.chip, a.H - y0), cw = min(a.chip, a.W - x0);
  const int32_t nty = (ch + TH - 1) / TH, ntx = (cw + TW - 1) / TW;
  uint32_t* hc = sh[tid & 7];
  const int32_t c0 = 4 * u;  // this thread's first tile column
  __syncthreads();
  for (int32_t t = part; t < nty * ntx; t += parts) {
    const int32_t ty = y0 + (t / ntx) * TH, tx = x0 + (t % ntx) * TW;
    const int32_t rows = min(TH, y0 + ch - ty), cols = min(TW, x0 + cw - tx);
    // stage tile columns -1 .. cols (clamped to the scene), rows -1 .. rows;
    // row group g stages rows g, g + RG, ...
    const bool vec = a.in_vec && (tx & 3) == 0 && tx + c0 + 3 < a.W && c0 < cols;
#pragma unroll
    for (int k = 0; k < (TH + 2 + RG - 1) / RG; ++k) {
      const int r = g + k * RG;
      if (r < rows + 2) {
        const int32_t y = min(max(ty - 1 + r, 0), a.H - 1);
        if (vec) {
          uint32_t v[4];
          value4(a, y, tx + c0, v);
          svw[r][u + 1] = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
        } else if (c0 <= cols) {
          for (int j = 0; j < 4 && c0 + j <= cols; ++j)
            svb[r * (4 * WPR) + c0 + j + 4] =
                (uint8_t)value_at(a, y, min(tx + c0 + j, a.W - 1));
        }
        if (u == 0) svb[r * (4 * WPR) + 3] = (uint8_t)value_at(a, y, max(tx - 1, 0));
        if (u == 1 && cols == TW)
          svb[r * (4 * WPR) + TW + 4] = (uint8_t)value_at(a, y, min(tx + TW, a.W - 1));
      }
    }
    __syncthreads();
    const int32_t rb = kTR * g;  // this thread's first tile row
    if (c0 < cols && rb < rows) {
      // input columns c0-1 .. c0+4 are bytes 3 .. 8 of words u, u+1, u+2
      auto col6 = [&](int r, uint32_t c[6]) {
        const uint32_t wl = svw[r][u], wm = svw[r][u + 1], wr = svw[r][u + 2];
        c[0] = wl >> 24;
#pragma unroll
        for (int j = 0; j < 4; ++j) c[1 + j] = (wm >> (8 * j)) & 255u;
        c[5] = wr & 255u;
      };
      uint32_t p0[6], p1[6];
      col6(rb, p0);
      col6(rb + 1, p1);
      const int nv = min(4, cols - c0);
      const int nr = min(kTR, rows - rb);
      uint8_t* out = a.vm + (int64_t)(ty + rb) * a.vm_pitch + tx + c0;
      for (int r = 0; r < nr; ++r) {
        uint32_t p2[6], lo3[6], md3[6], hi3[6];
        col6(rb + r + 2, p2);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          lo3[k] = min3u(p0[k], p1[k], p2[k]);
          md3[k] = med3u(p0[k], p1[k], p2[k]);
          hi3[k] = max3u(p0[k], p1[k], p2[k]);
        }
        uint32_t m[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          m[j] = med3u(max3u(lo3[j], lo3[j + 1], lo3[j + 2]),
                       med3u(md3[j], md3[j + 1], md3[j + 2]),
                       min3u(hi3[j], hi3[j + 1], hi3[j + 2]));
        if (nv == 4 && (tx & 3) == 0) {
          __builtin_nontemporal_store(m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24),
                                      (uint32_t*)(out + (int64_t)r * a.vm_pitch));
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < nv) out[(int64_t)r * a.vm_pitch + j] = (uint8_t)m[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nv) atomicAdd(&hc[m[j]], 1u);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          p0[k] = p1[k];
          p1[k] = p2[k];
        }
      }
    }
    __syncthreads();
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) sum += sh[k][tid];
  if (sum) atomicAdd(&a.hist[(int64_t)chip_id * 256 + tid], sum);
}

// Pass A for chips of 128 columns or more: 512-thread workgroups own 256 x 256
// tiles of one chip (a chip of side c has ceil(c/256)^2 of them) and run the
// fused labeller's chip walk over them (chip_walk.h): each wave walks 32 rows
// with a 3-row prefetch ring, medians in registers, a 32-copy LDS histogram.
// The tile's medians are then written to the median plane with nontemporal
// stores, and its histogram is added to the chip's.  Workgroup b serves XCD
// b mod 8, which owns a contiguous run of tiles.
constexpr int kWalkThreads = 512;
constexpr int kWalkTile = kWalkThreads / 64 * kWalkRows;  // 256

template <typename T>
__global__ __launch_bounds__(kWalkThreads, 4) void k_ex_walk(ExArgs a, int32_t tpc, int32_t ntx,
                                                             int32_t per_xcd) {
  __shared__ uint32_t hist[256 * kWalkCopies];
  const int32_t u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= a.nchips * tpc) return;
  const int32_t chip_id = u / tpc, part = u - chip_id * tpc;
  const int32_t cy = chip_id / a.ncx, cx = chip_id - cy * a.ncx;
  const int32_t y0 = cy * a.chip, x0 = cx * a.chip;
  const int32_t ch = min(a.chip, a.H - y0), cw = min(a.chip, a.W - x0);
  const int32_t ty = y0 + (part / ntx) * kWalkTile, tx = x0 + (part % ntx) * kWalkTile;
  const int32_t th = min(kWalkTile, y0 + ch - ty), tw = min(kWalkTile, x0 + cw - tx);
  if (th <= 0 || tw <= 0) return;  // edge chips have fewer tiles (uniform per block)

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool active = wave * kWalkRows < th;
  const bool vec = a.in_vec && (tx & 3) == 0;
  const char* const planes[3] = {(const char*)a.band[0], (const char*)a.band[1],
                                 (const char*)a.band[2]};
  const Walk<T> wk(planes, a.pitch_b, a.H, a.W, ty, tx, wave, lane);
  Raw<T> ring[kWalkPrefetch];
  if (active && vec) walk_prefetch<T>(wk, ring);
  for (int i = threadIdx.x; i < 256 * kWalkCopies / 4; i += kWalkThreads)
    ((uint4*)hist)[i] = make_uint4(0, 0, 0, 0);
  __syncthreads();

  if (active) {
    uint32_t vm[kWalkRows];
    // the rescale by 24-bit multiplies (the host launches this pass for
    // 16-bit scenes only when those constants exist for refl_max)
    walk_wave<T>(wk, vec, hist, th, tw, wave, lane, vm, ring, [&](uint32_t m) {
      if constexpr (sizeof(T) == 1) return m;
      return rescale24(m, a.x_sat, a.half, a.magic24, a.shift24);
    });
    const int32_t wy0 = wave * kWalkRows;
    const int nv = min(max(tw - 4 * lane, 0), 4);
    uint8_t* const col = a.vm + tx + 4 * lane;
#pragma unroll
    for (int k = 0; k < kWalkRows; ++k) {
      const int32_t r = wy0 + (wk.down ? k : kWalkRows - 1 - k);
      if (r >= th || nv == 0) continue;
      uint8_t* const q = col + (int64_t)(ty + r) * a.vm_pitch;
      if (nv == 4 && (tx & 3) == 0) {
        __builtin_nontemporal_store(vm[k], (uint32_t*)q);
      } else {
        for (int j = 0; j < nv; ++j) q[j] = (uint8_t)(vm[k] >> (8 * j));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const uint32_t bin = threadIdx.x;
    uint32_t sum = 0;
#pragma unroll 8
    for (uint32_t k = 0; k < kWalkCopies; ++k)
      sum += hist[bin * kWalkCopies + ((k + bin) & (kWalkCopies - 1))];
    if (sum) atomicAdd(&a.hist[(int64_t)chip_id * 256 + bin], sum);
  }
}

// ---- pass B: per-chip statistics -------------------------------------------------

typedef unsigned __int128 u128;

struct U192 {
  uint64_t w0, w1, w2;
};

__device__ __forceinline__ U192 mul_128_64(u128 a, uint64_t b) {
  const u128 lo = (u128)(uint64_t)a * b;
  const u128 hi = (u128)(uint64_t)(a >> 64) * b;
  const u128 mid = (lo >> 64) + (u128)(uint64_t)hi;
  return U192{(uint64_t)lo, (uint64_t)mid, (uint64_t)(hi >> 64) + (uint64_t)(mid >> 64)};
}

__device__ __forceinline__ int cmp192(const U192& a, const U192& b) {
  if (a.w2 != b.w2) return a.w2 > b.w2 ? 1 : -1;
  if (a.w1 != b.w1) return a.w1 > b.w1 ? 1 : -1;
  if (a.w0 != b.w0) return a.w0 > b.w0 ? 1 : -1;
  return 0;
}

template <typename T>
__device__ __forceinline__ T wave_scan_incl(T v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d);
  return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d));
  return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v = max(v, __shfl_xor(v, d));
  return v;
}

__global__ __launch_bounds__(64) void k_ex_stats(ExArgs a) {
  const int32_t chip = blockIdx.x;
  const int lane = threadIdx.x;
  const uint32_t* hg = a.hist + (int64_t)chip * 256;
  uint32_t h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) h[i] = hg[4 * lane + i];
  const uint32_t cl = h[0] + h[1] + h[2] + h[3];
  uint64_t sl = 0, ql = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t v = 4 * lane + i;
    sl += v * h[i];
    ql += v * v * h[i];
  }
  const uint32_t c_inc = wave_scan_incl(cl, lane);
  const uint64_t s_inc = wave_scan_incl(sl, lane);
  const uint32_t N = __shfl(c_inc, 63);
  const uint64_t S = __shfl(s_inc, 63);
  const uint64_t Q = wave_sum(ql);

  // Otsu over this lane's split points t = 4*lane + i (t <= 254):
  // sigma_B^2 N^2 = D^2 / (w0 w1), D = N*S0 - w0*S
  bool have = false;
  u128 bnum = 0;
  uint64_t bden = 1;
  uint32_t bt = 0;
  {
    uint32_t w0 = c_inc - cl;
    uint64_t s0 = s_inc - sl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t t = 4 * lane + i;
      w0 += h[i];
      s0 += (uint64_t)t * h[i];
      if (t < 255 && w0 > 0 && w0 < N) {
        const int64_t D = (int64_t)((uint64_t)N * s0) - (int64_t)((uint64_t)w0 * S);
        const uint64_t ad = (uint64_t)(D < 0 ? -D : D);
        const u128 num = (u128)ad * ad;
        const uint64_t den = (uint64_t)w0 * (N - w0);
        if (!have || cmp192(mul_128_64(num, bden), mul_128_64(bnum, den)) > 0) {
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
    const uint64_t olo = __shfl_xor((uint64_t)bnum, d);
    const uint64_t ohi = __shfl_xor((uint64_t)(bnum >> 64), d);
    const uint64_t oden = __shfl_xor(bden, d);
    const uint32_t ot = __shfl_xor(bt, d);
    const int ohave = __shfl_xor((int)have, d);
    const u128 onum = ((u128)ohi << 64) | olo;
    bool take = false;
    if (ohave) {
      if (!have) {
        take = true;
      } else {
        const int c = cmp192(mul_128_64(onum, bden), mul_128_64(bnum, oden));
        take = c > 0 || (c == 0 && ot < bt);
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
    const u128 var = (u128)N * Q - (u128)S * S;
    gate = cmp192(mul_128_64(bnum, a.eta_den), mul_128_64(var * bden, a.eta_num)) >= 0;
  }

  // truncation levels: (k+1)-th smallest and largest value, k = N >> clip_shift
  const uint32_t kk = N >> a.clip_shift;
  uint32_t lo_c = 256;
  int32_t hi_c = -1;
  {
    uint32_t cum = c_inc - cl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t v = 4 * lane + i;
      const uint32_t before = cum;
      cum += h[i];
      if (cum > kk && lo_c == 256) lo_c = v;
      if (N - before > kk) hi_c = (int32_t)v;
    }
  }
  const uint32_t lo = wave_min(lo_c);
  const uint32_t hi = (uint32_t)wave_max(hi_c);
  const bool stretch = gate && hi > lo;

  // table median -> filtered value; a1 / a2: smallest median whose filtered
  // value falls (last matching V-interval) in class >= 1 / >= 2
  uint32_t a1c = 256, a2c = 256;
  uint32_t packed = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t m = 4 * lane + i;
    uint32_t vc = m;
    if (stretch) {
      const uint32_t c = min(max(m, lo), hi);
      vc = ((c - lo) * 255u + (hi - lo) / 2u) / (hi - lo);
    }
    packed |= vc << (8 * i);
    int cls = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (a.lo[k][2] <= vc && vc <= a.hi[k][2]) cls = k;
    if (cls >= 1) a1c = min(a1c, m);
    if (cls >= 2) a2c = min(a2c, m);
  }
  ((uint32_t*)(a.lut + (int64_t)chip * 256))[lane] = packed;
  const uint32_t a1 = wave_min(a1c), a2 = wave_min(a2c);
  if (lane == 0 && a.chips) {
    sil_chip_info ci;
    ci.t = have ? (int32_t)bt : -1;
    ci.lo = (uint8_t)lo;
    ci.hi = (uint8_t)hi;
    ci.gate = gate;
    ci.stretch = stretch;
    ci.a1 = (uint16_t)a1;
    ci.a2 = (uint16_t)a2;
    a.chips[chip] = ci;
  }
}

// ---- pass C: masks, filtered colour, counts --------------------------------------

// 24-bit multiply(-add): full-rate forms the compiler does not pick by itself
// when it cannot see that the operands are 8-bit values.
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// 8-bit HSV hue (degrees / 2, 0..179) and saturation (0..255) of (r, g, b),
// rounded half up; red wins a tie for the maximum, then green.  rv = 1 / max(V, 1)
// and trcp[k] = 1 / max(k, 1), to within an ulp; numerators stay below 2^18.
// No branches: V = 0 and d = 0 give zero numerators, hence S = 0 and H = 0.
__device__ __forceinline__ void hue_sat(uint32_t r, uint32_t g, uint32_t b, uint32_t V, float rv,
                                        const float* trcp, uint32_t& H, uint32_t& S) {
  const uint32_t mn = min3u(r, g, b), d = V - mn;
  // S = floor((510 d + V) / (2V)); 1 / (2V) = rv / 2 exactly
  S = div_fma(mad24(d, 510u, V), 0.5f * rv, 0.25f * rv);
  // the sector position plus d (in [0, 6d]) for each possible maximum, then a select
  const uint32_t nr = d + g - b, ng = mad24(d, 3u, b) - r, nb = mad24(d, 5u, r) - g;
  const uint32_t np = V == r ? nr : (V == g ? ng : nb);
  // hue / 2 = floor((60 (np - d) + d) / (2d)), plus 180 to keep the numerator
  // non-negative: 60 np + 301 d
  const uint32_t top = mad24(np, 60u, mul24(d, 301u));
  const float rd2 = 0.5f * trcp[d];
  const uint32_t q = div_fma(top, rd2, 0.5f * rd2);
  H = min(q, q - 180u);  // q is in [150, 330]; below 180 the difference wraps high
}

// Tiles of 8 x 1024 pixels; thread t owns columns 4t .. 4t+3.  All rows'
// loads are issued before any use; the chips' median -> filtered-value tables
// of the tile are staged in LDS (when the tile touches at most kMaxTileChips
// chips, else read from the workspace).
// IN: 0 = 8-bit bands, 1 = 16-bit bands rescaled by to8, 2 = 16-bit bands
// rescaled by the 24-bit multiply-shift (when its constants exist).
// At most 80 VGPRs (six waves per SIMD: six 256-thread workgroups per CU):
// the filter variants otherwise take a few more and drop to five.
template <int IN, bool FILTER, bool HSALL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_ex_apply(
    ExArgs a, int32_t ntx, int64_t ntiles) {
  constexpr bool U16 = IN != 0;
  const auto rescale = [&](uint32_t x) -> uint32_t {
    if (IN == 2) return rescale24(x, a.x_sat, a.half, a.magic24, a.shift24);
    return to8<U16>(x, a);
  };
  __shared__ uint32_t scnt[kMaxTilePatches][3];
  __shared__ uint32_t slut[kMaxTileChips][64];
  // which masks admit each hue, saturation and filtered value: bit c = mask c,
  // and again as a 1 in byte c + 1, so that adding entries counts per mask
  __shared__ uint32_t tH[180], tS[256], tV[256];
  // reciprocals of 0..255 (1 at 0) for the per-pixel quotients
  __shared__ float trcp[256];
  static_assert(kThreads == 256, "one table entry per thread");
  const int tid = threadIdx.x, lane = tid & 63;
  {
    uint32_t bh = 0, bs = 0, bv = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bh |= (uint32_t)(a.lo[c][0] <= tid && tid <= a.hi[c][0]) << c;
      bs |= (uint32_t)(a.lo[c][1] <= tid && tid <= a.hi[c][1]) << c;
      bv |= (uint32_t)(a.lo[c][2] <= tid && tid <= a.hi[c][2]) << c;
    }
    const auto spread = [](uint32_t b) {
      return b | (b & 1u) << 8 | (b & 2u) << 15 | (b & 4u) << 22;
    };
    trcp[tid] = 1.0f / (float)max(tid, 1);
    if (tid < 180) tH[tid] = spread(bh);
    tS[tid] = spread(bs);
    tV[tid] = spread(bv);
  }
  const int32_t c0 = 4 * tid;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int32_t ty = (int32_t)(tile / ntx) * kTRC, tx = (int32_t)(tile % ntx) * kTW;
    const int32_t rows = min(kTRC, a.H - ty), cols = min(kTW, a.W - tx);
    const int32_t nv = max(0, min(4, cols - c0));  // this thread's pixels in the row
    const int32_t x = tx + c0;
    // chips and patches this tile touches
    int32_t cy0 = 0, cx0 = 0, ncx_t = 1;
    if (FILTER && a.lut_lds) {
      cy0 = ty / a.chip;
      cx0 = tx / a.chip;
      ncx_t = (tx + cols - 1) / a.chip - cx0 + 1;
      const int32_t nch = ((ty + rows - 1) / a.chip - cy0 + 1) * ncx_t;
      for (int i = tid; i < nch * 64; i += kThreads) {
        const int32_t k = i >> 6;
        const int64_t chip_id = (int64_t)(cy0 + k / ncx_t) * a.ncx + cx0 + k % ncx_t;
        slut[k][i & 63] = ((const uint32_t*)(a.lut + chip_id * 256))[i & 63];
      }
    }
    int32_t py0 = 0, px0 = 0, npx_t = 0;
    if (a.counts && a.cnt_lds) {
      py0 = ty / a.ph;
      px0 = tx / a.pw;
      npx_t = (tx + cols - 1) / a.pw - px0 + 1;
      const int32_t np = ((ty + rows - 1) / a.ph - py0 + 1) * npx_t;
      for (int i = tid; i < np * 3; i += kThreads) (&scnt[0][0])[i] = 0;
    }
    __syncthreads();

    // this thread's pixels' chip column among the tile's staged tables and
    // patch column among its counters, a byte each (both below 128 when staged;
    // pixels past the edge are masked and never used)
    uint32_t kcol4 = 0, pcol4 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (FILTER && a.lut_lds) kcol4 |= ((uint32_t)((x + j) / a.chip - cx0) & 255u) << (8 * j);
      if (a.counts && a.cnt_lds) pcol4 |= ((uint32_t)((x + j) / a.pw - px0) & 255u) << (8 * j);
    }
    // a thread's counts for its current patch: mask c in byte c + 1 of run (a
    // thread adds at most 4 x kTRC entries per tile, so no byte carries; byte 0
    // sums the entries' mask bits and is ignored)
    static_assert(4 * kTRC * 7 < 256, "per-tile counts must fit a byte");
    int32_t run_key = -1;
    uint32_t packed_run = 0;
    auto flush = [&]() {
      // the counts of this thread's current patch go to LDS; lanes of a wave
      // that share the patch are summed first
      uint32_t run[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) run[c] = (packed_run >> (8 * c + 8)) & 255u;
      const bool uni = __all(run_key == __shfl(run_key, 0));
      if (uni) {
#pragma unroll
        for (int c = 0; c < 3; ++c) run[c] = wave_sum(run[c]);
        if (lane == 0 && run_key >= 0)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (run[c]) atomicAdd(&scnt[run_key][c], run[c]);
      } else if (run_key >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (run[c]) atomicAdd(&scnt[run_key][c], run[c]);
      }
      packed_run = 0;
    };

    // one row's inputs, packed as loaded: the three bands (U16: two words of
    // two pixels each; 8-bit: one word of four) and four median bytes
    struct RowIn {
      uint32_t w[3][2];
      uint32_t vm;
    };
    const bool vec = a.in_vec && nv == 4;
    const auto load_row = [&](int32_t y, RowIn& o) {
#pragma unroll
      for (int i = 0; i < 3; ++i) o.w[i][0] = o.w[i][1] = 0;
      o.vm = 0;
      if (nv <= 0) return;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const uint8_t* row = a.band[i] + (int64_t)y * a.pitch_b;
        if (vec) {
          if (U16) {
            const uint2 w = *(const uint2*)(row + 2 * (int64_t)x);
            o.w[i][0] = w.x;
            o.w[i][1] = w.y;
          } else {
            o.w[i][0] = *(const uint32_t*)(row + x);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < nv) {
              const uint32_t v = raw_at<U16>(a, i, y, x + j);
              if (U16)
                o.w[i][j >> 1] |= v << (16 * (j & 1));
              else
                o.w[i][0] |= v << (8 * j);
            }
        }
      }
      if (FILTER) {
        const uint8_t* vrow = a.vm + (int64_t)y * a.vm_pitch + x;
        if (nv == 4) {
          o.vm = *(const uint32_t*)vrow;
        } else {
          for (int j = 0; j < nv; ++j) o.vm |= (uint32_t)vrow[j] << (8 * j);
        }
      }
    };
    const auto band_px = [](const RowIn& in, int i, int j) -> uint32_t {
      if (U16) return (in.w[i][j >> 1] >> (16 * (j & 1))) & 0xffffu;
      return (in.w[i][0] >> (8 * j)) & 255u;
    };

    // the next row's loads are issued before the current row is computed
    RowIn cur, nxt;
    load_row(ty, cur);
#pragma unroll 1
    for (int r = 0; r < rows; ++r) {
      const int32_t y = ty + r;
      if (r + 1 < rows) load_row(y + 1, nxt);
      const int32_t cyi = FILTER ? y / a.chip : 0;
      uint32_t bits4 = 0, rgbw[3] = {0, 0, 0};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int32_t key = -1;
        uint32_t bits = 0;
        if (j < nv) {
          const uint32_t bl = rescale(band_px(cur, 0, j)), gr = rescale(band_px(cur, 1, j)),
                         rd = rescale(band_px(cur, 2, j));
          const uint32_t V = max3u(bl, gr, rd);
          const float rv = trcp[V];
          uint32_t vc = V;
          if (FILTER) {
            const uint32_t m = (cur.vm >> (8 * j)) & 255u;
            if (a.lut_lds) {
              // a word read: a byte read here and the global one below would
              // be merged into one flat load, which waits on every load in flight
              const int32_t k = (cyi - cy0) * ncx_t + (int32_t)((kcol4 >> (8 * j)) & 255u);
              vc = (slut[k][m >> 2] >> (8 * (m & 3))) & 255u;
            } else {
              const int64_t chip_id = (int64_t)cyi * a.ncx + (x + j) / a.chip;
              vc = a.lut[chip_id * 256 + m];
            }
          }
          if (HSALL) {
            bits = tV[vc];
          } else {
            uint32_t Hh, Ss;
            hue_sat(rd, gr, bl, V, rv, trcp, Hh, Ss);
            bits = tH[Hh] & tS[Ss] & tV[vc];
          }
          // byte 0 of the entry (the mask bits) into byte j of bits4
          bits4 = __builtin_amdgcn_perm(bits, bits4, 0x03020100u + (4u << (8 * j)) - (j << (8 * j)));
          if (a.rgb) {
            // round(c vc / V): numerators below 2^17 (all zero when V = 0)
            const uint32_t cband[3] = {bl, gr, rd};
            const float hrv = 0.5f * rv;
#pragma unroll
            for (int i = 0; i < 3; ++i)
              rgbw[i] |= div_fma(mad24(cband[i], vc, V >> 1), rv, hrv) << (8 * j);
          }
          if (a.counts) {
            if (a.cnt_lds) {
              key = (y / a.ph - py0) * npx_t + (int32_t)((pcol4 >> (8 * j)) & 255u);
            } else {
              uint32_t* cp = a.counts + ((int64_t)(y / a.ph) * a.nx + (x + j) / a.pw) * 3;
#pragma unroll
              for (int c = 0; c < 3; ++c)
                if (bits >> c & 1u) atomicAdd(&cp[c], 1u);
            }
          }
        }
        if (a.counts && a.cnt_lds) {
          // wave-uniform test: every lane takes part in flush()
          if (__any(key != run_key && run_key >= 0 && key >= 0)) flush();
          if (key >= 0) run_key = key;
          packed_run += bits;
        }
      }
      if (nv > 0) {
        uint8_t* mrow = a.masks + (int64_t)y * a.mask_pitch + x;
        if (a.out_vec && nv == 4) {
          __builtin_nontemporal_store(bits4, (uint32_t*)mrow);
        } else {
          for (int j = 0; j < nv; ++j) mrow[j] = (uint8_t)(bits4 >> (8 * j));
        }
        if (a.rgb) {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            uint8_t* crow = a.rgb + ((int64_t)i * a.H + y) * a.rgb_pitch + x;
            if (a.out_vec && nv == 4) {
              __builtin_nontemporal_store(rgbw[i], (uint32_t*)crow);
            } else {
              for (int j = 0; j < nv; ++j) crow[j] = (uint8_t)(rgbw[i] >> (8 * j));
            }
          }
        }
      }
      cur = nxt;
    }
    if (a.counts && a.cnt_lds) {
      flush();
      __syncthreads();
      const int32_t np = ((ty + rows - 1) / a.ph - py0 + 1) * npx_t;
      for (int i = tid; i < np * 3; i += kThreads) {
        const uint32_t v = (&scnt[0][0])[i];
        if (v) {
          const int32_t k = i / 3, c = i - k * 3;
          const int32_t py = py0 + k / npx_t, px = px0 + k % npx_t;
          atomicAdd(&a.counts[((int64_t)py * a.nx + px) * 3 + c], v);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_ex_fill(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---- host ---------------------------------------------------------------------------

int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

// A multiply-shift for floor(n / d) over every numerator the rescale reaches
// below saturation (n = x * 255 + d/2 < 255 * d): the smallest shift whose
// rounded-up 32-bit magic checks out on all of them (Granlund-Montgomery).
bool derive_magic_uncached(uint32_t d, uint32_t* magic, uint32_t* shift) {
  const uint64_t nmax = 255ull * d - 1;
  for (uint32_t s = 0; s < 32; ++s) {
    const uint64_t m = ((1ull << (32 + s)) + d - 1) / d;
    if (m >= (1ull << 32)) break;
    bool ok = true;
    for (uint64_t x = 0; ok && x <= 65535; ++x) {
      const uint64_t n = x * 255 + d / 2;
      if (n > nmax) break;
      ok = ((n * m) >> (32 + s)) == n / d;
    }
    if (ok) {
      *magic = (uint32_t)m;
      *shift = s;
      return true;
    }
  }
  return false;
}

bool derive_magic(uint32_t d, uint32_t* magic, uint32_t* shift) {
  static std::mutex mu;
  static uint32_t cd = 0, cm = 0, cs = 0;
  static bool cok = false;
  std::lock_guard<std::mutex> lock(mu);
  if (cd != d) {
    cok = derive_magic_uncached(d, &cm, &cs);
    cd = d;
  }
  *magic = cm;
  *shift = cs;
  return cok;
}

struct Layout {
  int64_t nchips, vm_pitch, vm, hist, lut, total;
};

Layout layout(int32_t H, int32_t W, const sil_params* p) {
  Layout L{};
  const int64_t C = p->chip;
  L.nchips = ((H + C - 1) / C) * ((W + C - 1) / C);
  if (!p->filter) return L;
  // 128-byte rows: the median plane is written as whole cache lines
  L.vm_pitch = (W + 127) & ~int64_t(127);
  L.vm = 0;
  L.hist = align256((int64_t)H * L.vm_pitch);
  L.lut = align256(L.hist + L.nchips * 256 * 4);
  L.total = L.lut + L.nchips * 256;
  return L;
}

int validate_ex(int32_t nbands, const int32_t sel[3], int32_t H, int32_t W, int64_t pitch,
                int64_t mask_pitch, const sil_params* p) {
  if (!p || !sel) return SIL_EINVAL;
  if (p->abi != SIL_ABI_VERSION) return SIL_EINVAL;
  if (p->dtype != SIL_U8 && p->dtype != SIL_U16) return SIL_EINVAL;
  if (p->dtype == SIL_U16 && p->refl_max < 1) return SIL_EINVAL;
  if (p->filter > 1) return SIL_EINVAL;
  if (p->chip < 1 || p->clip_shift < 1 || p->clip_shift > 31) return SIL_EINVAL;
  if (p->eta_den < 1 || p->eta_num > p->eta_den) return SIL_EINVAL;
  if (p->patch_h < 1 || p->patch_w < 1) return SIL_EINVAL;
  if (H < 1 || W < 1 || pitch < W || mask_pitch < W || nbands < 1) return SIL_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (sel[i] < 0 || sel[i] >= nbands) return SIL_EINVAL;
  if (p->dtype == SIL_U16 && p->refl_max > 65535) return SIL_EUNSUPPORTED;
  if (p->filter == 1) {
    const int64_t ch = std::min<int64_t>(p->chip, H), cw = std::min<int64_t>(p->chip, W);
    if (ch * cw > kMaxChipPixels) return SIL_EUNSUPPORTED;
  }
  // int32 pixel and chip arithmetic in the kernels
  if ((int64_t)H * W > INT32_MAX || (int64_t)nbands * H * pitch > (INT64_MAX >> 2))
    return SIL_EUNSUPPORTED;
  return SIL_OK;
}

}  // namespace

extern "C" {

int sil_label_ex_validate(int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
                          int64_t pitch, int64_t mask_pitch, const sil_params* p) {
  return validate_ex(nbands, sel, H, W, pitch, mask_pitch, p);
}

int sil_label_ex_workspace(int32_t H, int32_t W, const sil_params* p, uint64_t* bytes) {
  if (!p || !bytes || H < 1 || W < 1 || p->chip < 1) return SIL_EINVAL;
  *bytes = (uint64_t)layout(H, W, p).total;
  return SIL_OK;
}

}  // extern "C"

namespace {

// The labelling of sil_label_ex with its workspace given as a device address.
int label_ex(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
             int64_t pitch, const sil_params* p, uint8_t* masks, int64_t mask_pitch,
             uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch, sil_chip_info* chips,
             void* workspace, uint64_t workspace_bytes, void* stream) {
  if (!scene || !masks) return SIL_EINVAL;
  int rc = validate_ex(nbands, sel, H, W, pitch, mask_pitch, p);
  if (rc != SIL_OK) return rc;
  if (rgb && rgb_pitch < W) return SIL_EINVAL;
  const int64_t esz = p->dtype == SIL_U16 ? 2 : 1;
  if (esz == 2 && ((uintptr_t)scene & 1)) return SIL_EINVAL;
  const Layout L = layout(H, W, p);
  if (p->filter && (!workspace || workspace_bytes < (uint64_t)L.total || (uintptr_t)workspace % 16))
    return SIL_EINVAL;
  if (L.nchips > INT32_MAX - 4096) return SIL_EUNSUPPORTED;

  ExArgs a{};
  for (int i = 0; i < 3; ++i)
    a.band[i] = (const uint8_t*)scene + (int64_t)sel[i] * H * pitch * esz;
  a.pitch_b = pitch * esz;
  a.H = H;
  a.W = W;
  a.u16 = esz == 2;
  a.refl_max = p->refl_max;
  a.half = p->refl_max / 2u;
  a.sat_n = 255u * p->refl_max;
  a.rd = 1.0f / (float)(p->refl_max ? p->refl_max : 1);
  if (esz == 2) a.use_magic = derive_magic(p->refl_max, &a.magic, &a.shift);
  if (esz == 2) {
    RescaleConst rc;
    if (derive_rescale(p->refl_max, &rc) && rc.fast24) {
      a.x_sat = rc.x_sat;
      a.magic24 = rc.magic;
      a.shift24 = rc.shift;
      a.fast24 = 1;
    }
  }
  a.filter = (int32_t)p->filter;
  a.chip = (int32_t)std::min<int64_t>(p->chip, std::max(H, W));
  a.ncx = (int32_t)((W + (int64_t)p->chip - 1) / p->chip);
  a.nchips = (int32_t)L.nchips;
  a.ph = (int32_t)std::min<int64_t>(p->patch_h, H);
  a.pw = (int32_t)std::min<int64_t>(p->patch_w, W);
  a.nx = (int32_t)((W + (int64_t)p->patch_w - 1) / p->patch_w);
  const int64_t ny = (H + (int64_t)p->patch_h - 1) / p->patch_h;
  // patches and chips an 8 x 1024 tile can touch
  const int64_t tp = (std::min<int64_t>(kTRC, H) - 1) / a.ph + 2;
  const int64_t tq = (std::min<int64_t>(kTW, W) - 1) / a.pw + 2;
  a.cnt_lds = tp * tq <= kMaxTilePatches;
  const int64_t tcy = (std::min<int64_t>(kTRC, H) - 1) / a.chip + 2;
  const int64_t tcx = (std::min<int64_t>(kTW, W) - 1) / a.chip + 2;
  a.lut_lds = tcy * tcx <= kMaxTileChips;
  const int64_t ain = esz == 2 ? 8 : 4;
  a.in_vec = a.pitch_b % ain == 0;
  for (int i = 0; i < 3; ++i) a.in_vec = a.in_vec && (uintptr_t)a.band[i] % ain == 0;
  a.out_vec = mask_pitch % 4 == 0 && (uintptr_t)masks % 4 == 0 &&
              (!rgb || (rgb_pitch % 4 == 0 && (uintptr_t)rgb % 4 == 0));
  memcpy(a.lo, p->lo, sizeof(a.lo));
  a.hs_all = 1;
  for (int c = 0; c < 3; ++c)
    if (p->lo[c][0] != 0 || p->hi[c][0] < 179 || p->lo[c][1] != 0 || p->hi[c][1] != 255)
      a.hs_all = 0;
  memcpy(a.hi, p->hi, sizeof(a.hi));
  a.clip_shift = p->clip_shift;
  a.eta_num = p->eta_num;
  a.eta_den = p->eta_den;
  if (p->filter) {
    a.vm_pitch = L.vm_pitch;
    a.vm = (uint8_t*)workspace + L.vm;
    a.hist = (uint32_t*)((uint8_t*)workspace + L.hist);
    a.lut = (uint8_t*)workspace + L.lut;
  }
  a.masks = masks;
  a.mask_pitch = mask_pitch;
  a.counts = counts;
  a.rgb = rgb;
  a.rgb_pitch = rgb_pitch;
  a.chips = chips;

  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  if (p->filter) {
    const int64_t nh = L.nchips * 256;
    hipLaunchKernelGGL(k_ex_fill, dim3((unsigned)std::min<int64_t>((nh + 255) / 256, 4096)),
                       dim3(256), 0, st, a.hist, nh);
    const int64_t cwid = std::min<int64_t>(a.chip, W);
    if (cwid >= 128 && a.pitch_b * (kWalkRows + 2) <= (int64_t)UINT32_MAX &&
        (!a.u16 || a.fast24)) {
      // the chip walk over 256 x 256 tiles (its 34-row window is addressed
      // with 32-bit offsets)
      const int32_t ntx = (int32_t)((cwid + kWalkTile - 1) / kWalkTile);
      const int32_t nty = (int32_t)((std::min<int64_t>(a.chip, H) + kWalkTile - 1) / kWalkTile);
      const int64_t units = (int64_t)L.nchips * ntx * nty;
      const int32_t per_xcd = (int32_t)((units + 7) / 8);
      const dim3 wgrid((unsigned)(per_xcd * 8));
      if (a.u16)
        hipLaunchKernelGGL(k_ex_walk<uint16_t>, wgrid, dim3(kWalkThreads), 0, st, a, ntx * nty,
                           ntx, per_xcd);
      else
        hipLaunchKernelGGL(k_ex_walk<uint8_t>, wgrid, dim3(kWalkThreads), 0, st, a, ntx * nty,
                           ntx, per_xcd);
      hipLaunchKernelGGL(k_ex_stats, dim3((unsigned)L.nchips), dim3(64), 0, st, a);
    } else {
    // the narrowest tile width that spans a chip
    const int tw = cwid <= 256 ? 256 : (cwid <= 512 ? 512 : kTW);
    const int64_t th = (int64_t)kTR * (kTW / tw);
    const int64_t tiles_per_chip = ((std::min<int64_t>(a.chip, H) + th - 1) / th) *
                                   ((cwid + tw - 1) / tw);
    const int32_t parts = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>((2048 + L.nchips - 1) / L.nchips, tiles_per_chip));
    const dim3 grid((unsigned)(L.nchips * parts));
    if (tw == 256)
      hipLaunchKernelGGL(k_ex_median<256>, grid, dim3(kThreads), 0, st, a, parts);
    else if (tw == 512)
      hipLaunchKernelGGL(k_ex_median<512>, grid, dim3(kThreads), 0, st, a, parts);
    else
      hipLaunchKernelGGL(k_ex_median<kTW>, grid, dim3(kThreads), 0, st, a, parts);
    hipLaunchKernelGGL(k_ex_stats, dim3((unsigned)L.nchips), dim3(64), 0, st, a);
    }
  }
  if (counts) {
    const int64_t nc = ny * a.nx * 3;
    hipLaunchKernelGGL(k_ex_fill, dim3((unsigned)std::min<int64_t>((nc + 255) / 256, 4096)),
                       dim3(256), 0, st, counts, nc);
  }
  const int32_t ntx = (W + kTW - 1) / kTW;
  const int64_t ntiles = (int64_t)((H + kTRC - 1) / kTRC) * ntx;
  const dim3 cgrid((unsigned)std::min<int64_t>(ntiles, 8192));
  const int in = a.u16 ? (a.fast24 ? 2 : 1) : 0;
#define SIL_EX_APPLY(I, F, HS)                                                             \
  if (in == I && a.filter == F && a.hs_all == HS)                                          \
    hipLaunchKernelGGL((k_ex_apply<I, F, HS>), cgrid, dim3(kThreads), 0, st, a, ntx, ntiles);
  SIL_EX_APPLY(2, 1, 1) SIL_EX_APPLY(2, 1, 0) SIL_EX_APPLY(2, 0, 1) SIL_EX_APPLY(2, 0, 0)
  SIL_EX_APPLY(1, 1, 1) SIL_EX_APPLY(1, 1, 0) SIL_EX_APPLY(1, 0, 1) SIL_EX_APPLY(1, 0, 0)
  SIL_EX_APPLY(0, 1, 1) SIL_EX_APPLY(0, 1, 0) SIL_EX_APPLY(0, 0, 1) SIL_EX_APPLY(0, 0, 0)
#undef SIL_EX_APPLY
  return hipGetLastError() == hipSuccess ? SIL_OK : SIL_EDEVICE;
}

// Workspace of sil_label_ex_noalloc: one array per device, held for the life
// of the process.  Host code uses the device address that hipGetSymbolAddress
// returns for the current device, never the array's own name.
constexpr uint64_t kScratchBytes = SIL_LABEL_EX_NOALLOC_MAX;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices];

// The current device's scratch address, looked up once per device.
void* device_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" {

int sil_label_ex(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
                 int64_t pitch, const sil_params* p, uint8_t* masks, int64_t mask_pitch,
                 uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch, sil_chip_info* chips,
                 void* workspace, uint64_t workspace_bytes, void* stream) {
  return label_ex(scene, nbands, sel, H, W, pitch, p, masks, mask_pitch, counts, rgb, rgb_pitch,
                  chips, workspace, workspace_bytes, stream);
}

int sil_label_ex_noalloc(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H,
                         int32_t W, int64_t pitch, const sil_params* p, uint8_t* masks,
                         int64_t mask_pitch, uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch,
                         sil_chip_info* chips, void* stream) {
  if (!scene || !masks) return SIL_EINVAL;
  const int rc = validate_ex(nbands, sel, H, W, pitch, mask_pitch, p);
  if (rc != SIL_OK) return rc;
  const uint64_t need = (uint64_t)layout(H, W, p).total;
  if (need > kScratchBytes) return SIL_EUNSUPPORTED;
  void* ws = nullptr;
  if (need) {
    ws = device_scratch();
    if (!ws) return SIL_EDEVICE;
  }
  return label_ex(scene, nbands, sel, H, W, pitch, p, masks, mask_pitch, counts, rgb, rgb_pitch,
                  chips, ws, need, stream);
}

}  // extern "C"
