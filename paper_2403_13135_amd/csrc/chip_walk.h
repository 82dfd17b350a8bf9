// chip_walk.h -- one wave's walk over 32 rows of a chip of a planar scene:
// V = max(B, G, R) per pixel, the exact 3x3 median with clamped scene borders
// (arXiv 2403.13135, section III-A, noise filtering), the 16->8-bit rescale
// and a per-chip 256-bin histogram in LDS.  Shared by the fused labeller
// (sil.hip) and the median pass of the general labeller (label_ex.hip); each
// includes it once, inside its own anonymous namespace.
//
// A wave owns chip rows [32w, 32w + 32) and lane l columns [4l, 4l + 4).  It
// walks its 34 input rows (one halo row above and below) once, keeping a
// three-row window of V in registers; horizontal neighbours come from the
// adjacent lanes through DPP wave shifts, and the chip's left and right halo
// columns are loaded with every row by lanes 0-31 and 32-63.  Even waves walk
// down and odd waves walk up, so the halo row two adjacent waves share is read
// by both at about the same time.  The rescale is applied after the median:
// order statistics commute with a non-decreasing map.

#ifndef SIL_CHIP_WALK_H
#define SIL_CHIP_WALK_H

#ifndef SIL_PREFETCH
#define SIL_PREFETCH 3
#endif

constexpr int kWalkRows = 32;             // output rows per wave
#ifndef SIL_HIST_COPIES
#define SIL_HIST_COPIES 32
#endif
constexpr int kWalkCopies = SIL_HIST_COPIES;  // LDS histogram copies (copy = lane % copies)
constexpr int kWalkPrefetch = SIL_PREFETCH;  // rows of loads in flight per wave

// The three order statistics as single VOP3 instructions.  Written out so that
// the compiler does not split them into two-operand min/max chains to share
// partial results between neighbouring rows, which costs more issue slots than
// the three-operand forms.
__device__ __forceinline__ uint32_t vmin3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t vmax3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t vmed3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
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

// Raw 4-pixel row segments of the three bands, plus one halo pixel per band
// (lanes 0-31 fetch the chip's left halo column, lanes 32-63 its right one,
// so every halo load instruction touches only two cache lines).  The four
// pixels of a band are packed as they lie in memory: two per 32-bit word for
// 16-bit scenes, four per word for 8-bit ones.
template <typename T>
struct Raw;
template <>
struct Raw<uint16_t> {
  uint2 v[3];
  uint32_t h[3];
};
template <>
struct Raw<uint8_t> {
  uint32_t v[3];
  uint32_t h[3];
};

// max over the three bands, 4 pixels.  PERM: first rearrange the 4 pixels
// by the byte selectors `sel` (v_perm_b32; see Walk).
template <typename T, bool PERM = false>
__device__ __forceinline__ void max_bands(const Raw<T>& r, uint32_t x[4],
                                          const uint32_t* sel = nullptr) {
  if constexpr (sizeof(T) == 2) {
    // two pixels per register: packed 16-bit maxima, then unpack
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    auto pmax = [](uint32_t a, uint32_t b, uint32_t c) {
      const u16x2 m = __builtin_elementwise_max(
          __builtin_elementwise_max(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)),
          __builtin_bit_cast(u16x2, c));
      return __builtin_bit_cast(uint32_t, m);
    };
    uint32_t m01 = pmax(r.v[0].x, r.v[1].x, r.v[2].x);
    uint32_t m23 = pmax(r.v[0].y, r.v[1].y, r.v[2].y);
    if constexpr (PERM) {
      const uint32_t a = __builtin_amdgcn_perm(m23, m01, sel[0]);
      m23 = __builtin_amdgcn_perm(m23, m01, sel[1]);
      m01 = a;
    }
    x[0] = m01 & 0xFFFFu;
    x[1] = m01 >> 16;
    x[2] = m23 & 0xFFFFu;
    x[3] = m23 >> 16;
  } else {
    uint32_t v[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) v[b] = PERM ? __builtin_amdgcn_perm(r.v[b], r.v[b], sel[0]) : r.v[b];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      x[j] = vmax3((v[0] >> (8 * j)) & 0xFFu, (v[1] >> (8 * j)) & 0xFFu, (v[2] >> (8 * j)) & 0xFFu);
  }
}

// Addresses of one wave's walk over a chip whose origin is (y0, x0): 34 input
// rows, chip rows -1..32 of the wave's band (down) or 32..-1 (up), clamped
// into the scene; the lane's four column offsets and its halo column, also
// clamped.  Rows are addressed from the walk's first row in each band: a
// wave-uniform 64-bit base per band plus a 32-bit per-lane offset (the walk
// spans 34 rows; callers refuse pitches for which 34 rows exceed 32 bits), so
// each load is a scalar-base + vector-offset load and the walk keeps few
// scalar registers live.
template <typename T>
struct Walk {
  const char* band[3];  // row `top` of each band
  int32_t base, top, last;
  uint32_t pitch;
  bool down;
  uint32_t coff[4];
  uint32_t hoff;
  // Vector loads (aligned scenes): each lane loads the aligned group of 4
  // columns at vcol, moved left so that it ends inside the scene's padded row
  // (the last group that holds column W-1), and `sel` rearranges the loaded
  // pixels so that column c reads column min(c, W-1), the clamped border.
  // Both are the identity away from the scene's right edge.
  uint32_t vcol;
  uint32_t sel[2];
  // planes: the blue, green and red planes (row 0); pitch in bytes
  __device__ __forceinline__ Walk(const char* const planes[3], int64_t pitch_b, int32_t H,
                                  int32_t W, int32_t y0, int32_t x0, int wave, int lane) {
    down = (wave & 1) == 0;
    base = y0 + wave * kWalkRows;
    last = H - 1;
    top = min(max(base - 1, 0), last);
    pitch = (uint32_t)pitch_b;
#pragma unroll
    for (int b = 0; b < 3; ++b) band[b] = planes[b] + (int64_t)top * pitch_b;
    const int32_t gx = x0 + 4 * lane;
#pragma unroll
    for (int j = 0; j < 4; ++j) coff[j] = (uint32_t)(min(gx + j, W - 1) * (int)sizeof(T));
    hoff = (uint32_t)(min(max(lane < 32 ? x0 - 1 : x0 + 4 * 64, 0), W - 1) * (int)sizeof(T));
    const int32_t g = min(gx, (W - 1) & ~3);  // first column of the loaded group
    vcol = (uint32_t)(g * (int)sizeof(T));
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (uint32_t)(min(gx + j, W - 1) - g);
    if constexpr (sizeof(T) == 2) {
      // byte selectors over {hi word : lo word} of two packed 16-bit pairs
      sel[0] = (2 * o[0]) | ((2 * o[0] + 1) << 8) | ((2 * o[1]) << 16) | ((2 * o[1] + 1) << 24);
      sel[1] = (2 * o[2]) | ((2 * o[2] + 1) << 8) | ((2 * o[3]) << 16) | ((2 * o[3] + 1) << 24);
    } else {
      sel[0] = o[0] | (o[1] << 8) | (o[2] << 16) | (o[3] << 24);
      sel[1] = 0;
    }
  }
  // byte offset, from row `top`, of the input row of walk step st (0..33)
  __device__ __forceinline__ uint32_t roff(int st) const {
    const int32_t r = down ? st - 1 : kWalkRows - st;
    return (uint32_t)(min(max(base + r, 0), last) - top) * pitch;
  }
};

// Walk step st into r.  VEC: one aligned vector per band at vcol (aligned
// scenes; max_bands applies `sel`).  Otherwise element loads at the 4
// (clamped) column offsets, packed the same way.  HALO: also the halo column
// (walks without the median skip it).
template <typename T, bool VEC, bool HALO = true>
__device__ __forceinline__ void load_step(const Walk<T>& wk, int st, Raw<T>& r) {
  const uint32_t ro = wk.roff(st);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const char* rb = wk.band[b];
    if constexpr (VEC) {
      if constexpr (sizeof(T) == 2)
        r.v[b] = *(const uint2*)(rb + (ro + wk.vcol));
      else
        r.v[b] = *(const uint32_t*)(rb + (ro + wk.vcol));
    } else {
      uint32_t e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) e[j] = *(const T*)(rb + (ro + wk.coff[j]));
      if constexpr (sizeof(T) == 2)
        r.v[b] = make_uint2(e[0] | (e[1] << 16), e[2] | (e[3] << 16));
      else
        r.v[b] = e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
    }
    if constexpr (HALO) r.h[b] = *(const T*)(rb + (ro + wk.hoff));
  }
}

// The first kWalkPrefetch rows of a vector walk (the loads it starts with).
template <typename T>
__device__ __forceinline__ void walk_prefetch(const Walk<T>& wk, Raw<T> (&ring)[kWalkPrefetch]) {
#pragma unroll
  for (int p = 0; p < kWalkPrefetch; ++p) load_step<T, true>(wk, p, ring[p]);
}

// One step of a wave's walk: take row `cur` into the three-row window of
// band maxima (horizontal neighbours from the adjacent lanes, the chip's halo
// columns from lanes 0 and 63); from step 2 on, the window's middle row gives
// an output row: 3x3 median, rescale, histogram (hist: kWalkCopies copies of
// 256 bins in LDS, adding inc & rowmask per pixel: 1 for pixels inside the
// chip), and the packed 8-bit medians.
template <typename T, bool PERM, class Rescale>
__device__ __forceinline__ uint32_t walk_row(const Raw<T>& cur, const uint32_t* sel,
                                             uint32_t (&w0)[6], uint32_t (&w1)[6],
                                             uint32_t (&w2)[6], bool out, uint32_t rowmask,
                                             const uint32_t inc[4], uint32_t* hist,
                                             uint32_t hist_lane, const Rescale& rescale) {
  uint32_t x[4];
  max_bands<T, PERM>(cur, x, sel);
  // lane 0 takes the left halo, lane 63 the right one (as the DPP fill value)
  const uint32_t hv = vmax3(cur.h[0], cur.h[1], cur.h[2]);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    w0[c] = w1[c];
    w1[c] = w2[c];
  }
  w2[0] = from_left(x[3], hv);
  w2[1] = x[0];
  w2[2] = x[1];
  w2[3] = x[2];
  w2[4] = x[3];
  w2[5] = from_right(x[0], hv);
  if (!out) return 0;

  uint32_t lo[6], mi[6], hi[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    lo[c] = vmin3(w0[c], w1[c], w2[c]);
    mi[c] = vmed3(w0[c], w1[c], w2[c]);
    hi[c] = vmax3(w0[c], w1[c], w2[c]);
  }
  uint32_t packed = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t m = vmed3(vmax3(lo[j], lo[j + 1], lo[j + 2]), vmed3(mi[j], mi[j + 1], mi[j + 2]),
                       vmin3(hi[j], hi[j + 1], hi[j + 2]));
    uint32_t v = rescale(m);
    atomicAdd(&hist[v * kWalkCopies + hist_lane], inc[j] & rowmask);
    packed |= v << (8 * j);
  }
  return packed;
}

// One wave's whole walk: median, rescale, histogram, and the packed 8-bit
// medians of its 32 rows in vm[] (row k of the band in vm[k] for down walks,
// vm[31 - k] for up walks).  ch, cw: the chip's extent from its origin.
//
// vec (aligned scenes) takes the vector walk, fully unrolled with a 3-row
// prefetch ring that holds the first rows on entry (walk_prefetch); at the
// scene's right edge the loads move left and `sel` clamps the columns.
// Otherwise the element walk: a rolled loop of element loads that waits for
// each row, slower but small, so the kernel carries one unrolled walk.
template <typename T, class Rescale>
__device__ __forceinline__ void walk_wave(const Walk<T>& wk, bool vec, uint32_t* hist,
                                          int32_t ch, int32_t cw, int wave, int lane,
                                          uint32_t vm[kWalkRows],
                                          Raw<T> (&ring)[kWalkPrefetch],
                                          const Rescale& rescale) {
  const bool down = wk.down;
  const int32_t wy0 = wave * kWalkRows;
  // histogram increments of the lane's 4 columns: 1 inside the chip, else 0
  uint32_t inc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) inc[j] = 4 * lane + j < cw ? 1u : 0u;
  const uint32_t hist_lane = (uint32_t)(lane & (kWalkCopies - 1));
  // rows of output step k inside the chip (wave-uniform)
  auto rowmask = [&](int k) { return wy0 + (down ? k : kWalkRows - 1 - k) < ch ? ~0u : 0u; };
  uint32_t w0[6], w1[6] = {0, 0, 0, 0, 0, 0}, w2[6] = {0, 0, 0, 0, 0, 0};

  if (vec) {
#pragma unroll
    for (int st = 0; st < kWalkRows + 2; ++st) {
      const Raw<T> cur = ring[st % kWalkPrefetch];
      if (st + kWalkPrefetch < kWalkRows + 2)
        load_step<T, true>(wk, st + kWalkPrefetch, ring[st % kWalkPrefetch]);
      const uint32_t packed =
          walk_row<T, true>(cur, wk.sel, w0, w1, w2, st >= 2, st >= 2 ? rowmask(st - 2) : 0u,
                            inc, hist, hist_lane, rescale);
      if (st >= 2) vm[st - 2] = packed;
    }
  } else {
#pragma unroll 1
    for (int st = 0; st < kWalkRows + 2; ++st) {
      Raw<T> cur;
      load_step<T, false>(wk, st, cur);
      const uint32_t packed =
          walk_row<T, false>(cur, nullptr, w0, w1, w2, st >= 2,
                             st >= 2 ? rowmask(st - 2) : 0u, inc, hist, hist_lane, rescale);
      if (st >= 2) {
        // static register indices in a rolled loop: shift the medians down
#pragma unroll
        for (int k = 0; k + 1 < kWalkRows; ++k) vm[k] = vm[k + 1];
        vm[kWalkRows - 1] = packed;
      }
    }
  }
}

#endif  // SIL_CHIP_WALK_H
