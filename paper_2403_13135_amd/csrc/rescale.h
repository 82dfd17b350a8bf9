// rescale.h -- the 16->8-bit reflectance rescale of the labeller (arXiv
// 2403.13135, section III-B: the HSV limits apply to 8-bit values):
// V8 = min(255, floor((x * 255 + refl_max / 2) / refl_max)), round half up of
// x * 255 / refl_max, saturating.  Division by refl_max runs as a
// multiply-shift (Granlund & Montgomery, "Division by invariant integers using
// multiplication", 1994) whose constants the host derives and verifies over
// every reachable numerator.  Shared by sil.hip and label_ex.hip; each
// includes it once, inside its own anonymous namespace.

#ifndef SIL_RESCALE_H
#define SIL_RESCALE_H

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
  // verified constants of the most recent full scales (callers that alternate
  // between a few scales do not re-verify); d = 0 marks an empty slot
  constexpr int kSlots = 16;
  static std::mutex mu;
  static RescaleConst cache[kSlots];
  static int next = 0;
  std::lock_guard<std::mutex> g(mu);
  for (int i = 0; i < kSlots; ++i)
    if (cache[i].d == d && d != 0) {
      *rc = cache[i];
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
  // prefer a 24-bit magic with shift >= 32 (full-rate 24-bit multiplies and
  // the product's high word on the device)
  for (int s = nb + l; s < 64 && !r.fast24; ++s) {
    uint64_t m = ((1ull << s) + d - 1) / d;
    if (m >= (1ull << 24)) break;
    if (s >= 32 && nmax < (1ull << 24) && check(m, s)) {
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
  cache[next] = r;
  next = (next + 1) % kSlots;
  *rc = r;
  return true;
}

// V8 of a 16-bit x with the constants of derive_rescale when fast24 is set
// (numerators below 2^24, magic below 2^24, shift >= 32): a 24-bit
// multiply-add, the high word of a 24 x 24-bit product and a 32-bit shift.
__device__ __forceinline__ uint32_t rescale24(uint32_t x, uint32_t x_sat, uint32_t half,
                                              uint32_t magic, uint32_t shift) {
  uint32_t n;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(n) : "v"(min(x, x_sat)), "v"(255u), "v"(half));
  uint32_t hi;
  asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(hi) : "s"(magic), "v"(n));
  return hi >> (shift - 32u);
}

#endif  // SIL_RESCALE_H
