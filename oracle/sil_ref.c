/*
 * sil_ref.c -- CPU oracle of the sea-ice auto-labeller (test infrastructure
 * only; see sil_ref.h for the definition and for who may use it).
 *
 * Written for a reader checking it against the paper by eye: every step runs
 * over the whole scene in the order the definition gives, with no blocking,
 * fusion or reordering.  Arithmetic is integer; products that can exceed 64
 * bits use unsigned __int128.
 */
#include "sil_ref.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- parameters -------------------------------------------------------- */

void sil_ref_params_default(sil_ref_params* p) {
  memset(p, 0, sizeof(*p));
  p->abi = SIL_REF_ABI_VERSION;
  p->dtype = SIL_REF_U8;
  p->refl_max = 10000; /* Sentinel-2 L1C/L2A quantification: 10000 = reflectance 1 */
  /* Section III-B: thick ice (0,0,205)-(185,255,255), thin ice
   * (0,0,31)-(185,255,204), open water (0,0,0)-(185,255,30).  Class ids are
   * ordered by V: 0 water, 1 thin ice, 2 thick ice. */
  const uint8_t lo[3][3] = {{0, 0, 0}, {0, 0, 31}, {0, 0, 205}};
  const uint8_t hi[3][3] = {{185, 255, 30}, {185, 255, 204}, {185, 255, 255}};
  memcpy(p->lo, lo, sizeof(lo));
  memcpy(p->hi, hi, sizeof(hi));
  p->filter = 1;
  p->chip = 256;       /* the 256x256 images of sections III-A and IV-A */
  p->clip_shift = 8;   /* k = N/256 pixels clipped at each tail */
  p->eta_num = 3;      /* gate: eta >= 3/4 */
  p->eta_den = 4;
  p->patch_h = 256;
  p->patch_w = 256;
}

const char* sil_ref_strerror(int code) {
  switch (code) {
    case SIL_REF_OK: return "ok";
    case SIL_REF_EINVAL: return "invalid argument";
    case SIL_REF_EUNSUPPORTED: return "unsupported parameters";
    default: return "unknown error";
  }
}

/* Number of classes whose V-interval holds v. */
static int classes_holding(uint32_t v, const sil_ref_params* p) {
  int n = 0;
  for (int c = 0; c < 3; ++c)
    if (p->lo[c][2] <= v && v <= p->hi[c][2]) ++n;
  return n;
}

int sil_ref_validate(int32_t nbands, const int32_t* sel, int32_t H, int32_t W,
                     int64_t pitch, int64_t label_pitch, const sil_ref_params* p) {
  if (!p || !sel) return SIL_REF_EINVAL;
  if (p->abi != SIL_REF_ABI_VERSION) return SIL_REF_EINVAL;
  if (p->dtype != SIL_REF_U8 && p->dtype != SIL_REF_U16) return SIL_REF_EINVAL;
  if (p->dtype == SIL_REF_U16 && p->refl_max < 1) return SIL_REF_EINVAL;
  if (p->filter > 1) return SIL_REF_EINVAL;
  if (p->chip < 1 || p->clip_shift < 1 || p->clip_shift > 31) return SIL_REF_EINVAL;
  if (p->eta_den < 1 || p->eta_num > p->eta_den) return SIL_REF_EINVAL;
  if (p->patch_h < 1 || p->patch_w < 1) return SIL_REF_EINVAL;
  if (H < 1 || W < 1 || pitch < W || label_pitch < W || nbands < 1) return SIL_REF_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (sel[i] < 0 || sel[i] >= nbands) return SIL_REF_EINVAL;
  /* Section III-B states the three ranges do not intersect. */
  for (uint32_t v = 0; v < 256; ++v)
    if (classes_holding(v, p) > 1) return SIL_REF_EINVAL;
  /* A V value in no range would leave a pixel unlabelled. */
  for (uint32_t v = 0; v < 256; ++v)
    if (classes_holding(v, p) == 0) return SIL_REF_EUNSUPPORTED;
  /* OpenCV 8-bit HSV: H in [0,179], S in [0,255].  Limits that do not span
   * those ranges would make the masks depend on hue/saturation. */
  for (int c = 0; c < 3; ++c)
    if (p->lo[c][0] != 0 || p->hi[c][0] < 179 || p->lo[c][1] != 0 || p->hi[c][1] != 255)
      return SIL_REF_EUNSUPPORTED;
  /* Exact Otsu comparisons below fit 128 bits for chips of at most 256^2. */
  if (p->filter == 1 && p->chip > 256) return SIL_REF_EUNSUPPORTED;
  return SIL_REF_OK;
}

int sil_ref_hist_dims(int32_t H, int32_t W, const sil_ref_params* p, int32_t* ny,
                      int32_t* nx) {
  if (!p || !ny || !nx || H < 1 || W < 1 || p->patch_h < 1 || p->patch_w < 1)
    return SIL_REF_EINVAL;
  *ny = (int32_t)(((int64_t)H + p->patch_h - 1) / p->patch_h);
  *nx = (int32_t)(((int64_t)W + p->patch_w - 1) / p->patch_w);
  return SIL_REF_OK;
}

/* ---- step 1: V plane --------------------------------------------------- */

/* round-half-up of x*255/refl_max, saturating at 255 */
uint8_t sil_ref_rescale(uint32_t x, uint32_t refl_max) {
  uint64_t q = ((uint64_t)x * 255u + refl_max / 2u) / refl_max;
  return (uint8_t)(q > 255u ? 255u : q);
}

void sil_ref_value_plane(const void* scene, int32_t nbands, const int32_t* sel,
                         int32_t H, int32_t W, int64_t pitch, uint32_t dtype,
                         uint32_t refl_max, uint8_t* V) {
  (void)nbands;
  const int64_t plane = (int64_t)H * pitch;
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      uint32_t m = 0;
      for (int i = 0; i < 3; ++i) {
        int64_t idx = sel[i] * plane + (int64_t)y * pitch + x;
        uint32_t v = dtype == SIL_REF_U8 ? ((const uint8_t*)scene)[idx]
                                         : ((const uint16_t*)scene)[idx];
        if (v > m) m = v;
      }
      V[(int64_t)y * W + x] = dtype == SIL_REF_U8 ? (uint8_t)m : sil_ref_rescale(m, refl_max);
    }
}

/* ---- step 3: 3x3 median, clamped border ------------------------------- */

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

void sil_ref_median3x3(const uint8_t* V, int32_t H, int32_t W, uint8_t* Vm) {
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      uint8_t w[9];
      int n = 0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
          w[n++] = V[(int64_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
      /* insertion sort, then the 5th smallest */
      for (int i = 1; i < 9; ++i)
        for (int j = i; j > 0 && w[j - 1] > w[j]; --j) {
          uint8_t t = w[j];
          w[j] = w[j - 1];
          w[j - 1] = t;
        }
      Vm[(int64_t)y * W + x] = w[4];
    }
}

/* ---- step 4: per-chip statistics --------------------------------------- */

uint8_t sil_ref_stretch(uint8_t m, uint8_t lo, uint8_t hi) {
  /* min-max normalisation of [lo,hi] to [0,255] after truncation to
   * [lo,hi]; round half up */
  uint32_t c = m < lo ? lo : (m > hi ? hi : m);
  uint32_t d = (uint32_t)hi - lo;
  return (uint8_t)(((c - lo) * 255u + d / 2u) / d);
}

int sil_ref_class_of(uint8_t vc, const sil_ref_params* p) {
  /* The three inRange masks; hue/saturation limits are vacuous (checked by
   * validation), so mask c holds iff lo_V[c] <= Vc <= hi_V[c]. */
  int label = -1;
  for (int c = 0; c < 3; ++c)
    if (p->lo[c][2] <= vc && vc <= p->hi[c][2]) label = c;
  return label;
}

static uint8_t filtered_value(uint8_t m, const sil_ref_chip_info* info) {
  return info->stretch ? sil_ref_stretch(m, info->lo, info->hi) : m;
}

/* 192-bit product of a 128-bit and a 64-bit unsigned integer, as three
 * 64-bit limbs (least significant first), and their comparison: the exact
 * Otsu and gate comparisons of chips beyond 256^2 pixels exceed 128 bits. */
typedef struct {
  uint64_t w[3];
} u192;

static u192 mul_128_64(u128 a, uint64_t b) {
  u128 lo = (u128)(uint64_t)a * b;
  u128 hi = (u128)(uint64_t)(a >> 64) * b;
  u192 r;
  r.w[0] = (uint64_t)lo;
  u128 mid = (lo >> 64) + (u128)(uint64_t)hi;
  r.w[1] = (uint64_t)mid;
  r.w[2] = (uint64_t)(hi >> 64) + (uint64_t)(mid >> 64);
  return r;
}

static int cmp_192(u192 a, u192 b) {
  for (int i = 2; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] > b.w[i] ? 1 : -1;
  return 0;
}

void sil_ref_chip_stats(const uint32_t* h, const sil_ref_params* p,
                        sil_ref_chip_info* info) {
  uint64_t N = 0, S = 0, Q = 0;
  for (uint32_t v = 0; v < 256; ++v) {
    N += h[v];
    S += (uint64_t)v * h[v];
    Q += (uint64_t)v * v * h[v];
  }

  /* Otsu: maximise the between-class variance over splits {v <= t} |
   * {v > t}.  With class weights w0, w1 and sums S0, S1,
   *   sigma_B^2 * N^2 = (w1*S0 - w0*S1)^2 / (w0*w1),
   * compared exactly as fractions num/den (192-bit cross products, so
   * chips of up to 2^27 pixels compare exactly); the smallest t wins ties. */
  int32_t best_t = -1;
  u128 best_num = 0;
  uint64_t best_den = 1;
  uint64_t w0 = 0, S0 = 0;
  for (uint32_t t = 0; t < 255; ++t) {
    w0 += h[t];
    S0 += (uint64_t)t * h[t];
    uint64_t w1 = N - w0, S1 = S - S0;
    if (w0 == 0 || w1 == 0) continue;
    __int128 diff = (__int128)w1 * S0 - (__int128)w0 * S1;
    u128 num = (u128)(diff < 0 ? -diff : diff);
    num *= num;
    uint64_t den = w0 * w1;
    if (best_t < 0 || cmp_192(mul_128_64(num, best_den), mul_128_64(best_num, den)) > 0) {
      best_t = (int32_t)t;
      best_num = num;
      best_den = den;
    }
  }
  info->t = best_t;

  /* Binary threshold on separability eta = sigma_B^2 / sigma_T^2 with
   *   sigma_T^2 * N^2 = N*Q - S^2. */
  info->gate = 0;
  if (best_t >= 0) {
    u128 var = (u128)N * Q - (u128)S * S;
    info->gate = cmp_192(mul_128_64(best_num, p->eta_den),
                         mul_128_64(var * best_den, p->eta_num)) >= 0;
  }

  /* Truncation levels: lo is the (k+1)-th smallest value, hi the (k+1)-th
   * largest, k = N >> clip_shift. */
  uint64_t k = N >> p->clip_shift;
  uint64_t cum = 0;
  int lo = 255;
  for (int v = 0; v < 256; ++v) {
    cum += h[v];
    if (cum > k) {
      lo = v;
      break;
    }
  }
  cum = 0;
  int hi = 0;
  for (int v = 255; v >= 0; --v) {
    cum += h[v];
    if (cum > k) {
      hi = v;
      break;
    }
  }
  info->lo = (uint8_t)lo;
  info->hi = (uint8_t)hi;
  info->stretch = info->gate && hi > lo;

  /* Debug summary: the smallest median value whose label reaches 1 and 2. */
  info->a1 = 256;
  info->a2 = 256;
  for (int m = 255; m >= 0; --m) {
    int c = sil_ref_class_of(filtered_value((uint8_t)m, info), p);
    if (c >= 1) info->a1 = (uint16_t)m;
    if (c >= 2) info->a2 = (uint16_t)m;
  }
}

/* ---- the whole labeller ------------------------------------------------ */

int sil_ref_label(const void* scene, int32_t nbands, const int32_t* sel, int32_t H,
                  int32_t W, int64_t pitch, const sil_ref_params* p, uint8_t* labels,
                  int64_t label_pitch, uint32_t* hist, sil_ref_chip_info* chips) {
  if (!scene || !labels || !hist) return SIL_REF_EINVAL;
  int rc = sil_ref_validate(nbands, sel, H, W, pitch, label_pitch, p);
  if (rc != SIL_REF_OK) return rc;
  int32_t ny, nx;
  sil_ref_hist_dims(H, W, p, &ny, &nx);

  const int64_t npx = (int64_t)H * W;
  uint8_t* V = malloc((size_t)npx);
  uint8_t* Vc = malloc((size_t)npx);
  if (!V || !Vc) {
    free(V);
    free(Vc);
    return SIL_REF_EINVAL;
  }

  /* 1. V plane */
  sil_ref_value_plane(scene, nbands, sel, H, W, pitch, p->dtype, p->refl_max, V);

  if (p->filter == 0) {
    /* 2. no filter */
    memcpy(Vc, V, (size_t)npx);
  } else {
    /* 3. median */
    uint8_t* Vm = malloc((size_t)npx);
    if (!Vm) {
      free(V);
      free(Vc);
      return SIL_REF_EINVAL;
    }
    sil_ref_median3x3(V, H, W, Vm);
    /* 4. per chip: statistics, then the stretch of every pixel */
    const int32_t C = (int32_t)p->chip;
    const int32_t ncy = (H + C - 1) / C, ncx = (W + C - 1) / C;
    for (int32_t cy = 0; cy < ncy; ++cy)
      for (int32_t cx = 0; cx < ncx; ++cx) {
        int32_t y0 = cy * C, y1 = y0 + C < H ? y0 + C : H;
        int32_t x0 = cx * C, x1 = x0 + C < W ? x0 + C : W;
        uint32_t h[256] = {0};
        for (int32_t y = y0; y < y1; ++y)
          for (int32_t x = x0; x < x1; ++x) h[Vm[(int64_t)y * W + x]]++;
        sil_ref_chip_info info;
        sil_ref_chip_stats(h, p, &info);
        if (chips) chips[(int64_t)cy * ncx + cx] = info;
        for (int32_t y = y0; y < y1; ++y)
          for (int32_t x = x0; x < x1; ++x)
            Vc[(int64_t)y * W + x] = filtered_value(Vm[(int64_t)y * W + x], &info);
      }
    free(Vm);
  }

  /* 5. masks -> label; 6. per-patch counts */
  memset(hist, 0, sizeof(uint32_t) * 3 * (size_t)ny * (size_t)nx);
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      int c = sil_ref_class_of(Vc[(int64_t)y * W + x], p);
      labels[(int64_t)y * label_pitch + x] = (uint8_t)c;
      int64_t py = y / (int64_t)p->patch_h, px = x / (int64_t)p->patch_w;
      hist[(py * nx + px) * 3 + c]++;
    }

  free(V);
  free(Vc);
  return SIL_REF_OK;
}

/* ---- general labeller: full HSV masks, any filter unit, filtered RGB ---- */

void sil_ref_hsv8(uint8_t r, uint8_t g, uint8_t b, uint8_t* h, uint8_t* s, uint8_t* v) {
  /* OpenCV's 8-bit HSV convention: V = max(R,G,B) in 0..255, S = 255*(V-min)/V
   * in 0..255, H = hue in degrees / 2 in 0..179 (hexcone model: the hue
   * angle is 60 degrees times the sector position).  Rounding is half up;
   * when two channels tie for the maximum, red takes precedence over green
   * and green over blue. */
  int32_t V = r > g ? r : g;
  V = V > b ? V : b;
  int32_t m = r < g ? r : g;
  m = m < b ? m : b;
  int32_t d = V - m;
  *v = (uint8_t)V;
  *s = V == 0 ? 0 : (uint8_t)((510 * d + V) / (2 * V));
  if (d == 0) {
    *h = 0;
    return;
  }
  /* sector position times d: red sector (g-b), green 2d + (b-r), blue 4d + (r-g) */
  int32_t num;
  if (V == r)
    num = g - b;
  else if (V == g)
    num = 2 * d + (b - r);
  else
    num = 4 * d + (r - g);
  /* hue / 2 = 30 * num / d, rounded half up: floor((60 num + d) / (2 d)) */
  int32_t top = 60 * num + d, bot = 2 * d;
  int32_t q = top >= 0 ? top / bot : -((-top + bot - 1) / bot);
  if (q < 0) q += 180;
  *h = (uint8_t)q;
}

void sil_ref_hsv8_many(const uint8_t* rgb, int64_t n, uint8_t* hsv) {
  for (int64_t i = 0; i < n; ++i)
    sil_ref_hsv8(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], &hsv[3 * i], &hsv[3 * i + 1],
                 &hsv[3 * i + 2]);
}

uint8_t sil_ref_filtered_band(uint8_t c, uint8_t v, uint8_t vc) {
  /* scale the pixel's colour so that its brightness becomes vc:
   * c' = c * vc / v, rounded half up; a black pixel stays black */
  if (v == 0) return 0;
  return (uint8_t)(((uint32_t)c * vc + v / 2u) / v);
}

int sil_ref_validate_ex(int32_t nbands, const int32_t* sel, int32_t H, int32_t W,
                        int64_t pitch, int64_t mask_pitch, const sil_ref_params* p) {
  if (!p || !sel) return SIL_REF_EINVAL;
  if (p->abi != SIL_REF_ABI_VERSION) return SIL_REF_EINVAL;
  if (p->dtype != SIL_REF_U8 && p->dtype != SIL_REF_U16) return SIL_REF_EINVAL;
  if (p->dtype == SIL_REF_U16 && p->refl_max < 1) return SIL_REF_EINVAL;
  if (p->filter > 1) return SIL_REF_EINVAL;
  if (p->chip < 1 || p->clip_shift < 1 || p->clip_shift > 31) return SIL_REF_EINVAL;
  if (p->eta_den < 1 || p->eta_num > p->eta_den) return SIL_REF_EINVAL;
  if (p->patch_h < 1 || p->patch_w < 1) return SIL_REF_EINVAL;
  if (H < 1 || W < 1 || pitch < W || mask_pitch < W || nbands < 1) return SIL_REF_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (sel[i] < 0 || sel[i] >= nbands) return SIL_REF_EINVAL;
  if (p->dtype == SIL_REF_U16 && p->refl_max > 65535) return SIL_REF_EUNSUPPORTED;
  /* the exact statistics hold for chips of at most 2^27 pixels */
  if (p->filter == 1) {
    int64_t ch = (int64_t)p->chip < H ? (int64_t)p->chip : H;
    int64_t cw = (int64_t)p->chip < W ? (int64_t)p->chip : W;
    if (ch * cw > ((int64_t)1 << 27)) return SIL_REF_EUNSUPPORTED;
  }
  return SIL_REF_OK;
}

int sil_ref_label_ex(const void* scene, int32_t nbands, const int32_t* sel, int32_t H,
                     int32_t W, int64_t pitch, const sil_ref_params* p, uint8_t* masks,
                     int64_t mask_pitch, uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch,
                     sil_ref_chip_info* chips) {
  if (!scene || !masks) return SIL_REF_EINVAL;
  int rc = sil_ref_validate_ex(nbands, sel, H, W, pitch, mask_pitch, p);
  if (rc != SIL_REF_OK) return rc;
  if (rgb && rgb_pitch < W) return SIL_REF_EINVAL;
  int32_t ny, nx;
  sil_ref_hist_dims(H, W, p, &ny, &nx);

  const int64_t npx = (int64_t)H * W;
  const int64_t plane = (int64_t)H * pitch;
  uint8_t* C8 = malloc((size_t)(3 * npx)); /* 8-bit blue, green, red planes */
  uint8_t* V = malloc((size_t)npx);
  uint8_t* Vc = malloc((size_t)npx);
  uint8_t* Vm = p->filter ? malloc((size_t)npx) : NULL;
  if (!C8 || !V || !Vc || (p->filter && !Vm)) {
    free(C8);
    free(V);
    free(Vc);
    free(Vm);
    return SIL_REF_EINVAL;
  }

  /* 1. each band to 8 bit (16-bit input: the same rescale as V), and V */
  for (int i = 0; i < 3; ++i)
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x) {
        int64_t idx = sel[i] * plane + (int64_t)y * pitch + x;
        uint32_t raw = p->dtype == SIL_REF_U8 ? ((const uint8_t*)scene)[idx]
                                               : ((const uint16_t*)scene)[idx];
        C8[i * npx + (int64_t)y * W + x] =
            p->dtype == SIL_REF_U8 ? (uint8_t)raw : sil_ref_rescale(raw, p->refl_max);
      }
  for (int64_t k = 0; k < npx; ++k) {
    uint8_t m = C8[k];
    if (C8[npx + k] > m) m = C8[npx + k];
    if (C8[2 * npx + k] > m) m = C8[2 * npx + k];
    V[k] = m;
  }

  /* 2-4. filtered brightness, exactly as the fused labeller but for any chip */
  if (p->filter == 0) {
    memcpy(Vc, V, (size_t)npx);
  } else {
    sil_ref_median3x3(V, H, W, Vm);
    const int64_t C = p->chip;
    const int64_t ncy = (H + C - 1) / C, ncx = (W + C - 1) / C;
    for (int64_t cy = 0; cy < ncy; ++cy)
      for (int64_t cx = 0; cx < ncx; ++cx) {
        int64_t y0 = cy * C, y1 = y0 + C < H ? y0 + C : H;
        int64_t x0 = cx * C, x1 = x0 + C < W ? x0 + C : W;
        uint32_t h[256] = {0};
        for (int64_t y = y0; y < y1; ++y)
          for (int64_t x = x0; x < x1; ++x) h[Vm[y * W + x]]++;
        sil_ref_chip_info info;
        sil_ref_chip_stats(h, p, &info);
        if (chips) chips[cy * ncx + cx] = info;
        for (int64_t y = y0; y < y1; ++y)
          for (int64_t x = x0; x < x1; ++x) Vc[y * W + x] = filtered_value(Vm[y * W + x], &info);
      }
  }

  /* 5. the three inRange masks on (H, S, Vc); H and S of the pixel's own
   * 8-bit colour (blue = sel[0], green = sel[1], red = sel[2]) */
  if (counts) memset(counts, 0, sizeof(uint32_t) * 3 * (size_t)ny * (size_t)nx);
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      uint8_t hh, ss, vv;
      sil_ref_hsv8(C8[2 * npx + k], C8[npx + k], C8[k], &hh, &ss, &vv);
      const uint8_t vc = Vc[k];
      uint8_t bits = 0;
      for (int c = 0; c < 3; ++c)
        if (p->lo[c][0] <= hh && hh <= p->hi[c][0] && p->lo[c][1] <= ss && ss <= p->hi[c][1] &&
            p->lo[c][2] <= vc && vc <= p->hi[c][2])
          bits |= (uint8_t)(1u << c);
      masks[(int64_t)y * mask_pitch + x] = bits;
      /* 6. per-patch mask counts */
      if (counts) {
        int64_t py = y / (int64_t)p->patch_h, px = x / (int64_t)p->patch_w;
        for (int c = 0; c < 3; ++c)
          if (bits >> c & 1u) counts[(py * nx + px) * 3 + c]++;
      }
      /* filtered colour image */
      if (rgb)
        for (int i = 0; i < 3; ++i)
          rgb[(int64_t)i * H * rgb_pitch + (int64_t)y * rgb_pitch + x] =
              sil_ref_filtered_band(C8[i * npx + k], V[k], vc);
    }

  free(C8);
  free(V);
  free(Vc);
  free(Vm);
  return SIL_REF_OK;
}

/* ---- colour rendering of the class ids (sections III-A, III-B) --------- */

void sil_ref_render_rgb(const uint8_t* labels, int32_t H, int32_t W, int64_t lpitch,
                        uint8_t* rgb, int64_t rgb_pitch) {
  for (int32_t y = 0; y < H; ++y) {
    for (int32_t x = 0; x < W; ++x) {
      const uint8_t c = labels[(int64_t)y * lpitch + x];
      uint8_t r = 0, g = 0, b = 0;
      if (c == 0) g = 255;      /* open water: green */
      else if (c == 1) b = 255; /* thin ice: blue */
      else if (c == 2) r = 255; /* thick ice: red */
      uint8_t* o = rgb + (int64_t)y * rgb_pitch + 3 * (int64_t)x;
      o[0] = r;
      o[1] = g;
      o[2] = b;
    }
  }
}
