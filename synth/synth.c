/*
 * synth.c -- seeded synthetic Sentinel-2-like scenes (input generator only).
 *
 * Holds none of the labelling method's arithmetic: it only draws pixels.
 * Integer-only given the host-built tables passed in, so any other copy of
 * it (for example on the device) can reproduce it bit for bit.
 *
 * Scene model:
 *   * ground truth: a jittered-grid Voronoi map of 3 classes (cell side G;
 *     one seed per cell; class = hash % 3; nearest seed by squared integer
 *     distance over the 5x5 surrounding cells, ties to the lowest row-major
 *     cell index);
 *   * per band b: v = clamp(mean[class] + NOISE[hash >> 52], 0, 255);
 *   * thin-cloud haze: v <- clamp(rhu(v + g*(40 + (128 - v)/4)), 0, 255),
 *     g in Q16 the maximum over the haze blobs of exp(-d^2 / 2 sigma^2);
 *   * shadow: v <- rhu(v*(1 - 0.4 g)), g over the shadow blobs;
 *   * 16-bit reflectance: each 8-bit v becomes x drawn uniformly by hash
 *     from the reflectance bin [v, v+1) * 10000/255.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct synth_blob {
  int64_t cy, cx; /* centre, pixels */
  int64_t s2;     /* sigma^2, pixels^2, >= 1 */
} synth_blob;

typedef struct synth_cfg {
  uint64_t seed;
  int32_t cell;            /* Voronoi cell side G */
  int32_t mean[3];         /* class means: water, thin ice, thick ice */
  const int8_t* noise;     /* 4096 entries */
  const uint32_t* gtab;    /* Q16 exp(-i/128), i = floor(64 d^2 / s2) */
  int32_t gtab_len;
  const synth_blob* haze;
  int32_t n_haze;
  const synth_blob* shadow;
  int32_t n_shadow;
} synth_cfg;

static uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* counter-based stream: u(seed, stream, index) */
uint64_t synth_hash(uint64_t seed, uint64_t stream, uint64_t index) {
  return mix64(mix64(seed ^ mix64(stream + 0x632BE59BD9B4E019ull)) + index);
}

enum { ST_SEED_Y = 1, ST_SEED_X = 2, ST_SEED_CLASS = 3, ST_NOISE = 16, ST_U16 = 32 };

static void cell_seed(const synth_cfg* c, int64_t gy, int64_t gx, int64_t ngx,
                      int64_t* sy, int64_t* sx, int* cls) {
  uint64_t id = (uint64_t)((gy + 2) * (ngx + 4) + (gx + 2));
  *sy = gy * c->cell + (int64_t)(synth_hash(c->seed, ST_SEED_Y, id) % (uint64_t)c->cell);
  *sx = gx * c->cell + (int64_t)(synth_hash(c->seed, ST_SEED_X, id) % (uint64_t)c->cell);
  *cls = (int)(synth_hash(c->seed, ST_SEED_CLASS, id) % 3u);
}

static uint32_t blob_g(const synth_cfg* c, const synth_blob* b, int n, int64_t y,
                       int64_t x) {
  uint32_t g = 0;
  for (int i = 0; i < n; ++i) {
    int64_t dy = y - b[i].cy, dx = x - b[i].cx;
    uint64_t d2 = (uint64_t)(dy * dy + dx * dx);
    uint64_t idx = d2 * 64u / (uint64_t)b[i].s2;
    uint32_t v = idx < (uint64_t)c->gtab_len ? c->gtab[idx] : 0u;
    if (v > g) g = v;
  }
  return g;
}

static int32_t clamp255(int64_t v) { return v < 0 ? 0 : (v > 255 ? 255 : (int32_t)v); }

/* truth may be NULL.  out8: [3][H][W] */
void synth_scene_u8(const synth_cfg* c, int32_t H, int32_t W, uint8_t* out8,
                    uint8_t* truth) {
  const int64_t G = c->cell;
  const int64_t ngx = (W + G - 1) / G;
  const int64_t plane = (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t y = 0; y < H; ++y) {
    int64_t gy = y / G;
    for (int32_t x = 0; x < W; ++x) {
      int64_t gx = x / G;
      /* nearest seed over the 5x5 neighbourhood, row-major tie order */
      int64_t best = INT64_MAX;
      int cls = 0;
      for (int64_t ny = gy - 2; ny <= gy + 2; ++ny)
        for (int64_t nx = gx - 2; nx <= gx + 2; ++nx) {
          int64_t sy, sx;
          int k;
          cell_seed(c, ny, nx, ngx, &sy, &sx, &k);
          int64_t d = (sy - y) * (sy - y) + (sx - x) * (sx - x);
          if (d < best) {
            best = d;
            cls = k;
          }
        }
      if (truth) truth[(int64_t)y * W + x] = (uint8_t)cls;
      uint32_t gh = blob_g(c, c->haze, c->n_haze, y, x);
      uint32_t gs = blob_g(c, c->shadow, c->n_shadow, y, x);
      for (int b = 0; b < 3; ++b) {
        uint64_t u = synth_hash(c->seed, ST_NOISE + b, (uint64_t)y * (uint64_t)W + x);
        int64_t v = clamp255(c->mean[cls] + c->noise[u >> 52]);
        /* haze: v + g (288 - v) / 4, round half up, in Q18 */
        v = clamp255(((v << 18) + (int64_t)gh * (288 - v) + (1 << 17)) >> 18);
        /* shadow: v (1 - 0.4 g) = v (5*2^16 - 2 g) / (5*2^16), round half up */
        v = (v * (327680 - 2 * (int64_t)gs) + 163840) / 327680;
        out8[b * plane + (int64_t)y * W + x] = (uint8_t)v;
      }
    }
  }
}

/* 16-bit reflectance from an 8-bit scene: the 8-bit value v is read as the
 * quantisation of a reflectance in [v, v+1)/255 of full scale 10000, and x
 * is drawn uniformly by hash from that bin (values up to 10039 occur, as
 * bright snow does above reflectance 1).  in8: [3][H][W]; out16: [3][H][pitch] */
void synth_u8_to_u16(uint64_t seed, int32_t H, int32_t W, const uint8_t* in8,
                     int64_t pitch, uint16_t* out16) {
  const int64_t plane8 = (int64_t)H * W, plane16 = (int64_t)H * pitch;
#pragma omp parallel for schedule(static)
  for (int32_t y = 0; y < H; ++y)
    for (int b = 0; b < 3; ++b)
      for (int32_t x = 0; x < W; ++x) {
        uint32_t v = in8[b * plane8 + (int64_t)y * W + x];
        uint64_t u = synth_hash(seed, ST_U16 + b, (uint64_t)y * (uint64_t)W + x);
        out16[b * plane16 + (int64_t)y * pitch + x] =
            (uint16_t)((v * 10000u + (uint32_t)(u % 10000u)) / 255u);
      }
}
