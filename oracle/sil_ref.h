/*
 * sil_ref.h -- CPU oracle of the sea-ice auto-labeller.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the GPU library computes, written from the paper
 * (arXiv 2403.13135, section III-A "Filtering Out the Thin Clouds and
 * Shadows", section III-B "Auto-labeling Method" and "Scaling
 * Auto-labeling").  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library; the two agree only through the written
 * definition of the method.
 *
 * Definition (every step integer-exact):
 *   1. V = max of the blue/green/red planes (section III-B: V of OpenCV's
 *      8-bit HSV is max(R,G,B)).  16-bit reflectance is rescaled to 8 bit by
 *      round-half-up of x*255/refl_max, saturating at 255.
 *   2. filter = 0: Vc = V, go to 5.
 *   3. 3x3 median of V, indices clamped at the scene border (the "noise
 *      filtering" of section III-A).
 *   4. Per chip (256x256 tiles anchored at the origin, partial at the
 *      edges): 256-bin histogram of the median, exact Otsu threshold and
 *      separability eta (the "Otsu thresholding"), a binary gate eta >=
 *      eta_num/eta_den (the "binary thresholding"), rank-k truncation levels
 *      lo/hi (the "truncated thresholding") and a min-max stretch of
 *      [lo,hi] to [0,255] (the "min-max normalization"), applied when the
 *      gate passes and hi > lo.
 *   5. Three inRange masks with the paper's inclusive HSV limits (section
 *      III-B); the hue and saturation limits must be vacuous, so each mask is
 *      an interval of V.  The label is the index of the one mask that holds.
 *   6. Per-patch class counts (the map-reduce of "Scaling Auto-labeling").
 *
 * Parity status: steps 1, 5 and 6 are fixed by the paper; the composition
 * and constants of steps 3-4 are a reading of an operation list the paper
 * gives without order or parameters.  That reading is pinned by independent
 * library routines and closed forms in the tests, not by the paper's
 * (unpublished) filter.
 */
#ifndef SIL_REF_H
#define SIL_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIL_REF_ABI_VERSION 1u

enum { SIL_REF_OK = 0, SIL_REF_EINVAL = -1, SIL_REF_EUNSUPPORTED = -2 };
enum { SIL_REF_U8 = 1, SIL_REF_U16 = 2 };

/* Field-for-field the same layout as the GPU library's parameter block. */
typedef struct sil_ref_params {
  uint32_t abi;        /* SIL_REF_ABI_VERSION */
  uint32_t dtype;      /* SIL_REF_U8 or SIL_REF_U16 */
  uint32_t refl_max;   /* 16-bit full scale mapped to V = 255 */
  uint8_t lo[3][3];    /* [class][H,S,V] inclusive lower limits */
  uint8_t hi[3][3];    /* [class][H,S,V] inclusive upper limits */
  uint8_t pad[2];
  uint32_t filter;     /* 0: thresholds only, 1: cloud/shadow filter */
  uint32_t chip;       /* filter unit side */
  uint32_t clip_shift; /* k = N >> clip_shift */
  uint32_t eta_num, eta_den;
  uint32_t patch_h, patch_w;
} sil_ref_params;

typedef struct sil_ref_chip_info {
  int32_t t;        /* Otsu threshold, -1 when no split exists */
  uint8_t lo, hi;   /* truncation levels */
  uint8_t gate;     /* eta >= eta_num/eta_den */
  uint8_t stretch;  /* gate && hi > lo */
  uint16_t a1, a2;  /* smallest median value labelled >= 1 / >= 2, 256 if none */
} sil_ref_chip_info;

void sil_ref_params_default(sil_ref_params* p);
const char* sil_ref_strerror(int code);
int sil_ref_validate(int32_t nbands, const int32_t* sel, int32_t H, int32_t W,
                     int64_t pitch, int64_t label_pitch, const sil_ref_params* p);
int sil_ref_hist_dims(int32_t H, int32_t W, const sil_ref_params* p, int32_t* ny,
                      int32_t* nx);

/* The whole labeller on host buffers.  scene: [nbands][H][pitch] elements of
 * the dtype; labels: [H][label_pitch]; hist: [ny][nx][3], overwritten;
 * chips (nullable, filter = 1 only): [ceil(H/chip)][ceil(W/chip)]. */
int sil_ref_label(const void* scene, int32_t nbands, const int32_t* sel, int32_t H,
                  int32_t W, int64_t pitch, const sil_ref_params* p, uint8_t* labels,
                  int64_t label_pitch, uint32_t* hist, sil_ref_chip_info* chips);

/* Individual steps, exported for unit pins. */
void sil_ref_value_plane(const void* scene, int32_t nbands, const int32_t* sel,
                         int32_t H, int32_t W, int64_t pitch, uint32_t dtype,
                         uint32_t refl_max, uint8_t* V);
uint8_t sil_ref_rescale(uint32_t x, uint32_t refl_max);
void sil_ref_median3x3(const uint8_t* V, int32_t H, int32_t W, uint8_t* Vm);
void sil_ref_chip_stats(const uint32_t* h, const sil_ref_params* p,
                        sil_ref_chip_info* info);
uint8_t sil_ref_stretch(uint8_t m, uint8_t lo, uint8_t hi);
int sil_ref_class_of(uint8_t vc, const sil_ref_params* p);

/* General labeller (the variants of the method): three inRange masks on full
 * HSV limits, a filter unit of any size up to a whole scene, and optionally
 * the filtered colour image.
 *   - H and S are those of the pixel's own 8-bit colour (OpenCV 8-bit
 *     convention: H = hue/2 in 0..179, S in 0..255, rounded half up); V is
 *     replaced by the filtered Vc.  Since H and S do not change when a colour
 *     is scaled, this is inRange on the HSV of the filtered colour image up to
 *     that image's rounding.
 *   - masks: [H][mask_pitch] bytes, bit c set iff mask c (0 water, 1 thin,
 *     2 thick) holds; limits are free (masks may overlap or leave pixels out).
 *   - counts (nullable): [ny][nx][3], pixels with bit c set per patch.
 *   - rgb (nullable): planar [3][H][rgb_pitch], plane i the filtered band
 *     sel[i]: c' = c * Vc / V rounded half up (0 where V = 0), so its maximum
 *     over the bands is exactly Vc.
 *   - chips (nullable, filter = 1): per-chip statistics as sil_ref_label.
 * Validation as sil_ref_label except: any H/S/V limits, any chip side (a
 * chip of more than 2^27 pixels is SIL_REF_EUNSUPPORTED). */
int sil_ref_validate_ex(int32_t nbands, const int32_t* sel, int32_t H, int32_t W,
                        int64_t pitch, int64_t mask_pitch, const sil_ref_params* p);
int sil_ref_label_ex(const void* scene, int32_t nbands, const int32_t* sel, int32_t H,
                     int32_t W, int64_t pitch, const sil_ref_params* p, uint8_t* masks,
                     int64_t mask_pitch, uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch,
                     sil_ref_chip_info* chips);
void sil_ref_hsv8(uint8_t r, uint8_t g, uint8_t b, uint8_t* h, uint8_t* s, uint8_t* v);
/* sil_ref_hsv8 over n interleaved (r, g, b) triples into (h, s, v) triples */
void sil_ref_hsv8_many(const uint8_t* rgb, int64_t n, uint8_t* hsv);
uint8_t sil_ref_filtered_band(uint8_t c, uint8_t v, uint8_t vc);

/* Colour rendering of a class-id plane (section III-A names the colours of
 * the labelled scenes: red for snow-covered / thick ice, blue for thin or
 * young ice, green for open water; section III-B merges the class masks, each
 * in its colour, into one image).  labels [H][lpitch] with 0 water, 1 thin,
 * 2 thick; rgb [H][rgb_pitch] interleaved (R, G, B): water (0, 255, 0), thin
 * (0, 0, 255), thick (255, 0, 0), any other id (0, 0, 0).  Bytes of rgb past
 * 3 W in a row are left as they are. */
void sil_ref_render_rgb(const uint8_t* labels, int32_t H, int32_t W, int64_t lpitch,
                        uint8_t* rgb, int64_t rgb_pitch);

#ifdef __cplusplus
}
#endif
#endif
