/*
 * sil.h -- C ABI of libsil, the GPU (gfx950) sea-ice auto-labeller.
 *
 * Method: arXiv 2403.13135, "A Parallel Workflow for Polar Sea-Ice
 * Classification using Auto-labeling of Sentinel-2 Imagery".
 *   - bands B2, B3, B4 (blue, green, red): section III-A;
 *   - thin-cloud/shadow filter built from the OpenCV operations the paper
 *     lists (HSV conversion, noise filtering, Otsu, truncated and binary
 *     thresholding, min-max normalisation): section III-A, "Filtering Out
 *     the Thin Clouds and Shadows";
 *   - HSV inRange segmentation with inclusive limits, water (0,0,0)-
 *     (185,255,30), thin ice (0,0,31)-(185,255,204), thick ice (0,0,205)-
 *     (185,255,255), non-intersecting masks merged into one label image:
 *     section III-B, "Auto-labeling Method";
 *   - per-patch class counts as the map-reduce output: section III-B,
 *     "Scaling Auto-labeling" (PySpark Map-Reduce).
 *
 * The filter composition the library implements (the paper lists the
 * operations without order or constants):
 *   V = max(B, G, R) (16-bit input: round-half-up of x*255/refl_max,
 *   saturating) -> 3x3 median with clamped borders -> per chip (chip x chip
 *   tiles anchored at the origin): 256-bin histogram, exact Otsu split t*
 *   (ties to the smallest t), gate eta = sigma_B^2/sigma_T^2 >= eta_num /
 *   eta_den, truncation levels lo/hi at rank k = N >> clip_shift from each
 *   tail, and, if the gate passes and hi > lo, the stretch
 *   Vc = ((clamp(Vm,lo,hi) - lo)*255 + (hi-lo)/2) div (hi-lo); else Vc = Vm.
 *   The label is the class whose V-interval holds Vc.
 *
 * Conventions for every entry point:
 *   - All arithmetic is integer; results are bit-exact and deterministic.
 *   - Device buffers are owned by the caller.  The library allocates no device
 *     or host memory per call and keeps no pointer after it returns.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     default stream).  Buffers must stay valid until that work completes.
 *   - Argument errors are detected before anything is enqueued and leave every
 *     output untouched.  A launch failure returns SIL_EDEVICE.  Faults during
 *     execution surface at the caller's next synchronisation of `stream`.
 *   - Thread-safe: no mutable global state besides a per-process cache of
 *     host-side derived constants guarded by a mutex.
 */
#ifndef SIL_H
#define SIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIL_ABI_VERSION 1u

/* Return codes. */
enum {
  SIL_OK = 0,
  SIL_EINVAL = -1,       /* bad pointer, size, pitch, band index or parameter */
  SIL_EUNSUPPORTED = -2, /* valid in the paper's model but outside this library */
  SIL_EDEVICE = -3       /* HIP launch error */
};

/* Input element types. */
enum { SIL_U8 = 1, SIL_U16 = 2 };

/* Labelling parameters.  sil_params_default() gives the paper's values. */
typedef struct sil_params {
  uint32_t abi;        /* must equal SIL_ABI_VERSION */
  uint32_t dtype;      /* SIL_U8 or SIL_U16 */
  uint32_t refl_max;   /* SIL_U16 only: reflectance full scale mapped to V = 255;
                          1..65535, default 10000 (Sentinel-2 quantification) */
  uint8_t lo[3][3];    /* [class][H,S,V] inclusive lower limits, class 0 water,
                          1 thin ice, 2 thick ice (section III-B) */
  uint8_t hi[3][3];    /* [class][H,S,V] inclusive upper limits */
  uint8_t pad[2];      /* zero */
  uint32_t filter;     /* 0: thresholds only (the paper's "original" images),
                          1: cloud/shadow filter, then thresholds (default) */
  uint32_t chip;       /* filter unit side in pixels, 1..256, default 256 */
  uint32_t clip_shift; /* truncation rank k = N >> clip_shift, 1..31, default 8 */
  uint32_t eta_num;    /* gate eta >= eta_num/eta_den, 0 <= num <= den, */
  uint32_t eta_den;    /*   den >= 1, default 3/4 */
  uint32_t patch_h;    /* count patch height, >= 1, default 256 */
  uint32_t patch_w;    /* count patch width, >= 1, default 256 */
} sil_params;

/* Per-chip filter statistics (optional debug output of sil_label). */
typedef struct sil_chip_info {
  int32_t t;       /* Otsu split t* in 0..254, -1 if the chip has one value */
  uint8_t lo, hi;  /* truncation levels */
  uint8_t gate;    /* 1 if eta >= eta_num/eta_den */
  uint8_t stretch; /* 1 if the min-max stretch was applied (gate && hi > lo) */
  uint16_t a1, a2; /* smallest median value labelled >= 1 and >= 2; 256 if none */
} sil_chip_info;

/* Fill *p with the paper's limits (section III-B) and the filter defaults
 * above.  p must be non-NULL. */
void sil_params_default(sil_params* p);

/* ABI version the library was built with (SIL_ABI_VERSION). */
uint32_t sil_abi_version(void);

/* Dimensions of the per-patch count array: ny = ceil(H/patch_h),
 * nx = ceil(W/patch_w).  Returns SIL_EINVAL on NULL pointers, H or W < 1, or
 * zero patch sides. */
int sil_hist_dims(int32_t H, int32_t W, const sil_params* p, int32_t* ny, int32_t* nx);

/* Check arguments exactly as sil_label does, without touching any buffer.
 * Same return codes as sil_label (never SIL_EDEVICE). */
int sil_validate(int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
                 int64_t pitch, int64_t label_pitch, const sil_params* p);

/* Label one scene and count classes per patch.
 *
 *   scene        device, planar [nbands][H][pitch] elements of p->dtype (plane
 *                stride H*pitch).  Any alignment and pitch is accepted;
 *                8-byte (u16) / 4-byte (u8) aligned rows take the vector path.
 *   nbands, sel  sel[0..2] are the plane indices of B2 (blue), B3 (green) and
 *                B4 (red), each in [0, nbands).
 *   H, W         scene height and width, >= 1; pitch >= W (elements).
 *   labels       device, [H][label_pitch] bytes, label_pitch >= W; every pixel
 *                (y < H, x < W) is written with 0 (water), 1 (thin ice) or
 *                2 (thick ice); bytes beyond W are not touched.
 *   hist         device, uint32 [ny][nx][3] (see sil_hist_dims), fully
 *                overwritten: hist[py][px][c] = number of pixels of class c in
 *                patch (py, px); patches are anchored at (0,0), partial at
 *                the right/bottom edges.
 *   chips        device, nullable; with filter = 1, [ceil(H/chip)][ceil(W/chip)]
 *                per-chip statistics.  Ignored when filter = 0.
 *   stream       hipStream_t or NULL.
 *
 * Errors:
 *   SIL_EINVAL        NULL scene/labels/hist/sel/p; H or W < 1; pitch < W;
 *                     label_pitch < W; nbands < 1; sel out of range; abi
 *                     mismatch; bad dtype, refl_max, filter, chip, clip_shift,
 *                     eta or patch; V-intervals that intersect (section III-B
 *                     states they do not).
 *   SIL_EUNSUPPORTED  V-intervals leaving a value unlabelled; hue/saturation
 *                     limits that do not span H in [0,179] and S in [0,255]
 *                     (OpenCV 8-bit HSV); class order along V other than
 *                     water <= thin <= thick; chip > 256; refl_max > 65535;
 *                     H*W beyond 2^31 chips or pixel offsets beyond int64;
 *                     with filter = 1, input rows of 2^32/34 bytes or more
 *                     (a chip walk addresses 34 rows with 32-bit offsets).
 *   SIL_EDEVICE       the kernel launch failed.
 */
int sil_label(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H,
              int32_t W, int64_t pitch, const sil_params* p, uint8_t* labels,
              int64_t label_pitch, uint32_t* hist, sil_chip_info* chips, void* stream);

/* Number of chips ceil(H/chip) * ceil(W/chip) of a scene (raster order:
 * chip id = cy * ceil(W/chip) + cx).  SIL_EINVAL on NULL or sizes < 1. */
int sil_chip_count(int32_t H, int32_t W, const sil_params* p, int32_t* nchips);

/* Scenes per sil_label_batch call. */
#define SIL_BATCH_MAX_JOBS 24

/* One scene's share of a batched launch: the scene and output buffers exactly
 * as for sil_label, plus the chip range [chip_begin, chip_begin + chip_count)
 * (raster order) to label in this call. */
typedef struct sil_job {
  const void* scene;     /* device, [nbands][H][pitch] */
  int32_t nbands;
  int32_t sel[3];
  int32_t H, W;
  int64_t pitch;
  uint8_t* labels;       /* device, [H][label_pitch] */
  int64_t label_pitch;
  uint32_t* hist;        /* device, [ceil(H/chip)][ceil(W/chip)][3] */
  sil_chip_info* chips;  /* device, nullable */
  int32_t chip_begin;
  int32_t chip_count;
} sil_job;

/* Label chip ranges of up to SIL_BATCH_MAX_JOBS scenes in ONE kernel launch
 * (the filter, segmentation and counts of section III of the paper, as in
 * sil_label).  Used for continuous batching: a long scene can be split over
 * several calls and small scenes share one launch.  Results of a chip do not
 * depend on which call labels it or what else that call contains.
 *
 * Requirements beyond sil_label's: filter = 1 and patch_h = patch_w = chip
 * (counts come straight from each chip), else SIL_EUNSUPPORTED; all jobs use
 * `p`.  Only the labels, counts and chip statistics of the listed chips are
 * written.  Errors: SIL_EINVAL for NULL/0/too many jobs or a chip range
 * outside the scene, plus every sil_label argument error of any job; nothing
 * is enqueued on error.  Allocates nothing; asynchronous on `stream`. */
int sil_label_batch(const sil_job* jobs, int32_t njobs, const sil_params* p, void* stream);

/* ---- General labeller: the variants of the method ------------------------
 *
 * sil_label_ex computes what sil_label does, generalised in the three ways
 * the paper leaves open to the fused kernel:
 *   - the three inRange masks of section III-B on FULL hue / saturation /
 *     value limits.  H and S are those of the pixel's own 8-bit colour in
 *     OpenCV's 8-bit convention (H = hue in degrees / 2, 0..179; S = 255 *
 *     (max - min) / max, 0..255; both rounded half up; red wins a tie for the
 *     maximum, then green); V is the filtered brightness Vc.  Scaling a colour
 *     leaves H and S unchanged, so this is inRange on the HSV of the filtered
 *     colour image up to that image's rounding.  Limits are free: masks may
 *     overlap or leave pixels in no mask, so the output is a bit mask;
 *   - a filter unit (p->chip) of any side, up to the whole scene (section
 *     III-A filters whole scenes; section IV uses 256 x 256 chips);
 *   - the filtered colour image, the U-Net's input in the inference workflow
 *     (section III-C): c' = (c * Vc + V/2) div V per 8-bit band (0 where
 *     V = 0), whose maximum over the bands is exactly Vc.
 * The filter (median, per-chip Otsu gate, truncation and stretch) is the same
 * definition as sil_label's; its exact comparisons are carried in 192 bits so
 * that chips of up to 2^27 pixels stay exact.
 *
 *   scene, nbands, sel, H, W, pitch   as sil_label; 16-bit scenes must be
 *                 2-byte aligned.
 *   masks         device, [H][mask_pitch] bytes, mask_pitch >= W: bit c of
 *                 pixel (y, x) is set iff mask c holds (c = 0 water, 1 thin
 *                 ice, 2 thick ice, the paper's three ranges).
 *   counts        device, nullable, uint32 [ny][nx][3] (sil_hist_dims), fully
 *                 overwritten: pixels of patch (py, px) with bit c set.
 *   rgb           device, nullable, planar [3][H][rgb_pitch] bytes, rgb_pitch
 *                 >= W: plane i is the filtered band sel[i].
 *   chips         device, nullable; with filter = 1 the per-chip statistics
 *                 [ceil(H/chip)][ceil(W/chip)] (a1/a2 refer to the last
 *                 V-interval holding the filtered value).
 *   workspace     device, caller-owned scratch of at least
 *                 sil_label_ex_workspace() bytes, 16-byte aligned (0 bytes
 *                 when filter = 0, where it may be NULL); its contents are not
 *                 kept between calls, and calls that share one workspace must
 *                 not overlap in time.
 *   stream        hipStream_t or NULL.
 *
 * Errors: SIL_EINVAL for NULL scene/masks/sel/p, a too small, NULL or
 * misaligned workspace with filter = 1, rgb_pitch < W with rgb, a misaligned 16-bit
 * scene, and sil_label's argument errors except those on H/S/V limits (any
 * limits are accepted) and chip > 256; SIL_EUNSUPPORTED for a chip of more
 * than 2^27 pixels (min(chip,H) * min(chip,W)), refl_max > 65535 or
 * H*W >= 2^31; SIL_EDEVICE on a launch failure.  Allocates nothing;
 * asynchronous on `stream`. */
int sil_label_ex_validate(int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
                          int64_t pitch, int64_t mask_pitch, const sil_params* p);

/* Workspace bytes sil_label_ex needs for an H x W scene under p (0 when
 * filter = 0).  SIL_EINVAL on NULL pointers, H or W < 1 or chip < 1. */
int sil_label_ex_workspace(int32_t H, int32_t W, const sil_params* p, uint64_t* bytes);

int sil_label_ex(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H, int32_t W,
                 int64_t pitch, const sil_params* p, uint8_t* masks, int64_t mask_pitch,
                 uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch, sil_chip_info* chips,
                 void* workspace, uint64_t workspace_bytes, void* stream);

/* sil_label_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and result as sil_label_ex without the workspace: the
 * workspace is a 32 MiB array that the library holds on each device for the
 * life of the process (SIL_LABEL_EX_NOALLOC_MAX bytes, enough for the
 * sil_label_ex_workspace() of e.g. a 4096 x 4096 scene with 256 x 256 chips or
 * a 5600 x 5600 one filtered as a whole).  Every call on a device shares that
 * array, so calls on one device must not overlap in time (their results are
 * undefined if they do); nothing in it is kept from one call to the next.
 * Errors: those of sil_label_ex, and SIL_EUNSUPPORTED (before anything is
 * enqueued) when the scene needs more workspace than the array holds;
 * SIL_EDEVICE if the array's device address cannot be obtained.  Calls no
 * allocator. */
#define SIL_LABEL_EX_NOALLOC_MAX (32ull << 20)
int sil_label_ex_noalloc(const void* scene, int32_t nbands, const int32_t sel[3], int32_t H,
                         int32_t W, int64_t pitch, const sil_params* p, uint8_t* masks,
                         int64_t mask_pitch, uint32_t* counts, uint8_t* rgb, int64_t rgb_pitch,
                         sil_chip_info* chips, void* stream);

/* Colour rendering of a class-id plane (section III-A labels scenes in red
 * for snow-covered / thick ice, blue for thin or young ice and green for open
 * water; section III-B merges the three class masks, each in its colour, into
 * one image).  labels: [H][lpitch] bytes, class ids 0 water, 1 thin ice,
 * 2 thick ice (as sil_label writes them); rgb: [H][rgb_pitch] bytes of
 * interleaved R, G, B, rgb_pitch >= 3 W.  Class 0 -> (0, 255, 0), 1 -> (0, 0,
 * 255), 2 -> (255, 0, 0), any other value -> (0, 0, 0).  Device pointers,
 * asynchronous on stream.  Errors (nothing enqueued): SIL_EINVAL for a NULL
 * pointer, H or W < 1, lpitch < W or rgb_pitch < 3 W; SIL_EDEVICE on a
 * launch failure. */
int sil_render_rgb(const uint8_t* labels, int32_t H, int32_t W, int64_t lpitch, uint8_t* rgb,
                   int64_t rgb_pitch, void* stream);

/* Human-readable text of a return code (static storage). */
const char* sil_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
