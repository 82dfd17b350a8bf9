/* Drives the oracle over random small scenes and parameter sets (the fused
 * labeller and the general one, the 8-bit HSV conversion and 2^27-pixel chip
 * statistics) so that tests/test_oracle_sanitized.py can run it under
 * AddressSanitizer and UndefinedBehaviorSanitizer. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "sil_ref.h"
static unsigned rng = 12345;
static unsigned nxt(void) { rng = rng * 1664525u + 1013904223u; return rng >> 8; }
int main(void) {
  for (int trial = 0; trial < 300; ++trial) {
    int H = 1 + nxt() % 70, W = 1 + nxt() % 70, u16 = nxt() & 1;
    int64_t pitch = W + nxt() % 5;
    sil_ref_params p; sil_ref_params_default(&p);
    p.dtype = u16 ? SIL_REF_U16 : SIL_REF_U8;
    int chips[] = {1, 3, 7, 16, 64, 256, 1 << 20};
    p.chip = chips[nxt() % 7];
    p.patch_h = 1 + nxt() % 40; p.patch_w = 1 + nxt() % 40;
    p.filter = nxt() % 4 != 0;
    int sel[3] = {0, 1, 2};
    size_t esz = u16 ? 2 : 1;
    unsigned char* scene = malloc(3 * H * pitch * esz);
    for (size_t i = 0; i < 3 * H * pitch; ++i) {
      if (u16) ((unsigned short*)scene)[i] = nxt() % 12000; else scene[i] = nxt() & 255;
    }
    int ny = (H + p.patch_h - 1) / p.patch_h, nx = (W + p.patch_w - 1) / p.patch_w;
    unsigned char* lab = malloc(H * W);
    unsigned* hist = malloc(ny * nx * 3 * 4);
    int ncy = (H + p.chip - 1) / p.chip, ncx = (W + p.chip - 1) / p.chip;
    sil_ref_chip_info* ci = malloc(sizeof(*ci) * ncy * ncx);
    int rc = sil_ref_label(scene, 3, sel, H, W, pitch, &p, lab, W, hist, ci);
    if (rc != 0 && !(rc == SIL_REF_EUNSUPPORTED && p.chip > 256 && p.filter)) { printf("label rc %d\n", rc); return 1; }
    // general labeller with free limits
    for (int c = 0; c < 3; ++c) for (int j = 0; j < 3; ++j) { p.lo[c][j] = nxt() & 255; p.hi[c][j] = nxt() & 255; }
    unsigned char* rgb = malloc(3 * H * W);
    rc = sil_ref_label_ex(scene, 3, sel, H, W, pitch, &p, lab, W, hist, rgb, W, ci);
    if (rc != 0) { printf("label_ex rc %d\n", rc); return 1; }
    free(scene); free(lab); free(hist); free(ci); free(rgb);
  }
  unsigned char rgbv[3 * 4096], hsv[3 * 4096];
  for (int i = 0; i < 3 * 4096; ++i) rgbv[i] = nxt() & 255;
  sil_ref_hsv8_many(rgbv, 4096, hsv);
  unsigned h[256]; for (int i = 0; i < 256; ++i) h[i] = 1u << 19;
  sil_ref_params p; sil_ref_params_default(&p); sil_ref_chip_info info;
  sil_ref_chip_stats(h, &p, &info);
  printf("ok t=%d gate=%d\n", info.t, info.gate);
  return 0;
}
