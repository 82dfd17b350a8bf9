"""Seeded synthetic Sentinel-2-like scenes: the input generator.

Stands in for the paper's Ross-Sea Sentinel-2 B2/B3/B4 exports (section III-A),
which are not available: 3 bands over a Voronoi map of open water, thin ice and
thick ice, Gaussian sensor noise, thin-cloud haze blobs and shadow blobs.  The
module holds none of the labelling method's arithmetic; it is shared by the
tests, the oracle runs and the benchmark.

Recipes:
  * ``config_small()``: 512x512 uint8, one haze and one shadow blob of sigma 96
    px, seed 1 (each blob covers about 15 % of the scene at g >= 1/2).
  * ``config_tile()``: 10980x10980 uint16 reflectance, 4 haze blobs covering
    ~10 % and 2 shadow blobs covering ~5 % (sigma ~832 px), seed 2.
"""
from .synth import (Blob, SceneSpec, blobs_for_coverage, coverage, config_small, config_tile,
                    generate, generate_u8, to_u16)

__all__ = ["Blob", "SceneSpec", "blobs_for_coverage", "coverage", "config_small", "config_tile",
           "generate", "generate_u8", "to_u16"]
