"""MI355X-native sea-ice auto-labeller (arXiv 2403.13135, sections III-A/III-B).

``sil.label(scene, params)`` runs the per-pixel thin-cloud/shadow filter,
the HSV threshold segmentation and the per-patch class counts in hand-written
gfx950 kernels behind the C ABI of ``include/sil.h``.
"""
from . import sil
from .sil import Params, SilError, label, hist_dims, validate

__all__ = ["sil", "Params", "SilError", "label", "hist_dims", "validate"]
