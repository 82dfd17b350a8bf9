"""CPU oracle of the sea-ice auto-labeller -- TEST INFRASTRUCTURE ONLY.

A plain single-threaded C implementation (``sil_ref.c``) of the labelling
method of arXiv 2403.13135 (section III-A "Filtering Out the Thin Clouds and
Shadows", section III-B "Auto-labeling Method" and "Scaling Auto-labeling"),
plus a ctypes wrapper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path (the GPU
library and its binding) never does.

Pinned functions (see ``tests/test_oracle_*.py``): V plane and 16-bit rescale,
3x3 median, Otsu threshold and separability, rank truncation, min-max stretch,
the inRange segmentation, per-patch counts.  The composition of the filter is
a reading of the paper's unordered operation list; it is pinned against
independent library routines and closed forms, not against the paper's own
(unpublished) filter.
"""
