"""CPU oracle of the cluster-adaptive IVF-PQ search — TEST INFRASTRUCTURE.

A plain, slow, obviously correct FP64 / int64 implementation of what the GPU
path computes, written from the paper (Sec. 2.1 stages CL, RC, LC, DC, TS;
Sec. 3.3-3.4 precision prediction; Sec. 4.1 DRM/TSM).  It shares no code with
the HIP library and imports nothing from it.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import or call it; the product never
does.

Pinned by the CPU tests against closed forms, brute force, library routines
and invariants, except where a function's docstring says "parity unpinned".
"""
from .search import (  # noqa: F401
    coarse_distances, select_probes, residual_f32, grid, e4m3_round_int,
    index_grid, lut_int, lut_f64, quantize_lut, mitchell_log2_q8,
    feature_u, svr_eval, bits_from_score, predict_pair_bits, dc_ts, search,
)
from .exact import exact_knn, recall_1_at, recall_at  # noqa: F401
from . import cl  # noqa: F401  (reduced-precision cluster locating)
