"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only *prepares inputs*: Gaussian-mixture corpora and query sets
shaped like the paper's workloads, an IVF-PQ index built from them (k-means
coarse quantiser, residual product quantiser, inverted lists, per-list size and
radius), and seeded parameter sets for the precision predictor.  It holds none
of the search method's arithmetic (no look-up tables, no quantisation of LUT
entries, no distance scans, no predictor evaluation): both the GPU path and the
oracle consume what it produces as plain arrays.
"""
from .synth import WORKLOADS, Workload, make_base, make_queries  # noqa: F401
from .ivfpq import build_index, lossless_index  # noqa: F401
from .model import random_model, rbf_table  # noqa: F401
