"""Seeded Gaussian-mixture workloads shaped like the paper's datasets.

The paper evaluates on SIFT100M / DEEP100M (uint8, d = 128 / 96, 10 000
queries; Sec. 5.1) and SIFT1M / GIST1M (d = 128 / 960; Sec. 5.4, Table 3).
None of those datasets is available here, so each workload below is a
synthetic stand-in with the dimensionality, value range and cluster structure
of the corresponding setting.  Every array is a pure function of
(workload, seed, sizes): numpy's PCG64 generator seeded per purpose.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int            # base vectors
    d: int            # dimensionality
    n_comp: int       # mixture components
    nq: int           # queries
    nlist: int        # IVF lists
    M: int            # PQ subspaces
    nprobe: int       # default probes per query (max for uneven mixes)
    k: int            # neighbours per query
    kind: str         # generator family, see make_base
    seed: int
    metric: str = "l2"
    integer_data: bool = False
    grid_kind: str = "u9"   # operand grid of the LUT build ("u9" | "e4m3")
    nprobe_lo: int = 0      # >0: per-query nprobe uniform in [nprobe_lo, nprobe]

    def scaled(self, n=None, nq=None, nlist=None):
        return dataclasses.replace(self, n=n or self.n, nq=nq or self.nq,
                                   nlist=nlist or self.nlist)


WORKLOADS = {
    # 20k x 32 fp32, 64-component isotropic mixture, IVF64 / PQ8.
    "tiny": Workload("tiny", 20_000, 32, 64, 100, 64, 8, 8, 10, "iso", 1001),
    # 1M x 128, values clipped to [0,255] and rounded (SIFT-like uint8 range).
    "mid": Workload("mid", 1_000_000, 128, 1024, 10_000, 1024, 16, 32, 10,
                    "uint8", 1002, integer_data=True),
    # the same shape with isotropic sigma-32 components (sensitivity run)
    "mid_iso": Workload("mid_iso", 1_000_000, 128, 1024, 10_000, 1024, 16, 32, 10,
                        "uint8iso", 1002, integer_data=True),
    # 10M x 96, 4096 components with Zipf(1.1) weights -> skewed lists.
    "skewed": Workload("skewed", 10_000_000, 96, 4096, 4096, 4096, 24, 128, 10,
                       "zipf", 1003, nprobe_lo=8),
    # 1M x 960, anisotropic per-dimension sigma (GIST-like dimensionality).
    "highdim": Workload("highdim", 1_000_000, 960, 512, 1000, 1024, 120, 64, 100,
                        "aniso", 1004, grid_kind="e4m3"),
    # 5M x 768 unit-normalised, inner product (embedding-style serving).
    "serving": Workload("serving", 5_000_000, 768, 2048, 100_000, 2048, 96, 256, 100,
                        "vmf", 1005, metric="ip"),
}

# sub-seed offsets, one per purpose, so that changing one size never shifts
# another array's random stream
_MEANS, _WEIGHTS, _SIGMA, _POINTS, _QUERIES, _TRAIN, _DRAWS = range(7)


def _rng(seed, purpose):
    return np.random.Generator(np.random.PCG64([seed, purpose]))


def _mixture_params(w: Workload):
    r = _rng(w.seed, _MEANS)
    if w.kind in ("uint8", "uint8iso"):
        means = r.uniform(48.0, 208.0, size=(w.n_comp, w.d))
    elif w.kind == "vmf":
        means = r.standard_normal(size=(w.n_comp, w.d))
        means /= np.linalg.norm(means, axis=1, keepdims=True)
    else:
        means = r.uniform(-10.0, 10.0, size=(w.n_comp, w.d))
    if w.kind == "zipf":
        ranks = np.arange(1, w.n_comp + 1, dtype=np.float64)
        weights = ranks ** -1.1
        weights = weights[_rng(w.seed, _WEIGHTS).permutation(w.n_comp)]
        weights /= weights.sum()
    else:
        weights = np.full(w.n_comp, 1.0 / w.n_comp)
    if w.kind == "aniso":
        sigma = _rng(w.seed, _SIGMA).uniform(0.1, 2.0, size=w.d)
    elif w.kind == "vmf":
        sigma = np.full(w.d, 0.75 / np.sqrt(w.d))
    elif w.kind == "uint8iso":
        sigma = np.full(w.d, ISO_SIGMA)
    else:
        sigma = np.full(w.d, 1.0)
    return means, weights, sigma


# The uint8 workload's components have a low-rank covariance: a 16-dimensional
# latent Gaussian mapped by a per-component random matrix (per-dimension
# spread LATENT_SIGMA) plus small isotropic noise.  Descriptor data such as
# SIFT has an intrinsic dimension of this order; isotropic 128-d clusters
# would make every member of a cluster nearly equidistant from a query.
LATENT_DIM, LATENT_SIGMA, NOISE_SIGMA = 16, 20.0, 2.0
# the harder-overlap variant of the mid workload: isotropic components of
# per-dimension sigma 32 (clipped to [0, 255] and rounded)
ISO_SIGMA = 32.0


def _latent_maps(w: Workload):
    r = _rng(w.seed, _SIGMA + 10)
    return r.standard_normal(size=(w.n_comp, w.d, LATENT_DIM)) * (LATENT_SIGMA / np.sqrt(LATENT_DIM))


def _draw(w: Workload, n: int, purpose: int, chunk: int = 1 << 18):
    means, weights, sigma = _mixture_params(w)
    r = _rng(w.seed, purpose)
    comp = r.choice(w.n_comp, size=n, p=weights)
    out = np.empty((n, w.d), dtype=np.float32)
    maps = _latent_maps(w) if w.kind == "uint8" else None
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        if maps is not None:
            z = r.standard_normal(size=(e - s, LATENT_DIM))
            x = means[comp[s:e]] + r.standard_normal(size=(e - s, w.d)) * NOISE_SIGMA
            cc = comp[s:e]
            order = np.argsort(cc, kind="stable")
            bounds = np.flatnonzero(np.diff(cc[order])) + 1
            for grp in np.split(order, bounds):
                x[grp] += z[grp] @ maps[cc[grp[0]]].T
            x = np.rint(np.clip(x, 0.0, 255.0))
        else:
            x = means[comp[s:e]] + r.standard_normal(size=(e - s, w.d)) * sigma
            if w.kind == "vmf":
                x /= np.linalg.norm(x, axis=1, keepdims=True)
            elif w.kind == "uint8iso":
                x = np.rint(np.clip(x, 0.0, 255.0))
        out[s:e] = x
    if w.kind == "vmf":
        # the serving corpus is stored in bf16: round to bf16 (nearest-even)
        out = _round_bf16(out)
    return out


def _round_bf16(x: np.ndarray) -> np.ndarray:
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def make_base(w: Workload) -> np.ndarray:
    """[n, d] float32 corpus of workload ``w``."""
    return _draw(w, w.n, _POINTS)


def make_queries(w: Workload, nq: int | None = None, train: bool = False) -> np.ndarray:
    """[nq, d] float32 queries from the same mixture (``train``: a disjoint
    stream used only to fit the precision predictor)."""
    return _draw(w, nq or w.nq, _TRAIN if train else _QUERIES)


def draw_nprobe(w: Workload, nq: int) -> np.ndarray:
    """Per-query probe counts: uniform in [nprobe_lo, nprobe] for uneven
    workloads, else the constant nprobe."""
    if w.nprobe_lo <= 0:
        return np.full(nq, w.nprobe, dtype=np.int32)
    r = _rng(w.seed, _DRAWS)
    return r.integers(w.nprobe_lo, w.nprobe + 1, size=nq).astype(np.int32)


def draw_k(w: Workload, nq: int, choices=(10, 50, 100)) -> np.ndarray:
    r = _rng(w.seed, _DRAWS + 1)
    return np.asarray(choices, dtype=np.int32)[r.integers(0, len(choices), size=nq)]


def random_queries(seed: int, nq: int, d: int, scale: float = 1.0) -> np.ndarray:
    r = _rng(seed, _QUERIES)
    return (r.standard_normal(size=(nq, d)) * scale).astype(np.float32)
