"""Python binding of the MI355X adaptive-precision IVF-PQ search library.

Thin ctypes marshalling over the C ABI declared in include/amp.h; every
function keeps the C name.  Numpy arrays are passed for host memory, torch
CUDA tensors (via data_ptr) for device memory.  No search arithmetic happens
here: if the HIP library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamp.so")

AMP_OK, AMP_EINVAL, AMP_ENOMEM, AMP_EDEVICE, AMP_EIO, AMP_EFORMAT = 0, -1, -2, -3, -4, -5
AMP_EBUSY, AMP_ECANCELED, AMP_EUNSUPPORTED, AMP_EOVERFLOW = -6, -7, -8, -9
AMP_L2, AMP_IP, AMP_L1 = 0, 1, 2
METRICS = {"l2": AMP_L2, "ip": AMP_IP, "l1": AMP_L1}
METRIC_NAMES = {v: k for k, v in METRICS.items()}
AMP_GRID_U9, AMP_GRID_E4M3 = 0, 1
AMP_MEM_HOST, AMP_MEM_DEVICE = 0, 1
AMP_POLICY_FP32, AMP_POLICY_FIXED, AMP_POLICY_ADAPTIVE, AMP_POLICY_EXPLICIT = 0, 1, 2, 3
AMP_LUT_BF16, AMP_LUT_F16, AMP_LUT_F8E4M3 = 1, 2, 3
AMP_F32, AMP_BF16 = 0, 1
AMP_N_STAGES = 9
STAGES = ("cl", "topn", "predict", "base", "queue", "scan1", "scan2", "merge", "total")
POLICIES = {"fp32": AMP_POLICY_FP32, "fixed": AMP_POLICY_FIXED,
            "adaptive": AMP_POLICY_ADAPTIVE, "explicit": AMP_POLICY_EXPLICIT}
AMP_CL_FP32, AMP_CL_FIXED, AMP_CL_ADAPTIVE = 0, 1, 2
CL_POLICIES = {"fp32": AMP_CL_FP32, "fixed": AMP_CL_FIXED, "adaptive": AMP_CL_ADAPTIVE}


class AmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Arrays(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", C.c_int32), ("nlist", C.c_int32), ("metric", C.c_int32),
                ("grid_kind", C.c_int32), ("grid_e", C.c_int32),
                ("centroids", C.c_void_p), ("codebook", C.c_void_p), ("list_offsets", C.c_void_p),
                ("ids", C.c_void_p), ("codes", C.c_void_p), ("radq", C.c_void_p)]


class _Model(C.Structure):
    _fields_ = [("n_sv", C.c_int32), ("sv", C.c_void_p), ("beta", C.c_void_p), ("table", C.c_void_p),
                ("beta0", C.c_int64), ("feat_lo", C.c_int64 * 5), ("feat_mul", C.c_int64 * 5),
                ("g_mul", C.c_uint64), ("theta", C.c_int64 * 3)]


class _Policy(C.Structure):
    _fields_ = [("kind", C.c_int32), ("fixed_bits", C.c_int32), ("allowed_bits_mask", C.c_uint32),
                ("lut_dtype", C.c_int32), ("margin_q40", C.c_int64), ("explicit_bits", C.c_void_p),
                ("granularity", C.c_int32)]


AMP_GRAN_PAIR, AMP_GRAN_SUBSPACE = 0, 1
GRANULARITIES = {"pair": AMP_GRAN_PAIR, "subspace": AMP_GRAN_SUBSPACE}


AMP_SEARCH_GRAPH = 1
AMP_SEARCH_DEVICE_SIZES = 2


class _LutExport(C.Structure):
    _fields_ = [("q", C.c_void_p), ("shift", C.c_void_p), ("base", C.c_void_p), ("t", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("mem", C.c_int32), ("stream", C.c_void_p), ("out_qdist", C.c_void_p),
                ("out_probes", C.c_void_p), ("out_bits", C.c_void_p), ("out_coarse", C.c_void_p),
                ("stage_ms", C.c_void_p), ("flags", C.c_uint32), ("q_dtype", C.c_int32), ("work", C.c_void_p),
                ("out_status", C.c_void_p), ("kmax", C.c_int32), ("npmax", C.c_int32),
                ("lut_export", C.POINTER(_LutExport)), ("cl_policy", C.c_int32), ("cl_bits", C.c_int32),
                ("out_cl_dist", C.c_void_p), ("out_cl_bits", C.c_void_p)]


class _ClMap(C.Structure):
    _fields_ = [("S", C.c_int32), ("P", C.c_int32), ("w", C.c_int32), ("o", C.c_float), ("ec", C.c_int32),
                ("assign", C.c_void_p), ("centre", C.c_void_p), ("radius", C.c_void_p), ("count", C.c_void_p)]


class _BuildParams(C.Structure):
    _fields_ = [("nlist", C.c_int32), ("M", C.c_int32), ("kmeans_iters", C.c_int32), ("metric", C.c_int32),
                ("grid_kind", C.c_int32), ("integer_data", C.c_int32), ("base_dtype", C.c_int32),
                ("seed", C.c_uint64)]


class _TrainParams(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("max_iter", C.c_int32), ("gamma", C.c_double),
                ("C", C.c_double), ("epsilon", C.c_double), ("tol", C.c_double),
                ("allowed_bits_mask", C.c_uint32), ("seed", C.c_uint64), ("granularity", C.c_int32)]


class _TrainReport(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("label_hist", C.c_int64 * 4), ("n_samples", C.c_int32),
                ("n_sv", C.c_int32), ("smo_iterations", C.c_int32), ("train_rmse", C.c_double)]


_lib = None
EXPORTS = ("amp_index_from_arrays", "amp_index_build", "amp_index_get_arrays", "amp_index_set_predictor", "amp_index_get_predictor",
           "amp_index_train_predictor", "amp_svr_fit",
           "amp_index_build_cl_map", "amp_index_get_cl_map", "amp_index_set_cl_predictor",
           "amp_index_get_cl_predictor", "amp_index_train_cl_predictor",
           "amp_index_to_device",
           "amp_index_save", "amp_index_load", "amp_index_info", "amp_search", "amp_search_noalloc",
           "amp_index_autotune", "amp_index_get_tuning", "amp_index_set_tuning",
           "amp_server_create", "amp_server_submit", "amp_server_cancel", "amp_server_flush",
           "amp_server_stats", "amp_server_destroy",
           "amp_index_free", "amp_status_str", "amp_last_error")


def lib():
    """Load libamp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_07156_amd/build.py")
        try:
            # load torch's HIP runtime first: the library then binds to the
            # same runtime (matched by soname), so device pointers and streams
            # are shared with torch in this process
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.amp_index_from_arrays.argtypes = [C.POINTER(_Arrays), C.POINTER(C.c_void_p)]
        L.amp_index_set_predictor.argtypes = [C.c_void_p, C.POINTER(_Model)]
        L.amp_index_get_predictor.argtypes = [C.c_void_p, C.POINTER(_Model), C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_int32]
        L.amp_index_train_predictor.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                                C.POINTER(_TrainParams), C.POINTER(_TrainReport)]
        L.amp_svr_fit.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                  C.c_int32, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.amp_index_build_cl_map.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64]
        L.amp_index_get_cl_map.argtypes = [C.c_void_p, C.POINTER(_ClMap)]
        L.amp_index_set_cl_predictor.argtypes = [C.c_void_p, C.POINTER(_Model)]
        L.amp_index_get_cl_predictor.argtypes = L.amp_index_get_predictor.argtypes
        L.amp_index_train_cl_predictor.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                                   C.POINTER(_TrainParams), C.POINTER(_TrainReport)]
        L.amp_index_to_device.argtypes = [C.c_void_p, C.c_int32]
        L.amp_index_save.argtypes = [C.c_void_p, C.c_char_p]
        L.amp_index_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.amp_index_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.amp_search.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(_Policy), C.POINTER(_Opts), C.c_void_p, C.c_void_p]
        L.amp_search_noalloc.argtypes = L.amp_search.argtypes
        L.amp_index_free.argtypes = [C.c_void_p]
        L.amp_index_free.restype = None
        L.amp_status_str.argtypes = [C.c_int32]
        L.amp_status_str.restype = C.c_char_p
        L.amp_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("amp_index_free", "amp_server_destroy", "amp_status_str", "amp_last_error"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def amp_status_str(status):
    return lib().amp_status_str(status).decode()


def amp_last_error():
    return lib().amp_last_error().decode()


def _check(status):
    if status != AMP_OK:
        raise AmpError(status, f"{amp_status_str(status)}: {amp_last_error()}")


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


class Index:
    """Owning wrapper of an amp_index handle."""

    def __init__(self, handle):
        self.handle = C.c_void_p(handle)

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.amp_index_free(self.handle)
            self.handle = C.c_void_p(None)

    def free(self):
        self.__del__()


def amp_index_from_arrays(ix):
    """``ix``: dict as produced by amp_data.build_index."""
    keep = dict(
        centroids=np.ascontiguousarray(ix["centroids"], dtype=np.float32),
        codebook=np.ascontiguousarray(ix["codebook"], dtype=np.float32),
        offsets=np.ascontiguousarray(ix["list_offsets"], dtype=np.int64),
        ids=np.ascontiguousarray(ix["ids"], dtype=np.int64),
        codes=np.ascontiguousarray(ix["codes"], dtype=np.uint8),
        radq=np.ascontiguousarray(ix["radq"], dtype=np.int32),
    )
    a = _Arrays(int(ix["d"]), int(ix["M"]), int(ix["nlist"]),
                METRICS[ix.get("metric", "l2")],
                AMP_GRID_U9 if ix.get("grid_kind", "u9") == "u9" else AMP_GRID_E4M3,
                int(ix["grid_e"]), _ptr(keep["centroids"]), _ptr(keep["codebook"]),
                _ptr(keep["offsets"]), _ptr(keep["ids"]), _ptr(keep["codes"]), _ptr(keep["radq"]))
    h = C.c_void_p()
    _check(lib().amp_index_from_arrays(C.byref(a), C.byref(h)))
    return Index(h.value)


def amp_index_build(base, nlist, M, iters=20, seed=0, integer_data=False, grid_kind="u9", metric="l2",
                    ids=None):
    """Build an index on the current device from host vectors ``base`` [n, d]
    (float32, or bfloat16 bit patterns as a uint16 array)."""
    if metric not in METRICS or grid_kind not in ("u9", "e4m3"):
        raise ValueError(f"unknown metric {metric!r} or grid kind {grid_kind!r}")
    bf16 = getattr(base, "dtype", None) == np.uint16
    x = np.ascontiguousarray(base, dtype=np.uint16 if bf16 else np.float32)
    if x.ndim != 2:
        raise ValueError("base must be [n, d]")
    idv = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    if idv is not None and idv.shape != (x.shape[0],):
        raise ValueError("ids must have one entry per vector")
    p = _BuildParams(int(nlist), int(M), int(iters), METRICS[metric],
                     AMP_GRID_U9 if grid_kind == "u9" else AMP_GRID_E4M3, int(bool(integer_data)),
                     AMP_BF16 if bf16 else AMP_F32, int(seed))
    h = C.c_void_p()
    _check(lib().amp_index_build(_ptr(x), int(x.shape[0]), int(x.shape[1]), _ptr(idv), C.byref(p), C.byref(h)))
    return Index(h.value)


def amp_index_get_arrays(index):
    """Copies of the index arrays, as a dict in the amp_index_from_arrays format."""
    a = _Arrays()
    _check(lib().amp_index_get_arrays(index.handle, C.byref(a)))
    info = amp_index_info(index)
    d, M, nl, n = a.d, a.M, a.nlist, info["n"]

    def arr(ptr, ctype, shape, dt):
        if n == 0 and ptr is None:
            return np.zeros(shape, dt)
        buf = (ctype * int(np.prod(shape))).from_address(ptr)
        return np.ctypeslib.as_array(buf).reshape(shape).astype(dt, copy=True)

    offs = arr(a.list_offsets, C.c_int64, (nl + 1,), np.int64)
    return dict(d=d, M=M, dsub=d // M, nlist=nl, metric=METRIC_NAMES[a.metric],
                grid_kind="u9" if a.grid_kind == AMP_GRID_U9 else "e4m3", grid_e=a.grid_e,
                centroids=arr(a.centroids, C.c_float, (nl, d), np.float32),
                codebook=arr(a.codebook, C.c_float, (M, 256, d // M), np.float32),
                list_offsets=offs, list_sizes=np.diff(offs).astype(np.int32),
                ids=arr(a.ids, C.c_int64, (n,), np.int64),
                codes=arr(a.codes, C.c_uint8, (n, M), np.uint8),
                radq=arr(a.radq, C.c_int32, (nl,), np.int32))


def amp_index_set_predictor(index, model):
    sv = np.ascontiguousarray(model["sv"], dtype=np.int32)
    beta = np.ascontiguousarray(model["beta"], dtype=np.int32)
    table = np.ascontiguousarray(model["table"], dtype=np.int32)
    m = _Model(int(model["n_sv"]), _ptr(sv), _ptr(beta), _ptr(table), int(model["beta0"]),
               (C.c_int64 * 5)(*[int(v) for v in model["feat_lo"]]),
               (C.c_int64 * 5)(*[int(v) for v in model["feat_mul"]]),
               int(model["g_mul"]), (C.c_int64 * 3)(*[int(v) for v in model["theta"]]))
    _check(lib().amp_index_set_predictor(index.handle, C.byref(m)))


def amp_index_get_predictor(index):
    """The index's predictor as a model dict (the format amp_index_set_predictor takes)."""
    m = _Model()
    st = lib().amp_index_get_predictor(index.handle, C.byref(m), None, None, None, 0)
    n = m.n_sv
    if st != AMP_OK and n == 0 and "no predictor" in amp_last_error():
        _check(st)
    sv = np.zeros((max(n, 1), 5), np.int32)
    beta = np.zeros(max(n, 1), np.int32)
    table = np.zeros(1024, np.int32)
    _check(lib().amp_index_get_predictor(index.handle, C.byref(m), _ptr(sv), _ptr(beta), _ptr(table), n))
    return dict(n_sv=n, sv=sv[:n], beta=beta[:n], table=table, beta0=m.beta0,
                feat_lo=np.array(m.feat_lo[:], np.int64), feat_mul=np.array(m.feat_mul[:], np.int64),
                g_mul=int(m.g_mul), theta=np.array(m.theta[:], np.int64))


def amp_index_train_predictor(index, train_queries, k, nprobe, n_samples=1280, gamma=1.0, C_=1.0,
                              epsilon=0.05, tol=1e-3, max_iter=0, allowed=(4, 8, 12, 16), seed=0,
                              granularity="pair"):
    """Fit and attach the precision predictor; returns the training report."""
    q = np.ascontiguousarray(train_queries, dtype=np.float32)
    mask = 0
    for b in allowed:
        mask |= 1 << int(b)
    p = _TrainParams(int(n_samples), int(max_iter), float(gamma), float(C_), float(epsilon), float(tol),
                     mask, int(seed), GRANULARITIES[granularity])
    r = _TrainReport()
    _check(lib().amp_index_train_predictor(index.handle, _ptr(q), int(q.shape[0]), int(k), int(nprobe),
                                           C.byref(p), C.byref(r)))
    return dict(n_pairs=r.n_pairs, label_hist=list(r.label_hist), n_samples=r.n_samples, n_sv=r.n_sv,
                smo_iterations=r.smo_iterations, train_rmse=r.train_rmse)


def amp_index_build_cl_map(index, S, P, iters=20, seed=0):
    """Vector space division for integer cluster locating (host)."""
    _check(lib().amp_index_build_cl_map(index.handle, int(S), int(P), int(iters), int(seed)))


def amp_index_get_cl_map(index):
    """Copies of the sub-space map: dict S, P, w, o (float32), ec, assign
    [nlist, S], centre [S, P, w], radius [S, P], count [S, P]."""
    m = _ClMap()
    _check(lib().amp_index_get_cl_map(index.handle, C.byref(m)))
    nl = amp_index_info(index)["nlist"]

    def arr(ptr, shape):
        buf = (C.c_int32 * int(np.prod(shape))).from_address(ptr)
        return np.ctypeslib.as_array(buf).reshape(shape).astype(np.int64, copy=True)

    return dict(S=m.S, P=m.P, w=m.w, o=np.float32(m.o), ec=m.ec, assign=arr(m.assign, (nl, m.S)),
                centre=arr(m.centre, (m.S, m.P, m.w)), radius=arr(m.radius, (m.S, m.P)),
                count=arr(m.count, (m.S, m.P)))


def _model_struct(model):
    sv = np.ascontiguousarray(model["sv"], dtype=np.int32)
    beta = np.ascontiguousarray(model["beta"], dtype=np.int32)
    table = np.ascontiguousarray(model["table"], dtype=np.int32)
    m = _Model(int(model["n_sv"]), _ptr(sv), _ptr(beta), _ptr(table), int(model["beta0"]),
               (C.c_int64 * 5)(*[int(v) for v in model["feat_lo"]]),
               (C.c_int64 * 5)(*[int(v) for v in model["feat_mul"]]),
               int(model["g_mul"]), (C.c_int64 * 3)(*[int(v) for v in model["theta"]]))
    return m, (sv, beta, table)


def amp_index_set_cl_predictor(index, model):
    m, keep = _model_struct(model)
    _check(lib().amp_index_set_cl_predictor(index.handle, C.byref(m)))


def amp_index_get_cl_predictor(index):
    """The index's CL predictor as a model dict."""
    m = _Model()
    st = lib().amp_index_get_cl_predictor(index.handle, C.byref(m), None, None, None, 0)
    n = m.n_sv
    if st != AMP_OK and n == 0 and "no CL predictor" in amp_last_error():
        _check(st)
    sv = np.zeros((max(n, 1), 5), np.int32)
    beta = np.zeros(max(n, 1), np.int32)
    table = np.zeros(1024, np.int32)
    _check(lib().amp_index_get_cl_predictor(index.handle, C.byref(m), _ptr(sv), _ptr(beta), _ptr(table), n))
    return dict(n_sv=n, sv=sv[:n], beta=beta[:n], table=table, beta0=m.beta0,
                feat_lo=np.array(m.feat_lo[:], np.int64), feat_mul=np.array(m.feat_mul[:], np.int64),
                g_mul=int(m.g_mul), theta=np.array(m.theta[:], np.int64))


def amp_index_train_cl_predictor(index, train_queries, nprobe, low=4, n_samples=1280, gamma=0.1, C_=10.0,
                                 epsilon=0.1, tol=1e-3, max_iter=0, seed=0):
    """Fit and attach the CL predictor (paper's CL setting gamma 0.1, C 10);
    returns the training report (label_hist[0]: low labels, [1]: 8 bits)."""
    q = np.ascontiguousarray(train_queries, dtype=np.float32)
    p = _TrainParams(int(n_samples), int(max_iter), float(gamma), float(C_), float(epsilon), float(tol), 0,
                     int(seed))
    r = _TrainReport()
    _check(lib().amp_index_train_cl_predictor(index.handle, _ptr(q), int(q.shape[0]), int(nprobe), int(low),
                                              C.byref(p), C.byref(r)))
    return dict(n_pairs=r.n_pairs, label_hist=list(r.label_hist)[:2], n_samples=r.n_samples, n_sv=r.n_sv,
                smo_iterations=r.smo_iterations, train_rmse=r.train_rmse)


def amp_svr_fit(K, y, C_=1.0, epsilon=0.1, tol=1e-3, max_iter=100000):
    """Test hook: the SVR solver of the trainer on a precomputed kernel."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    coef = np.zeros(len(y), np.float64)
    b, it = C.c_double(), C.c_int32()
    _check(lib().amp_svr_fit(_ptr(K), _ptr(y), len(y), float(C_), float(epsilon), float(tol), int(max_iter),
                             _ptr(coef), C.byref(b), C.byref(it)))
    return coef, b.value, it.value


class _TuneEntry(C.Structure):
    _fields_ = [("policy_kind", C.c_int32), ("nq_log2", C.c_int32), ("chunk", C.c_int64), ("chunk1", C.c_int64),
                ("narrow", C.c_int32), ("lut_dtype", C.c_int32), ("queue", C.c_int32), ("ms", C.c_float),
                ("ms_default", C.c_float),
                ("trials", C.c_int32)]


def _tune_dict(e):
    return {n: getattr(e, n) for n, _ in _TuneEntry._fields_}


def amp_index_autotune(index, queries, k, nprobe, policy="fixed", bits=16, allowed=(4, 8, 12, 16), margin_q40=0,
                       lut_dtype=0, repeats=5, granularity="pair"):
    """Time candidate search schedules for this batch shape on the current
    device and record the fastest in the index; returns the entry (dict)."""
    bf16 = getattr(queries, "dtype", None) == np.uint16
    q = np.ascontiguousarray(queries, dtype=np.uint16 if bf16 else np.float32)
    nq = int(q.shape[0])
    kk = np.atleast_1d(np.asarray(k, dtype=np.int32))
    npb = np.atleast_1d(np.asarray(nprobe, dtype=np.int32))
    per_query = int(kk.size > 1 or npb.size > 1)
    if per_query:
        kk = np.ascontiguousarray(np.broadcast_to(kk, (nq,)), dtype=np.int32)
        npb = np.ascontiguousarray(np.broadcast_to(npb, (nq,)), dtype=np.int32)
    pol, _ = make_policy(policy, bits, allowed, margin_q40, None, lut_dtype, granularity)
    e = _TuneEntry()
    _check(lib().amp_index_autotune(index.handle, _ptr(q), nq, _ptr(kk), _ptr(npb), per_query, C.byref(pol),
                                    AMP_BF16 if bf16 else AMP_F32, int(repeats), C.byref(e)))
    return _tune_dict(e)


def amp_index_get_tuning(index):
    n = C.c_int32()
    _check(lib().amp_index_get_tuning(index.handle, None, 0, C.byref(n)))
    arr = (_TuneEntry * max(1, n.value))()
    _check(lib().amp_index_get_tuning(index.handle, arr, n.value, C.byref(n)))
    return [_tune_dict(arr[i]) for i in range(n.value)]


def amp_index_set_tuning(index, entries):
    arr = (_TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        for n, _ in _TuneEntry._fields_:
            setattr(arr[i], n, e.get(n, -1 if n == "narrow" else 0))
    _check(lib().amp_index_set_tuning(index.handle, arr, len(entries)))


def amp_index_to_device(index, device=0):
    _check(lib().amp_index_to_device(index.handle, int(device)))


def amp_index_save(index, path):
    _check(lib().amp_index_save(index.handle, str(path).encode()))


def amp_index_load(path):
    h = C.c_void_p()
    _check(lib().amp_index_load(str(path).encode(), C.byref(h)))
    return Index(h.value)


def amp_index_info(index):
    d, M, nl, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().amp_index_info(index.handle, C.byref(d), C.byref(M), C.byref(nl), C.byref(n)))
    return dict(d=d.value, M=M.value, nlist=nl.value, n=n.value)


def make_policy(policy="fixed", bits=16, allowed=(4, 8, 12, 16), margin_q40=0,
                explicit_bits=None, lut_dtype=0, granularity="pair"):
    mask = 0
    for b in allowed:
        mask |= 1 << int(b)
    xb = None if explicit_bits is None else np.ascontiguousarray(explicit_bits, dtype=np.uint8)
    pol = _Policy(POLICIES[policy], int(bits), mask, int(lut_dtype), int(margin_q40), _ptr(xb),
                  GRANULARITIES[granularity])
    return pol, xb


def amp_search(index, queries, k, nprobe, policy="fixed", bits=16, allowed=(4, 8, 12, 16),
               margin_q40=0, explicit_bits=None, lut_dtype=0, want_qdist=True,
               want_probes=False, want_bits=False, want_coarse=False, stage_ms=False,
               out=None, stream=None, graph=False, q_dtype=None, work=False, kmax=None, npmax=None,
               want_status=False, cl_policy="fp32", cl_bits=0, want_cl_dist=False, want_cl_bits=False,
               granularity="pair", _entry="amp_search"):
    """Search a batch.

    Host mode (``queries`` a numpy array): returns a dict of numpy arrays.
    Device mode (``queries`` a torch CUDA tensor): ``out`` must be a dict of
    preallocated torch CUDA tensors ids [nq,kmax] int64, dist [nq,kmax] float32
    and optionally qdist / probes / bits / coarse / status (int32 [1]) /
    lut_q, lut_shift, lut_base, lut_t (the LUT export test hook) / cl_dist
    (int32 [nq, nlist]) / cl_bits (uint8 [nq, S, P]); work is enqueued
    on ``stream`` (a torch stream or raw handle) and the call returns at once.
    Device mode also takes ``k`` / ``nprobe`` as int32 CUDA tensors of nq
    entries (device-resident per-query sizes, bounded by ``kmax`` / ``npmax``).
    ``cl_policy`` "fixed" / "adaptive" selects integer cluster locating on
    8-bit codes (``cl_bits``: the fixed width, or the adaptive low width).
    """
    device = hasattr(queries, "data_ptr")
    nq = int(queries.shape[0])
    if q_dtype is None:
        q_dtype = "bf16" if str(getattr(queries, "dtype", "")) in ("uint16", "torch.bfloat16") else "f32"
    qd = AMP_BF16 if q_dtype == "bf16" else AMP_F32
    flags = AMP_SEARCH_GRAPH if graph else 0
    dev_sizes = hasattr(k, "data_ptr") or hasattr(nprobe, "data_ptr")
    if dev_sizes:
        if not (hasattr(k, "data_ptr") and hasattr(nprobe, "data_ptr")) or kmax is None or npmax is None:
            raise ValueError("device-resident sizes need both k and nprobe as device tensors and kmax / npmax")
        if tuple(k.shape) != (nq,) or tuple(nprobe.shape) != (nq,):
            raise ValueError("device k / nprobe must hold one entry per query")
        kk, npb, per_query = k, nprobe, 1
        kmax, npmax = int(kmax), int(npmax)
        flags |= AMP_SEARCH_DEVICE_SIZES
    else:
        kk = np.atleast_1d(np.asarray(k, dtype=np.int32))
        npb = np.atleast_1d(np.asarray(nprobe, dtype=np.int32))
        per_query = int(kk.size > 1 or npb.size > 1)
        if per_query:
            kk = np.ascontiguousarray(np.broadcast_to(kk, (nq,)), dtype=np.int32)
            npb = np.ascontiguousarray(np.broadcast_to(npb, (nq,)), dtype=np.int32)
        kmax, npmax = int(kk.max()), int(npb.max())
    pol, xb = make_policy(policy, bits, allowed, margin_q40, explicit_bits, lut_dtype, granularity)
    ms = np.zeros(AMP_N_STAGES, dtype=np.float32) if stage_ms else None
    wk = np.zeros(4, dtype=np.int64) if work else None
    fn = getattr(lib(), _entry)
    if device:
        o = out
        sh = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        exp = None
        if o.get("lut_q") is not None:
            exp = _LutExport(_ptr(o["lut_q"]), _ptr(o["lut_shift"]), _ptr(o["lut_base"]), _ptr(o.get("lut_t")))
        opts = _Opts(AMP_MEM_DEVICE, C.c_void_p(sh) if sh else None, _ptr(o.get("qdist")),
                     _ptr(o.get("probes")), _ptr(o.get("bits")), _ptr(o.get("coarse")), _ptr(ms),
                     flags, qd, _ptr(wk), _ptr(o.get("status")), kmax if dev_sizes else 0,
                     npmax if dev_sizes else 0, C.pointer(exp) if exp is not None else None,
                     CL_POLICIES[cl_policy], int(cl_bits), _ptr(o.get("cl_dist")), _ptr(o.get("cl_bits")))
        _check(fn(index.handle, _ptr(queries), nq, _ptr(kk), _ptr(npb), per_query,
                  C.byref(pol), C.byref(opts), _ptr(o["ids"]), _ptr(o["dist"])))
        if stage_ms:
            o["stage_ms"] = dict(zip(STAGES, ms.tolist()))
        if work:
            o["work"] = dict(zip(("scan_bytes", "live_pairs", "dead_pairs", "unit_bytes"), wk.tolist()))
        return o
    q = np.ascontiguousarray(queries, dtype=np.uint16 if qd == AMP_BF16 else np.float32)
    res = dict(ids=np.empty((nq, kmax), np.int64), dist=np.empty((nq, kmax), np.float32))
    if want_qdist:
        res["qdist"] = np.empty((nq, kmax), np.int64)
    if want_probes:
        res["probes"] = np.empty((nq, npmax), np.int32)
    if want_bits:
        res["bits"] = np.empty((nq, npmax), np.uint8)
    if want_coarse:
        info = amp_index_info(index)
        res["coarse"] = np.empty((nq, info["nlist"]), np.float32)
    if want_cl_dist:
        res["cl_dist"] = np.empty((nq, amp_index_info(index)["nlist"]), np.int32)
    if want_cl_bits:
        cm = _ClMap()
        _check(lib().amp_index_get_cl_map(index.handle, C.byref(cm)))
        res["cl_bits"] = np.empty((nq, cm.S, cm.P), np.uint8)
    st = np.zeros(1, np.int32) if want_status else None
    opts = _Opts(AMP_MEM_HOST, None, _ptr(res.get("qdist")), _ptr(res.get("probes")),
                 _ptr(res.get("bits")), _ptr(res.get("coarse")), _ptr(ms), flags, qd, _ptr(wk), _ptr(st), 0, 0,
                 None, CL_POLICIES[cl_policy], int(cl_bits), _ptr(res.get("cl_dist")), _ptr(res.get("cl_bits")))
    status = fn(index.handle, _ptr(q), nq, _ptr(kk), _ptr(npb), per_query,
                C.byref(pol), C.byref(opts), _ptr(res["ids"]), _ptr(res["dist"]))
    if want_status:
        res["status"] = int(status)
        if status not in (AMP_OK, AMP_EOVERFLOW):
            _check(status)
    else:
        _check(status)
    if stage_ms:
        res["stage_ms"] = dict(zip(STAGES, ms.tolist()))
    if work:
        res["work"] = dict(zip(("scan_bytes", "live_pairs", "dead_pairs", "unit_bytes"), wk.tolist()))
    return res


def amp_search_noalloc(index, queries, k, nprobe, **kw):
    """amp_search on the library's fixed scratch (no allocation): device mode
    only, per-query sizes as device tensors; see amp_search."""
    return amp_search(index, queries, k, nprobe, _entry="amp_search_noalloc", **kw)


# ------------------------------------------------------------------ serving loop
DONE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32)


class _ServerConfig(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("max_pending", C.c_int32), ("max_k", C.c_int32),
                ("max_nprobe", C.c_int32), ("batch_window_us", C.c_int32), ("q_dtype", C.c_int32),
                ("policy", _Policy)]


class _Request(C.Structure):
    _fields_ = [("query", C.c_void_p), ("k", C.c_int32), ("nprobe", C.c_int32), ("out_ids", C.c_void_p),
                ("out_dist", C.c_void_p), ("out_qdist", C.c_void_p), ("done", DONE_FN), ("user", C.c_void_p),
                ("policy", C.c_void_p), ("arrival_ns", C.c_int64)]


class _Report(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "rejected", "completed", "cancelled", "failed", "batches",
                                         "pending", "in_flight")] + \
               [(n, C.c_double) for n in ("elapsed_s", "qps", "mean_batch", "p50_ms", "p99_ms", "max_ms")]


class Server:
    """Owning wrapper of an amp_server handle.  Buffers and callbacks of
    submitted requests are kept alive here until flush()."""

    def __init__(self, handle, index, q_dtype):
        self.handle = C.c_void_p(handle)
        self.index = index  # the index must outlive the server
        self.q_dtype = q_dtype
        self._keep = []
        self._tl = threading.local()

    def submit_raw(self, query_addr, k, nprobe, ids_addr, dist_addr, qdist_addr=0, arrival_ns=0):
        """Fast path for load generators: host addresses as integers, no
        callback, default policy; the caller keeps the buffers alive until
        the request completes.  Returns the status (no exception)."""
        tl = self._tl
        if not hasattr(tl, "req"):
            tl.req = _Request()
            tl.ticket = C.c_uint64()
            tl.args = (self.handle, C.byref(tl.req), C.byref(tl.ticket))
            tl.fn = lib().amp_server_submit
        r = tl.req
        r.query, r.k, r.nprobe = query_addr, k, nprobe
        r.out_ids, r.out_dist, r.out_qdist = ids_addr, dist_addr, qdist_addr or None
        r.arrival_ns = arrival_ns
        return tl.fn(*tl.args)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.amp_server_destroy(self.handle)
            self.handle = C.c_void_p(None)
            self._keep = []


def amp_server_create(index, max_batch=1024, max_pending=0, max_k=100, max_nprobe=0, batch_window_us=0,
                      q_dtype="f32", policy="fixed", bits=16, allowed=(4, 8, 12, 16), margin_q40=0, lut_dtype=0,
                      granularity="pair"):
    pol, _ = make_policy(policy, bits, allowed, margin_q40, None, lut_dtype, granularity)
    qd = AMP_BF16 if q_dtype == "bf16" else AMP_F32
    cfg = _ServerConfig(int(max_batch), int(max_pending), int(max_k), int(max_nprobe), int(batch_window_us), qd, pol)
    h = C.c_void_p()
    _check(lib().amp_server_create(index.handle, C.byref(cfg), C.byref(h)))
    return Server(h.value, index, qd)


def amp_server_submit(server, query, k, nprobe, out_ids, out_dist, out_qdist=None, done=None, arrival_ns=0,
                      policy=None):
    """Queue one request.  ``query``: host row (float32, or uint16 bfloat16
    patterns for a BF16 server); ``out_*``: host numpy buffers of >= k
    entries; ``done(status)``: optional callable run on the server thread;
    ``policy``: None or a make_policy() tuple.  Returns the ticket."""
    q = np.ascontiguousarray(query, dtype=np.uint16 if server.q_dtype == AMP_BF16 else np.float32)
    cb = DONE_FN(lambda user, st: done(st)) if done is not None else DONE_FN()
    pol = policy[0] if policy is not None else None
    r = _Request(_ptr(q), int(k), int(nprobe), _ptr(out_ids), _ptr(out_dist), _ptr(out_qdist), cb, None,
                 C.cast(C.pointer(pol), C.c_void_p) if pol is not None else None, int(arrival_ns))
    t = C.c_uint64()
    _check(lib().amp_server_submit(server.handle, C.byref(r), C.byref(t)))
    server._keep.append((out_ids, out_dist, out_qdist, cb, pol))
    return t.value


def amp_server_cancel(server, ticket):
    _check(lib().amp_server_cancel(server.handle, C.c_uint64(ticket)))


def amp_server_flush(server):
    _check(lib().amp_server_flush(server.handle))
    server._keep = []


def amp_server_stats(server, reset=False):
    r = _Report()
    _check(lib().amp_server_stats(server.handle, C.byref(r), int(bool(reset))))
    return {n: getattr(r, n) for n, _ in _Report._fields_}


def amp_server_destroy(server):
    server.close()
