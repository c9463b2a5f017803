"""ctypes binding of libdh2.so (C ABI: include/dh2.h).

Argument marshalling only: every computation runs in the native library.
Device vectors are torch tensors (device memory and streams come from torch);
host geometry is numpy.  The library must be built first
(python -m paper_1809_04384_amd.build); loading fails loudly otherwise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdh2.so")

DH2_OK = 0
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_GEOMETRY", 3: "ERR_OOM", 4: "ERR_DEVICE", 5: "ERR_NUMERIC"}
FP64, FP32, BF16X3 = 0, 1, 2
RANKS_EXACT, RANKS_LEARNED = 0, 1
WEIGHTS_HOUSEHOLDER, WEIGHTS_GRAM = 0, 1
QUAD_DEFAULT, QUAD_PAPER = 0, 1
NORM_FROBENIUS, NORM_SPECTRAL = 0, 1
INSPECT = {"near": 1, "leaf_basis": 2, "transfer": 3, "rank_row": 4, "rank_col": 5,
           "sigma_row": 6, "sigma_col": 7, "omega": 8, "basis_weight": 9,
           "total_weight_row": 10, "total_weight_col": 11, "coupling": 12, "rank_pred_row": 13,
           "rank_pred_col": 14}

EXPORTED = ["dh2_build", "dh2_build_ex", "dh2_matvec", "dh2_matvec_profile", "dh2_free", "dh2_last_error",
            "dh2_get_stats", "dh2_plan_create", "dh2_plan_get_sizes", "dh2_plan_export",
            "dh2_plan_free", "dh2_inspect", "dh2_batch_create", "dh2_batch_run", "dh2_batch_free",
            "dh2_matvec_stream", "dh2_build_many", "dh2_matvec_noalloc", "dh2_plan_rank_features"]


class Dh2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("vertices", ctypes.c_void_p),
                ("n_triangles", ctypes.c_int64), ("triangles", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("eta1", ctypes.c_double),
                ("max_nrhs", ctypes.c_int32), ("norm", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("workspace_gb", ctypes.c_double),
                ("rank_mode", ctypes.c_int32), ("sketch_rank", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("weights", ctypes.c_int32), ("quadrature", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("k", ctypes.c_int32),
                ("n", ctypes.c_int64), ("n_clusters", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("depth", ctypes.c_int64), ("n_adm", ctypes.c_int64), ("n_near", ctypes.c_int64),
                ("n_slots", ctypes.c_int64), ("n_row_slots", ctypes.c_int64),
                ("n_col_slots", ctypes.c_int64), ("near_entries", ctypes.c_int64),
                ("coupling_entries", ctypes.c_int64), ("basis_entries", ctypes.c_int64),
                ("rank_max_row", ctypes.c_int32), ("rank_max_col", ctypes.c_int32),
                ("rank_mean_row", ctypes.c_double), ("rank_mean_col", ctypes.c_double),
                ("matvec_bytes", ctypes.c_double), ("matvec_bytes_per_rhs", ctypes.c_double),
                ("ms_structure", ctypes.c_double), ("ms_near", ctypes.c_double),
                ("ms_interp", ctypes.c_double), ("ms_basis_weights", ctypes.c_double),
                ("ms_block_weights", ctypes.c_double), ("ms_total_weights", ctypes.c_double),
                ("ms_truncation", ctypes.c_double), ("ms_projection", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("gemm_flops", ctypes.c_double),
                ("gemm_launches", ctypes.c_int64), ("qr_flops", ctypes.c_double),
                ("batches_basis_weights", ctypes.c_int64), ("batches_block_weights", ctypes.c_int64),
                ("batches_total_weights_row", ctypes.c_int64), ("batches_total_weights_col", ctypes.c_int64),
                ("batches_truncation", ctypes.c_int64),
                ("batches_projection", ctypes.c_int64), ("slots_straddled", ctypes.c_int64),
                ("coupling_regeneration", ctypes.c_double), ("sketch_slots", ctypes.c_int64),
                ("sketch_fallbacks", ctypes.c_int64), ("ms_rank_predict", ctypes.c_double),
                ("mv_variant", ctypes.c_int32 * 4), ("ms_autotune", ctypes.c_double),
                ("weights_gram", ctypes.c_int32), ("coupling_in_products", ctypes.c_double),
                ("touching_pairs", ctypes.c_int64)]


class PlanSizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("n", "n_clusters", "depth", "n_adm", "n_near", "n_dirs_total", "n_slots")]


_lib = None


def load():
    """Load libdh2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch provides device memory and streams; loading it first makes libdh2
    # bind to the same HIP runtime instead of a second copy
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdh2.so not found at %s: build it with "
                           "python -m paper_1809_04384_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.dh2_build.argtypes = [P, D, I32, D, I32, D, P]
    lib.dh2_build_ex.argtypes = [P, D, I32, D, I32, D, P, P]
    lib.dh2_matvec.argtypes = [P, P, P, I32]
    lib.dh2_matvec_profile.argtypes = [P, P, P, I32, P, P]
    lib.dh2_free.argtypes = [P]
    lib.dh2_free.restype = None
    lib.dh2_last_error.restype = ctypes.c_char_p
    lib.dh2_get_stats.argtypes = [P, P]
    lib.dh2_plan_create.argtypes = [P, D, I32, D, I32, D, P]
    lib.dh2_plan_get_sizes.argtypes = [P, P]
    lib.dh2_plan_export.argtypes = [P] * 13
    lib.dh2_plan_rank_features.argtypes = [P, D, I32, P]
    lib.dh2_plan_free.argtypes = [P]
    lib.dh2_plan_free.restype = None
    lib.dh2_inspect.argtypes = [P, I32, I64, P, P, P]
    lib.dh2_batch_create.argtypes = [P, P, P, I32, I32, P, P]
    lib.dh2_matvec_stream.argtypes = [P, P, P, I32, P]
    lib.dh2_matvec_noalloc.argtypes = [P, P, P, I32, P]
    lib.dh2_build_many.argtypes = [I32, P, P, P, P, P, P, P, I32, P]
    lib.dh2_batch_run.argtypes = [P]
    lib.dh2_batch_free.argtypes = [P]
    lib.dh2_batch_free.restype = None
    for name in ("dh2_build", "dh2_build_ex", "dh2_matvec", "dh2_matvec_profile", "dh2_get_stats", "dh2_plan_create",
                 "dh2_plan_get_sizes", "dh2_plan_export", "dh2_inspect", "dh2_batch_create", "dh2_batch_run",
                 "dh2_matvec_stream", "dh2_build_many", "dh2_matvec_noalloc", "dh2_plan_rank_features"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st):
    if st != DH2_OK:
        raise Dh2Error(st, load().dh2_last_error().decode())


def _geometry(V, T):
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    g = Geometry(V.shape[0], V.ctypes.data, T.shape[0], T.ctypes.data)
    return g, (V, T)


class Plan:
    """Host-only hierarchy (cluster tree, directions, block tree)."""

    def __init__(self, V, T, kappa, order, eta, leafsize, eta1=10.0):
        lib = load()
        g, keep = _geometry(V, T)
        self._p = ctypes.c_void_p()
        _check(lib.dh2_plan_create(ctypes.byref(g), kappa, order, eta, leafsize, eta1,
                                   ctypes.byref(self._p)))

    def export(self):
        lib = load()
        s = PlanSizes()
        _check(lib.dh2_plan_get_sizes(self._p, ctypes.byref(s)))
        nc, nd = s.n_clusters, s.n_dirs_total
        out = {
            "perm": np.empty(s.n, np.int64), "first": np.empty(nc, np.int64),
            "size": np.empty(nc, np.int64), "level": np.empty(nc, np.int32),
            "parent": np.empty(nc, np.int64), "box": np.empty((nc, 6)),
            "level_ndirs": np.empty(s.depth + 1, np.int32), "dirs": np.empty((nd, 3)),
            "sd": np.empty(nd, np.int32), "adm": np.empty((s.n_adm, 3), np.int64),
            "near": np.empty((s.n_near, 2), np.int64), "slots": np.empty((s.n_slots, 3), np.int64)}
        keys = ["perm", "first", "size", "level", "parent", "box", "level_ndirs", "dirs", "sd",
                "adm", "near", "slots"]
        _check(lib.dh2_plan_export(self._p, *[out[k].ctypes.data for k in keys]))
        return out

    def rank_features(self, tol, kind="row"):
        """Features of the learned rank predictor, (n_slots, 12) float32."""
        lib = load()
        s = PlanSizes()
        _check(lib.dh2_plan_get_sizes(self._p, ctypes.byref(s)))
        out = np.empty((s.n_slots, 12), dtype=np.float32)
        _check(lib.dh2_plan_rank_features(self._p, tol, 0 if kind == "row" else 1, out.ctypes.data))
        return out

    def __del__(self):
        if getattr(self, "_p", None) and _lib is not None:
            _lib.dh2_plan_free(self._p)
            self._p = None


class Handle:
    """A built DH^2 matrix on the current HIP device."""

    def __init__(self, V, T, kappa, order, eta, leafsize, tol, eta1=10.0, precision=FP64,
                 max_nrhs=16, stream=None, workspace_gb=0.0, norm=NORM_FROBENIUS, rank_mode=RANKS_EXACT,
                 sketch_rank=0, autotune=0, weights=0, quadrature=QUAD_DEFAULT):
        lib = load()
        g, keep = _geometry(V, T)
        opt = Options()
        opt.size = ctypes.sizeof(Options)
        opt.precision = precision
        opt.eta1 = eta1
        opt.max_nrhs = max_nrhs
        opt.stream = stream
        opt.workspace_gb = workspace_gb
        opt.norm = norm
        opt.rank_mode = rank_mode
        opt.sketch_rank = sketch_rank
        opt.autotune = autotune
        opt.weights = weights
        opt.quadrature = quadrature
        self.precision = precision
        self.max_nrhs = max_nrhs
        self.n = int(np.asarray(T).shape[0])
        self._h = ctypes.c_void_p()
        _check(lib.dh2_build_ex(ctypes.byref(g), kappa, order, eta, leafsize, tol,
                                ctypes.byref(opt), ctypes.byref(self._h)))

    def matvec_on(self, X, Y, stream):
        """Handle.matvec enqueued on another stream than the handle's (the
        products of a batch issued one after another, for comparison)."""
        lib = load()
        _check(lib.dh2_matvec_stream(self._h, X.data_ptr(), Y.data_ptr(), X.shape[0], stream))

    def matvec_noalloc(self, X, Y, stream=None):
        """Handle.matvec through dh2_matvec_noalloc: the staging lives in the
        library's static device scratch (no allocation); calls on one GPU must
        not overlap."""
        _check(load().dh2_matvec_noalloc(self._h, X.data_ptr(), Y.data_ptr(), X.shape[0], stream))

    def matvec_ptr(self, x_ptr, y_ptr, nrhs):
        """Y = Gtilde X for raw device pointers (column-major n x nrhs complex)."""
        _check(load().dh2_matvec(self._h, x_ptr, y_ptr, nrhs))

    def matvec(self, X, Y):
        """X, Y: device tensors of shape (nrhs, n), complex128 (FP64) or complex64
        (FP32), C-contiguous (= column-major n x nrhs)."""
        import torch
        want = torch.complex128 if self.precision == FP64 else torch.complex64
        for A in (X, Y):
            if A.dtype != want or not A.is_contiguous() or A.dim() != 2 or A.shape[1] != self.n:
                raise ValueError("X/Y must be contiguous %s tensors of shape (nrhs, %d)" % (want, self.n))
        if X.shape != Y.shape:
            raise ValueError("X and Y must have the same shape")
        self.matvec_ptr(X.data_ptr(), Y.data_ptr(), X.shape[0])

    PHASES = ("gather", "forward", "coupling", "backward", "near", "leaf_output", "scatter")

    def matvec_profile(self, X, Y):
        """Y = Gtilde X with per-phase event timing (synchronising).  Returns
        ({phase: ms}, near-field bytes streamed)."""
        ms = (ctypes.c_double * 7)()
        nb = ctypes.c_double()
        _check(load().dh2_matvec_profile(self._h, X.data_ptr(), Y.data_ptr(), X.shape[0], ms,
                                         ctypes.byref(nb)))
        return dict(zip(self.PHASES, list(ms))), nb.value

    def stats(self):
        s = Stats()
        s.size = ctypes.sizeof(Stats)
        _check(load().dh2_get_stats(self._h, ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in Stats._fields_ if f != "size"}
        out["mv_variant"] = list(out["mv_variant"])
        return out

    def inspect(self, what, index=0):
        lib = load()
        r, c = ctypes.c_int64(), ctypes.c_int64()
        code = INSPECT[what]
        _check(lib.dh2_inspect(self._h, code, index, None, ctypes.byref(r), ctypes.byref(c)))
        out = np.empty((c.value, r.value), dtype=np.complex128)   # column-major r x c
        _check(lib.dh2_inspect(self._h, code, index, out.ctypes.data, ctypes.byref(r), ctypes.byref(c)))
        return out.T

    def free(self):
        if getattr(self, "_h", None):
            load().dh2_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Y_i = Gtilde_i X_i for several handles as one graph launch (dh2_batch_*).
    X and Y are lists of device tensors laid out as for Handle.matvec; their
    memory is recorded, so later runs read and write the same tensors."""

    def __init__(self, handles, X, Y, stream=None):
        import torch
        lib = load()
        if not (len(handles) == len(X) == len(Y)) or not handles:
            raise ValueError("handles, X and Y must be non-empty lists of one length")
        nrhs = X[0].shape[0]
        for h, x, y in zip(handles, X, Y):
            want = torch.complex128 if h.precision == FP64 else torch.complex64
            for A in (x, y):
                if A.dtype != want or not A.is_contiguous() or A.dim() != 2 or A.shape != (nrhs, h.n):
                    raise ValueError("X/Y must be contiguous %s tensors of shape (%d, n)" % (want, nrhs))
        cnt = len(handles)
        hs = (ctypes.c_void_p * cnt)(*[h._h.value for h in handles])
        xs = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in X])
        ys = (ctypes.c_void_p * cnt)(*[y.data_ptr() for y in Y])
        self._keep = (list(handles), list(X), list(Y))
        self._b = ctypes.c_void_p()
        _check(lib.dh2_batch_create(hs, xs, ys, nrhs, cnt, stream, ctypes.byref(self._b)))

    def run(self):
        _check(load().dh2_batch_run(self._b))

    def free(self):
        if getattr(self, "_b", None):
            load().dh2_batch_free(self._b)
            self._b = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_many(problems, precision=FP64, max_nrhs=16, eta1=10.0, norm=NORM_FROBENIUS, threads=0,
               workspace_gb=0.0, weights=WEIGHTS_HOUSEHOLDER, autotune=0, quadrature=QUAD_DEFAULT):
    """Handles for many problems built side by side (dh2_build_many): problems is
    a list of (V, T, kappa, order, eta, leafsize, tol); every handle owns a
    stream of its own."""
    lib = load()
    cnt = len(problems)
    if cnt < 1:
        raise ValueError("no problems")
    geoms = (Geometry * cnt)()
    keep = []
    for i, (V, T, *_rest) in enumerate(problems):
        g, k = _geometry(V, T)
        geoms[i] = g
        keep.append(k)
    kap = (ctypes.c_double * cnt)(*[float(p[2]) for p in problems])
    order = (ctypes.c_int * cnt)(*[int(p[3]) for p in problems])
    eta = (ctypes.c_double * cnt)(*[float(p[4]) for p in problems])
    leaf = (ctypes.c_int * cnt)(*[int(p[5]) for p in problems])
    tol = (ctypes.c_double * cnt)(*[float(p[6]) for p in problems])
    opt = Options()
    opt.size = ctypes.sizeof(Options)
    opt.precision = precision
    opt.eta1 = eta1
    opt.max_nrhs = max_nrhs
    opt.workspace_gb = workspace_gb
    opt.weights = weights
    opt.autotune = autotune
    opt.norm = norm
    opt.quadrature = quadrature
    out = (ctypes.c_void_p * cnt)()
    _check(lib.dh2_build_many(cnt, geoms, kap, order, eta, leaf, tol, ctypes.byref(opt), threads, out))
    hs = []
    for i in range(cnt):
        h = Handle.__new__(Handle)
        h._h = ctypes.c_void_p(out[i])
        h.precision = precision
        h.max_nrhs = max_nrhs
        h.n = int(np.asarray(problems[i][1]).shape[0])
        hs.append(h)
    return hs
