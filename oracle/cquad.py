"""ctypes wrapper around the oracle's C product-rule sums (oracle/csrc/quad.c)."""
import ctypes
import math

import numpy as np

from . import build_oracle
from . import ses
from .quadrature import laplace_self_integral

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = build_oracle.build()
        lib = ctypes.CDLL(path)
        lib.oracle_pair_sums.restype = None
        lib.oracle_pair_sums.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
            ctypes.c_void_p]
        _lib = lib
    return _lib


def pair_sums(rows, cols, xq, wq, kappa):
    """Raw product-rule sums (see quad.c); returns complex [len(rows), len(cols)]."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    xq = np.ascontiguousarray(xq, dtype=np.float64)
    wq = np.ascontiguousarray(wq, dtype=np.float64)
    out = np.empty((len(rows), len(cols)), dtype=np.complex128)
    lib.oracle_pair_sums(len(rows), rows.ctypes.data, len(cols), cols.ctypes.data,
                         xq.shape[1], xq.ctypes.data, wq.ctypes.data, float(kappa),
                         out.ctypes.data)
    return out


def near_block(tri, rows, cols, kappa):
    """Near-field Galerkin block: Q16 x Q16 off the diagonal, singularity
    subtraction (closed-form Laplace part + Q16 x Q16 remainder) on it."""
    out = pair_sums(rows, cols, tri["x16"], tri["w16"], kappa)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    pos = {int(j): c for c, j in enumerate(cols)}
    for r, i in enumerate(rows):
        c = pos.get(int(i))
        if c is not None:
            P = tri["P"][i]
            out[r, c] = (laplace_self_integral(P[0], P[1], P[2]) + out[r, c]) / (4.0 * math.pi)
    return out


def far_block(tri, rows, cols, kappa):
    """Reference Galerkin block with the Q7 x Q7 product rule (i != j)."""
    return pair_sums(rows, cols, tri["x7"], tri["w7"], kappa)


def near_block_paper(tri, rows, cols, kappa):
    """Near-field Galerkin block with the paper's quadrature (Section 5):
    Duffy-Gauss of order 3 on both triangles (x9, w9) for pairs that share no
    vertex, Sauter-Erichsen-Schwab of order 5 for pairs that share a vertex,
    an edge, or are identical.  The touching rules are not symmetric in the
    two triangles, so a pair is always integrated with the triangle of lower
    index first: the matrix stays exactly symmetric."""
    out = pair_sums(rows, cols, tri["x9"], tri["w9"], kappa)
    V, T, vt = tri["V"], tri["T"], tri["vert_tris"]
    pos = {int(j): c for c, j in enumerate(cols)}
    for r, i in enumerate(np.asarray(rows)):
        cand = set()
        for v in T[int(i)]:
            cand.update(vt[int(v)])
        for j in sorted(cand):
            c = pos.get(j)
            if c is not None:
                lo, hi = min(int(i), j), max(int(i), j)
                out[r, c] = ses.ses_pair(V, T[lo], T[hi], kappa)
    return out
