"""Tensor Chebyshev interpolation on axis-parallel boxes (Section 2).

Points per axis: the m zeros of T_m, xhat_j = cos((2j+1) pi / (2m)), mapped
affinely onto [lo, hi].  Lagrange polynomials L_j(xhat) = prod_{l != j}
(xhat - xhat_l) / (xhat_j - xhat_l).  A box side of zero width maps every point
to xhat = 0 (all points of a flat box lie at its midpoint).  Tensor index
nu = jx + m (jy + m jz), k = m^3.
"""
import math

import numpy as np


def cheb_nodes(m):
    return np.array([math.cos((2 * j + 1) * math.pi / (2 * m)) for j in range(m)])


def lagrange_1d(xhat, nodes):
    """Values L_j(xhat) for an array of reference coordinates: [len(xhat), m]."""
    xhat = np.asarray(xhat, dtype=np.float64)
    m = len(nodes)
    out = np.ones((xhat.size, m))
    for j in range(m):
        for l in range(m):
            if l != j:
                out[:, j] *= (xhat.ravel() - nodes[l]) / (nodes[j] - nodes[l])
    return out


def to_reference(x, lo, hi):
    """Map physical coordinates of one axis onto [-1, 1]."""
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    if half == 0.0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return (np.asarray(x, dtype=np.float64) - mid) / half


def box_points(lo, hi, m):
    """Interpolation points xi_{t,nu} of a box: [k, 3]."""
    nodes = cheb_nodes(m)
    ax = [0.5 * (lo[d] + hi[d]) + 0.5 * (hi[d] - lo[d]) * nodes for d in range(3)]
    k = m ** 3
    out = np.empty((k, 3))
    for jz in range(m):
        for jy in range(m):
            for jx in range(m):
                nu = jx + m * (jy + m * jz)
                out[nu] = (ax[0][jx], ax[1][jy], ax[2][jz])
    return out


def box_lagrange(x, lo, hi, m):
    """Tensor Lagrange polynomials L_{t,nu}(x) for points x [np, 3]: [np, k]."""
    nodes = cheb_nodes(m)
    L = [lagrange_1d(to_reference(x[:, d], lo[d], hi[d]), nodes) for d in range(3)]
    npts = x.shape[0]
    out = np.empty((npts, m ** 3))
    for jz in range(m):
        for jy in range(m):
            for jx in range(m):
                out[:, jx + m * (jy + m * jz)] = L[0][:, jx] * L[1][:, jy] * L[2][:, jz]
    return out
