"""Cluster tree, directions and block tree (Section 2).

* Cluster tree (Definition 'cluster tree'; Section 5: standard binary space
  partitioning down to a leaf size).  Reading: split the index list at the
  midpoint of the longest side of the bounding box of the triangle centroids
  (ties -> lowest axis); indices with centroid coordinate < midpoint go to the
  first child, in stable order; a box of zero extent is split by position.
* Bounding boxes B_t: tight axis-parallel boxes of all vertices of the
  triangles in t (they contain the supports of the basis functions).
* Directions (Definition 'directions', Remark 'construction of directions'):
  per level d_l = max diam(B_t); D_l = {0} if kappa d_l <= eta1, else the
  6 m^2 projected centres of a face grid of the cube [-1,1]^3 with
  m = ceil(sqrt(2) kappa d_l / eta1).  sd_l(c) = nearest direction of D_{l+1}.
* Block tree (Definition 'block tree'): recursion from (root, root); a pair is
  an admissible leaf if the standard and parabolic conditions (eq.
  (admissibility), second and third line) hold with eta_2, then c_ts is the
  best approximation of (m_t - m_s)/|m_t - m_s| in D_l; otherwise it is an
  inadmissible leaf if t or s is a leaf, else the recursion visits all pairs
  of children.
Ties in nearest-direction searches go to the lowest index among candidates
within 1e-12 of the minimum.  All decisions use IEEE double arithmetic in a
fixed order (no fused operations), so the structure is reproducible.
"""
import math
from dataclasses import dataclass, field

import numpy as np

TIE = 1e-12


@dataclass
class Structure:
    n: int
    perm: np.ndarray            # cluster order -> triangle index
    first: np.ndarray           # [nc] first position in perm
    size: np.ndarray            # [nc]
    level: np.ndarray           # [nc]
    parent: np.ndarray          # [nc], -1 for the root
    children: list              # [nc] list of child ids (0 or 2)
    lo: np.ndarray              # [nc,3] box
    hi: np.ndarray              # [nc,3]
    depth: int
    dirs: list                  # per level: array [nd,3] (a single zero row if D_l = {0})
    dir_m: list                 # per level: grid parameter m_l (0 for D_l = {0})
    sd: list                    # per level l < depth: int array [nd_l] -> index in D_{l+1}
    adm: list = field(default_factory=list)     # list of (t, s, c)
    near: list = field(default_factory=list)    # list of (t, s)

    def idx(self, t):
        """Triangle indices of cluster t (the label t-hat)."""
        return self.perm[self.first[t]:self.first[t] + self.size[t]]

    def is_leaf(self, t):
        return len(self.children[t]) == 0

    def mid(self, t):
        return 0.5 * (self.lo[t] + self.hi[t])

    def diam(self, t):
        return _norm3(self.hi[t] - self.lo[t])


def _norm3(d):
    return math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])


def _dist_boxes(lo_t, hi_t, lo_s, hi_s):
    """Euclidean distance of two axis-parallel boxes."""
    acc = 0.0
    for d in range(3):
        g = max(0.0, lo_s[d] - hi_t[d], lo_t[d] - hi_s[d])
        acc += g * g
    return math.sqrt(acc)


def build_cluster_tree(V, T, leaf):
    n = T.shape[0]
    P = V[T]
    cen = ((P[:, 0] + P[:, 1]) + P[:, 2]) / 3.0
    vlo = np.minimum(np.minimum(P[:, 0], P[:, 1]), P[:, 2])
    vhi = np.maximum(np.maximum(P[:, 0], P[:, 1]), P[:, 2])

    first, size, level, parent, children, lo, hi = [], [], [], [], [], [], []
    perm = []

    def rec(ids, lev, par):
        me = len(first)
        first.append(len(perm) if False else -1)
        size.append(len(ids))
        level.append(lev)
        parent.append(par)
        children.append([])
        lo.append(vlo[ids].min(axis=0))
        hi.append(vhi[ids].max(axis=0))
        if len(ids) <= leaf:
            first[me] = len(perm)
            perm.extend(ids.tolist())
            return me
        c = cen[ids]
        clo = c.min(axis=0)
        chi = c.max(axis=0)
        ext = chi - clo
        d = 0
        for a in (1, 2):
            if ext[a] > ext[d]:
                d = a
        if ext[d] > 0.0:
            midv = 0.5 * (clo[d] + chi[d])
            m = c[:, d] < midv
            parts = [ids[m], ids[~m]]
        else:
            h = (len(ids) + 1) // 2
            parts = [ids[:h], ids[h:]]
        start = len(perm)
        for p in parts:
            children[me].append(rec(p, lev + 1, me))
        first[me] = start
        return me

    import sys
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 10000))
    try:
        rec(np.arange(n, dtype=np.int64), 0, -1)
    finally:
        sys.setrecursionlimit(old)
    return (np.asarray(perm, dtype=np.int64), np.asarray(first, dtype=np.int64),
            np.asarray(size, dtype=np.int64), np.asarray(level, dtype=np.int64),
            np.asarray(parent, dtype=np.int64), children,
            np.asarray(lo), np.asarray(hi))


def direction_grid(m):
    """6 m^2 unit directions: centres of an m x m grid on each face of [-1,1]^3,
    projected to the sphere; index f*m^2 + i*m + j, faces (+x,-x,+y,-y,+z,-z),
    the two free axes in ascending order take -1 + (2i+1)/m and -1 + (2j+1)/m."""
    out = np.empty((6 * m * m, 3))
    k = 0
    for f in range(6):
        ax = f // 2
        sgn = 1.0 if f % 2 == 0 else -1.0
        u, w = [a for a in range(3) if a != ax]
        for i in range(m):
            for j in range(m):
                c = [0.0, 0.0, 0.0]
                c[ax] = sgn
                c[u] = -1.0 + (2 * i + 1) / m
                c[w] = -1.0 + (2 * j + 1) / m
                r = _norm3(c)
                out[k] = (c[0] / r, c[1] / r, c[2] / r)
                k += 1
    return out


def nearest(u, D):
    """Index of the nearest direction: keys (u-c)_x^2 + (u-c)_y^2 + (u-c)_z^2
    summed in that order, lowest index among keys <= min + 1e-12."""
    dx = u[0] - D[:, 0]
    dy = u[1] - D[:, 1]
    dz = u[2] - D[:, 2]
    keys = dx * dx + dy * dy + dz * dz
    mn = keys.min()
    return int(np.nonzero(keys <= mn + TIE)[0][0])


def build_directions(st_level, st_diam, depth, kappa, eta1):
    dirs, dir_m = [], []
    for l in range(depth + 1):
        dl = max(st_diam[i] for i in range(len(st_level)) if st_level[i] == l)
        if kappa * dl <= eta1:
            dirs.append(np.zeros((1, 3)))
            dir_m.append(0)
        else:
            m = int(math.ceil(math.sqrt(2.0) * kappa * dl / eta1))
            dirs.append(direction_grid(m))
            dir_m.append(m)
    sd = []
    for l in range(depth):
        D1 = dirs[l + 1]
        sd.append(np.array([nearest(dirs[l][i], D1) for i in range(dirs[l].shape[0])],
                           dtype=np.int64))
    return dirs, dir_m, sd


def build_structure(V, T, kappa, eta, leaf, eta1=10.0):
    (perm, first, size, level, parent, children, lo, hi) = build_cluster_tree(V, T, leaf)
    nc = len(first)
    depth = int(level.max())
    diam = [_norm3(hi[t] - lo[t]) for t in range(nc)]
    dirs, dir_m, sd = build_directions(level, diam, depth, kappa, eta1)
    st = Structure(n=T.shape[0], perm=perm, first=first, size=size, level=level,
                   parent=parent, children=children, lo=lo, hi=hi, depth=depth,
                   dirs=dirs, dir_m=dir_m, sd=sd)
    mid = 0.5 * (lo + hi)

    adm, near = [], []
    # explicit stack instead of recursion; visiting order = recursive order
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        dist = _dist_boxes(lo[t], hi[t], lo[s], hi[s])
        md = max(diam[t], diam[s])
        if md <= eta * dist and kappa * max(diam[t] * diam[t], diam[s] * diam[s]) <= eta * dist:
            D = dirs[level[t]]
            if dir_m[level[t]] == 0:
                c = 0
            else:
                d = mid[t] - mid[s]
                r = _norm3(d)
                c = nearest((d[0] / r, d[1] / r, d[2] / r), D)
            adm.append((t, s, c))
        elif not children[t] or not children[s]:
            near.append((t, s))
        else:
            kids = [(t1, s1) for t1 in children[t] for s1 in children[s]]
            stack.extend(reversed(kids))
    st.adm = adm
    st.near = near
    return st
