"""Procedural triangulated surfaces used as inputs (Section 5 of the paper).

* Unit sphere: the double pyramid |x1|+|x2|+|x3| = 1 (eight faces), each face
  refined regularly into q^2 triangles, vertices pushed radially onto the unit
  sphere once at the end.  n = 8 q^2.
* Cube [-1,1]^3: every face split into two triangles along one diagonal, each
  refined regularly (equivalently a q x q grid of squares, each cut along the
  same diagonal).  n = 12 q^2.
* Ellipsoid: the sphere mesh with coordinates scaled by the three semi-axes.

Vertices are returned as float64 [nv, 3], triangles as int32 [n, 3] (0-based).
Shared vertices are merged through exact integer grid keys, so the output is
deterministic and platform independent.
"""
import numpy as np


def sphere_octahedral(q):
    """Sphere from the refined octahedron; faces in sign-bit order (x=bit0,
    y=bit1, z=bit2, bit set = negative), rows j, then i, 'up' then 'down'."""
    if q < 1:
        raise ValueError("q must be >= 1")
    keys = {}
    verts = []
    tris = []

    def vid(key):
        v = keys.get(key)
        if v is None:
            v = len(verts)
            keys[key] = v
            verts.append(key)
        return v

    for face in range(8):
        sx = -1 if face & 1 else 1
        sy = -1 if face & 2 else 1
        sz = -1 if face & 4 else 1

        def P(i, j):
            # integer coordinates of A + (i/q)(B-A) + (j/q)(C-A), scaled by q
            return (sx * (q - i - j), sy * i, sz * j)

        for j in range(q):
            for i in range(q - j):
                tris.append((vid(P(i, j)), vid(P(i + 1, j)), vid(P(i, j + 1))))
                if i + j <= q - 2:
                    tris.append((vid(P(i + 1, j)), vid(P(i + 1, j + 1)),
                                 vid(P(i, j + 1))))
    V = np.asarray(verts, dtype=np.float64) / float(q)
    r = np.sqrt(V[:, 0] * V[:, 0] + V[:, 1] * V[:, 1] + V[:, 2] * V[:, 2])
    V = V / r[:, None]
    return np.ascontiguousarray(V), np.asarray(tris, dtype=np.int32)


def ellipsoid_octahedral(q, axes=(1.0, 2.0, 3.0)):
    V, T = sphere_octahedral(q)
    V = V * np.asarray(axes, dtype=np.float64)[None, :]
    return np.ascontiguousarray(V), T


def cube_surface(q, lo=-1.0, hi=1.0):
    """Surface of the cube [lo,hi]^3, 2 q^2 triangles per face."""
    if q < 1:
        raise ValueError("q must be >= 1")
    keys = {}
    verts = []
    tris = []

    def vid(key):
        v = keys.get(key)
        if v is None:
            v = len(verts)
            keys[key] = v
            verts.append(key)
        return v

    for ax in range(3):
        u, w = [a for a in range(3) if a != ax]
        for side in (0, q):
            def P(i, j):
                p = [0, 0, 0]
                p[ax] = side
                p[u] = i
                p[w] = j
                return tuple(p)
            for j in range(q):
                for i in range(q):
                    a, b = vid(P(i, j)), vid(P(i + 1, j))
                    c, d = vid(P(i + 1, j + 1)), vid(P(i, j + 1))
                    tris.append((a, b, c))
                    tris.append((a, c, d))
    G = np.asarray(verts, dtype=np.float64)
    V = lo + (hi - lo) * (G / float(q))
    return np.ascontiguousarray(V), np.asarray(tris, dtype=np.int32)
