"""Galerkin discretisation pieces (Section 1, eq. (matrix); Section 5).

Piecewise-constant basis: phi_i is the indicator function of triangle T_i, so
g_ij = int_{T_i} int_{T_j} g(x,y) dy dx.

Rules (readings of the stated quadrature, see the design notes):
* far rule (Q7): the symmetric degree-5 seven-point rule of Radon on a
  triangle, used for interpolation bases and for admissible-block reference
  entries;
* near rule (Q16): 4x4 Gauss-Legendre on the unit square collapsed onto the
  triangle by the Duffy map (u,v) -> barycentric (1-u, u(1-v), uv), Jacobian
  u -- the Gauss/Duffy family of Section 5;
* self term i = j: singularity subtraction.  g = 1/(4 pi r) + rho(r)/(4 pi)
  with rho(r) = (exp(i kappa r) - 1)/r, bounded.  The Laplace part is
  integrated in closed form (laplace_self_integral), rho by Q16 x Q16 with
  rho(0) = i kappa.
"""
import math

import numpy as np


def kernel_g(x, y, kappa):
    """Helmholtz kernel exp(i kappa |x-y|) / (4 pi |x-y|), eq. (helmholtz)."""
    d = x - y
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
    return np.exp(1j * kappa * r) / (4.0 * math.pi * r)


def kernel_gc(x, y, c, kappa):
    """Directional remainder g_c(x,y) = exp(i kappa (|x-y| - <x-y,c>)) / (4 pi |x-y|)
    (Section 2, splitting of g into a plane wave and a smooth factor)."""
    d = x - y
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
    dc = d[..., 0] * c[0] + d[..., 1] * c[1] + d[..., 2] * c[2]
    return np.exp(1j * kappa * (r - dc)) / (4.0 * math.pi * r)


def gauss_legendre_01(npts):
    """Gauss-Legendre nodes and weights on [0,1] (numpy's rule, mapped)."""
    t, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (t + 1.0), 0.5 * w


def q7_rule():
    """Radon's degree-5 rule: barycentric points (3 columns) and weights summing
    to one (multiply by the triangle area)."""
    s15 = math.sqrt(15.0)
    a = (6.0 - s15) / 21.0
    b = (6.0 + s15) / 21.0
    wa = (155.0 - s15) / 1200.0
    wb = (155.0 + s15) / 1200.0
    lam = [(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0),
           (a, a, 1.0 - 2.0 * a), (a, 1.0 - 2.0 * a, a), (1.0 - 2.0 * a, a, a),
           (b, b, 1.0 - 2.0 * b), (b, 1.0 - 2.0 * b, b), (1.0 - 2.0 * b, b, b)]
    w = [9.0 / 40.0, wa, wa, wa, wb, wb, wb]
    return np.array(lam), np.array(w)


def q16_rule():
    """4x4 Gauss-Legendre collapsed by the Duffy map; weights sum to one."""
    u, wu = gauss_legendre_01(4)
    lam = []
    w = []
    for i in range(4):
        for j in range(4):
            lam.append((1.0 - u[i], u[i] * (1.0 - u[j]), u[i] * u[j]))
            w.append(2.0 * wu[i] * wu[j] * u[i])
    return np.array(lam), np.array(w)


def q9_rule():
    """3 x 3 Gauss-Legendre collapsed by the Duffy map (the paper's rule of order
    3 for pairs of triangles that share no vertex, Section 5); weights sum to one."""
    u, wu = gauss_legendre_01(3)
    lam = []
    w = []
    for i in range(3):
        for j in range(3):
            lam.append((1.0 - u[i], u[i] * (1.0 - u[j]), u[i] * u[j]))
            w.append(2.0 * wu[i] * wu[j] * u[i])
    return np.array(lam), np.array(w)


def triangle_data(V, T):
    """Per-triangle area, centroid, Q7 and Q16 physical points and weights.

    Returns dict with area [n], centroid [n,3], x7 [n,7,3], w7 [n,7],
    x16 [n,16,3], w16 [n,16], x9 [n,9,3], w9 [n,9] (the paper's rule), the
    vertex coordinates P [n,3,3], V, T and the triangles of every vertex.
    """
    P = V[T]                       # [n, 3 vertices, 3 coords]
    a, b, c = P[:, 0], P[:, 1], P[:, 2]
    e1 = b - a
    e2 = c - a
    cr = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                   e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                   e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], axis=1)
    area = 0.5 * np.sqrt(cr[:, 0] * cr[:, 0] + cr[:, 1] * cr[:, 1] + cr[:, 2] * cr[:, 2])
    centroid = ((a + b) + c) / 3.0
    l7, w7 = q7_rule()
    l16, w16 = q16_rule()
    l9, w9 = q9_rule()
    x7 = np.einsum("qv,nvd->nqd", l7, P)
    x16 = np.einsum("qv,nvd->nqd", l16, P)
    x9 = np.einsum("qv,nvd->nqd", l9, P)
    vert_tris = {}
    for i, tri in enumerate(np.asarray(T)):
        for v in tri:
            vert_tris.setdefault(int(v), []).append(i)
    return {"P": P, "area": area, "centroid": centroid,
            "x7": x7, "w7": area[:, None] * w7[None, :],
            "x16": x16, "w16": area[:, None] * w16[None, :],
            "x9": x9, "w9": area[:, None] * w9[None, :],
            "V": np.asarray(V, dtype=np.float64), "T": np.asarray(T), "vert_tris": vert_tris}


def laplace_self_integral(p0, p1, p2):
    """Closed form of int_T int_T 1/|x-y| dy dx for a flat triangle T.

    With edge lengths l_e, perimeter L and area A:
        (4 A^2 / 3) * sum_e (1/l_e) * log(L / (L - 2 l_e)).
    Derivation (written out in the design notes): the integral is
    homogeneous of degree 3; differentiating with respect to a scaling
    about one vertex (Reynolds transport) reduces it to line integrals of the
    triangle's potential over the opposite edge, and a second scaling about an
    endpoint of that edge reduces those to the classical closed forms for a
    point against a segment and two segments sharing a vertex.
    """
    l0 = _dist(p1, p2)
    l1 = _dist(p2, p0)
    l2 = _dist(p0, p1)
    e1 = np.asarray(p1, float) - np.asarray(p0, float)
    e2 = np.asarray(p2, float) - np.asarray(p0, float)
    cr = np.cross(e1, e2)
    A = 0.5 * math.sqrt(float(cr @ cr))
    L = l0 + l1 + l2
    s = 0.0
    for le in (l0, l1, l2):
        s += math.log(L / (L - 2.0 * le)) / le
    return 4.0 * A * A / 3.0 * s


def _dist(p, q):
    d = np.asarray(p, float) - np.asarray(q, float)
    return math.sqrt(float(d @ d))


def rho(r, kappa):
    """(exp(i kappa r) - 1) / r in the cancellation-free form, rho(0) = i kappa."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty(r.shape, dtype=np.complex128)
    z = r == 0.0
    nz = ~z
    rr = r[nz]
    s = np.sin(0.5 * kappa * rr)
    out[nz] = (-2.0 * s * s + 1j * np.sin(kappa * rr)) / rr
    out[z] = 1j * kappa
    return out


def self_entry(tri, i, kappa):
    """g_ii = (1/4pi) [ I_L(T_i) + sum_{p,q in Q16} w_p w_q rho(|x_p - x_q|) ]."""
    P = tri["P"][i]
    x = tri["x16"][i]
    w = tri["w16"][i]
    d = x[:, None, :] - x[None, :, :]
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
    reg = np.sum(w[:, None] * w[None, :] * rho(r, kappa))
    return (laplace_self_integral(P[0], P[1], P[2]) + reg) / (4.0 * math.pi)


def near_entry(tri, i, j, kappa):
    """Near-field entry with the Q16 x Q16 product rule (i != j), or the self term."""
    if i == j:
        return self_entry(tri, i, kappa)
    x = tri["x16"][i]
    y = tri["x16"][j]
    w = tri["w16"][i][:, None] * tri["w16"][j][None, :]
    return np.sum(w * kernel_g(x[:, None, :], y[None, :, :], kappa))


def far_entry(tri, i, j, kappa):
    """Reference entry with the Q7 x Q7 product rule (admissible blocks)."""
    x = tri["x7"][i]
    y = tri["x7"][j]
    w = tri["w7"][i][:, None] * tri["w7"][j][None, :]
    return np.sum(w * kernel_g(x[:, None, :], y[None, :, :], kappa))
