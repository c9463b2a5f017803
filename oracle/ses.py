"""The paper's quadrature for the Galerkin entries (Section 5): Sauter-Erichsen-
Schwab quadrature of order 5 for triangle pairs that share a vertex, an edge,
or are identical, and Gauss quadrature with the Duffy transformation of order
3 for every other pair.

TEST INFRASTRUCTURE ONLY: part of the oracle; the product library never
imports it.

Reference triangle: T^ = {(s1, s2) : 0 <= s2 <= s1 <= 1}, mapped onto a flat
triangle with ordered vertices (A, B, C) by chi(s) = A + s1 (B - A) + s2 (C - B)
(surface element 2 |T|).  A pair integral int_Ta int_Tb k(x, y) dy dx becomes
(2 |Ta|)(2 |Tb|) int_T^ int_T^ k(chi_a(s), chi_b(t)) dt ds, and the
Sauter-Schwab coordinates write the 4-d reference integral over the unit cube
in (xi, eta1, eta2, eta3) as a sum over regions, each with a polynomial
Jacobian that vanishes where x = y, so the 1/|x - y| singularity is removed
and tensor Gauss-Legendre rules converge exponentially.  The vertex order
fixes where the shared part lies: a shared vertex is A of both triangles, a
shared edge is A -> B of both (chi_a(s1, 0) = chi_b(s1, 0)), an identical pair
uses one order for both.

Regions (the map from the cube onto parts of T^ x T^ and its Jacobian), as
given for the three cases by Sauter and Schwab (Boundary Element Methods,
Section 5.2.3); every region's map and weight is checked in the tests by
integrating smooth functions exactly:
* identical (weight xi^3 eta1^2 eta2, six regions);
* common edge (weight xi^3 eta1^2 for the first region, xi^3 eta1^2 eta2 for
  the other four);
* common vertex (weight xi^3 eta2, two regions).
"""
import math

import numpy as np

from .quadrature import gauss_legendre_01

NQ_TOUCH = 5        # order of the Sauter-Erichsen-Schwab rules (Section 5)
NQ_REGULAR = 3      # order of the Duffy-Gauss rule on each triangle (Section 5)


def duffy_gauss_rule(n):
    """n x n Gauss-Legendre on the unit square collapsed onto a triangle by the
    Duffy map (u, v) -> barycentric (1 - u, u (1 - v), u v), Jacobian u; the
    weights sum to one (multiply by the area)."""
    u, wu = gauss_legendre_01(n)
    lam, w = [], []
    for i in range(n):
        for j in range(n):
            lam.append((1.0 - u[i], u[i] * (1.0 - u[j]), u[i] * u[j]))
            w.append(2.0 * wu[i] * wu[j] * u[i])
    return np.array(lam), np.array(w)


def _cube(nq):
    g, gw = gauss_legendre_01(nq)
    xi, e1, e2, e3 = np.meshgrid(g, g, g, g, indexing="ij")
    w = np.einsum("a,b,c,d->abcd", gw, gw, gw, gw)
    return xi.ravel(), e1.ravel(), e2.ravel(), e3.ravel(), w.ravel()


def ses_rule(kind, nq=NQ_TOUCH):
    """Points s, t (each [N, 2] in T^) and weights [N] of the rule for
    int_T^ int_T^ f(s, t) dt ds; kind 3 = identical, 2 = common edge,
    1 = common vertex."""
    xi, a, b, c, w = _cube(nq)
    S, Tt, W = [], [], []

    def add(s1, s2, t1, t2, wt):
        S.append(np.stack([s1, s2], axis=1))
        Tt.append(np.stack([t1, t2], axis=1))
        W.append(wt)

    if kind == 3:
        wt = w * xi ** 3 * a ** 2 * b
        add(xi, xi * (1 - a + a * b), xi * (1 - a * b * c), xi * (1 - a), wt)
        add(xi * (1 - a * b * c), xi * (1 - a), xi, xi * (1 - a + a * b), wt)
        add(xi, xi * a * (1 - b + b * c), xi * (1 - a * b), xi * a * (1 - b), wt)
        add(xi * (1 - a * b), xi * a * (1 - b), xi, xi * a * (1 - b + b * c), wt)
        add(xi * (1 - a * b * c), xi * a * (1 - b * c), xi, xi * a * (1 - b), wt)
        add(xi, xi * a * (1 - b), xi * (1 - a * b * c), xi * a * (1 - b * c), wt)
    elif kind == 2:
        w0 = w * xi ** 3 * a ** 2
        w1 = w0 * b
        add(xi, xi * a * c, xi * (1 - a * b), xi * a * (1 - b), w0)
        add(xi, xi * a, xi * (1 - a * b * c), xi * a * b * (1 - c), w1)
        add(xi * (1 - a * b), xi * a * (1 - b), xi, xi * a * b * c, w1)
        add(xi * (1 - a * b * c), xi * a * b * (1 - c), xi, xi * a, w1)
        add(xi * (1 - a * b * c), xi * a * (1 - b * c), xi, xi * a * b, w1)
    elif kind == 1:
        wt = w * xi ** 3 * b
        add(xi, xi * a, xi * b, xi * b * c, wt)
        add(xi * b, xi * b * c, xi, xi * a, wt)
    else:
        raise ValueError("kind must be 1, 2 or 3")
    return np.concatenate(S), np.concatenate(Tt), np.concatenate(W)


def ref_map(P, s):
    """chi(s) = A + s1 (B - A) + s2 (C - B) for ordered vertices P = [A, B, C]."""
    P = np.asarray(P, dtype=np.float64)
    return P[0] + s[:, :1] * (P[1] - P[0]) + s[:, 1:2] * (P[2] - P[1])


def area(P):
    P = np.asarray(P, dtype=np.float64)
    return 0.5 * float(np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0])))


def touching_order(Ta, Tb):
    """Kind (0 none, 1 vertex, 2 edge, 3 identical) of the vertex-index triples
    Ta, Tb and the vertex orders putting the shared part first (a shared vertex
    as A, a shared edge as A -> B of both)."""
    Ta = [int(v) for v in Ta]
    Tb = [int(v) for v in Tb]
    shared = [v for v in Ta if v in Tb]
    if len(shared) == 3:
        return 3, Ta, Ta
    if len(shared) == 2:
        p, q = shared
        oa = [p, q] + [v for v in Ta if v not in shared]
        ob = [p, q] + [v for v in Tb if v not in shared]
        return 2, oa, ob
    if len(shared) == 1:
        p = shared[0]
        return 1, [p] + [v for v in Ta if v != p], [p] + [v for v in Tb if v != p]
    return 0, Ta, Tb


def ses_pair(V, Ta, Tb, kappa, nq=NQ_TOUCH, kernel=None):
    """int_Ta int_Tb g(x, y) dy dx for a touching pair (vertex-index triples Ta,
    Tb into V), g = exp(i kappa r) / (4 pi r) unless another kernel(x, y) is
    given."""
    kind, oa, ob = touching_order(Ta, Tb)
    if kind == 0:
        raise ValueError("the triangles share no vertex")
    Pa, Pb = V[oa], V[ob]
    s, t, w = ses_rule(kind, nq)
    x, y = ref_map(Pa, s), ref_map(Pb, t)
    if kernel is None:
        d = x - y
        r = np.sqrt(np.einsum("nd,nd->n", d, d))
        f = np.exp(1j * kappa * r) / (4.0 * math.pi * r)
    else:
        f = kernel(x, y)
    return 4.0 * area(Pa) * area(Pb) * np.sum(w * f)


def regular_data(V, T, n=NQ_REGULAR):
    """Physical points [nt, n^2, 3] and weights [nt, n^2] of the Duffy-Gauss rule
    of order n on every triangle."""
    lam, w = duffy_gauss_rule(n)
    P = V[T]
    x = np.einsum("qv,nvd->nqd", lam, P)
    A = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    return x, A[:, None] * w[None, :]
