"""Pins for the oracle's Galerkin quadrature (Section 1 eq. (matrix), Section 5)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as Q

REF = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


def _rule_integral(lam, w, a, b):
    # reference right triangle, area 1/2
    x = lam @ REF
    return 0.5 * np.sum(w * x[:, 0] ** a * x[:, 1] ** b)


def _exact(a, b):
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("rule,deg", [("q7", 5), ("q16", 6)])
def test_polynomial_exactness_degree(rule, deg):
    lam, w = Q.q7_rule() if rule == "q7" else Q.q16_rule()
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            assert abs(_rule_integral(lam, w, a, b) - _exact(a, b)) < 1e-15
    # not exact one degree higher
    worst = max(abs(_rule_integral(lam, w, a, deg + 1 - a) - _exact(a, deg + 1 - a))
                for a in range(deg + 2))
    assert worst > 1e-8


def _potential_factory(P):
    """Potential of the uniform triangle at an in-plane point: sum over edges of
    the signed distance times log((RA+RB+L)/(RA+RB-L)).  Plain floats for speed."""
    edges = []
    for a in range(3):
        A, B, C = P[(a + 1) % 3], P[(a + 2) % 3], P[a]
        L = float(np.linalg.norm(B - A))
        nrm = np.cross(B - A, np.cross(C - A, B - A))
        nrm = nrm / np.linalg.norm(nrm)
        edges.append((tuple(map(float, A)), tuple(map(float, B)), L, tuple(map(float, nrm))))

    def pot(x0, x1, x2):
        s = 0.0
        for (A, B, L, nr) in edges:
            ra = math.sqrt((x0 - A[0]) ** 2 + (x1 - A[1]) ** 2 + (x2 - A[2]) ** 2)
            rb = math.sqrt((x0 - B[0]) ** 2 + (x1 - B[1]) ** 2 + (x2 - B[2]) ** 2)
            h = (x0 - A[0]) * nr[0] + (x1 - A[1]) * nr[1] + (x2 - A[2]) * nr[2]
            if ra + rb - L > 0:
                s += h * math.log((ra + rb + L) / (ra + rb - L))
        return s
    return pot


TRIS = [
    [[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]],
    [[0, 0, 0], [1, 0, 0], [0, 1, 0]],
    [[0.1, 0.2, 0.3], [1.3, -0.2, 0.5], [0.4, 0.9, -0.7]],
    [[0, 0, 0], [3, 0, 0], [0.2, 0.1, 0]],
]


@pytest.mark.parametrize("P", TRIS)
def test_laplace_self_integral_vs_adaptive_quadrature(P):
    """Closed form against an independent 2-D adaptive integration of the
    in-plane potential of the triangle."""
    P = np.asarray(P, dtype=float)
    a, b, c = P
    area2 = np.linalg.norm(np.cross(b - a, c - a))
    pot = _potential_factory(P)
    e1, e2 = b - a, c - a

    def f(v, u):
        return pot(a[0] + u * e1[0] + v * e2[0], a[1] + u * e1[1] + v * e2[1],
                   a[2] + u * e1[2] + v * e2[2])
    num, _ = integrate.dblquad(f, 0, 1, 0, lambda u: 1 - u, epsabs=1e-12, epsrel=1e-11)
    num *= area2
    assert abs(Q.laplace_self_integral(*P) - num) <= 1e-9 * num


def test_laplace_self_integral_invariances():
    P = np.array(TRIS[2])
    ref = Q.laplace_self_integral(*P)
    for perm in [(1, 2, 0), (2, 0, 1), (1, 0, 2)]:
        assert abs(Q.laplace_self_integral(*P[list(perm)]) - ref) <= 1e-14 * ref
    assert abs(Q.laplace_self_integral(*(2.0 * P)) - 8.0 * ref) <= 1e-14 * ref
    shift = np.array([0.25, -0.5, 1.0])
    assert abs(Q.laplace_self_integral(*(P + shift)) - ref) <= 1e-13 * ref


def test_rho_stable_form_and_limit():
    r = np.array([0.0, 1e-3, 0.1, 1.0, 3.0])
    kappa = 7.0
    rho = Q.rho(r, kappa)
    assert rho[0] == 1j * kappa
    direct = (np.exp(1j * kappa * r[1:]) - 1.0) / r[1:]
    assert np.max(np.abs(rho[1:] - direct)) < 1e-12
    assert abs(Q.rho(np.array([1e-9]), kappa)[0] - 1j * kappa) < 1e-7


def test_self_entry_kappa_zero_is_laplace():
    V = np.array(TRIS[2], dtype=float)
    T = np.array([[0, 1, 2]])
    tri = Q.triangle_data(V, T)
    g0 = Q.self_entry(tri, 0, 0.0)
    assert g0.imag == 0.0
    assert abs(g0.real - Q.laplace_self_integral(*V) / (4 * math.pi)) < 1e-15
    # continuity in kappa
    assert abs(Q.self_entry(tri, 0, 1e-7) - g0) < 1e-6


def test_directional_splitting_identity():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 3))
    y = rng.standard_normal((5, 3)) + 4.0
    c = np.array([1.0, 2.0, -2.0]) / 3.0
    kappa = 5.0
    lhs = Q.kernel_g(x, y, kappa)
    rhs = np.exp(1j * kappa * ((x - y) @ c)) * Q.kernel_gc(x, y, c, kappa)
    assert np.max(np.abs(lhs - rhs)) < 1e-15


def test_triangle_data_weights_and_points():
    V = np.array(TRIS[2], dtype=float)
    T = np.array([[0, 1, 2]])
    tri = Q.triangle_data(V, T)
    area = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
    assert abs(tri["area"][0] - area) < 1e-15
    assert abs(tri["w7"].sum() - area) < 1e-15
    assert abs(tri["w16"].sum() - area) < 1e-15
    # all quadrature points inside the triangle (positive barycentric coordinates)
    for key in ("x7", "x16"):
        A = np.stack([V[1] - V[0], V[2] - V[0]], axis=1)
        lam, *_ = np.linalg.lstsq(A, (tri[key][0] - V[0]).T, rcond=None)
        assert (lam > 0).all() and (lam.sum(axis=0) < 1).all()
