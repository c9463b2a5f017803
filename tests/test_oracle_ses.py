"""Pins of the oracle's version of the paper's quadrature (Section 5):
Sauter-Erichsen-Schwab rules for touching triangle pairs and the Duffy-Gauss
rule of order 3 (oracle/ses.py, oracle/quadrature.py q9_rule,
oracle/cquad.py near_block_paper).

* Every region map and weight of the three touching cases: smooth separable
  integrands f(x) h(y) over touching pairs (badly shaped triangles on
  purpose) equal the product of the two single-triangle integrals, computed
  by an independent high-order rule, to rounding.
* The singular case against closed forms: for kappa = 0 the identical-pair
  rule against the closed-form Laplace self integral, and the sum over the 16
  pairs of a triangle split into four (4 identical, 6 common-edge, 6
  common-vertex pairs) against the closed form of the whole triangle; both
  converge exponentially with the order, and the paper's order 5 is within
  1e-6.
* The Duffy-Gauss rule of order 3: exact for the monomials of total degree
  <= 4 on the reference triangle (closed form a! b! / (a + b + 2)!; the
  collapsed direction carries the Jacobian u, so degree 5 is not exact).
* The near block: touching pairs are found and take the touching rule in one
  orientation (the triangle of lower index first, so the block is exactly
  symmetric), the rest equal the 9 x 9 product rule.
"""
import math

import numpy as np
import pytest

from oracle import ses, cquad
from oracle.quadrature import laplace_self_integral, q9_rule, triangle_data

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

WELL = np.array([[0, 0, 0], [1, 0, 0], [0.45, 0.85, 0.05], [0.55, -0.8, 0.1],
                 [-0.5, 0.7, -0.2], [-0.6, -0.5, 0.1]], dtype=float)
CASES = {3: ([0, 1, 2], [0, 1, 2]), 2: ([0, 1, 2], [1, 0, 3]), 1: ([0, 1, 2], [4, 5, 0])}


def _single(V, tri, vec, n=30):
    lam, w = ses.duffy_gauss_rule(n)
    P = V[tri]
    x = lam @ P
    return ses.area(P) * np.sum(w * np.exp(1j * x @ vec) * (1.0 + x[:, 0] ** 2 * x[:, 1]))


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_touching_rules_integrate_smooth_functions(kind):
    V = np.random.default_rng(3).standard_normal((6, 3))      # far from equilateral
    a = np.array([0.7, -1.1, 0.4])
    b = np.array([-0.3, 0.9, 1.3])
    Ta, Tb = CASES[kind]
    exact = _single(V, Ta, a) * _single(V, Tb, b)

    def f(x, y):
        return (np.exp(1j * x @ a) * (1.0 + x[:, 0] ** 2 * x[:, 1])
                * np.exp(1j * y @ b) * (1.0 + y[:, 0] ** 2 * y[:, 1]))

    got = ses.ses_pair(V, Ta, Tb, 0.0, nq=16, kernel=f)
    assert abs(got - exact) <= 1e-13 * abs(exact)
    # constants: every rule's weights add up to |T^|^2 = 1/4
    assert abs(ses.ses_rule(kind, 3)[2].sum() - 0.25) < 1e-15


def test_identical_rule_against_the_closed_form():
    P = WELL[[0, 1, 2]]
    exact = laplace_self_integral(P[0], P[1], P[2]) / (4.0 * math.pi)
    errs = [abs(ses.ses_pair(WELL, [0, 1, 2], [0, 1, 2], 0.0, nq=q) - exact) / exact for q in (3, 5, 8)]
    assert errs[1] <= 1e-6                         # the paper's order 5
    assert errs[2] <= 1e-9 and errs[2] < errs[1] < errs[0]


def test_split_triangle_sum_against_the_closed_form():
    """A triangle split at its edge midpoints: the 16 pair integrals of the
    four parts (identical, common edge, common vertex) add up to the whole
    triangle's closed form; kappa = 0 so both sides are exact integrals."""
    T = np.array([[0, 0, 0], [1, 0, 0], [0.45, 0.85, 0.0]])
    mid = [(T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2]
    W = np.array([T[0], T[1], T[2], mid[0], mid[1], mid[2]])
    parts = [[0, 3, 5], [3, 1, 4], [5, 4, 2], [3, 4, 5]]
    kinds = {ses.touching_order(parts[i], parts[j])[0] for i in range(4) for j in range(4)}
    assert kinds == {1, 2, 3}
    exact = laplace_self_integral(*T) / (4.0 * math.pi)
    for nq, tol in ((5, 1e-6), (12, 1e-13)):
        tot = sum(ses.ses_pair(W, parts[i], parts[j], 0.0, nq=nq) for i in range(4) for j in range(4))
        assert abs(tot - exact) <= tol * exact


def test_touching_rule_symmetry_and_kappa():
    """g(x, y) = g(y, x): swapping the triangles gives the same entry to the
    rule's accuracy (the regions are not symmetric in the two triangles); for
    kappa > 0 the imaginary part tends to kappa |Ta| |Tb| / (4 pi) as kappa -> 0
    (sin(kappa r) / r -> kappa)."""
    for Ta, Tb in CASES.values():
        g1 = ses.ses_pair(WELL, Ta, Tb, 3.0)
        g2 = ses.ses_pair(WELL, Tb, Ta, 3.0)
        assert abs(g1 - g2) <= 1e-6 * abs(g1)
        g1 = ses.ses_pair(WELL, Ta, Tb, 3.0, nq=12)
        g2 = ses.ses_pair(WELL, Tb, Ta, 3.0, nq=12)
        assert abs(g1 - g2) <= 1e-13 * abs(g1)
        kap = 1e-4
        g = ses.ses_pair(WELL, Ta, Tb, kap)
        lim = kap * ses.area(WELL[Ta]) * ses.area(WELL[Tb]) / (4.0 * math.pi)
        assert abs(g.imag - lim) <= 1e-6 * lim


def test_duffy_gauss_order_3_exactness():
    lam, w = q9_rule()
    assert len(w) == 9 and abs(w.sum() - 1.0) < 1e-15
    # reference triangle (0,0), (1,0), (0,1): x = lam1, y = lam2, area 1/2
    x, y = lam[:, 1], lam[:, 2]
    for a in range(5):
        for b in range(5 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(0.5 * np.sum(w * x ** a * y ** b) - exact) <= 1e-15
    # not exact at degree 5 (u^6 in the collapsed direction)
    assert abs(0.5 * np.sum(w * x ** 5) - math.factorial(5) / math.factorial(7)) > 1e-10


def test_near_block_paper_rules():
    """A small strip of triangles: touching pairs take the touching rule, all
    others the 9 x 9 product rule; the block is symmetric."""
    V = np.array([[x, y, 0.1 * x * y] for y in (0.0, 1.0) for x in range(5)], dtype=float)
    T = []
    for x in range(4):
        T.append([x, x + 1, x + 5])
        T.append([x + 1, x + 6, x + 5])
    T = np.array(T)
    tri = triangle_data(V, T)
    kappa = 2.0
    idx = np.arange(len(T))
    blk = cquad.near_block_paper(tri, idx, idx, kappa)
    assert np.max(np.abs(blk - blk.T)) <= 1e-13 * np.max(np.abs(blk))
    for i in idx:
        for j in idx:
            kind = ses.touching_order(T[i], T[j])[0]
            if kind:
                lo, hi = min(i, j), max(i, j)
                ref = ses.ses_pair(V, T[lo], T[hi], kappa)
            else:
                d = tri["x9"][i][:, None, :] - tri["x9"][j][None, :, :]
                r = np.sqrt((d * d).sum(-1))
                ww = tri["w9"][i][:, None] * tri["w9"][j][None, :]
                ref = np.sum(ww * np.exp(1j * kappa * r) / (4.0 * math.pi * r))
            assert abs(blk[i, j] - ref) <= 1e-13 * abs(ref)
