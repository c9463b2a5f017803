"""Pins for tensor Chebyshev interpolation (Section 2)."""
import numpy as np
import pytest

from oracle.chebyshev import cheb_nodes, lagrange_1d, box_points, box_lagrange


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_lagrange_cardinal_and_partition_of_unity(m):
    nodes = cheb_nodes(m)
    assert np.allclose(np.polynomial.chebyshev.chebval(nodes, [0] * m + [1]), 0, atol=1e-14)
    L = lagrange_1d(nodes, nodes)
    assert np.max(np.abs(L - np.eye(m))) < 1e-14
    x = np.linspace(-1, 1, 37)
    assert np.max(np.abs(lagrange_1d(x, nodes).sum(axis=1) - 1)) < 1e-13


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_tensor_interpolation_exact_for_low_degree(m):
    rng = np.random.default_rng(m)
    lo = np.array([-0.3, 0.2, 1.0])
    hi = np.array([0.5, 0.9, 1.7])
    xi = box_points(lo, hi, m)
    x = lo + (hi - lo) * rng.random((50, 3))
    L = box_lagrange(x, lo, hi, m)
    deg = m - 1
    f = lambda p: (p[:, 0] ** deg) * (p[:, 1] ** deg) - 2.0 * p[:, 2] ** deg + p[:, 0] * p[:, 2]
    if m < 2:
        return
    assert np.max(np.abs(L @ f(xi) - f(x))) < 1e-12
    assert np.max(np.abs(L.sum(axis=1) - 1.0)) < 1e-13


def test_flat_box_interpolation_on_the_plane():
    """A box of zero width in z (cube faces): every point maps to xhat = 0 and
    interpolation of x,y polynomials of degree < m stays exact on the plane,
    whatever the z dependence of the function."""
    lo = np.array([0.0, 0.0, 1.0])
    hi = np.array([1.0, 1.0, 1.0])
    m = 3
    xi = box_points(lo, hi, m)
    assert np.all(xi[:, 2] == 1.0)
    rng = np.random.default_rng(0)
    x = np.column_stack([rng.random(20), rng.random(20), np.ones(20)])
    L = box_lagrange(x, lo, hi, m)
    f = lambda p: p[:, 0] ** 2 * p[:, 1] - 3.0 * p[:, 1] ** 2 + np.exp(p[:, 2])
    assert np.max(np.abs(L @ f(xi) - f(x))) < 1e-12
