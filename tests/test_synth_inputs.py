"""The seeded input generators shared by the oracle and the GPU path: mesh
sizes of each family, reproducibility, and the ranges of the batching recipe."""
import numpy as np

import synth


def test_mesh_families_have_the_stated_sizes():
    for q in (1, 3, 8):
        V, T = synth.sphere_octahedral(q)
        assert len(T) == 8 * q * q
        assert np.allclose(np.linalg.norm(V, axis=1), 1.0)          # vertices on the unit sphere
        V, T = synth.cube_surface(q)
        assert len(T) == 12 * q * q
        assert np.allclose(np.max(np.abs(V), axis=1), 1.0)          # vertices on the cube surface
        V, T = synth.ellipsoid_octahedral(q)
        assert len(T) == 8 * q * q
        assert np.allclose(np.sum((V / np.array([1.0, 2.0, 3.0])) ** 2, axis=1), 1.0)


def test_right_hand_sides_are_seeded():
    a = synth.complex_gaussian(100, 3, seed=4)
    b = synth.complex_gaussian(100, 3, seed=4)
    assert a.shape == (3, 100) and a.dtype == np.complex128
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.complex_gaussian(100, 3, seed=5))


def test_batch_recipe_ranges_and_reproducibility():
    ws = synth.batch_workloads()
    assert len(ws) == 64
    assert ws == synth.batch_workloads()
    assert {w.surface for w in ws} == {"sphere", "cube", "ellipsoid"}
    for w in ws:
        assert 4.0 <= w.kappa <= 24.0
        assert (w.order, w.leaf, w.tol) == (4, 32, 1e-5)
        # n rounded to the mesh family stays near [2048, 32768]
        assert 1800 <= w.n <= 33500
