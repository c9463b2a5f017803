"""Named workloads: mesh recipe plus the method parameters.

kappa  wave number, order m (k = m^3 interpolation points per cluster),
eta    the admissibility parameter eta_2, eta1 the direction parameter eta_1,
leaf   the maximal leaf-cluster size, tol the recompression tolerance,
nrhs   right-hand sides per matvec.
"""
from dataclasses import dataclass

from .meshes import sphere_octahedral, cube_surface, ellipsoid_octahedral


@dataclass(frozen=True)
class Workload:
    name: str
    surface: str          # "sphere" | "cube" | "ellipsoid"
    q: int                # refinement level (sphere n = 8 q^2, cube n = 12 q^2)
    kappa: float
    order: int
    leaf: int
    tol: float
    eta: float = 1.0
    eta1: float = 10.0
    nrhs: int = 1
    norm: str = "fro"     # error control of the recompression: "fro" | "spectral"

    @property
    def n(self):
        return (8 if self.surface in ("sphere", "ellipsoid") else 12) * self.q * self.q


def make_mesh(w):
    if w.surface == "sphere":
        return sphere_octahedral(w.q)
    if w.surface == "cube":
        return cube_surface(w.q)
    if w.surface == "ellipsoid":
        return ellipsoid_octahedral(w.q)
    raise ValueError(w.surface)


WORKLOADS = {
    # plain FP64 case: unit sphere n = 2048, kappa 4, m 4, leaf 32, tol 1e-6
    "sphere2k": Workload("sphere2k", "sphere", 16, 4.0, 4, 32, 1e-6),
    # unit sphere n = 32768, kappa 16, m 5, leaf 64, tol 1e-6
    "sphere32k": Workload("sphere32k", "sphere", 64, 16.0, 5, 64, 1e-6),
    # unit sphere n = 131072, kappa 32, m 5, leaf 64, tol 1e-4, 16 right-hand sides
    "sphere131k": Workload("sphere131k", "sphere", 128, 32.0, 5, 64, 1e-4, nrhs=16),
    # the spectral-norm experiment on the sphere at doubled wave numbers (Section 5):
    # n = 32768, kappa 32, m 4, leaf 32, eps 1e-4, spectral block-relative control
    "sphere32k_spec": Workload("sphere32k_spec", "sphere", 64, 32.0, 4, 32, 1e-4, norm="spectral"),
    # the largest row of the paper's unit-sphere table (spectral control) at its own
    # wave number: n = 131072, kappa 64, m 4, leaf 32, tol 1e-4
    "sphere131k_k64": Workload("sphere131k_k64", "sphere", 128, 64.0, 4, 32, 1e-4, norm="spectral"),
    # directional stress cases: every admissible block carries a direction c != 0
    # (small eta1 makes every level directional, larger eta admits blocks early)
    "dir512": Workload("dir512", "sphere", 8, 6.0, 3, 8, 1e-6, eta=8.0, eta1=1.0),
    "dir2k": Workload("dir2k", "sphere", 16, 8.0, 3, 16, 1e-6, eta=4.0, eta1=1.0),
    "dir8k": Workload("dir8k", "sphere", 32, 16.0, 4, 32, 1e-6, eta=4.0, eta1=2.0),
    # dir2k at the benchmark's tolerance 1e-4 (rank decisions far from FP32 rounding)
    "dir2k_t4": Workload("dir2k_t4", "sphere", 16, 8.0, 3, 16, 1e-4, eta=4.0, eta1=1.0),
    # the learned-rank family: side-2 cube, m 6 (k = 216), leaf 16, tol 1e-4, with kappa
    # scaled with sqrt(n) from kappa 64 at n = 524172 (q = 209), the largest member
    # being far beyond one GPU's memory at leaf 16; these are sizes that fit
    "cube7k_m6": Workload("cube7k_m6", "cube", 24, 7.35, 6, 16, 1e-4),
    "cube28k_m6": Workload("cube28k_m6", "cube", 48, 14.7, 6, 16, 1e-4),
    "cube110k_m6": Workload("cube110k_m6", "cube", 96, 29.4, 6, 16, 1e-4),
    # cube [-1,1]^3 (flat cluster boxes on the faces), low frequency and directional
    "cube768": Workload("cube768", "cube", 8, 4.0, 3, 16, 1e-6, eta=2.0),
    # order 6 (k = 216) on the same surface: inner clusters with full-width weights
    "cube768_m6": Workload("cube768_m6", "cube", 8, 4.0, 6, 16, 1e-6, eta=2.0),
    "cube1200dir": Workload("cube1200dir", "cube", 10, 4.0, 3, 16, 1e-6, eta=4.0, eta1=2.0),
}


def batch_workloads(count=64, seed=2024, n_lo=2048, n_hi=32768):
    """Problems of the batching form: surfaces drawn from sphere, side-2 cube
    and ellipsoid (axes 1:2:3), sizes n ~ U[n_lo, n_hi] rounded to the mesh
    family (sphere / ellipsoid n = 8 q^2, cube n = 12 q^2), kappa ~ U[4, 24],
    m = 4, leaf 32, tol 1e-5, eta 1, eta1 10."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        surface = ("sphere", "cube", "ellipsoid")[int(rng.integers(0, 3))]
        n = float(rng.uniform(n_lo, n_hi))
        q = max(1, int(round((n / (12.0 if surface == "cube" else 8.0)) ** 0.5)))
        kappa = float(rng.uniform(4.0, 24.0))
        out.append(Workload("batch%02d" % i, surface, q, round(kappa, 3), 4, 32, 1e-5))
    return out
