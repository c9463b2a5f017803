"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the compression method: it only produces
surface meshes (vertex and triangle arrays), right-hand sides and the named
workload parameter sets.
"""
from .meshes import sphere_octahedral, cube_surface, ellipsoid_octahedral
from .rhs import complex_gaussian
from .workloads import WORKLOADS, Workload, make_mesh, batch_workloads

__all__ = ["sphere_octahedral", "cube_surface", "ellipsoid_octahedral", "batch_workloads",
           "complex_gaussian", "WORKLOADS", "Workload", "make_mesh"]
