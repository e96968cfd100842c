"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Only geometry and random numbers live here: closed triangulated surfaces
(icosphere, sphere-swept box, ellipsoid, small polyhedra), seeded complex
coefficient vectors and seeded plane-wave directions/polarisation angles.
Nothing in this package evaluates the boundary-integral method itself.
"""
from .meshes import (icosphere, rounded_box, ellipsoid, tetrahedron, octahedron,
                     icosahedron, flat_plate, scene, mesh_stats)
from .vectors import (gaussian_coeffs, fibonacci_directions, plane_waves, serving_set, workload)

__all__ = ["icosphere", "rounded_box", "ellipsoid", "tetrahedron", "octahedron",
           "icosahedron", "flat_plate", "scene", "mesh_stats", "gaussian_coeffs",
           "fibonacci_directions", "plane_waves", "serving_set", "workload"]
