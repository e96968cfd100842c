"""Seeded coefficient vectors, plane-wave directions and the named workloads."""
import numpy as np

from . import meshes


def gaussian_coeffs(n_rows, nrhs, seed, dtype=np.complex128):
    """Column-major (n_rows x nrhs) block whose real and imaginary parts are
    i.i.d. N(0, 1), drawn from numpy's PCG64 generator with the given seed.
    Returned as a Fortran-ordered array so column r is contiguous."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nrhs, n_rows))
    im = rng.standard_normal((nrhs, n_rows))
    return np.asfortranarray((re + 1j * im).T.astype(dtype))


def fibonacci_directions(n, seed):
    """n incidence directions on a Fibonacci sphere and n polarisation angles.

    z_i = 1 - (2i+1)/n, azimuth_i = i*pi*(3 - sqrt 5) + phi0; phi0 and the
    polarisation angles psi_i are U[0, 2 pi) from the seed.  Returns
    (khat (n,3), psi (n,)); the incident field's propagation direction is
    khat and its polarisation is cos(psi) theta_hat + sin(psi) phi_hat."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * np.pi)
    psi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    i = np.arange(n)
    z = 1.0 - (2.0 * i + 1.0) / n
    az = i * np.pi * (3.0 - 5.0 ** 0.5) + phi0
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(az), s * np.sin(az), z], axis=1), psi


# Named workloads (lambda = 1, k = 2 pi).  Mesh recipes only: the surfaces,
# the leaf box edge and the seeds.  Sizes follow the configurations the
# method is benchmarked on.
_WORKLOADS = {
    # icosphere r = 0.5, 1 280 triangles / 1 920 RWG, 3 levels, 1 RHS
    "sphere_r0.5": dict(kind="icosphere", m=8, radius=0.5, leaf=0.25, nrhs=1, seed=1),
    # icosphere r = 3 at lambda/10 (25 920 triangles / 38 880 RWG), 6 levels, 1 RHS
    "sphere_r3": dict(kind="icosphere", m=36, radius=3.0, leaf=0.25, nrhs=1, seed=2),
    # sphere-swept 4 x 4 x 1 box, rho 0.2, lattice 0.073, 64 plane-wave RHS
    "box_4x4x1": dict(kind="rounded_box", dims=(4.0, 4.0, 1.0), rho=0.2, spacing=0.073,
                      leaf=0.25, nrhs=64, seed=3),
    # icosphere r = 8 (184 320 triangles / 276 480 RWG), 7 levels, 16 RHS
    "sphere_r8": dict(kind="icosphere", m=96, radius=8.0, leaf=0.25, nrhs=16, seed=4),
}


def workload(name):
    """Return (verts, tris, spec) for a named workload."""
    spec = dict(_WORKLOADS[name])
    if spec["kind"] == "icosphere":
        v, t = meshes.icosphere(spec["m"], spec["radius"])
    elif spec["kind"] == "rounded_box":
        v, t = meshes.rounded_box(spec["dims"], spec["rho"], spec["spacing"])
    else:
        raise KeyError(name)
    spec["name"] = name
    return v, t, spec
