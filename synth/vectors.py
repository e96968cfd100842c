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


def plane_waves(n, seed):
    """n plane waves: Fibonacci-sphere propagation directions and
    polarisations cos(psi) theta_hat + sin(psi) phi_hat (the spherical unit
    vectors at the propagation direction).  Returns (khat, pol), (n, 3) each."""
    khat, psi = fibonacci_directions(n, seed)
    th = np.arccos(np.clip(khat[:, 2], -1.0, 1.0))
    ph = np.arctan2(khat[:, 1], khat[:, 0])
    t_hat = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)
    p_hat = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
    pol = np.cos(psi)[:, None] * t_hat + np.sin(psi)[:, None] * p_hat
    return khat, pol


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
                      leaf=0.25, nrhs=64, seed=3, rhs="plane_waves"),
    # icosphere r = 8 (184 320 triangles / 276 480 RWG), 7 levels, 16 RHS
    "sphere_r8": dict(kind="icosphere", m=96, radius=8.0, leaf=0.25, nrhs=16, seed=4),
}


def serving_set(seed=5, n_geom=8, n_min=2000, n_max=150000):
    """Geometries of the serving workload: cycle sphere / rounded box /
    ellipsoid (semi-axes 1 : 0.75 : 0.5), RWG counts log-uniform in
    [n_min, n_max] from the seed, each scaled so its mean edge is a tenth of
    the wavelength (or its longest edge 0.12 if that is smaller, so touching
    triangles stay within adjacent 0.25-wavelength leaf boxes).
    Returns a list of (name, verts, tris)."""
    rng = np.random.default_rng(seed)
    targets = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_geom))
    out = []
    for i, nt in enumerate(targets):
        kind = ("sphere", "box", "ellipsoid")[i % 3]
        if kind == "box":
            n = max(4, int(round(np.sqrt(nt / 9.0))))
            v, t = meshes.rounded_box((1.0, 1.0, 0.25), 0.05, 1.0 / n)
        else:
            m = max(4, int(round(np.sqrt(nt / 30.0))))
            v, t = meshes.icosphere(m, 1.0) if kind == "sphere" else meshes.ellipsoid(m, (1.0, 0.75, 0.5))
        st = meshes.mesh_stats(v, t)
        scale = min(0.1 / st["mean_edge"], 0.12 / st["max_edge"])
        out.append(("%s_%d" % (kind, st["n_edges"]), v * scale, t))
    return out


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
