"""Seeded synthetic inputs for the discrete-dipole solve.

This module is shared by the oracle, the tests and the benchmark.  It holds
geometry (which lattice sites are occupied), material assignments, incidence
geometry and random draws -- and none of the scattering arithmetic: no
polarizabilities, no interaction tensor, no solver, no efficiencies.

Everything is returned as plain numpy arrays; every random draw comes from
``numpy.random.default_rng`` with a documented seed tuple so that a run can be
reproduced exactly.

Workloads (all in lattice units, dipole spacing d = 1):

* ``sphere_integer``: the integer sites with i^2+j^2+k^2 <= r^2 (the
  pseudosphere used to compare against Mie theory; "Applicability of the DDA").
* ``box_ellipsoid`` / ``box_sphere``: an ellipsoid inscribed in an
  nx x ny x nz box, site coordinates i-(n-1)/2, kept when sum (x/a)^2 <= 1
  (the ELLIPSOID target of "Target Generation: Isolated Finite Targets").
* ``brick``: every site of an nx x ny x nz box (the RCTGLPRSM target).
* ``orientation_angles`` / ``lab_axes_in_target_frame``: the (beta, Theta,
  Phi) target orientation angles and the lab-frame axes expressed in the
  target frame, following "Target Orientation" (section "Orientation of the
  Target in the Lab Frame", the inverse relations for x_LF, y_LF, z_LF) with
  the target axes a1, a2, a3 taken along the target-frame x, y, z.
"""
from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------


def sphere_integer(radius: float) -> np.ndarray:
    """Integer lattice sites (i, j, k) with i^2 + j^2 + k^2 <= radius^2.

    Returns int32 [N, 3] in lexicographic (i, j, k) order with k fastest.
    """
    r = int(math.floor(radius))
    g = np.arange(-r, r + 1)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    keep = (i * i + j * j + k * k) <= radius * radius + 1e-9
    return np.stack([i[keep], j[keep], k[keep]], axis=1).astype(np.int32)


def box_ellipsoid(n: tuple[int, int, int], semi: tuple[float, float, float]) -> np.ndarray:
    """Sites of an n[0] x n[1] x n[2] box whose centred coordinates
    c = i - (n-1)/2 satisfy sum (c/semi)^2 <= 1.  Returns the integer box
    indices, int32 [N, 3]."""
    axes = [np.arange(m) for m in n]
    i, j, k = np.meshgrid(*axes, indexing="ij")
    cx = (i - (n[0] - 1) / 2.0) / semi[0]
    cy = (j - (n[1] - 1) / 2.0) / semi[1]
    cz = (k - (n[2] - 1) / 2.0) / semi[2]
    keep = (cx * cx + cy * cy + cz * cz) <= 1.0 + 1e-12
    return np.stack([i[keep], j[keep], k[keep]], axis=1).astype(np.int32)


def box_sphere(n: int, radius: float) -> np.ndarray:
    """Sphere of the given radius centred in an n^3 box (``box_ellipsoid``)."""
    return box_ellipsoid((n, n, n), (radius, radius, radius))


def brick(nx: int, ny: int, nz: int) -> np.ndarray:
    """Every site of an nx x ny x nz box, int32 [N, 3]."""
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int32)


# --------------------------------------------------------------------------
# incidence geometry
# --------------------------------------------------------------------------


def orientation_angles(seed: int, count: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Random target orientations, uniform on SO(3): beta and Phi uniform in
    [0, 2pi), cos(Theta) uniform in [-1, 1].  Stream ``default_rng([seed, 3])``,
    drawn as three arrays of ``count`` (beta, then cos Theta, then Phi)."""
    rng = np.random.default_rng([seed, 3])
    beta = 2.0 * math.pi * rng.random(count)
    cos_theta = 2.0 * rng.random(count) - 1.0
    phi = 2.0 * math.pi * rng.random(count)
    return beta, np.arccos(cos_theta), phi


def lab_axes_in_target_frame(beta: float, theta: float, phi: float) -> np.ndarray:
    """Unit vectors x_LF, y_LF, z_LF expressed in the target frame (rows).

    x_LF is the propagation direction k-hat; y_LF and z_LF are the two
    linear polarizations e01 and e02.  Target axes a1, a2, a3 are the
    target-frame x, y, z axes."""
    cb, sb = math.cos(beta), math.sin(beta)
    ct, st = math.cos(theta), math.sin(theta)
    cp, sp = math.cos(phi), math.sin(phi)
    x_lf = [ct, -st * cb, st * sb]
    y_lf = [st * cp, ct * cb * cp - sb * sp, -(ct * sb * cp + cb * sp)]
    z_lf = [st * sp, ct * cb * sp + sb * cp, -(ct * sb * sp - cb * cp)]
    return np.array([x_lf, y_lf, z_lf], dtype=np.float64)


def incidences_for_orientations(seed: int, count: int) -> tuple[np.ndarray, np.ndarray]:
    """(khat [2*count, 3] float64, e0 [2*count, 3] complex128): for each
    orientation, two right-hand sides with polarizations y_LF and z_LF."""
    beta, theta, phi = orientation_angles(seed, count)
    kh, e0 = [], []
    for b, t, p in zip(beta, theta, phi):
        ax = lab_axes_in_target_frame(b, t, p)
        for pol in (1, 2):
            kh.append(ax[0])
            e0.append(ax[pol].astype(np.complex128))
    return np.array(kh), np.array(e0)


def lab_directions(theta_deg, phi_deg) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Scattering directions for incidence along x (the Lab Frame of "Target
    Orientation"): for scattering angle theta and scattering-plane angle phi
    (phi = 0: the x-y plane), the unit vector n of the direction and the unit
    vectors theta_s, phi_s of the two scattered polarizations, as three
    float64 arrays [n_dir, 3] (n, theta_s, phi_s a right-handed frame)."""
    t = np.radians(np.asarray(theta_deg, dtype=np.float64).reshape(-1))
    p = np.radians(np.asarray(phi_deg, dtype=np.float64).reshape(-1))
    ct, st, cp, sp = np.cos(t), np.sin(t), np.cos(p), np.sin(p)
    n = np.stack([ct, st * cp, st * sp], axis=-1)
    theta_s = np.stack([-st, ct * cp, ct * sp], axis=-1)
    phi_s = np.stack([np.zeros_like(t), -sp, cp], axis=-1)
    return n, theta_s, phi_s


def along_x_yz() -> tuple[np.ndarray, np.ndarray]:
    """Incidence along +x with the two linear polarizations y and z."""
    kh = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    e0 = np.array([[0, 1, 0], [0, 0, 1]], dtype=np.complex128)
    return kh, e0


# --------------------------------------------------------------------------
# seeded materials and sizes
# --------------------------------------------------------------------------


def sphere_radii(seed: int, count: int = 32) -> np.ndarray:
    """Radii of the ragged sphere batch: ``default_rng([seed, 33]).uniform(6, 20, count)``."""
    return np.random.default_rng([seed, 33]).uniform(6.0, 20.0, count)


def two_material_mask(seed: int, n: int = 40) -> np.ndarray:
    """True = material A for each site of an n^3 brick in ``brick`` order.
    Stream ``default_rng([seed, 5])`` for n = 40, ``[seed, 56]`` for the 6^3 instance."""
    stream = 5 if n == 40 else 56
    return np.random.default_rng([seed, stream]).random(n ** 3) < 0.5


def fd_sites(seed: int, n_sites: int = 64000, count: int = 20) -> np.ndarray:
    """Sites checked by finite differences: ``default_rng([seed, 55]).choice``."""
    return np.random.default_rng([seed, 55]).choice(n_sites, count, replace=False)


def random_vectors(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Complex128 standard-normal test vectors, ``default_rng([seed, 7])``."""
    rng = np.random.default_rng([seed, 7])
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


# --------------------------------------------------------------------------
# the workloads, by name
# --------------------------------------------------------------------------

M_WATERLIKE = 1.33 + 0.01j


def workload(name: str, seed: int = 0) -> dict:
    """Sites, per-site refractive index, size parameter, incidences, tolerance.

    Names: 'sphere389' (N=389 pseudosphere, x=1, tol 1e-8),
    'ellipsoid51k' (64x48x32 ellipsoid with semi-axes 32/24/16, x=5, tol 1e-5),
    'brick48' (48x24x16 brick, x=4, 64 random orientations x 2 polarizations),
    'sphere1m' (radius-64 sphere in a 128^3 box, x=20, tol 1e-5),
    'twomat40' (40^3 two-material brick, x=6), 'twomat6' (its 6^3 instance,
    same kd as the 40^3 case), 'au_brick' (16x32x32 gold brick, x=3.093665),
    'au_sphere_nf' (gold pseudosphere of the near-field example, N = 59728)."""
    if name == "sphere389":
        ijk = sphere_integer(4.5)
        kh, e0 = along_x_yz()
        m = np.full(len(ijk), M_WATERLIKE)
        return dict(ijk=ijk, m=m, x=1.0, khat=kh, e0=e0, tol=1e-8)
    if name == "ellipsoid51k":
        ijk = box_ellipsoid((64, 48, 32), (32.0, 24.0, 16.0))
        kh, e0 = along_x_yz()
        m = np.full(len(ijk), 1.5 + 0.02j)
        return dict(ijk=ijk, m=m, x=5.0, khat=kh, e0=e0, tol=1e-5)
    if name == "brick48":
        ijk = brick(48, 24, 16)
        kh, e0 = incidences_for_orientations(seed, 64)
        m = np.full(len(ijk), 1.6 + 0.1j)
        return dict(ijk=ijk, m=m, x=4.0, khat=kh, e0=e0, tol=1e-5)
    if name == "sphere1m":
        ijk = box_sphere(128, 64.0)
        kh, e0 = along_x_yz()
        m = np.full(len(ijk), M_WATERLIKE)
        return dict(ijk=ijk, m=m, x=20.0, khat=kh, e0=e0, tol=1e-5)
    if name in ("twomat40", "twomat6"):
        n = 40 if name == "twomat40" else 6
        ijk = brick(n, n, n)
        mask = two_material_mask(seed, n)
        m = np.where(mask, 1.5 + 0.01j, 2.0 + 0.5j)
        # the 6^3 instance keeps the 40^3 case's kd: x scales with N^(1/3)
        x = 6.0 if n == 40 else 6.0 * (n / 40.0)
        kh = np.array([[1.0, 0.0, 0.0]])
        e0 = np.array([[0, 1, 0]], dtype=np.complex128)
        return dict(ijk=ijk, m=m, x=x, khat=kh, e0=e0, tol=1e-5)
    if name == "au_brick":
        ijk = brick(16, 32, 32)
        kh, e0 = along_x_yz()
        m = np.full(len(ijk), 0.9656 + 1.8628j)
        return dict(ijk=ijk, m=m, x=3.093665, khat=kh, e0=e0, tol=1e-5)
    if name == "au_sphere_nf":
        # the guide's near-field example: a 48^3-box pseudosphere of diameter
        # 48.49 sites (N = 59728), m = 0.96+1.01i, x = 5, extended by half
        # the box on every side
        ijk = box_sphere(48, 48.49 / 2)
        kh, e0 = along_x_yz()
        m = np.full(len(ijk), 0.96 + 1.01j)
        return dict(ijk=ijk, m=m, x=5.0, khat=kh, e0=e0, tol=1e-5, nf_ext=(0.5,) * 6, polarizability="GKDLDR")
    raise KeyError(name)


def sphere_batch(seed: int = 0, count: int = 32) -> list[np.ndarray]:
    """The ragged batch: integer-site spheres with radii ``sphere_radii``."""
    return [sphere_integer(r) for r in sphere_radii(seed, count)]
