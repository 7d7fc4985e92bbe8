"""The electric field in and near the target on an extended lattice (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): never imported by the
product path.

The guide's section "Near-Field Calculations" (and "Additional Nearfield
Calculation?") takes a solved polarization P and evaluates, at every point j
of a rectangular lattice volume that contains the target, the incident field
E_inc,j and the field E_sca,j radiated by the target's dipoles, the dipole at
j itself excluded; the total field is E_inc + E_sca.  In the guide's sign
convention the off-diagonal blocks of A are minus the dipole field tensor, so
E_sca,j = - sum_{l != j} A_jl P_l.  The volume grows the target's bounding box
by the fractions r1..r6 of its extents on the -x, +x, -y, +y, -z, +z sides.

The guide's readnf program reports E along a line between two points; it does
not state how values between lattice points are formed.  Reading: trilinear
interpolation of the lattice values (``line_field``).  The printed track of
the gold-sphere example is reproduced this way to its printed digits and not
with the nearest lattice point (``tests/test_oracle_pins.py``).

Every function here is the definition written out: a direct O(N) sum per
point, no FFT.  Lattice units (d = 1), k = kd, P [N, 3] complex for one
right-hand side.
"""
from __future__ import annotations

import numpy as np


def extension(n, r):
    """Lattice points added below and above the bounding box on each axis.

    ``n`` = box extents (nx, ny, nz) in sites, ``r`` = (r1, ..., r6).  The
    guide extends X1..X2 to X1 - r1 Lx .. X2 + r2 Lx with Lx the box extent;
    on the lattice that is round(r1 nx) points below and round(r2 nx) above
    (reading: L = n d, the box's width in sites; the gold-sphere example's
    48-site box with r = 0.5 on every side becomes the printed 96 sites)."""
    n = [int(v) for v in n]
    r = [float(v) for v in r]
    lo = [int(np.floor(r[2 * a] * n[a] + 0.5)) for a in range(3)]
    hi = [int(np.floor(r[2 * a + 1] * n[a] + 0.5)) for a in range(3)]
    return lo, hi


def extended_box(ijk, r):
    """(origin, dims): lattice coordinates of the extended volume's first
    point and its extents, for target sites ``ijk`` [N, 3] and fractions r."""
    ijk = np.asarray(ijk, dtype=np.int64)
    lo_t = ijk.min(axis=0)
    n = ijk.max(axis=0) - lo_t + 1
    e_lo, e_hi = extension(n, r)
    origin = lo_t - np.asarray(e_lo)
    dims = n + np.asarray(e_lo) + np.asarray(e_hi)
    return origin.astype(np.int64), dims.astype(np.int64)


def scattered_field(ijk, P, k: float, points) -> np.ndarray:
    """E_sca at lattice points ``points`` [np, 3]: the sum over every dipole l
    not at the point of the field of an oscillating dipole P_l (Draine 1988),

        E = exp(ikr)/r [ k^2 (n x P) x n + (1/r^2 - ik/r)(3 n (n.P) - P) ],

    with R = r_point - r_l, r = |R|, n = R/r.  Returns [np, 3] complex."""
    rs = np.asarray(ijk, dtype=np.float64)
    P = np.asarray(P, dtype=np.complex128)
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    out = np.zeros((len(pts), 3), dtype=np.complex128)
    for i, pt in enumerate(pts):
        R = pt - rs
        dist = np.sqrt(np.sum(R * R, axis=1))
        keep = dist > 0
        R, dist, pl = R[keep], dist[keep], P[keep]
        n = R / dist[:, None]
        ndp = np.sum(n * pl, axis=1)
        pref = np.exp(1j * k * dist) / dist
        far = k * k * (pl - n * ndp[:, None])                       # (n x P) x n
        near = ((1.0 / dist ** 2 - 1j * k / dist)[:, None]) * (3.0 * n * ndp[:, None] - pl)
        out[i] = np.sum(pref[:, None] * (far + near), axis=0)
    return out


def incident_field(points, k: float, khat, e0) -> np.ndarray:
    """E_inc = e exp(i k khat . r) at lattice points, e = e0/|e0|, phase origin
    at lattice index (0, 0, 0) (the same convention as the solve's E_inc)."""
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    e = np.asarray(e0, dtype=np.complex128)
    e = e / np.linalg.norm(e)
    return np.exp(1j * k * (pts @ np.asarray(khat, dtype=np.float64)))[:, None] * e[None, :]


def box_points(origin, dims) -> np.ndarray:
    """Every point of the box in box-scan order (x fastest, then y, then z)."""
    nx, ny, nz = (int(v) for v in dims)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + np.asarray(origin, dtype=np.int64)


def nearfield(ijk, P, k: float, khat, e0, r):
    """(origin, dims, E_inc, E_sca) on the whole extended volume, fields
    [nz, ny, nx, 3] in box-scan order.  O(N x volume): small targets only."""
    origin, dims = extended_box(ijk, r)
    pts = box_points(origin, dims)
    shape = (int(dims[2]), int(dims[1]), int(dims[0]), 3)
    return (origin, dims, incident_field(pts, k, khat, e0).reshape(shape),
            scattered_field(ijk, P, k, pts).reshape(shape))


def line_points(a, b, n_ab: int) -> np.ndarray:
    """n_ab equally spaced points from a to b inclusive (lattice units)."""
    t = np.linspace(0.0, 1.0, int(n_ab))
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a[None, :] + t[:, None] * (b - a)[None, :]


def trilinear(field_at, pts) -> np.ndarray:
    """Trilinear interpolation of a lattice field: ``field_at(q)`` returns the
    field [m, 3] at integer lattice points q [m, 3]; ``pts`` [np, 3] real."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    base = np.floor(pts).astype(np.int64)
    frac = pts - base
    corners = np.array([[dx, dy, dz] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], dtype=np.int64)
    q = (base[:, None, :] + corners[None, :, :]).reshape(-1, 3)
    uniq, inv = np.unique(q, axis=0, return_inverse=True)
    vals = np.asarray(field_at(uniq))[np.ravel(inv)].reshape(len(pts), 8, 3)
    w = np.ones((len(pts), 8))
    for c, (dx, dy, dz) in enumerate(corners):
        for a, dd in enumerate((dx, dy, dz)):
            w[:, c] *= frac[:, a] if dd else 1.0 - frac[:, a]
    return np.sum(w[:, :, None] * vals, axis=1)


def line_field(ijk, P, k: float, khat, e0, a, b, n_ab: int) -> np.ndarray:
    """Total field E_inc + E_sca at n_ab points from a to b (lattice units),
    trilinear between lattice points (the readnf reading above)."""
    def field_at(q):
        return incident_field(q, k, khat, e0) + scattered_field(ijk, P, k, q)
    return trilinear(field_at, line_points(a, b, n_ab))
