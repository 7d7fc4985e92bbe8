"""Ewald summation of the dipole interaction over an infinite cubic lattice.

Test infrastructure (CPU).  It pins the oracle's polarizability against the
property the lattice-dispersion-relation prescription is defined by (Draine &
Goodman 1993, the LATTDR option of "Dipole Polarizabilities"): on an infinite
cubic lattice of unit spacing, dipoles P_l = e exp(i K . r_l) with the
continuum wavevector K = m k khat are a free mode of the lattice when
1/alpha e + T(K) e = 0, with

    T(K) = sum_{l != 0} A(r_l) exp(i K . r_l),

A the off-diagonal interaction block of the DDA matrix,
A(R) = -(k^2 + grad grad) exp(i k R)/R.  The sum converges only
conditionally, so it is split (Ewald) into a rapidly converging real-space
part and a reciprocal-lattice part:

    exp(ikR)/R = g1(R) + g2(R),
    g1(R) = [exp(ikR) erfc(eta R + ik/2eta) + exp(-ikR) erfc(eta R - ik/2eta)] / 2R,
    sum_l exp(iK.r_l) g2(r - r_l) = 4 pi sum_G exp((k^2 - q^2)/4 eta^2)
                                   exp(i q.r) / (q^2 - k^2),   q = K + G,

G running over the reciprocal lattice 2 pi Z^3.  The l = 0 term of the smooth
part g2 is removed again; its value (k^2 + grad grad) g2 at R = 0 follows from
the Taylor series of g2 = [2i sin kR + exp(ikR) erf(eta R + ic) +
exp(-ikR) erf(eta R - ic)] / 2R, c = k / 2 eta:

    (k^2 + grad grad) g2 |_0 = [ (2/3) i k^3 - (2/3) k^3 erfi(c)
                                 + (4 eta / 3 sqrt(pi)) exp(c^2) (k^2 - eta^2) ] I.

The formulas are analytic in k, so for complex k with Im k > 0 (where the
direct sum converges absolutely) the Ewald value can be checked against brute
force; the tests do that first.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def _cube(n: int, skip_origin: bool) -> np.ndarray:
    g = np.arange(-n, n + 1)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    if skip_origin:
        pts = pts[np.any(pts != 0, axis=1)]
    return pts.astype(np.float64)


def interaction_sum(K, k, eta: float = 2.0, n_real: int = 5, n_recip: int = 6) -> np.ndarray:
    """T(K) = sum_{l != 0} A(r_l) exp(i K . r_l) (3x3 complex) by Ewald
    summation on the unit cubic lattice; K real [3], k real or complex."""
    K = np.asarray(K, dtype=np.float64)
    k = complex(k)
    sp = math.sqrt(math.pi)
    eye = np.eye(3)
    # real-space part: (k^2 + grad grad) g1 at the lattice points l != 0
    L = _cube(n_real, True)
    R = np.sqrt(np.sum(L * L, axis=1))
    n = L / R[:, None]
    c = k / (2.0 * eta)
    up = np.exp(1j * k * R) * special.erfc(eta * R + 1j * c)
    um = np.exp(-1j * k * R) * special.erfc(eta * R - 1j * c)
    E = np.exp(-eta * eta * R * R + c * c)
    s0 = up + um
    s1 = 1j * k * (up - um) - (4.0 * eta / sp) * E              # (u+ + u-)'
    s2 = -k * k * s0 + (8.0 * eta ** 3 * R / sp) * E            # (u+ + u-)''
    h = s0 / (2.0 * R)
    h1 = s1 / (2.0 * R) - s0 / (2.0 * R * R)
    h2 = s2 / (2.0 * R) - s1 / (R * R) + s0 / R ** 3
    nn = n[:, :, None] * n[:, None, :]
    F1 = (k * k * h)[:, None, None] * eye + h2[:, None, None] * nn + (h1 / R)[:, None, None] * (eye - nn)
    ph = np.exp(1j * (L @ K))
    real = np.einsum("l,lab->ab", ph, F1)
    # reciprocal part: (k^2 + grad grad) of the smooth sum at r = 0
    q = K[None, :] + 2.0 * math.pi * _cube(n_recip, False)
    q2 = np.sum(q * q, axis=1)
    wgt = 4.0 * math.pi * np.exp((k * k - q2) / (4.0 * eta * eta)) / (q2 - k * k)
    recip = np.einsum("g,gab->ab", wgt, k * k * eye[None] - q[:, :, None] * q[:, None, :])
    # the l = 0 term of the smooth part
    self_term = ((2.0 / 3.0) * 1j * k ** 3 - (2.0 / 3.0) * k ** 3 * special.erfi(c)
                 + (4.0 * eta / (3.0 * sp)) * np.exp(c * c) * (k * k - eta * eta)) * eye
    # A = -(k^2 + grad grad) exp(ikR)/R
    return -(real + recip - self_term)


def interaction_sum_direct(K, k, block, n: int) -> np.ndarray:
    """The same sum taken directly over the cube |l|_inf <= n, l != 0, with
    ``block(R, k)`` the 3x3 interaction block (for Im k > 0 only, where it
    converges absolutely)."""
    K = np.asarray(K, dtype=np.float64)
    out = np.zeros((3, 3), dtype=np.complex128)
    for l in _cube(n, True):
        out += block(l, k) * np.exp(1j * float(l @ K))
    return out
