"""Far-field scattering amplitudes, the amplitude matrix and the Mueller
matrix of a dipole array (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): never imported by the
product path.

The scattered field of the dipoles P_j at r_j (lattice units, d = 1) is, far
away in direction n, E_s = (k^2 e^{ikr} / r) (I - n n) . sum_j P_j
exp(-i k n . r_j) (Draine 1988).  The guide ("Scattering by Finite Targets:
The Mueller Matrix") writes (E_s . theta_s, E_s . phi_s) = e^{ikr}/(kr) f
(E_i . e01*, E_i . e02*), so f_ml = k^3 e_m . sum_j P_j^(l) exp(-i k n . r_j)
with e_1 = theta_s, e_2 = phi_s and P^(l) the solution for incident
polarization e0l.  The amplitude matrix (S2 S3; S4 S1) of Bohren & Huffman
(1983) follows from the guide's relation between the two, and the Mueller
elements from Bohren & Huffman's definitions.
"""
from __future__ import annotations

import numpy as np


def amplitude_vectors(ijk, P, k: float, n_hat) -> np.ndarray:
    """A(n) = k^3 sum_j P_j exp(-i k n . r_j) for directions n ([nd, 3]);
    P is [N, 3]; returns [nd, 3] complex."""
    r = np.asarray(ijk, dtype=np.float64)
    n = np.atleast_2d(np.asarray(n_hat, dtype=np.float64))
    ph = np.exp(-1j * k * (n @ r.T))          # [nd, N]
    return k ** 3 * (ph @ np.asarray(P, dtype=np.complex128))


def lab_directions(theta_deg, phi_deg):
    """Scattering direction n and the unit vectors theta_s, phi_s for
    incidence along x (the guide's Lab Frame): n = x cos t + (y cos p +
    z sin p) sin t, phi = 0 being the x-y scattering plane."""
    t = np.radians(np.asarray(theta_deg, dtype=np.float64))
    p = np.radians(np.asarray(phi_deg, dtype=np.float64))
    n = np.stack([np.cos(t), np.sin(t) * np.cos(p), np.sin(t) * np.sin(p)], axis=-1)
    th = np.stack([-np.sin(t), np.cos(t) * np.cos(p), np.cos(t) * np.sin(p)], axis=-1)
    ph = np.stack([np.zeros_like(t), -np.sin(p), np.cos(p)], axis=-1)
    return n, th, ph


def f_matrix(A1, A2, theta_hat, phi_hat) -> np.ndarray:
    """f[d, m, l]: m = 0 (theta_s), 1 (phi_s); l = 0, 1 (incident e01, e02)."""
    f = np.empty((len(theta_hat), 2, 2), dtype=np.complex128)
    for l, A in enumerate((A1, A2)):
        f[:, 0, l] = np.sum(theta_hat * A, axis=1)
        f[:, 1, l] = np.sum(phi_hat * A, axis=1)
    return f


def amplitude_matrix(f, e01, e02, phi_deg) -> np.ndarray:
    """(S2 S3; S4 S1) per direction: with a = e01* . y, b = e01* . z,
    c = e02* . y, d = e02* . z and the incident components parallel and
    perpendicular to the scattering plane (e_par = y cos p + z sin p,
    e_perp = e_par x x), S = -i (f11 f12; -f21 -f22) (a b; c d) R with
    R = (cos p  sin p; sin p  -cos p)."""
    e01 = np.asarray(e01, dtype=np.complex128)
    e02 = np.asarray(e02, dtype=np.complex128)
    M = np.array([[np.conj(e01[1]), np.conj(e01[2])], [np.conj(e02[1]), np.conj(e02[2])]])
    p = np.radians(np.asarray(phi_deg, dtype=np.float64))
    out = np.empty((len(f), 2, 2), dtype=np.complex128)
    for i in range(len(f)):
        F = np.array([[f[i, 0, 0], f[i, 0, 1]], [-f[i, 1, 0], -f[i, 1, 1]]])
        R = np.array([[np.cos(p[i]), np.sin(p[i])], [np.sin(p[i]), -np.cos(p[i])]])
        out[i] = -1j * F @ M @ R
    return out


def mueller(S) -> dict:
    """Bohren & Huffman's 16 Mueller elements from (S2 S3; S4 S1) per
    direction (their eq. 3.16)."""
    S2, S3, S4, S1 = S[:, 0, 0], S[:, 0, 1], S[:, 1, 0], S[:, 1, 1]
    a1, a2, a3, a4 = (np.abs(x) ** 2 for x in (S1, S2, S3, S4))
    c = np.conj
    return dict(
        S11=0.5 * (a2 + a3 + a4 + a1), S12=0.5 * (a2 - a3 + a4 - a1),
        S13=np.real(S2 * c(S3) + S1 * c(S4)), S14=np.imag(S2 * c(S3) - S1 * c(S4)),
        S21=0.5 * (a2 + a3 - a4 - a1), S22=0.5 * (a2 - a3 - a4 + a1),
        S23=np.real(S2 * c(S3) - S1 * c(S4)), S24=np.imag(S2 * c(S3) + S1 * c(S4)),
        S31=np.real(S2 * c(S4) + S1 * c(S3)), S32=np.real(S2 * c(S4) - S1 * c(S3)),
        S33=np.real(S1 * c(S2) + S3 * c(S4)), S34=np.imag(S2 * c(S1) + S4 * c(S3)),
        S41=np.imag(S4 * c(S2) + S1 * c(S3)), S42=np.imag(S4 * c(S2) - S1 * c(S3)),
        S43=np.imag(S1 * c(S2) - S3 * c(S4)), S44=np.real(S1 * c(S2) - S3 * c(S4)),
    )


def q_bk(A_back, theta_hat, phi_hat, k: float, a_eff_over_d: float) -> float:
    """Backscattering efficiency of one incident polarization: the
    differential cross section at theta = 180 deg, (|f_1l|^2 + |f_2l|^2)/k^2,
    over pi a_eff^2."""
    f1 = np.sum(theta_hat * A_back)
    f2 = np.sum(phi_hat * A_back)
    return float((abs(f1) ** 2 + abs(f2) ** 2) / k ** 2 / (np.pi * a_eff_over_d ** 2))


def angular_averages(ijk, P, k: float, khat, a_eff_over_d: float, n_theta: int = 48, n_phi: int = 64):
    """Q_sca, g = <cos theta> and <cos^2 theta> of one incident polarization
    (the guide's "Averaging over Scattering Directions" quantities): the
    differential cross section (|f_1|^2 + |f_2|^2)/k^2 integrated over all
    directions n = cos t khat + sin t (cos p u + sin p v) with Gauss-Legendre
    nodes in cos t and n_phi equally spaced p (exact for the band-limited
    far field once the nodes resolve it)."""
    kh = np.asarray(khat, dtype=np.float64)
    kh = kh / np.linalg.norm(kh)
    u = np.cross(kh, [1.0, 0.0, 0.0] if abs(kh[0]) < 0.9 else [0.0, 1.0, 0.0])
    u = u / np.linalg.norm(u)
    v = np.cross(kh, u)
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    p = np.arange(n_phi) * 2 * np.pi / n_phi
    MU, PP = np.meshgrid(mu, p, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    n = (MU[..., None] * kh + st[..., None] * (np.cos(PP)[..., None] * u + np.sin(PP)[..., None] * v)).reshape(-1, 3)
    A = amplitude_vectors(ijk, P, k, n)
    # |f_1|^2 + |f_2|^2 = |A|^2 - |n . A|^2 (the transverse part)
    dcs = (np.sum(np.abs(A) ** 2, axis=1) - np.abs(np.sum(n * A, axis=1)) ** 2) / k ** 2
    w = (wmu[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).reshape(-1)
    csca = np.sum(w * dcs)
    g = np.sum(w * dcs * MU.reshape(-1)) / csca
    c2 = np.sum(w * dcs * MU.reshape(-1) ** 2) / csca
    return float(csca / (np.pi * a_eff_over_d ** 2)), float(g), float(c2)
