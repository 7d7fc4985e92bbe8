"""The polarizability prescriptions pinned by the lattice dispersion relation
(no GPU).

Draine & Goodman (1993) define LATTDR ("Dipole Polarizabilities") by asking
that an infinite cubic lattice of point dipoles carry a transverse plane wave
of wavevector K = m k khat -- the continuum's -- to order (kd)^2: the
coefficients b1, b2, b3 and the direction-and-polarization factor S are what
make the lattice sum's (kd)^2 term vanish, and the -(2/3) i (kd)^3 term is what
makes a lossless lattice lossless.  So, with T(K) the Ewald-summed lattice
interaction (tests/lattice_sums.py),

    R(k) = e^* . (1/alpha I + T(m k khat)) . e     (|e| = 1)

must be purely real and O(k^4) for every direction, polarization and real m.
A dropped or mis-read term (S from (khat . e)^2, e not normalised, S without
the modulus for elliptical e, the radiative-reaction sign, m^2 missing on b3)
leaves an O(k^2) or O(k^3) remainder, which the planted-mistake test checks.
Oblique incidence is what makes S nonzero; every printed example has khat on a
lattice axis and e transverse, where S = 0.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import dense

import lattice_sums as ls

K_SMALL = (0.05, 0.1)


def _cases():
    """(khat, e) pairs: an axis, two oblique directions with both linear and
    an elliptical polarization, and two of the random orientations of the
    48x24x16 brick's right-hand sides."""
    kh = np.array([0.36, 0.48, 0.8])
    e1 = np.array([0.8, -0.6, 0.0])
    e2 = np.cross(kh, e1)
    kr, er = w.incidences_for_orientations(0, 2)
    return [
        (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])),
        (kh, e1), (kh, e2), (kh, e1 + 0.5j * e2),
        (np.ones(3) / math.sqrt(3.0), np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)),
        (kr[0], er[0]), (kr[3], er[3]),
    ]


MATERIALS = (1.33, 1.7, 2.5)


def _remainder(m, k, khat, e, scheme=dense.LATTDR):
    eps = m * m
    khat = np.asarray(khat, dtype=np.float64)
    e = np.asarray(e, dtype=np.complex128)
    e = e / np.linalg.norm(e)
    T = ls.interaction_sum(math.sqrt(eps) * k * khat, k)
    ainv = dense.alpha_inverse(m, k, khat, e, scheme)
    return complex(np.conj(e) @ (np.diag(ainv) + T) @ e)


def _dispersion_violations(scheme=dense.LATTDR):
    """Cases where R(k) is not a real O(k^4) remainder: |R| > k^4, |Im R| >
    1e-12, or R(0.1)/R(0.05) outside 16 +- 1."""
    bad = []
    for m in MATERIALS:
        for khat, e in _cases():
            r = [_remainder(m, k, khat, e, scheme) for k in K_SMALL]
            ratio = (r[1] / r[0]).real if r[0] != 0 else float("inf")
            if (any(abs(v) > k ** 4 for v, k in zip(r, K_SMALL)) or any(abs(v.imag) > 1e-12 for v in r)
                    or abs(ratio - 16.0) > 1.0):
                bad.append((m, tuple(np.round(khat, 3)), r))
    return bad


def test_ewald_sum_equals_direct_sum_where_it_converges():
    """For Im k > 0 the direct lattice sum converges absolutely; the Ewald
    value matches it, and does not depend on the splitting parameter."""
    K = np.array([0.3, -0.2, 0.5])
    k = 0.4 + 1.5j
    direct = ls.interaction_sum_direct(K, k, dense.interaction_block, 24)
    for eta in (1.6, 2.0, 2.6):
        ew = ls.interaction_sum(K, k, eta=eta, n_real=6, n_recip=7)
        assert np.abs(ew - direct).max() <= 1e-12 * np.abs(direct).max(), eta


def test_ewald_sum_independent_of_splitting_at_real_k():
    K = 1.7 * 0.1 * np.array([0.36, 0.48, 0.8])
    a = ls.interaction_sum(K, 0.1, eta=1.5, n_real=7, n_recip=5)
    b = ls.interaction_sum(K, 0.1, eta=2.4, n_real=4, n_recip=8)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_static_limit_is_clausius_mossotti():
    """k -> 0 along the continuum dispersion: -e.T.e -> 4 pi/(eps-1) + 4 pi/3,
    the Lorentz local field, i.e. 1/alpha_CM (textbook)."""
    for m in MATERIALS:
        khat = np.array([0.36, 0.48, 0.8])
        e = np.array([0.8, -0.6, 0.0])
        k = 1e-3
        T = ls.interaction_sum(m * k * khat, k)
        val = -(e @ T @ e)
        assert abs(val.real - dense.alpha_cm_inverse(m * m)) <= 1e-5 * abs(dense.alpha_cm_inverse(m * m))


@pytest.mark.parametrize("scheme", [dense.LATTDR, dense.GKDLDR])
def test_prescription_satisfies_the_lattice_dispersion_relation(scheme):
    """R(k) real and O(k^4) for every case (GKDLDR's diagonal tensor has the
    same projection on e as LATTDR's scalar, so it passes too)."""
    assert _dispersion_violations(scheme) == []


def _mutant(kind):
    """The oracle's alpha_inverse with one plausible mistake planted."""
    b1, b2, b3 = dense.LDR_B1, dense.LDR_B2, dense.LDR_B3

    def ainv(m_rel, k, khat, e0, scheme=dense.LATTDR):
        eps = complex(m_rel) ** 2
        khat = np.asarray(khat, dtype=np.float64)
        e = np.asarray(e0, dtype=np.complex128)
        if kind != "unnormalised":
            e = e / np.linalg.norm(e)
        rr = (2.0 / 3.0) * 1j * k ** 3
        base = dense.alpha_cm_inverse(eps) + (rr if kind == "radiation_sign" else -rr)
        if kind == "khat_dot_e":
            s = abs(np.dot(khat, e)) ** 2
        elif kind == "no_modulus":
            s = np.sum(khat ** 2 * e ** 2)
        else:
            s = float(np.sum(khat ** 2 * np.abs(e) ** 2))
        b3e = b3 if kind == "b3_without_eps" else eps * b3
        v = base + (b1 + eps * b2 + b3e * s) * k * k
        return np.array([v, v, v], dtype=np.complex128)
    return ainv


@pytest.mark.parametrize("kind", ["khat_dot_e", "unnormalised", "no_modulus", "radiation_sign", "b3_without_eps"])
def test_pin_rejects_planted_mistakes(monkeypatch, kind):
    """Each planted mistake in the oracle's polarizability breaks the
    dispersion relation for at least one case.  The unnormalised-e mutant is
    fed e scaled by 2, as a caller may pass it."""
    mut = _mutant(kind)
    if kind == "unnormalised":
        monkeypatch.setattr(dense, "alpha_inverse", lambda m, k, kh, e, s=dense.LATTDR: mut(m, k, kh, 2.0 * e, s))
    else:
        monkeypatch.setattr(dense, "alpha_inverse", mut)
    assert _dispersion_violations() != []
