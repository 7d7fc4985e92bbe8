"""Dense FP64 reference of the DDA linear system and its efficiencies.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): never imported by the
product path.

Units: lattice spacing d = 1, incident amplitude |E0| = 1, so every length is
in units of d and k below is the dimensionless kd.

Sources.  The guide (Draine & Flatau, DDSCAT 7.2 User Guide) states the
problem A P = E ("Choice of Iterative Algorithm", eq. AP=E), the definitions of
a_eff, x and the validity bound ("Applicability of the DDA"), the ambient
medium rule ("Application to Targets in Dielectric Media"), the incident
polarization convention ("Incident Polarization State") and the stopping test
(eq. err_tol).  It only names the sources of the remaining formulas, which are
written out here from those sources:

* interaction tensor and the Q_ext / Q_abs expressions: Draine (1988), the
  paper the guide cites for "the DDA formulae";
* LATTDR: Draine & Goodman (1993), cited in "Dipole Polarizabilities";
* GKDLDR: Gutkowicz-Krusin & Draine (2004), same section;
* Q_pha: the phase-lag efficiency defined in "What Does It Calculate?",
  evaluated as the real part of the forward-scattering sum (optical theorem);
* closed-form Q_sca: the angular integral of the far field of N dipoles,
  done analytically (spherical Bessel functions), exact for any N.
"""
from __future__ import annotations

import math

import numpy as np

# Lattice-dispersion-relation coefficients (Draine & Goodman 1993, eq. 3.8 there).
LDR_B1 = -1.891531
LDR_B2 = 0.1648469
LDR_B3 = -1.7700004

LATTDR = "LATTDR"
GKDLDR = "GKDLDR"


# --------------------------------------------------------------------------
# sizes ("Applicability of the DDA": V = N d^3, a_eff = (3V/4pi)^(1/3), x = k a_eff)
# --------------------------------------------------------------------------


def aeff_over_d(n_sites: int) -> float:
    """a_eff / d = (3N / 4 pi)^(1/3)."""
    return (3.0 * n_sites / (4.0 * math.pi)) ** (1.0 / 3.0)


def kd_from_size_parameter(x: float, n_sites: int) -> float:
    """kd = x / (a_eff/d), with x = 2 pi a_eff / lambda_medium."""
    return x / aeff_over_d(n_sites)


def kd_from_physical(wavelength: float, aeff: float, n_sites: int, m_medium: float = 1.0) -> float:
    """kd for vacuum wavelength and effective radius in the same physical units.
    In an ambient medium the wavelength is lambda_vac / m_medium
    ("Application to Targets in Dielectric Media", eq. lambda_medium)."""
    k = 2.0 * math.pi * m_medium / wavelength
    d = aeff / aeff_over_d(n_sites)
    return k * d


# --------------------------------------------------------------------------
# polarizability ("Dipole Polarizabilities")
# --------------------------------------------------------------------------


def alpha_cm_inverse(eps: complex) -> complex:
    """Clausius-Mossotti 1/alpha for d = 1: (4 pi / 3)(eps + 2)/(eps - 1)."""
    return (4.0 * math.pi / 3.0) * (eps + 2.0) / (eps - 1.0)


def alpha_inverse(m_rel: complex, k: float, khat, e0, scheme: str = LATTDR) -> np.ndarray:
    """Diagonal of 1/alpha (units d^-3) for one site, as a complex [3] array.

    LATTDR (Draine & Goodman 1993):
        1/alpha = 1/alpha_CM + (b1 + eps b2 + eps b3 S) k^2 - (2/3) i k^3,
        S = sum_mu khat_mu^2 |e_mu|^2  (e normalised; for real e this is the
        published sum of (khat_mu e_mu)^2), the same for all three axes.
    GKDLDR (Gutkowicz-Krusin & Draine 2004): the same form with S replaced by
        khat_mu^2 on axis mu, giving a diagonal tensor in the target frame.
    """
    eps = complex(m_rel) ** 2
    khat = np.asarray(khat, dtype=np.float64)
    e = np.asarray(e0, dtype=np.complex128)
    e = e / np.linalg.norm(e)
    base = alpha_cm_inverse(eps) - (2.0 / 3.0) * 1j * k ** 3
    if scheme == LATTDR:
        s = float(np.sum(khat ** 2 * np.abs(e) ** 2))
        v = base + (LDR_B1 + eps * LDR_B2 + eps * LDR_B3 * s) * k * k
        return np.array([v, v, v], dtype=np.complex128)
    if scheme == GKDLDR:
        return np.array(
            [base + (LDR_B1 + eps * LDR_B2 + eps * LDR_B3 * khat[mu] ** 2) * k * k for mu in range(3)],
            dtype=np.complex128,
        )
    raise ValueError(scheme)


def alpha_inverse_derivative(m_rel: complex, k: float, khat, e0, scheme: str = LATTDR) -> np.ndarray:
    """d(1/alpha)/d eps for one site, complex [3]: -4 pi/(eps-1)^2 + (b2 + b3 S) k^2."""
    eps = complex(m_rel) ** 2
    khat = np.asarray(khat, dtype=np.float64)
    e = np.asarray(e0, dtype=np.complex128)
    e = e / np.linalg.norm(e)
    base = -4.0 * math.pi / (eps - 1.0) ** 2
    if scheme == LATTDR:
        s = float(np.sum(khat ** 2 * np.abs(e) ** 2))
        v = base + (LDR_B2 + LDR_B3 * s) * k * k
        return np.array([v, v, v], dtype=np.complex128)
    return np.array([base + (LDR_B2 + LDR_B3 * khat[mu] ** 2) * k * k for mu in range(3)],
                    dtype=np.complex128)


def site_alpha_inverse(m_sites, k, khat, e0, scheme=LATTDR) -> np.ndarray:
    """[N, 3] diagonal of 1/alpha for every site (sites with equal m share a value)."""
    m_sites = np.asarray(m_sites, dtype=np.complex128)
    uniq, inv = np.unique(m_sites, return_inverse=True)
    table = np.array([alpha_inverse(m, k, khat, e0, scheme) for m in uniq])
    return table[inv.ravel()]


# --------------------------------------------------------------------------
# interaction matrix (Draine 1988)
# --------------------------------------------------------------------------


def interaction_block(R, k: float) -> np.ndarray:
    """3x3 off-diagonal block A_jl for separation R = r_j - r_l != 0:

        A_jl = exp(i k r)/r [ k^2 (n n - I) + (i k r - 1)/r^2 (3 n n - I) ],

    n = R/r.  -A_jl P_l is the field at r_j of an oscillating dipole P_l."""
    R = np.asarray(R, dtype=np.float64)
    r = float(np.linalg.norm(R))
    n = R / r
    nn = np.outer(n, n)
    eye = np.eye(3)
    return np.exp(1j * k * r) / r * (k * k * (nn - eye) + (1j * k * r - 1.0) / (r * r) * (3.0 * nn - eye))


def assemble(ijk, alpha_inv_sites, k: float) -> np.ndarray:
    """Dense 3N x 3N complex A: A_jl off the diagonal, diag(1/alpha_j) on it.
    Row/column index 3*j + mu (site j, Cartesian axis mu)."""
    r = np.asarray(ijk, dtype=np.float64)
    n = len(r)
    R = r[:, None, :] - r[None, :, :]                       # [N, N, 3]
    dist = np.sqrt(np.sum(R * R, axis=-1))
    np.fill_diagonal(dist, 1.0)
    nhat = R / dist[..., None]
    nn = nhat[..., :, None] * nhat[..., None, :]            # [N, N, 3, 3]
    eye = np.eye(3)
    pref = np.exp(1j * k * dist) / dist
    blk = pref[..., None, None] * (k * k * (nn - eye)
                                   + ((1j * k * dist - 1.0) / dist ** 2)[..., None, None] * (3.0 * nn - eye))
    idx = np.arange(n)
    blk[idx, idx] = 0.0
    a_inv = np.asarray(alpha_inv_sites, dtype=np.complex128)
    for mu in range(3):
        blk[idx, idx, mu, mu] = a_inv[:, mu]
    return blk.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def apply_rows(ijk, alpha_inv_sites, k: float, x, rows) -> np.ndarray:
    """(A x)_j for the listed sites j only, by the direct O(N) sum over l of
    A_jl x_l (the definition of the product; used to check products of
    targets far too large for a dense A).  Returns [len(rows), 3]."""
    r = np.asarray(ijk, dtype=np.float64)
    x = np.asarray(x, dtype=np.complex128)
    a_inv = np.asarray(alpha_inv_sites, dtype=np.complex128)
    out = np.zeros((len(rows), 3), dtype=np.complex128)
    for i, j in enumerate(rows):
        R = r[j] - r
        dist = np.sqrt(np.sum(R * R, axis=1))
        mask = dist > 0
        R, dist, xl = R[mask], dist[mask], x[mask]
        nhat = R / dist[:, None]
        pref = np.exp(1j * k * dist) / dist
        c_iso = pref * (-k * k - (1j * k * dist - 1.0) / dist ** 2)
        c_nn = pref * (k * k + 3.0 * (1j * k * dist - 1.0) / dist ** 2)
        ndotx = np.sum(nhat * xl, axis=1)
        out[i] = np.sum(c_iso[:, None] * xl + (c_nn * ndotx)[:, None] * nhat, axis=0) + a_inv[j] * x[j]
    return out


def incident_field(ijk, k: float, khat, e0) -> np.ndarray:
    """E_inc at every site, [N, 3]: e exp(i k khat . r_j), with e = e0/|e0|
    ("Incident Polarization State": the library normalises e01).  Phase origin
    at lattice index (0, 0, 0)."""
    r = np.asarray(ijk, dtype=np.float64)
    e = np.asarray(e0, dtype=np.complex128)
    e = e / np.linalg.norm(e)
    ph = np.exp(1j * k * (r @ np.asarray(khat, dtype=np.float64)))
    return ph[:, None] * e[None, :]


def solve_dense(A: np.ndarray, E: np.ndarray) -> np.ndarray:
    """P from A P = E by LU (LAPACK zgesv); E and P are [N, 3]."""
    return np.linalg.solve(A, E.reshape(-1)).reshape(-1, 3)


# --------------------------------------------------------------------------
# efficiencies (Draine 1988; "What Does It Calculate?")
# --------------------------------------------------------------------------


def q_prefactor(k: float, n_sites: int) -> float:
    """c_Q = 4 pi k / (pi a_eff^2) with a_eff in units of d."""
    a = aeff_over_d(n_sites)
    return 4.0 * math.pi * k / (math.pi * a * a)


def q_ext(E, P, k) -> float:
    """Q_ext = c_Q sum_j Im(E_j^* . P_j)."""
    return q_prefactor(k, len(P)) * float(np.sum(np.imag(np.conj(E) * P)))


def q_abs(P, alpha_inv_sites, k) -> float:
    """Q_abs = c_Q sum_j { Im[P_j . (1/alpha_j)^* P_j^*] - (2/3) k^3 |P_j|^2 }."""
    a_inv = np.asarray(alpha_inv_sites)
    term = np.imag(P * np.conj(a_inv) * np.conj(P)) - (2.0 / 3.0) * k ** 3 * np.abs(P) ** 2
    return q_prefactor(k, len(P)) * float(np.sum(term))


def q_pha(E, P, k) -> float:
    """Q_pha = (c_Q / 2) sum_j Re(E_j^* . P_j)."""
    return 0.5 * q_prefactor(k, len(P)) * float(np.sum(np.real(np.conj(E) * P)))


def _sph_j012(x):
    """Spherical Bessel j0, j1, j2 for x > 0 (upward recurrence is stable for
    the moderate orders used here); small x uses the series."""
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-3
    xs = np.where(small, 1.0, x)
    s, c = np.sin(xs), np.cos(xs)
    j0 = s / xs
    j1 = s / xs ** 2 - c / xs
    j2 = (3.0 / xs ** 2 - 1.0) * s / xs - 3.0 * c / xs ** 2
    x2 = x * x
    j0 = np.where(small, 1.0 - x2 / 6.0, j0)
    j1 = np.where(small, x / 3.0 - x * x2 / 30.0, j1)
    j2 = np.where(small, x2 / 15.0, j2)
    return j0, j1, j2


def q_sca_closed_form(ijk, P, k: float, block: int = 2048) -> float:
    """Exact Q_sca of N point dipoles, O(N^2):

        C_sca = k^4 sum_{j,l} P_j^* . [ int dOmega (I - n n) exp(i k n.(r_j - r_l)) ] . P_l
              = 4 pi k^4 sum_{j,l} P_j^* . [ (j0(u) - j1(u)/u) I + j2(u) Rhat Rhat ] . P_l,

    u = k |r_j - r_l|; the j = l term is (2/3)|P_j|^2.  Q = C / (pi a_eff^2)."""
    r = np.asarray(ijk, dtype=np.float64)
    P = np.asarray(P, dtype=np.complex128)
    n = len(r)
    total = 0.0
    for s0 in range(0, n, block):
        rj = r[s0:s0 + block]
        Pj = np.conj(P[s0:s0 + block])
        R = rj[:, None, :] - r[None, :, :]
        dist = np.sqrt(np.sum(R * R, axis=-1))
        u = k * dist
        j0, j1, j2 = _sph_j012(u)
        same = dist < 0.5
        us = np.where(same, 1.0, u)
        iso = np.where(same, 2.0 / 3.0, j0 - j1 / us)
        aniso = np.where(same, 0.0, j2 / np.where(same, 1.0, dist ** 2))
        dots = Pj @ P.T                                        # sum_mu Pj*_mu P_l,mu
        pr = np.einsum("jla,ja->jl", R, Pj)                    # R . Pj*
        rp = np.einsum("jla,la->jl", R, P)                     # R . P_l
        total += float(np.real(np.sum(iso * dots + aniso * pr * rp)))
    a = aeff_over_d(n)
    return 4.0 * math.pi * k ** 4 * total / (math.pi * a * a)


# --------------------------------------------------------------------------
# the guide's error measure (eq. err_tol) and the true residual
# --------------------------------------------------------------------------


def residuals(A: np.ndarray, P, E) -> tuple[float, float]:
    """(|E - A P| / |E|, |A^H A P - A^H E| / |A^H E|)."""
    p = np.asarray(P).reshape(-1)
    e = np.asarray(E).reshape(-1)
    r = A @ p - e
    ah = A.conj().T
    return (float(np.linalg.norm(r) / np.linalg.norm(e)),
            float(np.linalg.norm(ah @ r) / np.linalg.norm(ah @ e)))


# --------------------------------------------------------------------------
# one whole solve
# --------------------------------------------------------------------------


def solve_case(ijk, m_sites, x: float, khat, e0, scheme: str = LATTDR, m_medium: float = 1.0,
               with_qsca: bool = True) -> dict:
    """Dense solve of one right-hand side; returns P, E, 1/alpha, k and the Q's."""
    n = len(ijk)
    k = kd_from_size_parameter(x, n)
    m_rel = np.asarray(m_sites, dtype=np.complex128) / m_medium
    ainv = site_alpha_inverse(m_rel, k, khat, e0, scheme)
    A = assemble(ijk, ainv, k)
    E = incident_field(ijk, k, khat, e0)
    P = solve_dense(A, E)
    out = dict(P=P, E=E, alpha_inv=ainv, k=k, A=A,
               qext=q_ext(E, P, k), qabs=q_abs(P, ainv, k), qpha=q_pha(E, P, k))
    if with_qsca:
        out["qsca"] = q_sca_closed_form(ijk, P, k)
    return out
