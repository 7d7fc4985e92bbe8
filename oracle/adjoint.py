"""Gradients of Q_abs and Q_ext with respect to the per-site permittivity,
by the adjoint of the dense solve (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The guide computes no derivatives; this follows from its statement of the
problem (A P = E, "Choice of Iterative Algorithm") and the efficiency formulas
of ``oracle.dense``.  The only entries of A that depend on eps_j are the
diagonal 1/alpha_j, a holomorphic function of eps_j with derivative h_j
(``dense.alpha_inverse_derivative``); A is complex symmetric (A = A^T), so the
adjoint system has the same matrix as the forward one.

Convention for a real objective Q and complex eps_j:
    grad_j = dQ/dRe(eps_j) + i dQ/dIm(eps_j).

Q_ext = c_Q Im(E^H P):  with A lam = c_Q conj(E),
    grad_j = i conj( -h_j . (lam_j * P_j) )
Q_abs = c_Q sum w_j |P_j|^2,  w = -Im(1/alpha) - (2/3) k^3:  with A lam = c_Q w conj(P),
    grad_j = 2 conj( -h_j . (lam_j * P_j) ) - i c_Q sum_mu conj(h_j,mu) |P_j,mu|^2
where "." sums over the three axes without conjugation.
"""
from __future__ import annotations

import numpy as np

from . import dense


def adjoint_rhs(E, P, alpha_inv_sites, k, w_qabs: float, w_qext: float) -> list:
    """The two adjoint right-hand sides (Q_abs part, Q_ext part), [N, 3] each."""
    cq = dense.q_prefactor(k, len(P))
    w = -np.imag(alpha_inv_sites) - (2.0 / 3.0) * k ** 3
    return [w_qabs * cq * w * np.conj(P), w_qext * cq * np.conj(E)]


def gradient_from_adjoint(P, lam_abs, lam_ext, h_sites, k, w_qabs: float) -> np.ndarray:
    """Combine the adjoint solutions into grad_j (complex [N])."""
    cq = dense.q_prefactor(k, len(P))
    implicit_abs = 2.0 * np.conj(-np.sum(h_sites * lam_abs * P, axis=1))
    explicit_abs = -1j * w_qabs * cq * np.sum(np.conj(h_sites) * np.abs(P) ** 2, axis=1)
    implicit_ext = 1j * np.conj(-np.sum(h_sites * lam_ext * P, axis=1))
    return implicit_abs + explicit_abs + implicit_ext


def gradient_dense(ijk, m_sites, x: float, khat, e0, w_qabs: float = 1.0, w_qext: float = 0.0,
                   scheme: str = dense.LATTDR) -> tuple[np.ndarray, dict]:
    """grad of (w_qabs Q_abs + w_qext Q_ext) with respect to eps_j = m_j^2, by
    one forward and one adjoint dense solve (LU reused)."""
    sol = dense.solve_case(ijk, m_sites, x, khat, e0, scheme, with_qsca=False)
    k = sol["k"]
    m_sites = np.asarray(m_sites, dtype=np.complex128)
    uniq, inv = np.unique(m_sites, return_inverse=True)
    htab = np.array([dense.alpha_inverse_derivative(m, k, khat, e0, scheme) for m in uniq])
    h = htab[inv.ravel()]
    g_abs, g_ext = adjoint_rhs(sol["E"], sol["P"], sol["alpha_inv"], k, w_qabs, w_qext)
    lam = np.linalg.solve(sol["A"], np.stack([g_abs.reshape(-1), g_ext.reshape(-1)], axis=1))
    grad = gradient_from_adjoint(sol["P"], lam[:, 0].reshape(-1, 3), lam[:, 1].reshape(-1, 3), h, k, w_qabs)
    return grad, sol


def objective_dense(ijk, eps_sites, x: float, khat, e0, w_qabs=1.0, w_qext=0.0, scheme=dense.LATTDR) -> float:
    """w_qabs Q_abs + w_qext Q_ext for per-site permittivities (for finite differences)."""
    m = np.sqrt(np.asarray(eps_sites, dtype=np.complex128))
    sol = dense.solve_case(ijk, m, x, khat, e0, scheme, with_qsca=False)
    return w_qabs * sol["qabs"] + w_qext * sol["qext"]
