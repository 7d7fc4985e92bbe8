"""Mie theory for a homogeneous sphere (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The guide judges DDA accuracy against exact Mie results for spheres
("Applicability of the DDA", Figs. 1-4, which compare with the equal-volume
sphere of radius a_eff).  Written from the equations of Bohren & Huffman
(1983), ch. 4: coefficients a_n, b_n from the logarithmic derivative
D_n(mx) (downward recurrence) and the Riccati-Bessel functions psi_n, xi_n
(upward recurrence), truncated at n_max = x + 4 x^(1/3) + 2 (Wiscombe 1980).
"""
from __future__ import annotations

import math

import numpy as np


def coefficients(m: complex, x: float):
    """Mie a_n, b_n for n = 1..n_max."""
    m = complex(m)
    nmax = int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    mx = m * x
    nstart = int(max(nmax, abs(mx))) + 16
    D = np.zeros(nstart + 1, dtype=np.complex128)
    for n in range(nstart, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    psi_m1, psi_0 = math.cos(x), math.sin(x)
    chi_m1, chi_0 = -math.sin(x), math.cos(x)
    xi_prev = complex(psi_0, -chi_0)
    a = np.zeros(nmax, dtype=np.complex128)
    b = np.zeros(nmax, dtype=np.complex128)
    psi_prev, chi_prev = psi_0, chi_0
    psi_pp, chi_pp = psi_m1, chi_m1
    for n in range(1, nmax + 1):
        psi = (2 * n - 1) / x * psi_prev - psi_pp
        chi = (2 * n - 1) / x * chi_prev - chi_pp
        xi = complex(psi, -chi)
        ta = D[n] / m + n / x
        tb = D[n] * m + n / x
        a[n - 1] = (ta * psi - psi_prev) / (ta * xi - xi_prev)
        b[n - 1] = (tb * psi - psi_prev) / (tb * xi - xi_prev)
        psi_pp, psi_prev = psi_prev, psi
        chi_pp, chi_prev = chi_prev, chi
        xi_prev = complex(psi_prev, -chi_prev)
    return a, b


def efficiencies(m: complex, x: float) -> dict:
    """Q_ext, Q_sca, Q_abs and Q_back for relative index m and size parameter x."""
    a, b = coefficients(m, x)
    n = np.arange(1, len(a) + 1)
    qext = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * np.real(a + b)))
    qsca = 2.0 / x ** 2 * float(np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2)))
    back = np.sum((2 * n + 1) * (-1.0) ** n * (a - b))
    return dict(qext=qext, qsca=qsca, qabs=qext - qsca, qback=float(abs(back) ** 2 / x ** 2))
