"""Right-hand sides that make a Krylov solver break down in its first step
(test infrastructure, CPU).  From x0 = 0, BiCGSTAB and BiCGstab(2) divide by
<rhat, A b> = b^H A b (rhat = r0 = b) and QMR for complex-symmetric A by
b^T A b; a b that zeroes that form stops them at once.

* b^T A b = 0: b = u + theta w with theta a root of the quadratic
  (w^T A w) theta^2 + 2 (u^T A w) theta + u^T A u = 0 (A = A^T), exact up to
  rounding for any A.
* b^H A b = 0 needs 0 in the numerical range of A, which a passive target
  (Im eps >= 0) never has: its b^H A b has a negative imaginary part (the
  absorbed plus scattered power).  A gain material (Im eps < 0) with Re eps
  below -2 makes both the Hermitian and the skew-Hermitian part indefinite;
  b then comes from minimising |b^H A b|^2 / |b|^4 from a seeded start.
  On a 2 x 2 x 2 cube of it (x = 1) BiCGSTAB restarted with the shadow
  residual conj(b) converges in about a dozen iterations; on larger cubes the
  strongly indefinite system breaks the restarted iteration down again.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

# eps = -3 - i: Re(1/alpha_CM) < 0 and gain, so 0 lies inside A's numerical range
GAIN_M = np.sqrt(-3.0 - 1.0j)


def bilinear_zero(A: np.ndarray, seed: int = 0) -> np.ndarray:
    """b with b^T A b = 0 (unit norm)."""
    rng = np.random.default_rng([seed, 91])
    n = A.shape[0]
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a2, a1, a0 = v @ A @ v, 2 * (u @ A @ v), u @ A @ u
    theta = np.roots([a2, a1, a0])[0]
    b = u + theta * v
    return b / np.linalg.norm(b)


def hermitian_zero(A: np.ndarray, seed: int = 0, starts: int = 8) -> np.ndarray:
    """b with b^H A b = 0 (unit norm), where A's numerical range holds 0."""
    n = A.shape[0]

    def f(x):
        b = x[:n] + 1j * x[n:]
        nb = float(np.vdot(b, b).real)
        z = np.vdot(b, A @ b)
        val = abs(z) ** 2 / nb ** 2
        g_re = A.T @ b.conj() + A @ b          # d(b^H A b) along Re b
        g_im = 1j * (A.T @ b.conj()) - 1j * (A @ b)
        d_re = 2 * np.real(np.conj(z) * g_re) / nb ** 2 - 4 * val * b.real / nb
        d_im = 2 * np.real(np.conj(z) * g_im) / nb ** 2 - 4 * val * b.imag / nb
        return val, np.concatenate([d_re, d_im])

    rng = np.random.default_rng([seed, 92])
    best = None
    for _ in range(starts):
        r = minimize(f, rng.standard_normal(2 * n), jac=True, method="L-BFGS-B",
                     options={"maxiter": 20000, "gtol": 1e-20, "ftol": 1e-32})
        if best is None or r.fun < best.fun:
            best = r
    b = best.x[:n] + 1j * best.x[n:]
    return b / np.linalg.norm(b)
