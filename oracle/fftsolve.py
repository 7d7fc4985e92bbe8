"""FFT-embedded interaction matrix and plain BiCGSTAB, FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): never imported by the
product path.

The off-diagonal part of A depends only on r_j - r_l, so on a cubic lattice it
is a three-level block-Toeplitz matrix; embedded in a circulant on a
zero-padded grid it is applied with three-dimensional FFTs (Goodman, Draine &
Flatau 1990, the method the guide names in "Choice of FFT Algorithm" and in
its acknowledgments of the FFT convolution code).  The padded extent along each
axis is 2n if that is a product of powers of 2, 3 and 5, otherwise the smallest
such number >= 2n - 1 (any extent >= 2n - 1 holds every separation
-(n-1)..(n-1) without wrap-around; the guide's "extension" of the
computational volume to 2^i 3^j 5^k sizes is the same idea).

BiCGSTAB is van der Vorst (1992), the PBCGST option of "Choice of Iterative
Algorithm", with x0 = 0 (the guide's usual starting guess), shadow residual
r^ = r0 and conjugated inner products <u, v> = sum conj(u) v.  It stops when
|E - A P| / |E| < tol, checked after the half step (s) and after the full step.
``qmr_sym`` is the QMRCCG option and ``bicgstab_l`` (l = 2) the PBCGS2
option of the same section (see their docstrings).
"""
from __future__ import annotations

import os

import numpy as np

# threads for scipy's FFT (-1: all CPUs); the CPU-baseline timing sets it to
# the host's CPU share and reports it
WORKERS = int(os.environ.get("DDA_ORACLE_FFT_WORKERS", "-1"))

try:  # scipy's FFT is a library primitive with a thread-pool option
    import scipy.fft as _fft

    def _fftn(a, axes):
        return _fft.fftn(a, axes=axes, workers=WORKERS)

    def _ifftn(a, axes):
        return _fft.ifftn(a, axes=axes, workers=WORKERS)
except Exception:  # pragma: no cover
    def _fftn(a, axes):
        return np.fft.fftn(a, axes=axes)

    def _ifftn(a, axes):
        return np.fft.ifftn(a, axes=axes)

from . import dense


def is_smooth235(m: int) -> bool:
    for p in (2, 3, 5):
        while m % p == 0:
            m //= p
    return m == 1


def padded_extent(n: int) -> int:
    """2n when 2,3,5-smooth, else the smallest 2,3,5-smooth integer >= 2n-1."""
    if is_smooth235(2 * n):
        return 2 * n
    m = max(2 * n - 1, 1)
    while not is_smooth235(m):
        m += 1
    return m


class FFTOperator:
    """A (for one right-hand side's 1/alpha) applied by FFT convolution."""

    def __init__(self, ijk, alpha_inv_sites, k: float):
        ijk = np.asarray(ijk, dtype=np.int64)
        self.lo = ijk.min(axis=0)
        self.pos = ijk - self.lo
        self.n = tuple(int(v) for v in self.pos.max(axis=0) + 1)
        self.M = tuple(padded_extent(v) for v in self.n)
        self.k = k
        self.alpha_inv = np.asarray(alpha_inv_sites, dtype=np.complex128)
        self.ghat = self._green_hat()

    def _offsets(self, axis):
        """Signed lattice separation stored at each padded index (None = empty slot)."""
        n, M = self.n[axis], self.M[axis]
        off = np.zeros(M)
        valid = np.zeros(M, dtype=bool)
        for m in range(M):
            if m <= n - 1:
                off[m], valid[m] = m, True
            elif m >= M - (n - 1):
                off[m], valid[m] = m - M, True
        return off, valid

    def _green_hat(self):
        """FFT of the six distinct components of the off-diagonal tensor,
        sampled at every separation on the padded grid (zero at R = 0 and in
        the empty slots).  Order: xx, xy, xz, yy, yz, zz."""
        ox, vx = self._offsets(0)
        oy, vy = self._offsets(1)
        oz, vz = self._offsets(2)
        X, Y, Z = np.meshgrid(ox, oy, oz, indexing="ij")
        V = vx[:, None, None] & vy[None, :, None] & vz[None, None, :]
        r = np.sqrt(X * X + Y * Y + Z * Z)
        V &= r > 0
        rs = np.where(V, r, 1.0)
        k = self.k
        pref = np.exp(1j * k * rs) / rs
        c_iso = pref * (-k * k - (1j * k * rs - 1.0) / rs ** 2)
        c_nn = pref * (k * k + 3.0 * (1j * k * rs - 1.0) / rs ** 2) / rs ** 2
        comps = []
        R = (X, Y, Z)
        for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)):
            g = c_nn * R[a] * R[b] + (c_iso if a == b else 0.0)
            comps.append(np.where(V, g, 0.0))
        return _fftn(np.stack(comps), axes=(1, 2, 3))

    def apply(self, x):
        """y = A x for x of shape [N, 3]."""
        x = np.asarray(x, dtype=np.complex128)
        grid = np.zeros((3,) + self.M, dtype=np.complex128)
        p = self.pos
        for a in range(3):
            grid[a][p[:, 0], p[:, 1], p[:, 2]] = x[:, a]
        xh = _fftn(grid, axes=(1, 2, 3))
        g = self.ghat
        full = ((g[0], g[1], g[2]), (g[1], g[3], g[4]), (g[2], g[4], g[5]))
        yh = np.stack([full[a][0] * xh[0] + full[a][1] * xh[1] + full[a][2] * xh[2] for a in range(3)])
        y = _ifftn(yh, axes=(1, 2, 3))
        out = np.stack([y[a][p[:, 0], p[:, 1], p[:, 2]] for a in range(3)], axis=1)
        return out + self.alpha_inv * x


def bicgstab(apply, b, tol: float, max_iter: int, x0=None):
    """Plain BiCGSTAB (van der Vorst 1992) on [N, 3] complex vectors.

    Returns (x, info) with info = dict(iters, matvecs, rel_residual (recursive),
    converged)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    matvecs = 0
    if x0 is None:
        r = b.copy()
    else:
        r = b - apply(x)
        matvecs += 1
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    if np.linalg.norm(r) / bnorm < tol:
        return x, dict(iters=0, matvecs=matvecs, rel_residual=float(np.linalg.norm(r) / bnorm), converged=True)
    for it in range(1, max_iter + 1):
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p)
        matvecs += 1
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        sn = np.linalg.norm(s) / bnorm
        if sn < tol:
            x = x + alpha * p
            return x, dict(iters=it, matvecs=matvecs, rel_residual=float(sn), converged=True)
        t = apply(s)
        matvecs += 1
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        rn = np.linalg.norm(r) / bnorm
        if rn < tol:
            return x, dict(iters=it, matvecs=matvecs, rel_residual=float(rn), converged=True)
    return x, dict(iters=max_iter, matvecs=matvecs, rel_residual=float(rn), converged=False)


def qmr_sym(apply, b, tol: float, max_iter: int, x0=None, trace=None):
    """QMR for complex-symmetric A (the guide's QMRCCG option of "Choice of
    Iterative Algorithm"), read as conjugate orthogonal CG (COCG; van der
    Vorst & Melissen 1990) followed by quasi-minimal-residual smoothing
    (Zhou & Walker 1994) of its iterates and residuals.

    COCG is CG with the unconjugated bilinear form u^T v, which A = A^T makes
    a valid Petrov-Galerkin condition: rho_k = r_k^T r_k, p_k = r_k +
    (rho_k / rho_{k-1}) p_{k-1}, alpha_k = rho_k / (p_k^T A p_k), x_{k+1} =
    x_k + alpha_k p_k, r_{k+1} = r_k - alpha_k A p_k.  The smoothing keeps
    tau_k (1/tau_k^2 = 1/tau_{k-1}^2 + 1/|r_k|^2, tau_0 = |r_0|) and replaces
    (y, s) by the convex combination (tau_k^2/tau_{k-1}^2)(y, s) +
    (tau_k^2/|r_k|^2)(x_k, r_k), so that s_k = b - A y_k.  It stops when
    |s_k| / |b| < tol and returns y.  ``trace``, if a list, receives
    dict(r, s, y, tau2) after every step (for the pins).

    Returns (y, info) with info = dict(iters, matvecs, rel_residual (of s),
    converged)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    matvecs = 0
    if x0 is None:
        r = b.copy()
    else:
        r = b - apply(x)
        matvecs += 1
    y = x.copy()
    s = r.copy()
    tau2 = float(np.vdot(r, r).real)
    if trace is not None:
        trace.append(dict(r=r.copy(), s=s.copy(), y=y.copy(), tau2=tau2))
    sn = np.sqrt(tau2) / bnorm
    if sn < tol:
        return y, dict(iters=0, matvecs=matvecs, rel_residual=float(sn), converged=True)
    p = np.zeros_like(b)
    rho_old = None
    for it in range(1, max_iter + 1):
        rho = np.sum(r * r)
        beta = 0.0 if rho_old is None else rho / rho_old
        p = r + beta * p
        q = apply(p)
        matvecs += 1
        alpha = rho / np.sum(p * q)
        x = x + alpha * p
        r = r - alpha * q
        rho_old = rho
        nu2 = float(np.vdot(r, r).real)
        tau2_new = 1.0 / (1.0 / tau2 + 1.0 / nu2)
        w_old, w_new = tau2_new / tau2, tau2_new / nu2
        s = w_old * s + w_new * r
        y = w_old * y + w_new * x
        tau2 = tau2_new
        if trace is not None:
            trace.append(dict(r=r.copy(), s=s.copy(), y=y.copy(), tau2=tau2))
        sn = np.linalg.norm(s) / bnorm
        if sn < tol:
            return y, dict(iters=it, matvecs=matvecs, rel_residual=float(sn), converged=True)
    return y, dict(iters=max_iter, matvecs=matvecs, rel_residual=float(sn), converged=False)


def bicgstab_l(apply, b, tol: float, max_iter: int, ell: int = 2, x0=None, trace=None):
    """BiCGstab(l) (Sleijpen & Fokkema 1993; the guide's PBCGS2 option of
    "Choice of Iterative Algorithm" is l = 2), conjugated inner products,
    shadow residual r~ = r0.  One outer iteration takes l BiCG steps, each
    extending the search vectors u_0..u_j and residuals r_0..r_j by one
    product, then a minimal-residual step: r_0 - sum_j gamma_j r_j is
    minimised over gamma by modified Gram-Schmidt on r_1..r_l.  Stops when
    |r| / |b| < tol after an outer iteration.  ``trace``, if a list, receives
    dict(x, r, r_bicg) after every outer iteration, r_bicg being the BiCG
    residual the minimal-residual step started from (for the pins).

    Returns (x, info) with info = dict(iters (outer), matvecs, rel_residual,
    converged)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    matvecs = 0
    if x0 is None:
        r = b.copy()
    else:
        r = b - apply(x)
        matvecs += 1
    rt = r.copy()
    u = np.zeros_like(b)
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    rn = np.linalg.norm(r) / bnorm
    if rn < tol:
        return x, dict(iters=0, matvecs=matvecs, rel_residual=float(rn), converged=True)
    for it in range(1, max_iter + 1):
        rs = [r] + [None] * ell
        us = [u] + [None] * ell
        rho0 = -omega * rho0
        # BiCG part
        for j in range(ell):
            rho1 = np.vdot(rt, rs[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                us[i] = rs[i] - beta * us[i]
            us[j + 1] = apply(us[j])
            matvecs += 1
            alpha = rho0 / np.vdot(rt, us[j + 1])
            for i in range(j + 1):
                rs[i] = rs[i] - alpha * us[i + 1]
            rs[j + 1] = apply(rs[j])
            matvecs += 1
            x = x + alpha * us[0]
        r_bicg = rs[0]
        # minimal-residual part (modified Gram-Schmidt)
        tau = np.zeros((ell + 1, ell + 1), dtype=np.complex128)
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=np.complex128)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = np.vdot(rs[i], rs[j]) / sigma[i]
                rs[j] = rs[j] - tau[i, j] * rs[i]
            sigma[j] = np.vdot(rs[j], rs[j]).real
            gp[j] = np.vdot(rs[j], rs[0]) / sigma[j]
        g = np.zeros(ell + 1, dtype=np.complex128)
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1, dtype=np.complex128)
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * rs[0]
        rs[0] = rs[0] - gp[ell] * rs[ell]
        us[0] = us[0] - g[ell] * us[ell]
        for j in range(1, ell):
            us[0] = us[0] - g[j] * us[j]
            x = x + gpp[j] * rs[j]
            rs[0] = rs[0] - gp[j] * rs[j]
        r, u = rs[0], us[0]
        if trace is not None:
            trace.append(dict(x=x.copy(), r=r.copy(), r_bicg=r_bicg.copy()))
        rn = np.linalg.norm(r) / bnorm
        if rn < tol:
            return x, dict(iters=it, matvecs=matvecs, rel_residual=float(rn), converged=True)
    return x, dict(iters=max_iter, matvecs=matvecs, rel_residual=float(rn), converged=False)


SOLVERS = {"bicgstab": bicgstab, "qmr": qmr_sym, "bicgstab2": bicgstab_l}


def solve_case(ijk, m_sites, x: float, khat, e0, tol: float, scheme: str = dense.LATTDR,
               m_medium: float = 1.0, max_iter: int = 1000, solver: str = "bicgstab") -> dict:
    """FFT-BiCGSTAB solve of one right-hand side; returns P, E, the Q's and
    solver counts (Q_sca = Q_ext - Q_abs here; the closed form is O(N^2))."""
    n = len(ijk)
    k = dense.kd_from_size_parameter(x, n)
    m_rel = np.asarray(m_sites, dtype=np.complex128) / m_medium
    ainv = dense.site_alpha_inverse(m_rel, k, khat, e0, scheme)
    op = FFTOperator(ijk, ainv, k)
    E = dense.incident_field(ijk, k, khat, e0)
    P, info = SOLVERS[solver](op.apply, E, tol, max_iter)
    qe, qa = dense.q_ext(E, P, k), dense.q_abs(P, ainv, k)
    true_res = float(np.linalg.norm(E - op.apply(P)) / np.linalg.norm(E))
    return dict(P=P, E=E, alpha_inv=ainv, k=k, op=op, qext=qe, qabs=qa, qsca=qe - qa,
                qpha=dense.q_pha(E, P, k), true_residual=true_res, **info)
