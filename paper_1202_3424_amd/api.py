"""Python binding of the C ABI (include/dda.h).

Argument marshalling only: device memory and streams come from PyTorch, every
step of the solve runs in the HIP kernels of libdda.so.  Importing this module
loads the library and fails loudly if it is not built.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi

_lib = _abi.load()


class DDAError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.dda_last_error().decode()
        super().__init__(f"{where}: {_abi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, where: str, allow=()):
    if status != _abi.DDA_OK and status not in allow:
        raise DDAError(status, where)
    return status


def last_error() -> str:
    return _lib.dda_last_error().decode()


# ------------------------------------------------------------------ contexts

_contexts: dict = {}


def context(device: int | None = None) -> ctypes.c_void_p:
    """The library context bound to ``device`` and torch's current stream there."""
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    h = _contexts.get(key)
    if h is None:
        h = ctypes.c_void_p()
        _check(_lib.dda_ctx_create(dev, ctypes.c_void_p(stream), ctypes.byref(h)), "dda_ctx_create")
        _contexts[key] = h
    return h


# ------------------------------------------------------------------ options

_POLZ = {"LATTDR": _abi.DDA_LATTDR, "GKDLDR": _abi.DDA_GKDLDR}
_PREC = {"fp64": _abi.DDA_FP64, "fp32_matvec": _abi.DDA_FP32_MATVEC}
_SOLVER = {"bicgstab": _abi.DDA_BICGSTAB, "qmr": _abi.DDA_QMR_SYM, "bicgstab2": _abi.DDA_BICGSTAB2}


@dataclass
class Options:
    """Solve options (see dda_opts).  ``for_size_parameter`` builds the
    wavelength/a_eff pair of a given x = 2 pi a_eff m_medium / lambda."""
    wavelength: float = 2 * math.pi
    aeff: float = 1.0
    m_medium: float = 1.0
    tol: float = 1e-5
    max_iter: int = 1000
    polarizability: str = "LATTDR"
    precision: str = "fp64"
    solver: str = "bicgstab"
    recompute_green: bool = False
    final_checks: bool = True
    autotune: bool = True
    graphs: bool = True
    share_launches: bool = True
    kernel_variant: int = 0

    @classmethod
    def for_size_parameter(cls, x: float, **kw) -> "Options":
        m_med = kw.get("m_medium", 1.0)
        return cls(wavelength=2 * math.pi * m_med / x, aeff=1.0, **kw)

    def c(self) -> _abi.Opts:
        flags = 0
        if self.recompute_green:
            flags |= _abi.DDA_FLAG_RECOMPUTE_GREEN
        if not self.final_checks:
            flags |= _abi.DDA_FLAG_NO_FINAL_CHECKS
        if not self.autotune:
            flags |= _abi.DDA_FLAG_NO_AUTOTUNE
        if not self.graphs:
            flags |= _abi.DDA_FLAG_NO_GRAPH
        if not self.share_launches:
            flags |= _abi.DDA_FLAG_SEPARATE_TARGETS
        return _abi.Opts(self.wavelength, self.aeff, self.m_medium, self.tol, int(self.max_iter),
                         _POLZ[self.polarizability], _SOLVER[self.solver], _PREC[self.precision], flags,
                         int(self.kernel_variant))


def _incidences(khat, e0) -> ctypes.Array:
    kh = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    ee = np.atleast_2d(np.asarray(e0, dtype=np.complex128))
    if kh.shape != ee.shape or kh.shape[1] != 3:
        raise ValueError("khat and e0 must both be [n_rhs, 3]")
    arr = (_abi.Incidence * len(kh))()
    for q in range(len(kh)):
        for m in range(3):
            arr[q].khat[m] = float(kh[q, m])
            arr[q].e0[m] = _abi.C64(float(ee[q, m].real), float(ee[q, m].imag))
    return arr


def _dev_c128(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.complex128 and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a complex128 CUDA tensor of shape {tuple(shape)}")
    return t.contiguous()


# ------------------------------------------------------------------ targets

class Target:
    """A target uploaded to the device: occupied lattice sites ``ijk``
    (int [N, 3]) and per-site complex refractive index ``m`` ([N])."""

    def __init__(self, ijk, m, device: int | None = None):
        ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32))
        if ijk.ndim != 2 or ijk.shape[1] != 3:
            raise ValueError("ijk must be [N, 3]")
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(m, dtype=np.complex128), (len(ijk),)))
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.ctx = context(self.device)
        self.n_sites = len(ijk)
        h = ctypes.c_void_p()
        _check(_lib.dda_target_create(self.ctx, self.n_sites, ijk.ctypes.data, m.ctypes.data, ctypes.byref(h)),
               "dda_target_create")
        self._h = h
        box = (ctypes.c_int32 * 3)()
        grid = (ctypes.c_int32 * 3)()
        _check(_lib.dda_target_geometry(h, box, grid), "dda_target_geometry")
        self.box = tuple(box)
        self.grid = tuple(grid)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.dda_target_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_dict(r: _abi.Result) -> dict:
    return dict(qext=r.qext, qabs=r.qabs, qsca=r.qsca, qpha=r.qpha, rel_residual=r.rel_residual,
                normal_eq_residual=r.normal_eq_residual, kd=r.kd, aeff_d=r.aeff_d, iters=r.iters,
                matvecs=r.matvecs, status=r.status, restarts=r.restarts, refinements=r.refinements)


# ------------------------------------------------------------------ calls

def apply(target: Target, opts: Options, khat, e0, x: torch.Tensor) -> torch.Tensor:
    """y = A x for each right-hand side (x: complex128 CUDA [n_rhs, N, 3])."""
    inc = _incidences(khat, e0)
    x = _dev_c128(x, (len(inc), target.n_sites, 3), "x")
    y = torch.empty_like(x)
    o = opts.c()
    _check(_lib.dda_apply(target.ctx, target.handle, ctypes.byref(o), len(inc), inc, x.data_ptr(), y.data_ptr()),
           "dda_apply")
    return y


def apply_noalloc(target: Target, opts: Options, khat, e0, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """y = A x into the caller's y (complex128 CUDA [n_rhs, N, 3]) with the
    library's fixed work memory (dda_apply_noalloc: no device allocation; the
    target's tensor FFT for these options must already be built)."""
    inc = _incidences(khat, e0)
    x = _dev_c128(x, (len(inc), target.n_sites, 3), "x")
    _dev_c128(y, (len(inc), target.n_sites, 3), "y")
    if not y.is_contiguous():
        raise ValueError("y must be contiguous")
    o = opts.c()
    _check(_lib.dda_apply_noalloc(target.ctx, target.handle, ctypes.byref(o), len(inc), inc, x.data_ptr(),
                                  y.data_ptr()), "dda_apply_noalloc")
    return y


def solve(target: Target, opts: Options, khat, e0, P0: torch.Tensor | None = None, want_P: bool = True,
          raise_on_failure: bool = False):
    """Solve A P = E for every incidence; returns (P or None, [result dict])."""
    inc = _incidences(khat, e0)
    n = len(inc)
    P = torch.empty((n, target.n_sites, 3), dtype=torch.complex128, device=f"cuda:{target.device}") if want_P else None
    p0 = _dev_c128(P0, (n, target.n_sites, 3), "P0") if P0 is not None else None
    res = (_abi.Result * n)()
    o = opts.c()
    st = _lib.dda_solve(target.ctx, target.handle, ctypes.byref(o), n, inc, P.data_ptr() if P is not None else None,
                        p0.data_ptr() if p0 is not None else None, res)
    allow = () if raise_on_failure else (_abi.DDA_E_NOT_CONVERGED, _abi.DDA_E_BREAKDOWN, _abi.DDA_E_NONFINITE)
    _check(st, "dda_solve", allow)
    return P, [_result_dict(r) for r in res]


def solve_rhs(target: Target, opts: Options, khat, e0, b: torch.Tensor, x0: torch.Tensor | None = None):
    """Solve A x = b for caller-given right-hand sides (complex128 CUDA
    [n_rhs, N, 3]); A is the matrix of the given incidences.  Returns (x,
    [result dict]) (the efficiency fields are zero)."""
    inc = _incidences(khat, e0)
    n = len(inc)
    b = _dev_c128(b, (n, target.n_sites, 3), "b")
    x = torch.empty_like(b)
    p0 = _dev_c128(x0, (n, target.n_sites, 3), "x0") if x0 is not None else None
    res = (_abi.Result * n)()
    o = opts.c()
    st = _lib.dda_solve_rhs(target.ctx, target.handle, ctypes.byref(o), n, inc, b.data_ptr(), x.data_ptr(),
                            p0.data_ptr() if p0 is not None else None, res)
    _check(st, "dda_solve_rhs", (_abi.DDA_E_NOT_CONVERGED, _abi.DDA_E_BREAKDOWN, _abi.DDA_E_NONFINITE))
    return x, [_result_dict(r) for r in res]


def solve_batched(targets, opts, rhs_target, khat, e0, want_P: bool = True):
    """Several targets, each with its own right-hand sides, in one call.
    ``opts`` is one Options per target.  Returns ([P per rhs], [result dict])."""
    inc = _incidences(khat, e0)
    n = len(inc)
    rt = np.asarray(rhs_target, dtype=np.int32)
    if rt.shape != (n,):
        raise ValueError("rhs_target must have one entry per right-hand side")
    hs = (ctypes.c_void_p * len(targets))(*[t.handle.value for t in targets])
    oa = (_abi.Opts * len(targets))(*[o.c() for o in opts])
    Ps = []
    ptrs = (ctypes.c_void_p * n)()
    for q in range(n):
        t = targets[int(rt[q])]
        if want_P:
            P = torch.empty((t.n_sites, 3), dtype=torch.complex128, device=f"cuda:{t.device}")
            ptrs[q] = P.data_ptr()
            Ps.append(P)
        else:
            Ps.append(None)
    res = (_abi.Result * n)()
    st = _lib.dda_solve_batched(targets[0].ctx, len(targets), hs, oa, n, rt.ctypes.data, inc, ptrs, res)
    _check(st, "dda_solve_batched", (_abi.DDA_E_NOT_CONVERGED, _abi.DDA_E_BREAKDOWN, _abi.DDA_E_NONFINITE))
    return Ps, [_result_dict(r) for r in res]


def grad_eps(target: Target, opts: Options, khat, e0, P: torch.Tensor, w_qabs: float = 1.0, w_qext: float = 0.0):
    """Gradient of w_qabs Q_abs + w_qext Q_ext with respect to eps_j = m_j^2
    (dQ/dRe eps + i dQ/dIm eps), by one adjoint solve.  P: [N, 3] solution."""
    inc = _incidences(khat, e0)
    if len(inc) != 1:
        raise ValueError("grad_eps takes one incidence")
    P = _dev_c128(P, (target.n_sites, 3), "P")
    g = torch.empty(target.n_sites, dtype=torch.complex128, device=P.device)
    r = _abi.Result()
    o = opts.c()
    st = _lib.dda_grad_eps(target.ctx, target.handle, ctypes.byref(o), inc, P.data_ptr(), float(w_qabs),
                           float(w_qext), g.data_ptr(), ctypes.byref(r))
    _check(st, "dda_grad_eps", (_abi.DDA_E_NOT_CONVERGED,))
    return g, _result_dict(r)


class QEff(torch.autograd.Function):
    """(Q_abs, Q_ext) of a target as a differentiable function of the per-site
    permittivity eps ([N] complex128).  Backward runs one adjoint solve.

        q = QEff.apply(eps, ijk, opts, khat, e0)   # q = tensor([Q_abs, Q_ext])
    """

    @staticmethod
    def forward(ctx, eps, ijk, opts, khat, e0):
        m = torch.sqrt(eps.detach().to("cpu", torch.complex128)).numpy()
        tgt = Target(ijk, m)
        P, res = solve(tgt, opts, [khat], [e0], raise_on_failure=True)
        ctx.tgt, ctx.opts, ctx.khat, ctx.e0 = tgt, opts, khat, e0
        ctx.save_for_backward(P[0])
        ctx.eps_device = eps.device
        return torch.tensor([res[0]["qabs"], res[0]["qext"]], dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, gq):
        (P,) = ctx.saved_tensors
        g = gq.detach().to("cpu", torch.float64)
        grad, _ = grad_eps(ctx.tgt, ctx.opts, ctx.khat, ctx.e0, P, float(g[0]), float(g[1]))
        return grad.to(ctx.eps_device), None, None, None, None


def set_timing(categories=True, device: int | None = None) -> None:
    """Start (clearing totals) or stop per-kernel-category GPU timing.
    ``categories``: True (all), False (stop) or an iterable of category names."""
    if categories is True:
        mask = (1 << _abi.DDA_TIMING_CATEGORIES) - 1
    elif categories is False or categories is None:
        mask = 0
    else:
        mask = 0
        for name in categories:
            mask |= 1 << _abi.TIMING_NAMES.index(name)
    _check(_lib.dda_ctx_set_timing(context(device), mask), "dda_ctx_set_timing")


def far_field(target: "Target", opts: Options, P: torch.Tensor, n_hat, theta_hat, phi_hat):
    """Scattering amplitudes f [n_rhs, n_dir, 2] (complex128: theta, phi
    components) and differential cross sections dcs [n_rhs, n_dir] of the
    solution P [n_rhs, n_sites, 3] (device, complex128) for the given
    orthonormal direction frames (dda_far_field)."""
    if P.dim() == 2:
        P = P.unsqueeze(0)
    P = P.to(torch.complex128).contiguous()
    nh = np.ascontiguousarray(np.asarray(n_hat, dtype=np.float64).reshape(-1, 3))
    th = np.ascontiguousarray(np.asarray(theta_hat, dtype=np.float64).reshape(-1, 3))
    ph = np.ascontiguousarray(np.asarray(phi_hat, dtype=np.float64).reshape(-1, 3))
    n_rhs, n_dir = P.shape[0], nh.shape[0]
    f = np.zeros((n_rhs, n_dir, 2), dtype=np.complex128)
    dcs = np.zeros((n_rhs, n_dir), dtype=np.float64)
    o = opts.c()
    _check(_lib.dda_far_field(target.ctx, target.handle, ctypes.byref(o), n_rhs, P.data_ptr(), n_dir,
                              nh.ctypes.data, th.ctypes.data, ph.ctypes.data, f.ctypes.data, dcs.ctypes.data),
           "dda_far_field")
    return f, dcs


def scattering_averages(target: "Target", opts: Options, khat, e0, P: torch.Tensor, n_theta: int = 48,
                        n_phi: int = 64) -> list:
    """[{qsca, g, cos2}] per right-hand side: Q_sca, <cos theta> and
    <cos^2 theta> by quadrature of the far field (dda_scattering_averages)."""
    if P.dim() == 2:
        P = P.unsqueeze(0)
    P = P.to(torch.complex128).contiguous()
    inc = _incidences(khat, e0)
    n = len(inc)
    out = np.zeros((n, 3), dtype=np.float64)
    o = opts.c()
    _check(_lib.dda_scattering_averages(target.ctx, target.handle, ctypes.byref(o), n, inc, P.data_ptr(),
                                        int(n_theta), int(n_phi), out.ctypes.data), "dda_scattering_averages")
    return [dict(qsca=float(r[0]), g=float(r[1]), cos2=float(r[2])) for r in out]


def nearfield_volume(target: "Target", ext) -> tuple[np.ndarray, np.ndarray]:
    """(origin, dims) of the near-field volume: the target's bounding box
    grown by round(r_i n_a) points per side, ext = (r1..r6) for -x, +x, -y,
    +y, -z, +z (dda_nearfield_volume)."""
    r = np.ascontiguousarray(np.asarray(ext, dtype=np.float64).reshape(6))
    org = np.zeros(3, dtype=np.int32)
    dims = np.zeros(3, dtype=np.int32)
    _check(_lib.dda_nearfield_volume(target.handle, r.ctypes.data, org.ctypes.data, dims.ctypes.data),
           "dda_nearfield_volume")
    return org, dims


def nearfield(target: "Target", opts: Options, ext, khat, e0, P: torch.Tensor, incident: bool = True):
    """E_inc and E_sca [n_rhs, dims z, dims y, dims x, 3] (device, complex128)
    on the near-field volume for the solution P [n_rhs, n_sites, 3]; returns
    (origin, dims, E_inc or None, E_sca) (dda_nearfield)."""
    if P.dim() == 2:
        P = P.unsqueeze(0)
    P = P.to(torch.complex128).contiguous()
    inc = _incidences(khat, e0)
    n = len(inc)
    _dev_c128(P, (n, target.n_sites, 3), "P")
    org, dims = nearfield_volume(target, ext)
    shape = (n, int(dims[2]), int(dims[1]), int(dims[0]), 3)
    esca = torch.empty(shape, dtype=torch.complex128, device=P.device)
    einc = torch.empty(shape, dtype=torch.complex128, device=P.device) if incident else None
    r = np.ascontiguousarray(np.asarray(ext, dtype=np.float64).reshape(6))
    o = opts.c()
    _check(_lib.dda_nearfield(target.ctx, target.handle, ctypes.byref(o), r.ctypes.data, n, inc, P.data_ptr(),
                              einc.data_ptr() if einc is not None else None, esca.data_ptr()), "dda_nearfield")
    return org, dims, einc, esca


def field_line(E: torch.Tensor, origin, a, b, n_points: int, device: int | None = None) -> torch.Tensor:
    """Trilinear values [n_rhs, n_points, 3] of the lattice field E [n_rhs,
    dims z, dims y, dims x, 3] (first point at ``origin``) at n_points equally
    spaced points from a to b (lattice coordinates; dda_field_line)."""
    if E.dim() == 4:
        E = E.unsqueeze(0)
    n, nz, ny, nx, _ = E.shape
    E = _dev_c128(E, (n, nz, ny, nx, 3), "E")
    org = np.ascontiguousarray(np.asarray(origin, dtype=np.int32).reshape(3))
    dims = np.array([nx, ny, nz], dtype=np.int32)
    pa = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(3))
    pb = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(3))
    out = torch.empty((n, int(n_points), 3), dtype=torch.complex128, device=E.device)
    _check(_lib.dda_field_line(context(E.device.index if device is None else device), n, org.ctypes.data,
                               dims.ctypes.data, E.data_ptr(), pa.ctypes.data, pb.ctypes.data, int(n_points),
                               out.data_ptr()), "dda_field_line")
    return out


def mueller(f1, f2, e01, e02, phi_deg) -> np.ndarray:
    """Mueller matrices [n_dir, 4, 4] in the Lab Frame from the amplitudes
    f1, f2 [n_dir, 2] of the incident polarizations e01, e02 (dda_mueller)."""
    f1 = np.ascontiguousarray(np.asarray(f1, dtype=np.complex128).reshape(-1, 2))
    f2 = np.ascontiguousarray(np.asarray(f2, dtype=np.complex128).reshape(-1, 2))
    e1 = np.ascontiguousarray(np.asarray(e01, dtype=np.complex128).reshape(3))
    e2 = np.ascontiguousarray(np.asarray(e02, dtype=np.complex128).reshape(3))
    ph = np.ascontiguousarray(np.asarray(phi_deg, dtype=np.float64).reshape(-1))
    n_dir = f1.shape[0]
    if f2.shape[0] != n_dir or ph.shape[0] != n_dir:
        raise ValueError("f1, f2 and phi_deg must have the same number of directions")
    S = np.zeros((n_dir, 16), dtype=np.float64)
    _check(_lib.dda_mueller(n_dir, f1.ctypes.data, f2.ctypes.data, e1.ctypes.data, e2.ctypes.data, ph.ctypes.data,
                            S.ctypes.data), "dda_mueller")
    return S.reshape(n_dir, 4, 4)


def tuned_variants(target: "Target", n_rhs: int, precision: str = "fp64") -> tuple:
    """(y forward, z with tensor, y inverse) strided-pass variants the
    autotuner chose for this target, right-hand-side count and precision, or
    (-1, -1, -1) before any such solve."""
    out = (ctypes.c_int32 * 3)()
    _check(_lib.dda_ctx_tuned_variants(target.ctx, target._h, int(n_rhs), _PREC[precision], out),
           "dda_ctx_tuned_variants")
    return tuple(int(v) for v in out)


def get_timing(device: int | None = None) -> dict:
    """{category: (total ms of the timed launches, timed launches, all
    launches)} accumulated since set_timing."""
    t = _abi.Timing()
    _check(_lib.dda_ctx_get_timing(context(device), ctypes.byref(t)), "dda_ctx_get_timing")
    return {name: (t.ms[i], int(t.launches[i]), int(t.all_launches[i])) for i, name in enumerate(_abi.TIMING_NAMES)}


def set_timing_sample(every: int, device: int | None = None) -> None:
    """Time every ``every``-th launch of each recorded category only."""
    _check(_lib.dda_ctx_set_timing_sample(context(device), int(every)), "dda_ctx_set_timing_sample")
