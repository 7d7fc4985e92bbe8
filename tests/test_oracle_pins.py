"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test names what fixes the expected value: the guide's printed worked
example, textbook limits, brute-force quadrature, finite differences, or
exact algebraic identities of the physics (energy conservation).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as w
from oracle import adjoint, dense, farfield, fftsolve, mie, nearfield

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- worked example

def _worked():
    with open(os.path.join(GOLDEN, "worked_example_au_brick.json")) as f:
        return json.load(f)


def test_worked_example_lattice_constants():
    """d/a_eff and kd printed in the .avg header of the guide's sample run."""
    g = _worked()
    ijk = w.brick(*g["shape"])
    assert len(ijk) == g["n_sites"]
    # one unit in the last printed place (the sample run is a single-precision build)
    assert abs(1.0 / dense.aeff_over_d(len(ijk)) - g["d_over_aeff"]) < 1e-8
    assert abs(dense.kd_from_size_parameter(g["x"], len(ijk)) - g["kd"]) < 5e-6


def test_worked_example_efficiencies_gkdldr():
    """The whole pipeline (interaction tensor, FFT embedding, GKDLDR
    polarizability, E_inc, Q_ext/Q_abs/Q_pha) reproduces the printed
    efficiencies of the 16x32x32 gold brick to the printed digits (1e-4
    relative: the guide solved with PBCGS2 to TOL 1e-5)."""
    g = _worked()
    d = w.workload("au_brick")
    m = np.full(len(d["ijk"]), complex(*g["m"]))
    r = fftsolve.solve_case(d["ijk"], m, g["x"], d["khat"][0], d["e0"][0], tol=1e-7, scheme=dense.GKDLDR)
    for key in ("qext", "qabs", "qsca", "qpha"):
        assert abs(r[key] - g[key]) <= 1e-4 * abs(g[key]) + 5e-6, (key, r[key], g[key])


def test_worked_example_discriminates_lattdr():
    """The printed Q_ext is not reproduced by the LATTDR prescription (it
    differs by ~0.26%), so the example pins the GKDLDR reading."""
    g = _worked()
    d = w.workload("au_brick")
    m = np.full(len(d["ijk"]), complex(*g["m"]))
    r = fftsolve.solve_case(d["ijk"], m, g["x"], d["khat"][0], d["e0"][0], tol=1e-6, scheme=dense.LATTDR)
    assert abs(r["qext"] - g["qext"]) > 1e-3 * g["qext"]


# ---------------------------------------------------------------- interaction tensor

def _psi(r, k):
    rr = np.linalg.norm(r)
    return np.exp(1j * k * rr) / rr


@pytest.mark.parametrize("k", [0.0, 0.3, 1.1])
@pytest.mark.parametrize("R", [(1, 0, 0), (1, 2, -1), (-3, 1, 2), (0, -2, 5)])
def test_interaction_tensor_is_dipole_field(k, R):
    """-A_jl P is the field of an oscillating point dipole P at r_l:
    E = k^2 psi P + grad(P . grad psi), psi = exp(ikr)/r.  The Hessian of psi
    is taken by central finite differences, independently of the closed form
    (k = 0 is the static dipole field)."""
    R = np.array(R, dtype=np.float64)
    h = 2e-4
    H = np.zeros((3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for a in range(3):
        for b in range(3):
            H[a, b] = (_psi(R + h * eye[a] + h * eye[b], k) - _psi(R + h * eye[a] - h * eye[b], k)
                       - _psi(R - h * eye[a] + h * eye[b], k) + _psi(R - h * eye[a] - h * eye[b], k)) / (4 * h * h)
    field = k * k * _psi(R, k) * eye + H
    A = dense.interaction_block(R, k)
    assert np.allclose(A, -field, rtol=0, atol=2e-6 * np.abs(field).max())


def test_matrix_complex_symmetric_not_hermitian():
    """A = A^T exactly (reciprocity); A != A^H for an absorbing target."""
    ijk = w.sphere_integer(2.2)
    k = 0.4
    ainv = dense.site_alpha_inverse(np.full(len(ijk), 1.5 + 0.1j), k, [1, 0, 0], [0, 1, 0])
    A = dense.assemble(ijk, ainv, k)
    assert np.array_equal(A, A.T)
    assert np.abs(A - A.conj().T).max() > 1e-3


def test_assembly_blocks_match_pairwise_formula():
    """Vectorised assembly agrees with the per-pair block and the 1/alpha diagonal."""
    rng = np.random.default_rng(3)
    ijk = rng.integers(-3, 4, size=(40, 3))
    ijk = np.unique(ijk, axis=0)
    k = 0.7
    ainv = dense.site_alpha_inverse(np.full(len(ijk), 1.7 + 0.2j), k, [0, 0, 1], [1, 0, 0])
    A = dense.assemble(ijk, ainv, k)
    for j, l in [(0, 1), (5, 17), (len(ijk) - 1, 2)]:
        assert np.allclose(A[3 * j:3 * j + 3, 3 * l:3 * l + 3], dense.interaction_block(ijk[j] - ijk[l], k), atol=1e-14)
    assert np.allclose(np.diag(A)[:3], ainv[0])


# ---------------------------------------------------------------- FFT embedding

@pytest.mark.parametrize("shape", ["sphere", "ragged", "odd_pad", "line"])
def test_fft_embedding_equals_dense(shape):
    """The circulant embedding reproduces the dense product (any padded extent
    >= 2n-1 is exact), including odd and 5-smooth extents (n=13 -> 25)."""
    rng = np.random.default_rng(11)
    if shape == "sphere":
        ijk = w.sphere_integer(3.3)
    elif shape == "ragged":
        ijk = np.unique(rng.integers(0, 7, size=(150, 3)) * np.array([1, 1, 2]), axis=0)
    elif shape == "odd_pad":
        ijk = np.array([[i, j, 0] for i in range(13) for j in range(2)])
    else:
        ijk = np.array([[0, 0, i] for i in range(9)])
    k = 0.55
    ainv = dense.site_alpha_inverse(np.full(len(ijk), 1.4 + 0.05j), k, [0.6, 0.8, 0], [0, 0, 1])
    A = dense.assemble(ijk, ainv, k)
    op = fftsolve.FFTOperator(ijk, ainv, k)
    x = w.random_vectors(5, (len(ijk), 3))
    y = op.apply(x).reshape(-1)
    assert np.abs(y - A @ x.reshape(-1)).max() <= 1e-12 * np.abs(y).max()


def test_padded_extents():
    """2n when 2,3,5-smooth, else the smallest smooth extent >= 2n-1."""
    assert [fftsolve.padded_extent(n) for n in (1, 9, 13, 17, 41, 64, 48, 32, 40, 128)] == \
        [2, 18, 25, 36, 81, 128, 96, 64, 80, 256]


# ---------------------------------------------------------------- polarizability

def test_polarizability_reduces_to_clausius_mossotti():
    """kd -> 0: both LDR prescriptions tend to the Clausius-Mossotti value
    alpha = (3/4pi)(eps-1)/(eps+2) d^3."""
    for m in (1.33 + 0.01j, 2 + 1j):
        eps = m * m
        a_cm = 3.0 / (4 * math.pi) * (eps - 1) / (eps + 2)
        for scheme in (dense.LATTDR, dense.GKDLDR):
            ainv = dense.alpha_inverse(m, 1e-6, [1, 0, 0], [0, 1, 0], scheme)
            assert np.allclose(1.0 / ainv, a_cm, rtol=1e-10)


def test_radiative_reaction_makes_real_m_lossless():
    """For real m the only imaginary part of 1/alpha is radiative reaction,
    so Q_abs = 0 and Q_ext = Q_sca (energy conservation, Draine 1988)."""
    ijk = w.sphere_integer(2.5)
    s = dense.solve_case(ijk, np.full(len(ijk), 1.5 + 0j), 1.2, [1, 0, 0], [0, 1, 0])
    assert abs(s["qabs"]) < 1e-13
    assert abs(s["qext"] - s["qsca"]) < 1e-12 * s["qext"]


# ---------------------------------------------------------------- efficiencies

@pytest.mark.parametrize("scheme", [dense.LATTDR, dense.GKDLDR])
def test_optical_theorem_at_lu_solution(scheme):
    """Q_ext = Q_abs + Q_sca with Q_sca from the independent far-field
    integral, at the exact (LU) solution, on the N=389 pseudosphere and on an
    elliptically polarised oblique wave."""
    d = w.workload("sphere389")
    s = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0], scheme)
    assert abs(s["qext"] - s["qabs"] - s["qsca"]) < 1e-12 * s["qext"]
    kh = np.array([0.36, 0.48, 0.8])
    e0 = np.array([0.8, -0.6, 0]) + 1j * np.cross(kh, [0.8, -0.6, 0])
    s = dense.solve_case(d["ijk"], np.full(389, 2.0 + 0.5j), 2.0, kh, e0, scheme)
    assert abs(s["qext"] - s["qabs"] - s["qsca"]) < 1e-11 * s["qext"]


def test_qsca_closed_form_matches_angular_quadrature():
    """The analytic angular integral equals brute-force quadrature of
    k^4 |sum_j (P_j - n (n.P_j)) exp(-i k n.r_j)|^2 over the sphere."""
    rng = np.random.default_rng(2)
    ijk = np.unique(rng.integers(-3, 4, size=(25, 3)), axis=0)
    P = w.random_vectors(9, (len(ijk), 3))
    k = 0.9
    mu, wt = np.polynomial.legendre.leggauss(96)
    phi = np.linspace(0, 2 * math.pi, 192, endpoint=False)
    st = np.sqrt(1 - mu ** 2)
    n = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)), np.outer(mu, np.ones_like(phi))], -1)
    ph = np.exp(-1j * k * np.einsum("tpa,ja->tpj", n, ijk))
    F = np.einsum("tpj,ja->tpa", ph, P)
    Fperp = F - n * np.einsum("tpa,tpa->tp", n, F)[..., None]
    integrand = k ** 4 * np.sum(np.abs(Fperp) ** 2, axis=-1)
    csca = float(np.sum(wt[:, None] * integrand) * (2 * math.pi / len(phi)))
    a = dense.aeff_over_d(len(ijk))
    q_quad = csca / (math.pi * a * a)
    assert abs(dense.q_sca_closed_form(ijk, P, k) - q_quad) < 1e-10 * q_quad


def test_sphere_polarizations_equal():
    """The pseudosphere is symmetric under y <-> z, so both polarizations
    give the same efficiencies."""
    d = w.workload("sphere389")
    q = [dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][i], d["e0"][i], with_qsca=False) for i in range(2)]
    assert abs(q[0]["qext"] - q[1]["qext"]) < 1e-13
    assert abs(q[0]["qabs"] - q[1]["qabs"]) < 1e-13


def test_single_dipole():
    """One dipole: P = alpha E and energy balance Q_ext = Q_abs + Q_sca."""
    ijk = np.zeros((1, 3), dtype=np.int32)
    s = dense.solve_case(ijk, [1.7 + 0.3j], 0.3, [0, 0, 1], [1, 0, 0])
    assert np.allclose(s["P"][0], s["E"][0] / s["alpha_inv"][0])
    assert abs(s["qext"] - s["qabs"] - s["qsca"]) < 1e-14 * s["qext"]


def test_rayleigh_limit():
    """Small x at fixed N: the DDA sphere tends to the Rayleigh absorption
    and scattering efficiencies of a small sphere (textbook) to within the
    discretisation error of a 389-site pseudosphere (~1%)."""
    d = w.workload("sphere389")
    m = 1.33 + 0.01j
    F = (m * m - 1) / (m * m + 2)
    x = 0.01
    s = dense.solve_case(d["ijk"], d["m"], x, d["khat"][0], d["e0"][0])
    assert abs(s["qabs"] / (4 * x * F.imag) - 1) < 0.02
    assert abs(s["qsca"] / (8 / 3 * x ** 4 * abs(F) ** 2) - 1) < 0.02


# ---------------------------------------------------------------- Mie

def test_mie_rayleigh_limit():
    m = 1.5 + 0.1j
    F = (m * m - 1) / (m * m + 2)
    x = 1e-3
    q = mie.efficiencies(m, x)
    assert abs(q["qabs"] / (4 * x * F.imag) - 1) < 1e-5
    assert abs(q["qsca"] / (8 / 3 * x ** 4 * abs(F) ** 2) - 1) < 1e-5


def test_mie_lossless_and_extinction_paradox():
    assert abs(mie.efficiencies(1.5, 3.0)["qabs"]) < 1e-13
    assert abs(mie.efficiencies(1.5 + 0.5j, 300.0)["qext"] - 2.0) < 0.06


def test_dda_vs_mie_sphere389():
    """'Accurate to a few percent' ("Applicability of the DDA"): the N=389
    pseudosphere at x=1, m=1.33+0.01i is within 3% of Mie in all three Q."""
    d = w.workload("sphere389")
    s = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0])
    q = mie.efficiencies(1.33 + 0.01j, 1.0)
    for key in ("qext", "qabs", "qsca"):
        assert abs(s[key] / q[key] - 1) < 0.03, key


# ---------------------------------------------------------------- solver

def test_bicgstab_matches_lu():
    d = w.workload("sphere389")
    lu = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], with_qsca=False)
    it = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], tol=1e-10)
    assert it["converged"] and it["true_residual"] < 1e-9
    assert np.abs(it["P"] - lu["P"]).max() < 1e-8 * np.abs(lu["P"]).max()
    assert abs(it["qext"] - lu["qext"]) < 1e-9


def test_qmr_matches_lu():
    """QMR (COCG with quasi-minimal-residual smoothing) reaches the LU
    solution of the same system."""
    d = w.workload("sphere389")
    lu = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], with_qsca=False)
    it = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], tol=1e-10, solver="qmr")
    assert it["converged"] and it["true_residual"] < 1e-9
    assert np.abs(it["P"] - lu["P"]).max() < 1e-8 * np.abs(lu["P"]).max()
    assert abs(it["qext"] - lu["qext"]) < 1e-9


def _qmr_trace(name="sphere389", pol=0, steps=12):
    d = w.workload(name)
    k = dense.kd_from_size_parameter(d["x"], len(d["ijk"]))
    ainv = dense.site_alpha_inverse(d["m"], k, d["khat"][pol], d["e0"][pol], dense.LATTDR)
    A = dense.assemble(d["ijk"], ainv, k)
    E = dense.incident_field(d["ijk"], k, d["khat"][pol], d["e0"][pol])
    trace = []
    fftsolve.qmr_sym(lambda v: (A @ v.reshape(-1)).reshape(v.shape), E, 1e-14, steps, trace=trace)
    return A, E, trace


def test_qmr_smoothed_residual_is_residual_of_smoothed_iterate():
    """The smoothing must carry (y, s) together: s_k = E - A y_k at every
    step, and tau_k decreases with |s_k| <= sqrt(k+1) tau_k (the
    quasi-minimal residual bound)."""
    A, E, trace = _qmr_trace()
    en = np.linalg.norm(E)
    for k, t in enumerate(trace):
        res = E.reshape(-1) - A @ t["y"].reshape(-1)
        assert np.linalg.norm(res - t["s"].reshape(-1)) < 1e-11 * en, k
        assert np.linalg.norm(t["s"]) <= math.sqrt(k + 1) * math.sqrt(t["tau2"]) * (1 + 1e-12), k
        if k:
            assert t["tau2"] < trace[k - 1]["tau2"]


def test_cocg_residuals_are_bilinearly_orthogonal():
    """COCG's residuals are orthogonal in the unconjugated form u^T v (the
    Galerkin condition that A = A^T permits), not in the Hermitian one."""
    A, E, trace = _qmr_trace(steps=8)
    rs = [t["r"].reshape(-1) for t in trace]
    herm = 0.0
    for j in range(len(rs)):
        for k in range(j + 1, len(rs)):
            scale = np.linalg.norm(rs[j]) * np.linalg.norm(rs[k])
            assert abs(np.sum(rs[j] * rs[k])) < 1e-9 * scale, (j, k)
            herm = max(herm, abs(np.vdot(rs[j], rs[k])) / scale)
    assert herm > 1e-3


def test_bicgstab2_matches_lu():
    d = w.workload("sphere389")
    lu = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], with_qsca=False)
    it = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][1], d["e0"][1], tol=1e-10, solver="bicgstab2")
    assert it["converged"] and it["true_residual"] < 1e-9
    assert np.abs(it["P"] - lu["P"]).max() < 1e-8 * np.abs(lu["P"]).max()


def test_bicgstab_l_with_l1_is_bicgstab():
    """BiCGstab(1) is BiCGSTAB (van der Vorst 1992): the same iterates, step
    by step, from an independent formulation of the recurrences."""
    A, E, _ = _qmr_trace(steps=1)
    op = lambda v: (A @ v.reshape(-1)).reshape(v.shape)
    tr = []
    fftsolve.bicgstab_l(op, E, 1e-14, 6, ell=1, trace=tr)
    for k in range(1, 7):
        xk, _ = fftsolve.bicgstab(op, E, 1e-30, k)
        assert np.linalg.norm(tr[k - 1]["x"] - xk) <= 1e-9 * np.linalg.norm(xk), k


def test_bicgstab2_residual_consistent_and_minimal():
    """After every outer iteration of BiCGstab(2) the recursive residual is
    E - A x, and it is no larger than the BiCG residual the minimal-residual
    step started from."""
    A, E, _ = _qmr_trace(steps=1)
    op = lambda v: (A @ v.reshape(-1)).reshape(v.shape)
    tr = []
    fftsolve.bicgstab_l(op, E, 1e-14, 5, ell=2, trace=tr)
    en = np.linalg.norm(E)
    for t in tr:
        res = E.reshape(-1) - A @ t["x"].reshape(-1)
        assert np.linalg.norm(res - t["r"].reshape(-1)) < 1e-10 * en
        assert np.linalg.norm(t["r"]) <= np.linalg.norm(t["r_bicg"]) * (1 + 1e-12)


def _err_tol_by_differences(A, P, E):
    """eq. err_tol without forming A^H: phi(P) = |A P - E|^2 / 2 has the
    gradient dphi/dRe P + i dphi/dIm P = A^H (A P - E), and at P = 0 that is
    -A^H E.  Central differences of the quadratic phi are exact up to rounding."""
    p0 = np.asarray(P, dtype=np.complex128).reshape(-1)
    e = np.asarray(E, dtype=np.complex128).reshape(-1)

    def grad(p):
        phi = lambda v: 0.5 * float(np.sum(np.abs(A @ v - e) ** 2))
        h = 1e-4 * max(np.abs(p).max(), 1.0)
        g = np.zeros(len(p), dtype=np.complex128)
        for i in range(len(p)):
            for unit in (1.0, 1j):
                d = np.zeros(len(p), dtype=np.complex128)
                d[i] = unit * h
                g[i] += unit * (phi(p + d) - phi(p - d)) / (2 * h)
        return g

    return float(np.linalg.norm(grad(p0)) / np.linalg.norm(grad(np.zeros_like(p0))))


def _err_tol_case():
    """A 20-site ragged target of a lossy material at oblique elliptical
    incidence (A far from Hermitian), and a P away from the solution."""
    rng = np.random.default_rng(41)
    ijk = np.unique(rng.integers(0, 4, size=(26, 3)), axis=0)[:20].astype(np.int32)
    kh = np.array([0.36, 0.48, 0.8])
    e0 = np.array([0.8, -0.6, 0.0]) + 0.4j * np.cross(kh, [0.8, -0.6, 0.0])
    s = dense.solve_case(ijk, np.full(len(ijk), 2.0 + 0.7j), 1.2, kh, e0, with_qsca=False)
    P = s["P"] + 0.05 * np.abs(s["P"]).max() * w.random_vectors(12, s["P"].shape)
    return s, P


def test_normal_equation_residual_definition():
    """eq. err_tol |A^H A P - A^H E| / |A^H E|: zero at the LU solution, and
    at a P away from it equal to the value found from finite differences of
    |A P - E|^2 (which never forms A^H)."""
    d = w.workload("sphere389")
    s = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0], with_qsca=False)
    true_r, ne_r = dense.residuals(s["A"], s["P"], s["E"])
    assert true_r < 1e-13 and ne_r < 1e-12
    s, P = _err_tol_case()
    fd = _err_tol_by_differences(s["A"], P, s["E"])
    true_r, ne_r = dense.residuals(s["A"], P, s["E"])
    assert abs(ne_r - fd) <= 1e-7 * fd and true_r > 1e-3


def test_err_tol_pin_rejects_transpose_for_adjoint(monkeypatch):
    """Planted in the oracle: A^T in place of A^H (for the complex-symmetric A
    that is A itself) changes the value beyond the pin's tolerance."""
    def residuals_t(A, P, E):
        p = np.asarray(P).reshape(-1)
        e = np.asarray(E).reshape(-1)
        r = A @ p - e
        return (float(np.linalg.norm(r) / np.linalg.norm(e)),
                float(np.linalg.norm(A.T @ r) / np.linalg.norm(A.T @ e)))
    monkeypatch.setattr(dense, "residuals", residuals_t)
    s, P = _err_tol_case()
    fd = _err_tol_by_differences(s["A"], P, s["E"])
    assert abs(dense.residuals(s["A"], P, s["E"])[1] - fd) > 1e-3 * fd


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("weights", [(1.0, 0.0), (0.0, 1.0)])
def test_adjoint_gradient_matches_finite_differences(weights):
    """Central differences of Q_abs (and of Q_ext) with respect to Re and Im
    of eps_j on the 6^3 two-material target (dense solves)."""
    d = w.workload("twomat6")
    kh, e0 = d["khat"][0], d["e0"][0]
    grad, sol = adjoint.gradient_dense(d["ijk"], d["m"], d["x"], kh, e0, *weights)
    eps = np.asarray(d["m"]) ** 2
    for j in (0, 37, 101, 215):
        h = 1e-4 * abs(eps[j])
        fd = []
        for step in (h, 1j * h):
            ep, em = eps.copy(), eps.copy()
            ep[j] += step
            em[j] -= step
            fd.append((adjoint.objective_dense(d["ijk"], ep, d["x"], kh, e0, *weights)
                       - adjoint.objective_dense(d["ijk"], em, d["x"], kh, e0, *weights)) / (2 * h))
        fdc = fd[0] + 1j * fd[1]
        assert abs(grad[j] - fdc) < 1e-6 * abs(grad).max(), (j, grad[j], fdc)


# ---------------------------------------------------------------- inputs

def test_orientation_frames():
    """Lab axes in the target frame are orthonormal, right-handed, and hit
    the guide's printed special cases: Theta=90, Phi=0, beta=0 puts a1 along
    y_LF and a2 along -x_LF; beta=90 puts a2 along z_LF."""
    for b, t, p in zip(*w.orientation_angles(0, 16)):
        ax = w.lab_axes_in_target_frame(b, t, p)
        assert np.allclose(ax @ ax.T, np.eye(3), atol=1e-14)
        assert np.allclose(np.cross(ax[0], ax[1]), ax[2], atol=1e-14)
    ax = w.lab_axes_in_target_frame(0.0, math.pi / 2, 0.0)
    # a1 (TF x) along y_LF: y_LF = +x_TF;  a2 (TF y) along -x_LF: x_LF = -y_TF
    assert np.allclose(ax[1], [1, 0, 0], atol=1e-15) and np.allclose(ax[0], [0, -1, 0], atol=1e-15)
    ax = w.lab_axes_in_target_frame(math.pi / 2, math.pi / 2, 0.0)
    assert np.allclose(ax[2], [0, 1, 0], atol=1e-15)
    kh, e0 = w.incidences_for_orientations(0, 4)
    assert np.allclose(np.cross(kh[0], np.conj(e0[0])), e0[1])


def test_workload_sizes():
    assert len(w.workload("sphere389")["ijk"]) == 389
    assert len(w.workload("ellipsoid51k")["ijk"]) == 51488
    assert len(w.box_sphere(128, 64.0)) == 1099136


def test_apply_rows_matches_dense():
    """The O(N)-per-row product equals rows of the dense product."""
    ijk = np.unique(np.random.default_rng(4).integers(-4, 5, size=(120, 3)), axis=0)
    k = 0.45
    ainv = dense.site_alpha_inverse(np.full(len(ijk), 1.5 + 0.2j), k, [0, 1, 0], [1, 0, 0])
    A = dense.assemble(ijk, ainv, k)
    x = w.random_vectors(2, (len(ijk), 3))
    rows = [0, 7, len(ijk) - 1]
    ref = (A @ x.reshape(-1)).reshape(-1, 3)[rows]
    assert np.abs(dense.apply_rows(ijk, ainv, k, x, rows) - ref).max() < 1e-12 * np.abs(ref).max()


def test_bicgstab2_iterations_near_the_printed_worked_example():
    """The guide prints 18 PBCGS2 iterations per polarization for its gold
    brick at TOL 1e-5; plain BiCGstab(2) lands within a few of that (plain
    BiCGSTAB needs about twice as many)."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example_au_brick.json")))
    d = w.workload("au_brick")
    r = fftsolve.solve_case(d["ijk"], d["m"], g["x"], d["khat"][0], d["e0"][0], tol=1e-5,
                            scheme=dense.GKDLDR, solver="bicgstab2")
    assert r["converged"] and abs(r["iters"] - g["pbcgs2_iterations"][0]) <= 3
    for key in ("qext", "qabs"):
        assert abs(r[key] - g[key]) <= 1e-4 * abs(g[key]) + 5e-6


# ---------------------------------------------------------------- far field


def _au_brick_P(tol=1e-9):
    d = w.workload("au_brick")
    Ps, k = [], None
    for q in range(2):
        r = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][q], d["e0"][q], tol=tol, scheme=dense.GKDLDR)
        Ps.append(r["P"])
        k = r["k"]
    return d, Ps, k


def test_worked_example_mueller_matrix_matches_printed():
    """The guide's printed Mueller elements of the gold brick at 74
    directions (phi = 0 and 90 deg), its polarization column and Q_bk."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example_au_brick_mueller.json")))
    rows = np.array(g["rows"])
    d, Ps, k = _au_brick_P()
    n, th, ph = farfield.lab_directions(rows[:, 0], rows[:, 1])
    A1 = farfield.amplitude_vectors(d["ijk"], Ps[0], k, n)
    A2 = farfield.amplitude_vectors(d["ijk"], Ps[1], k, n)
    M = farfield.mueller(farfield.amplitude_matrix(farfield.f_matrix(A1, A2, th, ph), d["e0"][0], d["e0"][1],
                                                   rows[:, 1]))
    s11 = rows[:, 3]
    assert np.all(np.abs(M["S11"] - s11) <= 2e-4 * s11)
    assert np.all(np.abs(M["S12"] - rows[:, 4]) <= 2e-4 * s11)
    assert np.all(np.abs(M["S21"] - rows[:, 5]) <= 1e-3 * s11)
    assert np.all(np.abs(M["S22"] - rows[:, 6]) <= 1e-3 * s11)
    assert np.all(np.abs(-M["S12"] / M["S11"] - rows[:, 2]) <= 1e-4)
    assert np.all(np.abs(M["S31"]) <= 1e-4) and np.all(np.abs(M["S41"]) <= 1e-4)
    a = dense.aeff_over_d(len(d["ijk"]))
    nb, thb, phb = farfield.lab_directions([180.0], [0.0])
    for P in Ps:
        qbk = farfield.q_bk(farfield.amplitude_vectors(d["ijk"], P, k, nb)[0], thb[0], phb[0], k, a)
        assert abs(qbk - g["qbk"]) <= 2e-4 * g["qbk"]


def test_forward_amplitude_gives_q_ext():
    """Optical theorem: Q_ext = 4 Im(e0* . A(k)) / (k^2 a^2) from the forward
    amplitude equals the extinction sum over dipoles (oblique, elliptical)."""
    d = w.workload("sphere389")
    kh = np.array([0.36, 0.48, 0.8])
    e0 = np.array([0.8, -0.6, 0]) + 1j * np.cross(kh, [0.8, -0.6, 0])
    e0 = e0 / np.linalg.norm(e0)
    s = dense.solve_case(d["ijk"], d["m"], d["x"], kh, e0, with_qsca=False)
    A = farfield.amplitude_vectors(d["ijk"], s["P"], s["k"], kh[None, :])[0]
    a = dense.aeff_over_d(len(d["ijk"]))
    qe = 4 * np.imag(np.vdot(e0, A)) / (s["k"] ** 2 * a ** 2)
    assert abs(qe - s["qext"]) < 1e-12 * abs(s["qext"])


def test_angular_integral_of_far_field_is_q_sca():
    """The differential cross section (|f_1|^2 + |f_2|^2)/k^2 integrated
    over all directions (Gauss-Legendre in cos theta, uniform in phi) equals
    the closed-form Q_sca."""
    d = w.workload("sphere389")
    s = dense.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0])
    mu, wmu = np.polynomial.legendre.leggauss(48)
    phis = np.arange(64) * 2 * np.pi / 64
    T, Pp = np.meshgrid(np.degrees(np.arccos(mu)), np.degrees(phis), indexing="ij")
    n, th, ph = farfield.lab_directions(T.ravel(), Pp.ravel())
    A = farfield.amplitude_vectors(d["ijk"], s["P"], s["k"], n)
    dcs = (np.abs(np.sum(th * A, axis=1)) ** 2 + np.abs(np.sum(ph * A, axis=1)) ** 2) / s["k"] ** 2
    csca = np.sum(dcs.reshape(T.shape) * wmu[:, None]) * (2 * np.pi / 64)
    a = dense.aeff_over_d(len(d["ijk"]))
    assert abs(csca / (np.pi * a ** 2) - s["qsca"]) < 1e-8 * s["qsca"]


def test_mueller_elements_match_the_stokes_construction():
    """Each of the 16 element formulas against the matrix construction
    M = T (J kron J*) T^-1, with J = (S2 S3; S4 S1) acting on (E_par, E_perp)
    and T the map from E (x) E* to the Stokes vector (I, Q, U, V); a Mueller
    matrix of one amplitude matrix is non-depolarizing, sum S_ij^2 = 4 S11^2."""
    rng = np.random.default_rng(3)
    S = rng.normal(size=(20, 2, 2)) + 1j * rng.normal(size=(20, 2, 2))
    M = farfield.mueller(S)
    T = np.array([[1, 0, 0, 1], [1, 0, 0, -1], [0, 1, 1, 0], [0, 1j, -1j, 0]])
    Ti = np.linalg.inv(T)
    for n in range(len(S)):
        Mk = T @ np.kron(S[n], np.conj(S[n])) @ Ti
        assert np.abs(Mk.imag).max() < 1e-12
        for i in range(4):
            for j in range(4):
                assert abs(M[f"S{i + 1}{j + 1}"][n] - Mk[i, j].real) < 1e-12 * max(1.0, abs(Mk[0, 0])), (i, j)
        frob = sum(M[f"S{i + 1}{j + 1}"][n] ** 2 for i in range(4) for j in range(4))
        assert abs(frob - 4 * M["S11"][n] ** 2) < 1e-10 * M["S11"][n] ** 2


def test_worked_example_angular_averages_near_printed():
    """<cos theta> and <cos^2 theta> of the gold brick by converged
    quadrature against the guide's printed g(1) = 0.41463 and <cos^2> =
    0.75169, which the guide evaluates on its own 962-direction set
    (ETASCA = 0.5): agreement within that rule's 0.3%; Q_sca from the same
    quadrature equals Q_ext - Q_abs."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example_au_brick.json")))
    d, Ps, k = _au_brick_P()
    a = dense.aeff_over_d(len(d["ijk"]))
    for q in range(2):
        qs, gg, c2 = farfield.angular_averages(d["ijk"], Ps[q], k, d["khat"][q], a, 32, 48)
        assert abs(gg - g["g1"]) <= 3e-3 * g["g1"]
        assert abs(c2 - g["cos2"]) <= 3e-3 * g["cos2"]
        assert abs(qs - g["qsca"]) <= 2e-4 * g["qsca"]


# ---------------------------------------------------------------- near field

def _nf_track():
    with open(os.path.join(GOLDEN, "nearfield_au_sphere_track.json")) as f:
        return json.load(f)


def test_nearfield_example_lattice_and_extended_volume():
    """The near-field example's header: N = 59728 sites in the 48^3 box, the
    printed kd = 0.20619 and d = 1.6408e-2 um at a_eff = 0.39789 um, and the
    extended volume of 96^3 points for r = 0.5 on every side."""
    g = _nf_track()
    d = w.workload("au_sphere_nf")
    assert len(d["ijk"]) == g["header"]["n_sites"]
    assert abs(dense.kd_from_size_parameter(d["x"], len(d["ijk"])) - g["header"]["kd"][0]) < 5e-6
    # half a unit in the last printed place (1.6408E-02)
    assert abs(g["header"]["aeff_um"] / dense.aeff_over_d(len(d["ijk"])) - g["header"]["d_um"]) < 5e-7
    origin, dims = nearfield.extended_box(d["ijk"], d["nf_ext"])
    assert list(dims) == g["header"]["dims"] and list(origin) == [-24, -24, -24]


def _au_sphere_solution():
    d = w.workload("au_sphere_nf")
    res = fftsolve.solve_case(d["ijk"], d["m"], d["x"], d["khat"][0], d["e0"][0], 1e-5,
                              scheme=dense.GKDLDR, solver="bicgstab2")
    return d, res


def test_nearfield_printed_readnf_track():
    """E = E_inc + E_sca along the x_TF axis through the gold sphere (the
    guide's printed readnf output, 52 rows): GKDLDR solve to tol 1e-5, then
    the direct-sum near field, trilinear between lattice points.  Positions:
    lattice = x_TF / d + 23.5 (the box centre), E_inc phase 1 at the centre.
    The nearest-lattice-point reading misses the printed values by 1e-2."""
    g = _nf_track()
    d, res = _au_sphere_solution()
    k = res["k"]
    dl = g["header"]["aeff_um"] / dense.aeff_over_d(len(d["ijk"]))
    c = 23.5
    a = np.array(g["line_um"]["a"]) / dl + c
    b = np.array(g["line_um"]["b"]) / dl + c
    rows = np.array(g["rows"])
    printed = rows[:, 3::2] + 1j * rows[:, 4::2]
    E = nearfield.line_field(d["ijk"], res["P"], k, d["khat"][0], d["e0"][0], a, b, len(rows))
    E *= np.exp(-1j * k * c)           # phase origin at the sphere's centre
    assert np.abs(E - printed).max() < 3e-4
    # positions as printed (4 digits) agree too, within their rounding
    pts = nearfield.line_points(a, b, len(rows))
    assert np.abs(pts[:, 0] - (rows[:, 0] / dl + c)).max() < 0.01
    near = nearfield.incident_field(np.rint(pts), k, d["khat"][0], d["e0"][0]) + \
        nearfield.scattered_field(d["ijk"], res["P"], k, np.rint(pts))
    assert np.abs(near * np.exp(-1j * k * c) - printed).max() > 1e-2


def test_nearfield_satisfies_the_dda_equations_at_the_sites():
    """At every target site the field of the others plus E_inc is the local
    field that polarizes it: P_j = alpha_j (E_inc,j + E_sca,j) for the LU
    solution (the system A P = E, stated point by point), two materials and
    an oblique elliptical incidence."""
    ijk = w.brick(4, 3, 3)
    mask = np.arange(len(ijk)) % 3 == 0
    m = np.where(mask, 1.5 + 0.02j, 2.2 + 0.4j)
    kh = np.array([0.6, 0.0, 0.8])
    e0 = np.array([0.8, 0.3j, -0.6])
    case = dense.solve_case(ijk, m, 1.1, kh, e0, scheme=dense.LATTDR)
    k, P = case["k"], case["P"]
    E = nearfield.incident_field(ijk, k, kh, e0) + nearfield.scattered_field(ijk, P, k, ijk)
    assert np.abs(case["alpha_inv"] * P - E).max() < 1e-11 * np.abs(E).max()
    # on the extended volume the target's own sites carry the same fields
    origin, dims, Ei, Es = nearfield.nearfield(ijk, P, k, kh, e0, (0.5, 0.25, 0.0, 1.0, 0.4, 0.4))
    pts = nearfield.box_points(origin, dims)
    flat = (Ei + Es).reshape(-1, 3)
    idx = [int(np.flatnonzero((pts == s).all(axis=1))[0]) for s in ijk]
    assert np.abs(flat[idx] - E).max() < 1e-12 * np.abs(E).max()
    assert list(dims) == [4 + 2 + 1, 3 + 0 + 3, 3 + 1 + 1]


def test_nearfield_far_zone_is_the_far_field_amplitude():
    """Far away along n the dipole sum becomes (e^{ikR} / kR) (I - n n) A(n)
    / k^2 ... i.e. E_sca R e^{-ikR} -> (I - n n) A(n) / k, with A(n) the
    far-field amplitude vector pinned by the guide's printed Mueller table."""
    ijk = w.sphere_integer(2.5)
    kh, e0 = w.along_x_yz()
    case = dense.solve_case(ijk, np.full(len(ijk), 1.4 + 0.05j), 0.8, kh[0], e0[0])
    k, P = case["k"], case["P"]
    n = np.array([0.36, -0.48, 0.8])
    R = 1e7
    E = nearfield.scattered_field(ijk, P, k, (R * n)[None, :])[0] * R * np.exp(-1j * k * R)
    A = farfield.amplitude_vectors(ijk, P, k, n[None, :])[0]
    expect = (A - n * (n @ A)) / k
    assert np.abs(E - expect).max() < 1e-5 * np.abs(expect).max()


def test_nearfield_static_dipole_and_interaction_tensor():
    """k -> 0: one dipole's field is (3 n (n.P) - P) / r^3 (electrostatics).
    At finite k the field equals -A_jl P_l with the interaction block that
    finite differences of exp(ikr)/r pin."""
    P = np.array([[0.3, -0.2 + 0.1j, 0.5]])
    site = np.array([[0, 0, 0]])
    r = np.array([[2.0, -1.0, 3.0]])
    rn = np.linalg.norm(r[0])
    n = r[0] / rn
    E0 = nearfield.scattered_field(site, P, 1e-9, r)[0]
    assert np.abs(E0 - (3 * n * (n @ P[0]) - P[0]) / rn ** 3).max() < 1e-12
    E1 = nearfield.scattered_field(site, P, 0.7, r)[0]
    assert np.abs(E1 + dense.interaction_block(r[0], 0.7) @ P[0]).max() < 1e-14
    # no self term: the field at the dipole's own site is zero
    assert not nearfield.scattered_field(site, P, 0.7, site).any()


def test_trilinear_reproduces_linear_fields():
    """Trilinear interpolation is exact for a field linear in position."""
    B = np.array([[1.0, 2.0j, -0.5], [0.3, 0.0, 1j], [2.0, -1.0, 0.25]])
    c0 = np.array([0.1, -2j, 3.0])
    lin = lambda q: c0[None, :] + np.asarray(q, float) @ B
    pts = nearfield.line_points([-1.3, 0.25, 2.0], [4.7, 3.5, -1.1], 23)
    assert np.abs(nearfield.trilinear(lin, pts) - lin(pts)).max() < 1e-12
    assert np.allclose(pts[0], [-1.3, 0.25, 2.0]) and np.allclose(pts[-1], [4.7, 3.5, -1.1])


# ---------------------------------------------------------------- breakdown right-hand sides

def test_breakdown_right_hand_sides_zero_their_forms():
    """The right-hand sides the GPU breakdown tests use: b^H A b vanishes to
    rounding for the gain target (0 in its numerical range) while b^T A b does
    not, so a restart with the conjugate shadow residual can proceed; for a
    passive target b^H A b stays away from 0 (its imaginary part is minus the
    extinguished power), while b^T A b can be zeroed."""
    import breakdown_rhs as br
    cube = w.brick(2, 2, 2)
    k = dense.kd_from_size_parameter(1.0, len(cube))
    A = dense.assemble(cube, dense.site_alpha_inverse(np.full(len(cube), br.GAIN_M), k, [1, 0, 0], [0, 1, 0]), k)
    b = br.hermitian_zero(A)
    nAb = np.linalg.norm(A @ b)
    assert abs(np.vdot(b, A @ b)) <= 1e-15 * nAb and abs(b @ A @ b) >= 0.05 * nAb
    ijk = w.brick(3, 3, 3)
    k = dense.kd_from_size_parameter(1.0, len(ijk))
    Ap = dense.assemble(ijk, dense.site_alpha_inverse(np.full(len(ijk), 1.5 + 0.1j), k, [1, 0, 0], [0, 1, 0]), k)
    bp = br.bilinear_zero(Ap)
    assert abs(bp @ Ap @ bp) <= 1e-14 * np.linalg.norm(Ap @ bp)
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = rng.standard_normal(81) + 1j * rng.standard_normal(81)
        assert np.vdot(u, Ap @ u).imag < 0
