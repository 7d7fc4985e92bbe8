// HIP kernels of the DDA solve for gfx950, other than the matvec passes
// (dda_passes.h): the interaction-tensor sampling and its FFT, 1/alpha,
// E_inc, the BiCGSTAB updates and their reductions, the efficiency sums, the
// adjoint right-hand side and gradient, and small utilities.
#include <stdexcept>
#include "dda_kernels.h"

namespace dda {

namespace {

template <typename C> __device__ __forceinline__ C to_c(double2 u) {
    C c;
    c.x = u.x;
    c.y = u.y;
    return c;
}
template <typename C> __device__ __forceinline__ double2 to_d(C u) {
    double2 c;
    c.x = (double)u.x;
    c.y = (double)u.y;
    return c;
}
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }


__host__ __device__ inline int pad_len(int L) { return L | 1; }
template <typename C> __host__ inline size_t fft_smem(int L, int nlines) {
    return ((size_t)((L + 1) & ~1) + (size_t)nlines * pad_len(L)) * sizeof(C) + 8 * (NT / 64) * sizeof(double) + 64;
}

// Forward FFT along x of every line of a two-slab three-component FP64 grid
// (the interaction tensor; slab = grid z).
__global__ __launch_bounds__(NT) void k_xgrid3(Geo g, double2* grid, const double2* tw64, int XL) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mx = g.M[0], My = g.M[1];
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * XL;
    const int nl = min(XL, My - y0);
    const int nlines = 3 * nl;
    const int Lp = pad_len(Mx);
    double2* tws = (double2*)smem;
    double2* lds = tws + ((Mx + 1) & ~1);
    load_twiddles<double>(tws, tw64, g.ax[0]);
    double2* gq = grid + (long long)blockIdx.z * g.npts * 3 + ((long long)z * My + y0) * Mx * 3;
    const int tot = nl * Mx * 3;
    for (int idx = threadIdx.x; idx < tot; idx += NT) {
        const int c = idx % 3;
        const int rest = idx / 3;
        const int e = rest % Mx;
        const int yo = rest / Mx;
        lds[(yo * 3 + c) * Lp + e] = gq[idx];
    }
    __syncthreads();
    fft_lines<double, -1>(lds, tws, nlines, Lp, g.ax[0]);
    for (int idx = threadIdx.x; idx < tot; idx += NT) {
        const int c = idx % 3;
        const int rest = idx / 3;
        const int e = rest % Mx;
        const int yo = rest / Mx;
        gq[idx] = lds[(yo * 3 + c) * Lp + e];
    }
}

// ------------------------------------------------------------------ setup

// Signed lattice separation held by padded index m on an axis of box extent
// n and padded extent M; false for the empty slots between +(n-1) and -(n-1).
__device__ __forceinline__ bool sep(int m, int n, int M, int& d) {
    if (m <= n - 1) { d = m; return true; }
    if (m >= M - (n - 1)) { d = m - M; return true; }
    return false;
}

// Off-diagonal interaction tensor (Draine 1988) sampled at every separation:
// A_jl = exp(ikr)/r [k^2 (nn - I) + (ikr - 1)/r^2 (3nn - I)], stored as its six
// distinct components xx, xy, xz, yy, yz, zz; zero at R = 0 and empty slots.
__global__ __launch_bounds__(NT) void k_green_sample(Geo g, double kd, double2* G) {
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= g.npts) return;
    const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
    const int mx = (int)(i % Mx);
    const int my = (int)((i / Mx) % My);
    const int mz = (int)(i / ((long long)Mx * My));
    int dx, dy, dz;
    // component c in slab c / 3, position c % 3
    double2* out0 = G + i * 3;
    double2* out1 = G + (g.npts + i) * 3;
    const bool ok = sep(mx, g.n[0], Mx, dx) && sep(my, g.n[1], My, dy) && sep(mz, g.n[2], Mz, dz);
    if (!ok || (dx == 0 && dy == 0 && dz == 0)) {
        for (int c = 0; c < 3; ++c) out0[c] = out1[c] = double2{0.0, 0.0};
        return;
    }
    const double X = dx, Y = dy, Z = dz;
    const double r2 = X * X + Y * Y + Z * Z;
    const double r = sqrt(r2);
    double sn, cs;
    sincos(kd * r, &sn, &cs);
    const double2 pref = {cs / r, sn / r};                       // exp(ikr)/r
    const double2 ikr1 = {-1.0 / r2, kd * r / r2};               // (ikr - 1)/r^2
    // A = pref [ (-k^2 - (ikr-1)/r^2) I + (k^2 + 3(ikr-1)/r^2) R R / r^2 ]
    const double2 ciso = cmul(pref, double2{-kd * kd - ikr1.x, -ikr1.y});
    const double2 cnn = cscale(cmul(pref, double2{kd * kd + 3.0 * ikr1.x, 3.0 * ikr1.y}), 1.0 / r2);
    const double R[3] = {X, Y, Z};
    const int ab[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int c = 0; c < 6; ++c) {
        double2 v = cscale(cnn, R[ab[c][0]] * R[ab[c][1]]);
        if (ab[c][0] == ab[c][1]) v = cadd(v, ciso);
        (c < 3 ? out0 : out1)[c % 3] = v;
    }
}

// Keep the octant 0..M/2 of the tensor FFT, scaled by 1/M so that the
// inverse transforms of the product need no further normalisation.
__global__ __launch_bounds__(NT) void k_green_octant(Geo g, const double2* G, double2* gh64, float2* gh32) {
    const long long nh = (long long)g.H[0] * g.H[1] * g.H[2];
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= nh) return;
    const int hx = (int)(i % g.H[0]);
    const int hy = (int)((i / g.H[0]) % g.H[1]);
    const int hz = (int)(i / ((long long)g.H[0] * g.H[1]));
    const long long src = (((long long)hz * g.M[1] + hy) * g.M[0] + hx) * 3;
    const double sc = 1.0 / (double)g.npts;
    for (int c = 0; c < 6; ++c) {
        const double2 v = cscale(G[(c < 3 ? 0 : g.npts * 3) + src + c % 3], sc);
        if (gh64) gh64[i * 6 + c] = v;
        if (gh32) gh32[i * 6 + c] = float2{(float)v.x, (float)v.y};
    }
}

// 1/alpha (or its derivative with respect to eps, scheme + 2) per
// (right-hand side, material): "Dipole Polarizabilities".
//   LATTDR (Draine & Goodman 1993): 1/alpha = 1/alpha_CM
//       + (b1 + eps b2 + eps b3 S) (kd)^2 - (2/3) i (kd)^3,
//       S = sum_mu khat_mu^2 |e_mu|^2, 1/alpha_CM = (4 pi/3)(eps+2)/(eps-1).
//   GKDLDR (Gutkowicz-Krusin & Draine 2004): S -> khat_mu^2 on axis mu.
__global__ void k_alpha(int nrhs, int nmat, const double2* mats, double m_medium, const double* khat,
                        const double2* e0, double kd, int scheme, double2* out, int ostride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrhs * nmat) return;
    const int q = i / nmat, mt = i % nmat;
    const double b1 = -1.891531, b2 = 0.1648469, b3 = -1.7700004;
    const double pi = 3.14159265358979323846;
    // refractive index relative to the ambient medium
    const double2 m = {mats[mt].x / m_medium, mats[mt].y / m_medium};
    const double2 eps = cmul(m, m);
    const double* kh = khat + q * 3;
    const double2* e = e0 + q * 3;
    double S = 0.0;
    for (int mu = 0; mu < 3; ++mu) S += kh[mu] * kh[mu] * (e[mu].x * e[mu].x + e[mu].y * e[mu].y);
    const double k2 = kd * kd;
    const double2 em1 = {eps.x - 1.0, eps.y};
    const bool deriv = scheme >= 2;
    const int sch = scheme & 1;
    for (int mu = 0; mu < 3; ++mu) {
        const double Smu = sch ? kh[mu] * kh[mu] : S;
        double2 v;
        if (!deriv) {
            const double2 cm = cscale(cdiv(double2{eps.x + 2.0, eps.y}, em1), 4.0 * pi / 3.0);
            const double2 ldr = cscale(cadd(double2{b1, 0.0}, cscale(eps, b2 + b3 * Smu)), k2);
            v = cadd(cm, ldr);
            v.y -= (2.0 / 3.0) * k2 * kd;
        } else {
            // d/deps: -4 pi/(eps-1)^2 + (b2 + b3 S) k^2
            const double2 d = cdiv(double2{-4.0 * pi, 0.0}, cmul(em1, em1));
            v = cadd(d, double2{(b2 + b3 * Smu) * k2, 0.0});
        }
        out[((long long)q * ostride + mt) * 3 + mu] = v;
    }
}

// E_inc at every site: e exp(i kd khat . r), "Incident Polarization State".
__global__ __launch_bounds__(NT) void k_einc(SiteArgs a, const int* coords, const double* khat, const double2* e0) {
    const int q = blockIdx.y;
    const double* kh = khat + q * 3;
    const double2* e = e0 + q * 3;
    const int ns = a.rg ? a.rg[q].nsites : a.nsites;
    const double kdq = rhs_kd(a, q);
    coords += 3LL * rhs_site_off(a, q);
    for (int s = blockIdx.x * NT + threadIdx.x; s < ns; s += gridDim.x * NT) {
        const double ph = kdq * (kh[0] * coords[s * 3 + 0] + kh[1] * coords[s * 3 + 1] + kh[2] * coords[s * 3 + 2]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double2 w = {cs, sn};
        double2* b = a.b + (long long)q * a.n3 + (long long)s * 3;
        for (int c = 0; c < 3; ++c) b[c] = cmul(e[c], w);
    }
}

// ------------------------------------------------------------------ Krylov

// Cold start x = 0: r = rhat = b, p = v = 0; rho = |b|^2.
__global__ __launch_bounds__(NT) void k_init_cold(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const long long vb = (long long)q * a.n3;
    double acc[1] = {0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 bb = a.b[vb + i];
        a.r[vb + i] = bb;
        a.rhat[vb + i] = bb;
        a.x[vb + i] = double2{0.0, 0.0};
        a.p[vb + i] = double2{0.0, 0.0};
        a.v[vb + i] = double2{0.0, 0.0};
        acc[0] += bb.x * bb.x + bb.y * bb.y;
    }
    publish_partial<1>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// Warm start: x already holds P0 and r = b - A P0.  rhat = r, p = v = 0.
__global__ __launch_bounds__(NT) void k_init_warm(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const long long vb = (long long)q * a.n3;
    double acc[2] = {0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 rr = a.r[vb + i];
        const double2 bb = a.b[vb + i];
        a.rhat[vb + i] = rr;
        a.p[vb + i] = double2{0.0, 0.0};
        a.v[vb + i] = double2{0.0, 0.0};
        acc[0] += rr.x * rr.x + rr.y * rr.y;
        acc[1] += bb.x * bb.x + bb.y * bb.y;
    }
    publish_partial<2>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// The end of the latest BiCGSTAB iteration, where still pending (see
// RhsState::pend): x += alpha p + omega s, r = s - omega t, or x += alpha p
// after a half-step convergence.  During the iteration the next pass-1
// scatter applies it; this kernel applies it once the iteration has
// stopped, or before a restart.  A FIN_FLUSH finalize then clears the flag.
__global__ __launch_bounds__(NT) void k_bicg_flush(SiteArgs a) {
    const int q = blockIdx.y;
    const RhsState* st = a.st + q;
    const int pend = st->pend;
    if (pend == 0) return;
    const double2 alpha = st->alpha, omega = st->omega;
    const long long vb = (long long)q * a.n3;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)gridDim.x * NT) {
        const double2 s = a.r[vb + i];
        double2 xx = cadd(a.x[vb + i], cmul(alpha, a.p[vb + i]));
        if (pend == 1) {
            xx = cadd(xx, cmul(omega, s));
            a.r[vb + i] = csub(s, cmul(omega, a.t[vb + i]));
        }
        a.x[vb + i] = xx;
    }
}

// One restart after a breakdown, from the current x and r: p = v = 0 and
// the shadow residual rhat = conj(r), so that rho = <rhat, r> = r^T r.  A
// shadow residual rhat = r would repeat a breakdown met in the first step
// after a start (<r, A r> = 0 again); for A = A^T, <conj(r), A r> = r^T A r
// is the bilinear form, independent of the Hermitian one.  Sums r^T r and
// |r|^2 (= |rhat|^2).
__global__ __launch_bounds__(NT) void k_restart(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const RhsState* st = a.st + q;
    if (st->status != ST_BREAKDOWN || st->restarts > 0) return;
    const long long vb = (long long)q * a.n3;
    double acc[3] = {0.0, 0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 rr = a.r[vb + i];
        a.rhat[vb + i] = cconj(rr);
        a.p[vb + i] = double2{0.0, 0.0};
        a.v[vb + i] = double2{0.0, 0.0};
        acc[0] += rr.x * rr.x - rr.y * rr.y;
        acc[1] += 2.0 * rr.x * rr.y;
        acc[2] += rr.x * rr.x + rr.y * rr.y;
    }
    publish_partial<3>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// ------------------------------------------------------------------ QMR
// QMR for complex-symmetric A ("Choice of Iterative Algorithm", QMRCCG): COCG
// (van der Vorst & Melissen 1990) -- CG with the bilinear form u^T v -- whose
// iterates and residuals are smoothed (Zhou & Walker 1994) so that the
// smoothed residual s = b - A y has quasi-minimal norm.  Vectors: x, r, p
// (COCG), v = A p, rhat = s, t = y.  A smoothing step (w_old, w_new) is
// computed by the finalize after an update and applied by the next scatter
// (or by k_qmr_final); pend marks it as not yet applied.

// Start: cold r = b, x = 0 (warm: r = b - A x already).  p = 0, s = r,
// y = x; sums r^T r, |r|^2, |b|^2.
__global__ __launch_bounds__(NT) void k_qmr_init(SiteArgs a, int cold) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const long long vb = (long long)q * a.n3;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 bb = a.b[vb + i];
        double2 rr;
        if (cold) {
            rr = bb;
            a.r[vb + i] = rr;
            a.x[vb + i] = double2{0.0, 0.0};
        } else {
            rr = a.r[vb + i];
        }
        a.p[vb + i] = double2{0.0, 0.0};
        a.rhat[vb + i] = rr;
        a.t[vb + i] = cold ? double2{0.0, 0.0} : a.x[vb + i];
        acc[0] += rr.x * rr.x - rr.y * rr.y;
        acc[1] += 2.0 * rr.x * rr.y;
        acc[2] += rr.x * rr.x + rr.y * rr.y;
        acc[3] += bb.x * bb.x + bb.y * bb.y;
    }
    publish_partial<4>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// x += alpha p, r -= alpha v; sums r^T r, |r|^2 and Re <s, r> (for the
// norm of the next smoothed residual).
__global__ __launch_bounds__(NT) void k_qmr_update(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const RhsState* st = a.st + q;
    if (st->status != ST_ACTIVE) return;
    const double2 alpha = st->alpha;
    const long long vb = (long long)q * a.n3;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        a.x[vb + i] = cadd(a.x[vb + i], cmul(alpha, a.p[vb + i]));
        const double2 rr = csub(a.r[vb + i], cmul(alpha, a.v[vb + i]));
        a.r[vb + i] = rr;
        const double2 sm = a.rhat[vb + i];
        acc[0] += rr.x * rr.x - rr.y * rr.y;
        acc[1] += 2.0 * rr.x * rr.y;
        acc[2] += rr.x * rr.x + rr.y * rr.y;
        acc[3] += sm.x * rr.x + sm.y * rr.y;
    }
    publish_partial<4>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// x and y <- the smoothed iterate: w_old y + w_new x if a step is pending,
// else y.  A FIN_QFINAL finalize then clears the pending flag, so applying
// both again leaves x unchanged.
__global__ __launch_bounds__(NT) void k_qmr_final(SiteArgs a) {
    const int q = blockIdx.y;
    const RhsState* st = a.st + q;
    const bool pend = st->pend != 0;
    const double wo = st->w_old, wn = st->w_new;
    const long long vb = (long long)q * a.n3;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)gridDim.x * NT) {
        double2 y = a.t[vb + i];
        if (pend) {
            const double2 xx = a.x[vb + i];
            y = double2{wo * y.x + wn * xx.x, wo * y.y + wn * xx.y};
            a.t[vb + i] = y;
        }
        a.x[vb + i] = y;
    }
}

// Breakdown tests compare a quantity with the norms that bound it: an inner
// product <u, v> (or u^T v) is taken as zero when |<u, v>| <= BD_EPS |u| |v|,
// the size of its FP64 rounding error over millions of terms (a single test
// on exact zero would almost never fire).  bound2 is |u|^2 |v|^2.
constexpr double BD_EPS = 1e-12;
__device__ __forceinline__ bool vanishes(double2 z, double bound2) {
    return z.x * z.x + z.y * z.y <= BD_EPS * BD_EPS * bound2;
}

// QMR state from the start sums: r^T r = (acc0, acc1), |r|^2 = acc2, |b|^2 =
// acc3.  The first smoothing step is (0, 1): y = x, s = r.
__device__ void qmr_start(RhsState* st, const double* acc) {
    st->bnorm2 = acc[3];
    st->rnorm2 = acc[2];
    st->snorm2 = acc[2];
    st->tau2 = acc[2];
    st->rho = double2{acc[0], acc[1]};
    st->beta = double2{0.0, 0.0};
    st->w_old = 0.0;
    st->w_new = 1.0;
    st->pend = 1;
    st->sconv = 0;
    if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(acc[2]) || !isfinite(acc[3])) {
        st->status = ST_NONFINITE;
    } else if (acc[2] <= st->tol2 * acc[3]) {
        st->status = ST_CONVERGED;
    } else {
        st->status = vanishes(double2{acc[0], acc[1]}, acc[2] * acc[2]) ? ST_BREAKDOWN : ST_ACTIVE;
    }
}

// ------------------------------------------------------------------ BiCGstab(2)
// End of a BiCGstab(2) iteration ("Choice of Iterative Algorithm", PBCGS2;
// Sleijpen & Fokkema 1993): the minimal-residual combination
// x += g1 r_0 + g2 r_1, r_0 -= g1 r_1 + g2 r_2, u_0 -= g1 u_1 + g2 u_2;
// sums <rhat, r_0> and |r_0|^2 for the next iteration.
__global__ __launch_bounds__(NT) void k_b2_update(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const RhsState* st = a.st + q;
    if (st->status != ST_ACTIVE) return;
    const double2 g1 = st->g1, g2 = st->g2;
    const long long vb = (long long)q * a.n3;
    double acc[3] = {0.0, 0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 r0 = a.r[vb + i], r1 = a.t[vb + i];
        a.x[vb + i] = cadd(a.x[vb + i], cadd(cmul(g1, r0), cmul(g2, r1)));
        const double2 rn = csub(r0, cadd(cmul(g1, r1), cmul(g2, a.r2[vb + i])));
        a.r[vb + i] = rn;
        a.p[vb + i] = csub(a.p[vb + i], cadd(cmul(g1, a.v[vb + i]), cmul(g2, a.u2[vb + i])));
        const double2 w = cdotc(a.rhat[vb + i], rn);
        acc[0] += w.x;
        acc[1] += w.y;
        acc[2] += rn.x * rn.x + rn.y * rn.y;
    }
    publish_partial<3>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// ------------------------------------------------------------------ far field
// Scattering amplitudes ("Scattering by Finite Targets: The Mueller Matrix";
// Draine 1988): per direction n and right-hand side, A = k^3 sum_j P_j
// exp(-i k n . r_j), then f_1 = theta . A, f_2 = phi . A and the differential
// cross section (|f_1|^2 + |f_2|^2) / k^2.  dirs holds n, theta, phi per
// direction.  On the lattice the phase factor separates by axis,
// exp(-i k n . r) = w_x(x) w_y(y) w_z(z), so one workgroup per direction
// tabulates the n_x + n_y + n_z factors of its direction in LDS and every
// term costs two complex products instead of a sine and cosine; the
// right-hand sides are taken FR at a time over the same factors, and DW
// directions at a time over the same loaded sites (each site's P is read
// once for all DW).  per > 0: direction d belongs to right-hand side d / per
// alone (every right-hand side with its own direction set in one launch;
// DW divides per) and its results go to entry d; there FR is 1.  Each term
// is accumulated as four fused multiply-adds in a fixed order.
// Deterministic sums (each direction: fixed per-thread order, then the
// workgroup reduction; the same for every DW and FR).
template <int DW, int FR>
__global__ __launch_bounds__(NT) void k_farfield(int nsites, const int* coords, const double2* P, long long n3,
                                                 int nrhs, const double* dirs, double k, int lox, int loy, int loz,
                                                 int nx, int ny, int nz, double2* f, double* dcs, int ndir,
                                                 int per) {
    extern __shared__ double2 wtab[];     // [DW][nx + ny + nz] phase factors of the group's directions
    __shared__ double sh[6 * FR * NT / 64];   // block_sum scratch: one value per wave and sum
    const int d0 = blockIdx.x * DW;
    const int nt = nx + ny + nz;
    for (int i = threadIdx.x; i < DW * nt; i += NT) {
        const int j = i / nt, ii = i % nt;
        const int d = min(d0 + j, ndir - 1);   // past the end: a copy of the last direction, not stored
        const double* dv = dirs + (long long)d * 9;
        const int a = ii < nx ? 0 : (ii < nx + ny ? 1 : 2);
        const int c = a == 0 ? lox + ii : (a == 1 ? loy + (ii - nx) : loz + (ii - nx - ny));
        double sn, cs;
        sincos(-k * dv[a] * c, &sn, &cs);
        wtab[i] = double2{cs, sn};
    }
    __syncthreads();
    const double k3 = k * k * k;
    // per = 0: the right-hand sides FR at a time along the grid's y
    const int qa = per > 0 ? d0 / per : (int)blockIdx.y * FR;
    const int qb = per > 0 ? qa + 1 : min(nrhs, qa + FR);
    for (int q0 = qa; q0 < qb; q0 += FR) {
        double acc[DW][6 * FR];
#pragma unroll
        for (int j = 0; j < DW; ++j)
#pragma unroll
            for (int i = 0; i < 6 * FR; ++i) acc[j][i] = 0.0;
        // a thread's sites s, s + NT, s + 2 NT, ... in that order, two per
        // iteration with both sites' loads issued first
        for (int s0 = threadIdx.x; s0 < nsites; s0 += 2 * NT) {
            int cc[2][3];
            double2 pv[2][FR][3];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int s = min(s0 + h * NT, nsites - 1);   // past the end: loaded, not added
                cc[h][0] = coords[s * 3 + 0] - lox;
                cc[h][1] = nx + coords[s * 3 + 1] - loy;
                cc[h][2] = nx + ny + coords[s * 3 + 2] - loz;
#pragma unroll
                for (int r = 0; r < FR; ++r) {
                    const double2* Pq = P + (long long)(q0 + r) * n3 + (long long)s * 3;
#pragma unroll
                    for (int c = 0; c < 3; ++c) pv[h][r][c] = q0 + r < qb ? Pq[c] : double2{0.0, 0.0};
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && s0 + NT >= nsites) break;
#pragma unroll
                for (int j = 0; j < DW; ++j) {
                    const double2* wt = wtab + j * nt;
                    const double2 w = cmul(cmul(wt[cc[h][0]], wt[cc[h][1]]), wt[cc[h][2]]);
#pragma unroll
                    for (int r = 0; r < FR; ++r) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double& ar = acc[j][6 * r + 2 * c];
                            double& ai = acc[j][6 * r + 2 * c + 1];
                            ar = fma(pv[h][r][c].x, w.x, ar);
                            ar = fma(-pv[h][r][c].y, w.y, ar);
                            ai = fma(pv[h][r][c].x, w.y, ai);
                            ai = fma(pv[h][r][c].y, w.x, ai);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < DW; ++j) {
            block_sum<6 * FR>(acc[j], sh);
            const int d = d0 + j;
            if (threadIdx.x == 0 && d < ndir) {
                const double* dv = dirs + (long long)d * 9;
                for (int r = 0; r < FR && q0 + r < qb; ++r) {
                    double2 f1 = {0.0, 0.0}, f2 = {0.0, 0.0};
                    for (int c = 0; c < 3; ++c) {
                        const double2 A = {k3 * acc[j][6 * r + 2 * c], k3 * acc[j][6 * r + 2 * c + 1]};
                        f1 = cadd(f1, double2{dv[3 + c] * A.x, dv[3 + c] * A.y});
                        f2 = cadd(f2, double2{dv[6 + c] * A.x, dv[6 + c] * A.y});
                    }
                    const long long o = per > 0 ? (long long)d : (long long)(q0 + r) * ndir + d;
                    f[o * 2 + 0] = f1;
                    f[o * 2 + 1] = f2;
                    dcs[o] = (f1.x * f1.x + f1.y * f1.y + f2.x * f2.x + f2.y * f2.y) / (k * k);
                }
            }
            __syncthreads();
        }
    }
}

// Direction sets of the angular averages ("Averaging over Scattering
// Directions"): for right-hand side q with incidence direction k, the frame
// (k, u, v), u the unit vector along k x e (e the x axis, or y where k is
// near x) and v = k x u, and the directions n = mu_i k + sqrt(1 - mu_i^2)
// (cos p_j u + sin p_j v), p_j = 2 pi j / n_phi, with their theta and phi
// unit vectors: dirs [ng][n_theta][n_phi][9] (n, theta, phi).
__global__ __launch_bounds__(NT) void k_avg_dirs(int ng, const double* kh, const double* mu, int n_theta, int n_phi,
                                                 double* dirs) {
    const long long nd = (long long)n_theta * n_phi;
    const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
    if (idx >= (long long)ng * nd) return;
    const int q = (int)(idx / nd);
    const int i = (int)((idx % nd) / n_phi);
    const int j = (int)(idx % n_phi);
    const double* k = kh + 3 * q;
    const bool nx = fabs(k[0]) < 0.9;
    const double e[3] = {nx ? 1.0 : 0.0, nx ? 0.0 : 1.0, 0.0};
    double u[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2], k[0] * e[1] - k[1] * e[0]};
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (double& x : u) x /= un;
    const double v[3] = {k[1] * u[2] - k[2] * u[1], k[2] * u[0] - k[0] * u[2], k[0] * u[1] - k[1] * u[0]};
    const double ct = mu[i], st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double p = 2.0 * M_PI * j / n_phi;
    double sp, cp;
    sincos(p, &sp, &cp);
    double* D = dirs + idx * 9;
    for (int m = 0; m < 3; ++m) {
        const double t = cp * u[m] + sp * v[m];
        D[m] = ct * k[m] + st * t;
        D[3 + m] = ct * t - st * k[m];
        D[6 + m] = -sp * u[m] + cp * v[m];
    }
}

// ------------------------------------------------------------------ near field
// ("Near-Field Calculations".)  The extended volume is a lattice box of
// dims[0] x dims[1] x dims[2] points starting at lattice point org, every
// point a site of the product's target; its site vectors are in box-scan
// order.  k_nf_place copies the solution P (caller order) into that vector
// at the target's sites (every other point is zeroed beforehand).
__global__ __launch_bounds__(NT) void k_nf_place(int nsites, const int* perm, const int* coords, const double2* P,
                                                 int ox, int oy, int oz, int nx, int ny, long long n3x,
                                                 double2* x) {
    const int q = blockIdx.y;
    const long long n3 = 3LL * nsites;
    for (int s = blockIdx.x * NT + threadIdx.x; s < nsites; s += gridDim.x * NT) {
        const long long i = ((long long)(coords[s * 3 + 2] - oz) * ny + (coords[s * 3 + 1] - oy)) * nx +
                            (coords[s * 3 + 0] - ox);
        const double2* src = P + (long long)q * n3 + (long long)perm[s] * 3;
        double2* dst = x + (long long)q * n3x + i * 3;
        for (int c = 0; c < 3; ++c) dst[c] = src[c];
    }
}

// E_sca = -(off-diagonal product) at every point of the extended volume (v
// holds that product: the diagonal was zero), and E_inc = e exp(i kd khat . r)
// with r the point's lattice coordinates.  Either output may be null.
__global__ __launch_bounds__(NT) void k_nf_out(long long npts, int ox, int oy, int oz, int nx, int ny,
                                               const double* khat, const double2* e0, double kd, const double2* v,
                                               double2* einc, double2* esca) {
    const int q = blockIdx.y;
    const double* kh = khat + q * 3;
    const double2* e = e0 + q * 3;
    const long long base = (long long)q * npts * 3;
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < npts; i += (long long)gridDim.x * NT) {
        if (esca)
            for (int c = 0; c < 3; ++c) {
                const double2 y = v[base + i * 3 + c];
                esca[base + i * 3 + c] = double2{-y.x, -y.y};
            }
        if (einc) {
            const long long xy = (long long)nx * ny;
            const int z = (int)(i / xy), y = (int)((i / nx) % ny), x = (int)(i % nx);
            const double ph = kd * (kh[0] * (x + ox) + kh[1] * (y + oy) + kh[2] * (z + oz));
            double sn, cs;
            sincos(ph, &sn, &cs);
            const double2 w = {cs, sn};
            for (int c = 0; c < 3; ++c) einc[base + i * 3 + c] = cmul(e[c], w);
        }
    }
}

// Trilinear values of a lattice field E [nrhs][dims z][dims y][dims x][3]
// (first point at lattice point org) at n points p_i = a + (b - a) i / (n - 1)
// (p_0 = a when n = 1).  The host has checked that a and b lie in the box,
// so every p_i does; the lower corner is clamped so that a point on the upper
// face takes weight 1 on it.
__global__ __launch_bounds__(NT) void k_field_line(const double2* E, int ox, int oy, int oz, int nx, int ny, int nz,
                                                   double ax, double ay, double az, double bx, double by, double bz,
                                                   int n, double2* out) {
    const int q = blockIdx.y;
    const long long npts = (long long)nx * ny * nz;
    const double2* Eq = E + (long long)q * npts * 3;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const double t = n > 1 ? (double)i / (double)(n - 1) : 0.0;
        const double p[3] = {ax + t * (bx - ax) - ox, ay + t * (by - ay) - oy, az + t * (bz - az) - oz};
        const int dim[3] = {nx, ny, nz};
        int b0[3];
        double f[3];
        for (int d = 0; d < 3; ++d) {
            int c = (int)floor(p[d]);
            c = c < 0 ? 0 : c;
            c = c > dim[d] - 2 ? (dim[d] >= 2 ? dim[d] - 2 : 0) : c;
            b0[d] = c;
            f[d] = dim[d] >= 2 ? p[d] - c : 0.0;
        }
        double2 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int corner = 0; corner < 8; ++corner) {
            const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
            if ((dx && nx < 2) || (dy && ny < 2) || (dz && nz < 2)) continue;
            const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
            const long long j = ((long long)(b0[2] + dz) * ny + (b0[1] + dy)) * nx + (b0[0] + dx);
            for (int c = 0; c < 3; ++c) {
                const double2 v = Eq[j * 3 + c];
                acc[c].x += w * v.x;
                acc[c].y += w * v.y;
            }
        }
        for (int c = 0; c < 3; ++c) out[((long long)q * n + i) * 3 + c] = acc[c];
    }
}

// Efficiency sums at the solution x (Draine 1988):
//   red[3] = sum Im(E* . P), red[4] = sum (-Im(1/alpha) - (2/3) k^3) |P|^2,
//   red[5] = sum Re(E* . P).
__global__ __launch_bounds__(NT) void k_qsum(SiteArgs a) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.y;
    const long long vb = (long long)q * a.n3;
    const double2* ai = a.ainv + (long long)q * a.nmat * 3;
    const double kdq = rhs_kd(a, q);
    const double rr = (2.0 / 3.0) * kdq * kdq * kdq;
    const int* mat = a.mat + rhs_site_off(a, q);
    double acc[3] = {0.0, 0.0, 0.0};
    const int sb = rhs_site_blocks(a, q);
    if ((int)blockIdx.x >= sb) return;
    const long long n3q = rhs_n3(a, q);
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n3q; i += (long long)sb * NT) {
        const double2 P = a.x[vb + i];
        const double2 E = a.b[vb + i];
        const double2 w = cdotc(E, P);
        const int s = (int)(i / 3), c = (int)(i % 3);
        const double2 d = ai[mat[s] * 3 + c];
        acc[0] += w.y;
        acc[1] += (-d.y - rr) * (P.x * P.x + P.y * P.y);
        acc[2] += w.x;
    }
    publish_partial<3>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blockIdx.x, a.maxblk, sh);
}

// Each k_finalize thread's sum of the partials of slot i = blockIdx.x,
// right-hand side q = blockIdx.y: thread t adds workgroups t, t + NT, ...
// in that order, as sum_partials does.
__global__ __launch_bounds__(NT) void k_chain_sums(SiteArgs a, int nblk) {
    const int i = blockIdx.x, q = blockIdx.y;
    if (nblk == NBLK_PASS) nblk = a.rg[q].pass_blocks;
    else if (nblk == NBLK_SITE) nblk = a.rg[q].site_blocks;
    const double* part = a.partials + ((long long)q * PSTRIDE + i) * a.maxblk;
    double acc = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblk; b += NT) acc += part[b];
    a.chains[((long long)q * PSTRIDE + i) * NT + threadIdx.x] = acc;
}

// The workgroup sums of k_finalize: from the partials, or from the chains
// k_chain_sums formed of them (the same values, so the same tree).
template <int NV>
__device__ __forceinline__ void fin_sums(double (&acc)[NV], const SiteArgs& a, int q, const double* part, int nblk,
                                         bool chained, double* sh) {
    if (chained) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = a.chains[((long long)q * PSTRIDE + i) * NT + threadIdx.x];
        block_sum<NV>(acc, sh);
    } else {
        sum_partials<NV>(acc, part, nblk, a.maxblk, sh);
    }
}

// Turn the partial sums of a producer kernel into the right-hand side's
// scalars and status.  One workgroup per right-hand side; it applies the
// same skip rule as the producer so a skipped right-hand side is untouched.
// chained: k_chain_sums ran before it.
__global__ __launch_bounds__(NT) void k_finalize(SiteArgs a, int kind, int nblk, int chained) {
    __shared__ double sh[8 * NT / 64];
    const int q = blockIdx.x;
    RhsState* st = a.st + q;
    const double* part = a.partials + (long long)q * a.maxblk * PSTRIDE;
    bool run;
    switch (kind) {
        case FIN_V: case FIN_T: run = st->status == ST_ACTIVE; break;
        case FIN_RESTART: run = st->status == ST_BREAKDOWN && st->restarts == 0; break;
        case FIN_REFINE: case FIN_QREFINE: run = st->status == ST_CONVERGED && !st->checked; break;
        case FIN_QV: case FIN_QUPD: case FIN_B_BETA: case FIN_B_MR: case FIN_B_UPD:
            run = st->status == ST_ACTIVE;
            break;
        default: run = true; break;
    }
    if (!run) return;
    if (nblk == NBLK_PASS) nblk = a.rg[q].pass_blocks;
    else if (nblk == NBLK_SITE) nblk = a.rg[q].site_blocks;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int ns = fin_slots(kind);
    if (ns == 8) {
        fin_sums<8>(acc, a, q, part, nblk, chained, sh);
    } else if (ns == 4) {
        double a4[4];
        fin_sums<4>(a4, a, q, part, nblk, chained, sh);
        for (int i = 0; i < 4; ++i) acc[i] = a4[i];
    } else {
        double a3[3];
        fin_sums<3>(a3, a, q, part, nblk, chained, sh);
        acc[0] = a3[0];
        acc[1] = a3[1];
        acc[2] = a3[2];
    }
    if (threadIdx.x != 0) return;
    switch (kind) {
        case FIN_V: {
            // <rhat, v>, and |v|^2 in slot 2
            const double2 rv = {acc[0], acc[1]};
            st->pend = 0;   // the scatter before this product applied it
            st->matvecs += 1;
            if (!finite2(rv) || !isfinite(acc[2])) st->status = ST_NONFINITE;
            else if (vanishes(rv, st->rhat2 * acc[2])) st->status = ST_BREAKDOWN;
            else st->alpha = cdiv(st->rho, rv);
            break;
        }
        case FIN_T: {
            // slots 5-7, from the scatter of s: |s|^2 and <rhat, s>.  A
            // half-step convergence ends the iteration with x += alpha p
            // pending (the product t = A s is then not used).  Otherwise
            // omega = <t, s> / |t|^2 from slots 0-4 (the gather of t), and
            // the end of the iteration from the sums alone (r = s - omega t
            // itself is formed later, by the next scatter or the flush):
            // rho' = <rhat, r> = <rhat, s> - omega <rhat, t>, and |r|^2 =
            // |s|^2 - |<t, s>|^2 / |t|^2 since omega t is the projection of
            // s on t
            const double2 ts = {acc[0], acc[1]}, rt = {acc[3], acc[4]}, rs = {acc[6], acc[7]};
            const double tt = acc[2];
            st->matvecs += 1;
            st->snorm2 = acc[5];
            st->rs = rs;
            if (!isfinite(acc[5]) || !finite2(rs)) {
                st->status = ST_NONFINITE;
                break;
            }
            if (acc[5] <= st->tol2 * st->bnorm2) {
                st->sconv = 1;
                st->iters += 1;
                st->rnorm2 = acc[5];
                st->pend = 2;
                st->status = ST_CONVERGED;
                break;
            }
            if (!finite2(ts) || !isfinite(tt) || !finite2(rt)) {
                st->status = ST_NONFINITE;
                break;
            }
            const double2 alpha = st->alpha;
            const double2 omega = tt == 0.0 ? double2{0.0, 0.0} : double2{ts.x / tt, ts.y / tt};
            const double2 rho_new = csub(st->rs, cmul(omega, rt));
            const double r2 = tt == 0.0 ? st->snorm2 : fmax(st->snorm2 - (ts.x * ts.x + ts.y * ts.y) / tt, 0.0);
            st->omega = omega;
            st->iters += 1;
            st->rnorm2 = r2;
            st->pend = 1;
            if (r2 <= st->tol2 * st->bnorm2) {
                st->status = ST_CONVERGED;
            } else if (vanishes(rho_new, st->rhat2 * r2) || vanishes(ts, tt * acc[5])) {
                // <rhat, r'> = 0, or <t, s> = 0 (omega = 0: no stabilising step)
                st->status = ST_BREAKDOWN;
            } else {
                st->beta = cmul(cdiv(rho_new, st->rho), cdiv(alpha, omega));
                st->rho = rho_new;
            }
            if (st->status == ST_ACTIVE && st->iters >= st->max_iter) st->status = ST_MAXITER;
            break;
        }
        case FIN_FLUSH:
            st->pend = 0;
            break;
        case FIN_COLD:
            st->bnorm2 = acc[0];
            st->rnorm2 = acc[0];
            st->rhat2 = acc[0];
            st->rho = double2{acc[0], 0.0};
            st->alpha = double2{1.0, 0.0};
            st->omega = double2{1.0, 0.0};
            st->beta = double2{0.0, 0.0};
            st->iters = 0;
            st->matvecs = 0;
            st->sconv = 0;
            st->pend = 0;
            st->restarts = 0;
            st->status = isfinite(acc[0]) ? (acc[0] > 0.0 ? ST_ACTIVE : ST_CONVERGED) : ST_NONFINITE;
            break;
        case FIN_WARM:
            st->bnorm2 = acc[1];
            st->rnorm2 = acc[0];
            st->rhat2 = acc[0];
            st->rho = double2{acc[0], 0.0};
            st->alpha = double2{1.0, 0.0};
            st->omega = double2{1.0, 0.0};
            st->beta = double2{0.0, 0.0};
            st->iters = 0;
            st->matvecs = 1;
            st->sconv = 0;
            st->pend = 0;
            st->restarts = 0;
            if (!isfinite(acc[0]) || !isfinite(acc[1])) st->status = ST_NONFINITE;
            else st->status = (acc[0] <= st->tol2 * acc[1]) ? ST_CONVERGED : ST_ACTIVE;
            break;
        case FIN_RESTART:
            // rho = r^T r (rhat = conj(r)), |rhat|^2 = |r|^2
            st->rho = double2{acc[0], acc[1]};
            st->rhat2 = acc[2];
            st->rnorm2 = acc[2];
            st->alpha = double2{1.0, 0.0};
            st->omega = double2{1.0, 0.0};
            st->beta = double2{0.0, 0.0};
            st->sconv = 0;
            st->pend = 0;
            st->restarts += 1;
            if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(acc[2])) st->status = ST_NONFINITE;
            else st->status = vanishes(st->rho, acc[2] * acc[2]) ? ST_BREAKDOWN : ST_ACTIVE;
            break;
        case FIN_REFINE:
            // r holds the FP64 residual b - A x: keep converged or iterate on from x
            st->matvecs += 1;
            st->rnorm2 = acc[0];
            if (!isfinite(acc[0])) {
                st->status = ST_NONFINITE;
            } else if (acc[0] > st->tol2 * st->bnorm2) {
                st->rho = double2{acc[0], 0.0};
                st->rhat2 = acc[0];
                st->alpha = double2{1.0, 0.0};
                st->omega = double2{1.0, 0.0};
                st->beta = double2{0.0, 0.0};
                st->sconv = 0;
                st->pend = 0;
                st->pad0 += 1;
                st->status = st->iters >= st->max_iter ? ST_MAXITER : ST_ACTIVE;
            } else {
                st->checked = 1;
            }
            break;
        case FIN_QV: {
            // mu = p^T A p; the scatter has applied the pending smoothing
            // step; |v|^2 and |p|^2 in slots 2 and 3
            const double2 mu = {acc[0], acc[1]};
            st->matvecs += 1;
            st->pend = 0;
            if (!finite2(mu) || !isfinite(acc[2]) || !isfinite(acc[3])) st->status = ST_NONFINITE;
            else if (vanishes(mu, acc[2] * acc[3])) st->status = ST_BREAKDOWN;
            else st->alpha = cdiv(st->rho, mu);
            break;
        }
        case FIN_QUPD: {
            // next smoothing step: 1/tau^2 += 1/|r|^2, weights tau^2/tau_old^2
            // and tau^2/|r|^2; |s_next|^2 from |s|^2, Re <s, r>, |r|^2
            const double2 rho_new = {acc[0], acc[1]};
            const double nu2 = acc[2], sr = acc[3];
            st->iters += 1;
            st->rnorm2 = nu2;
            if (!finite2(rho_new) || !isfinite(nu2) || !isfinite(sr)) {
                st->status = ST_NONFINITE;
                break;
            }
            double wo = 0.0, wn = 1.0, t2 = 0.0;
            if (nu2 > 0.0) {
                t2 = 1.0 / (1.0 / st->tau2 + 1.0 / nu2);
                wo = t2 / st->tau2;
                wn = t2 / nu2;
            }
            const double s2 = fmax(wo * wo * st->snorm2 + 2.0 * wo * wn * sr + wn * wn * nu2, 0.0);
            st->tau2 = t2;
            st->w_old = wo;
            st->w_new = wn;
            st->pend = 1;
            st->snorm2 = s2;
            if (s2 <= st->tol2 * st->bnorm2) {
                st->status = ST_CONVERGED;
            } else if (vanishes(rho_new, nu2 * nu2)) {   // r^T r against |r|^2
                st->status = ST_BREAKDOWN;
            } else {
                st->beta = cdiv(rho_new, st->rho);
                st->rho = rho_new;
            }
            if (st->status == ST_ACTIVE && st->iters >= st->max_iter) st->status = ST_MAXITER;
            break;
        }
        case FIN_QFINAL:
            st->pend = 0;
            break;
        case FIN_B_BETA: {
            // rho_1 = <rhat, r_1>: beta = alpha rho_1 / rho_0, rho_0 <- rho_1
            const double2 rho1 = {acc[0], acc[1]};   // |r_1|^2 in slot 2
            st->matvecs += 1;
            if (!finite2(rho1) || !isfinite(acc[2])) st->status = ST_NONFINITE;
            else if (vanishes(rho1, st->rhat2 * acc[2])) st->status = ST_BREAKDOWN;
            else {
                st->beta = cmul(st->alpha, cdiv(rho1, st->rho));
                st->rho = rho1;
            }
            break;
        }
        case FIN_B_MR: {
            // modified Gram-Schmidt on r_1, r_2: tau = <r_1,r_2>/s1,
            // s2 = |r_2 - tau r_1|^2, g'1 = <r_1,r_0>/s1,
            // g'2 = <r_2 - tau r_1, r_0>/s2; g2 = g'2, g1 = g'1 - tau g2
            st->matvecs += 1;
            bool ok = true;
            for (int i = 0; i < 8; ++i) ok = ok && isfinite(acc[i]);
            if (!ok) {
                st->status = ST_NONFINITE;
                break;
            }
            const double s1 = acc[0];
            const double2 c12 = {acc[1], acc[2]}, c10 = {acc[4], acc[5]}, c20 = {acc[6], acc[7]};
            if (!(s1 > 0.0)) {
                st->status = ST_BREAKDOWN;
                break;
            }
            const double2 tau = {c12.x / s1, c12.y / s1};
            const double s2 = acc[3] - (c12.x * c12.x + c12.y * c12.y) / s1;
            if (!(s2 > BD_EPS * BD_EPS * acc[3])) {   // r_2 parallel to r_1 within rounding
                st->status = ST_BREAKDOWN;
                break;
            }
            const double2 gp1 = {c10.x / s1, c10.y / s1};
            const double2 num = csub(c20, cmul(cconj(tau), c10));
            const double2 g2 = {num.x / s2, num.y / s2};
            st->g2 = g2;
            st->g1 = csub(gp1, cmul(tau, g2));
            st->omega = g2;
            break;
        }
        case FIN_B_UPD: {
            // convergence on |r_0|; rho_0 <- -omega rho_0, then the first
            // BiCG step's beta = alpha <rhat, r_0> / rho_0
            const double2 rho1 = {acc[0], acc[1]};
            const double2 om = st->omega;
            st->iters += 1;
            st->rnorm2 = acc[2];
            if (!isfinite(acc[2]) || !finite2(rho1)) {
                st->status = ST_NONFINITE;
            } else if (acc[2] <= st->tol2 * st->bnorm2) {
                st->status = ST_CONVERGED;
            } else if (vanishes(rho1, st->rhat2 * acc[2]) || (om.x == 0.0 && om.y == 0.0)) {
                st->status = ST_BREAKDOWN;
            } else {
                const double2 rho0 = cmul(double2{-om.x, -om.y}, st->rho);
                st->beta = cmul(st->alpha, cdiv(rho1, rho0));
                st->rho = rho1;
            }
            if (st->status == ST_ACTIVE && st->iters >= st->max_iter) st->status = ST_MAXITER;
            break;
        }
        case FIN_QCOLD:
        case FIN_QWARM:
            qmr_start(st, acc);
            st->iters = 0;
            st->matvecs = kind == FIN_QWARM ? 1 : 0;
            st->restarts = 0;
            break;
        case FIN_QREFINE:
            // r holds the FP64 residual b - A x of a converged solution
            st->matvecs += 1;
            st->rnorm2 = acc[2];
            if (!isfinite(acc[2])) {
                st->status = ST_NONFINITE;
            } else if (acc[2] > st->tol2 * st->bnorm2) {
                qmr_start(st, acc);
                st->pad0 += 1;
                if (st->status == ST_ACTIVE && st->iters >= st->max_iter) st->status = ST_MAXITER;
            } else {
                st->checked = 1;
            }
            break;
        case FIN_QSUM:
            st->red[3] = acc[0];
            st->red[4] = acc[1];
            st->red[5] = acc[2];
            break;
        case FIN_RES:
            st->red[0] = acc[0];
            break;
        default:  // FIN_CONJ
            st->red[a.slot] = acc[0];
            break;
    }
}

// Adjoint right-hand side for the gradient of w_abs Q_abs + w_ext Q_ext
// (with b holding E on entry, g on exit):
//   g = c_Q [ w_abs (-Im(1/alpha) - (2/3) k^3) conj(P) + w_ext conj(E) / (2i) ]
__global__ __launch_bounds__(NT) void k_adjoint_rhs(SiteArgs a, const double2* P, double cq_abs, double cq_ext) {
    const double2* ai = a.ainv;
    const double rr = (2.0 / 3.0) * a.kd * a.kd * a.kd;
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < a.n3; i += (long long)gridDim.x * NT) {
        const int s = (int)(i / 3), c = (int)(i % 3);
        const double2 d = ai[a.mat[s] * 3 + c];
        const double wabs = -d.y - rr;
        const double2 pc = cconj(P[i]);
        const double2 ec = cconj(a.b[i]);
        // conj(E)/(2i) = -i conj(E)/2
        const double2 ext = {0.5 * ec.y, -0.5 * ec.x};
        a.b[i] = cadd(cscale(pc, cq_abs * wabs), cscale(ext, cq_ext));
    }
}

// grad_j = 2 conj(-sum_mu h_mu lam_mu P_mu) - i w_abs c_Q sum_mu conj(h_mu) |P_mu|^2
__global__ __launch_bounds__(NT) void k_grad(SiteArgs a, const double2* P, const double2* dainv, double cq_abs,
                                            double2* grad) {
    for (int s = blockIdx.x * NT + threadIdx.x; s < a.nsites; s += gridDim.x * NT) {
        double2 imp = {0.0, 0.0};
        double2 expl = {0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            const double2 h = dainv[a.mat[s] * 3 + c];
            const double2 lam = a.x[(long long)s * 3 + c];
            const double2 p = P[(long long)s * 3 + c];
            imp = cadd(imp, cmul(h, cmul(lam, p)));
            expl = cadd(expl, cscale(cconj(h), p.x * p.x + p.y * p.y));
        }
        // 2 conj(-imp) = (-2 imp.x, 2 imp.y);  -i cq expl = (cq expl.y, -cq expl.x)
        grad[s] = double2{-2.0 * imp.x + cq_abs * expl.y, 2.0 * imp.y - cq_abs * expl.x};
    }
}

__global__ __launch_bounds__(NT) void k_permute(int nrhs, int nsites, int width, const int* perm, const double2* src,
                                               double2* dst, int to_sorted) {
    const long long per = (long long)nsites * width;
    const long long tot = per * nrhs;
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < tot; i += (long long)gridDim.x * NT) {
        const long long q = i / per;
        const long long rem = i % per;
        const int s = (int)(rem / width), c = (int)(rem % width);
        const long long caller = q * per + (long long)perm[s] * width + c;
        if (to_sorted) dst[i] = src[caller];
        else dst[caller] = src[i];
    }
}

__global__ __launch_bounds__(NT) void k_fill(double2* p, long long n) {
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
        p[i] = double2{0.0, 0.0};
}

__global__ void k_set_state(RhsState* st, int nrhs, double tol2, int max_iter) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nrhs) return;
    RhsState s = {};
    s.tol2 = tol2;
    s.max_iter = max_iter;
    s.status = ST_ACTIVE;
    st[q] = s;
}

inline int blocks_for(long long n, int cap) {
    long long b = (n + NT - 1) / NT;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

// ------------------------------------------------------------------ launchers

LaunchEvents& launch_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

int x_lines_per_tile(const Geo& g, int nrhs, bool fp32) {
    // compile-time lengths: one x-line (three components) per workgroup
    if (ct_length(g.M[0])) return 1;
    // otherwise as many lines as fit one tile, but no fewer than ~2048
    // workgroups when the problem allows it
    const int emax = fp32 ? Tile<float>::EMAX : Tile<double>::EMAX;
    int cap = emax / (3 * g.M[0]);
    if (cap < 1) cap = 1;
    const long long lines = (long long)g.n[1] * g.n[2] * nrhs;
    long long xl = lines / 2048;
    if (xl < 1) xl = 1;
    if (xl > cap) xl = cap;
    return (int)xl;
}

int x_pass_blocks(const Geo& g, int nrhs, bool fp32) {
    const int xl = x_lines_per_tile(g, nrhs, fp32);
    return ((g.n[1] + xl - 1) / xl) * g.n[2];
}

int site_blocks_for(long long n3, int nrhs) {
    // ~2048 workgroups over all right-hand sides, at least one element per thread
    long long b = (2048 + nrhs - 1) / nrhs;
    const long long most = (n3 + NT - 1) / NT;
    if (b > most) b = most;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

int strided_cols_per_tile(int L, int nc, bool fp32) {
    const int emax = fp32 ? Tile<float>::EMAX : Tile<double>::EMAX;
    int tx = emax / (nc * L);
    if (tx < 1) tx = 1;
    int p = 1;
    while (p * 2 <= tx && p * 2 <= 16) p *= 2;
    return p;
}

void launch_xgrid3(const Geo& g, double2* grid, const double2* tw, hipStream_t s) {
    int XL = Tile<double>::EMAX / (3 * g.M[0]);
    if (XL < 1) throw std::invalid_argument("x extent above the LDS line tile");
    dim3 grd((g.M[1] + XL - 1) / XL, g.M[2], 2);
    hipLaunchKernelGGL(k_xgrid3, grd, dim3(NT), fft_smem<double2>(g.M[0], 3 * XL), s, g, grid, tw, XL);
}

void launch_green_sample(const Geo& g, double kd, double2* G, hipStream_t s) {
    hipLaunchKernelGGL(k_green_sample, dim3((unsigned)((g.npts + NT - 1) / NT)), dim3(NT), 0, s, g, kd, G);
}

void launch_green_octant(const Geo& g, const double2* G, double2* gh64, float2* gh32, hipStream_t s) {
    const long long nh = (long long)g.H[0] * g.H[1] * g.H[2];
    hipLaunchKernelGGL(k_green_octant, dim3((unsigned)((nh + NT - 1) / NT)), dim3(NT), 0, s, g, G, gh64, gh32);
}

void launch_alpha(int nrhs, int nmat, const double2* mats, double m_medium, const double* khat, const double2* e0,
                  double kd, int scheme, double2* ainv, hipStream_t s, int ostride) {
    const int n = nrhs * nmat;
    hipLaunchKernelGGL(k_alpha, dim3((n + 63) / 64), dim3(64), 0, s, nrhs, nmat, mats, m_medium, khat, e0, kd, scheme,
                       ainv, ostride > 0 ? ostride : nmat);
}

void launch_einc(const SiteArgs& a, const int* coords, const double* khat, const double2* e0, hipStream_t s) {
    hipLaunchKernelGGL(k_einc, dim3(blocks_for(a.nsites, 1024), a.nrhs), dim3(NT), 0, s, a, coords, khat, e0);
}

void launch_init_cold(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_init_cold, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_init_warm(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_init_warm, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_bicg_flush(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_flush, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_restart(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_restart, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_qmr_init(const SiteArgs& a, bool cold, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_qmr_init, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a, cold ? 1 : 0);
}
void launch_qmr_update(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_qmr_update, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_b2_update(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_b2_update, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_qmr_final(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_qmr_final, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
// directions per workgroup of the far field: four where the direction sets
// allow it and the launch still has at least FF_MIN_WG workgroups (each
// site's P then serves four directions), else one
constexpr int FF_DW = 4;
constexpr int FF_MIN_WG = 512;
void launch_farfield(int nsites, const int* coords, const double2* P, int nrhs, const double* dirs, int ndir,
                     double k, const int lo[3], const int n[3], double2* f, double* dcs, hipStream_t s) {
    const size_t nt = (size_t)(n[0] + n[1] + n[2]);
    const int npair = (nrhs + 1) / 2;   // grid y: the right-hand sides two at a time
    if ((long long)((ndir + FF_DW - 1) / FF_DW) * npair >= FF_MIN_WG) {
        hipLaunchKernelGGL((k_farfield<FF_DW, 2>), dim3((ndir + FF_DW - 1) / FF_DW, npair), dim3(NT),
                           FF_DW * nt * sizeof(double2), s, nsites, coords, P, 3LL * nsites, nrhs, dirs, k, lo[0],
                           lo[1], lo[2], n[0], n[1], n[2], f, dcs, ndir, 0);
    } else {
        hipLaunchKernelGGL((k_farfield<1, 2>), dim3(ndir, npair), dim3(NT), nt * sizeof(double2), s, nsites, coords,
                           P, 3LL * nsites, nrhs, dirs, k, lo[0], lo[1], lo[2], n[0], n[1], n[2], f, dcs, ndir, 0);
    }
}
void launch_avg_dirs(int ng, const double* kh, const double* mu, int n_theta, int n_phi, double* dirs,
                     hipStream_t s) {
    const long long tot = (long long)ng * n_theta * n_phi;
    hipLaunchKernelGGL(k_avg_dirs, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, s, ng, kh, mu, n_theta, n_phi,
                       dirs);
}
void launch_farfield_sets(int nsites, const int* coords, const double2* P, int nrhs, const double* dirs, int per,
                          double k, const int lo[3], const int n[3], double2* f, double* dcs, hipStream_t s) {
    const size_t nt = (size_t)(n[0] + n[1] + n[2]);
    const int ndt = per * nrhs;
    if (per % FF_DW == 0 && ndt >= FF_DW * FF_MIN_WG) {
        hipLaunchKernelGGL((k_farfield<FF_DW, 1>), dim3(ndt / FF_DW), dim3(NT), FF_DW * nt * sizeof(double2), s, nsites,
                           coords, P, 3LL * nsites, nrhs, dirs, k, lo[0], lo[1], lo[2], n[0], n[1], n[2], f, dcs,
                           ndt, per);
    } else {
        hipLaunchKernelGGL((k_farfield<1, 1>), dim3(ndt), dim3(NT), nt * sizeof(double2), s, nsites, coords, P,
                           3LL * nsites, nrhs, dirs, k, lo[0], lo[1], lo[2], n[0], n[1], n[2], f, dcs, ndt, per);
    }
}
void launch_nf_place(int nsites, const int* perm, const int* coords, const double2* P, int nrhs, const int org[3],
                     const int dims[3], double2* x, hipStream_t s) {
    const long long n3x = 3LL * dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_nf_place, dim3(blocks_for(nsites, 4096), nrhs), dim3(NT), 0, s, nsites, perm, coords, P,
                       org[0], org[1], org[2], dims[0], dims[1], n3x, x);
}
void launch_nf_out(int nrhs, const int org[3], const int dims[3], const double* khat, const double2* e0, double kd,
                   const double2* v, double2* einc, double2* esca, hipStream_t s) {
    const long long npts = (long long)dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_nf_out, dim3(blocks_for(npts, 4096), nrhs), dim3(NT), 0, s, npts, org[0], org[1], org[2],
                       dims[0], dims[1], khat, e0, kd, v, einc, esca);
}
void launch_field_line(int nrhs, const int org[3], const int dims[3], const double2* E, const double a[3],
                       const double b[3], int n, double2* out, hipStream_t s) {
    hipLaunchKernelGGL(k_field_line, dim3(blocks_for(n, 1024), nrhs), dim3(NT), 0, s, E, org[0], org[1], org[2],
                       dims[0], dims[1], dims[2], a[0], a[1], a[2], b[0], b[1], b[2], n, out);
}
void launch_qsum(const SiteArgs& a, int site_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_qsum, dim3(site_blocks, a.nrhs), dim3(NT), 0, s, a);
}
void launch_finalize(const SiteArgs& a, int kind, int nblk, hipStream_t s) {
    // the largest count a right-hand side can have: its own, or in a ragged
    // batch the launch's (a.maxblk)
    const int most = nblk >= 0 ? nblk : a.maxblk;
    const int chained = a.chains && nblk != 0 && most >= FIN_CHAIN_MIN;
    if (chained)
        hipLaunchKernelGGL(k_chain_sums, dim3(fin_slots(kind), a.nrhs), dim3(NT), 0, s, a, nblk);
    hipLaunchKernelGGL(k_finalize, dim3(a.nrhs), dim3(NT), 0, s, a, kind, nblk, chained);
}

void launch_permute(int nrhs, int nsites, int width, const int* perm, const double2* src, double2* dst,
                    bool to_sorted, hipStream_t s) {
    const long long tot = (long long)nrhs * nsites * width;
    hipLaunchKernelGGL(k_permute, dim3(blocks_for(tot, 4096)), dim3(NT), 0, s, nrhs, nsites, width, perm, src, dst,
                       to_sorted ? 1 : 0);
}

void launch_fill(double2* p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 4096)), dim3(NT), 0, s, p, n);
}

void launch_set_state(RhsState* st, int nrhs, double tol, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_set_state, dim3((nrhs + 63) / 64), dim3(64), 0, s, st, nrhs, tol * tol, max_iter);
}

void launch_adjoint_rhs(const SiteArgs& a, const double2* P_sorted, double w_qabs, double w_qext, hipStream_t s) {
    const double pi = 3.14159265358979323846;
    const double aeff = cbrt(3.0 * a.nsites / (4.0 * pi));
    const double cq = 4.0 * pi * a.kd / (pi * aeff * aeff);
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(blocks_for(a.n3, 4096)), dim3(NT), 0, s, a, P_sorted, cq * w_qabs,
                       cq * w_qext);
}

void launch_grad(const SiteArgs& a, const double2* dainv, double w_qabs, double2* grad, hipStream_t s) {
    const double pi = 3.14159265358979323846;
    const double aeff = cbrt(3.0 * a.nsites / (4.0 * pi));
    const double cq = 4.0 * pi * a.kd / (pi * aeff * aeff);
    // P (sorted) is passed in a.in
    hipLaunchKernelGGL(k_grad, dim3(blocks_for(a.nsites, 4096)), dim3(NT), 0, s, a, a.in, dainv, cq * w_qabs, grad);
}

}  // namespace dda
