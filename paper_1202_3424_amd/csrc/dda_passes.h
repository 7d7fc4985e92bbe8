// The five passes of the FFT matrix-vector product y = A x, as kernel
// templates instantiated per grid precision (dda_passes_f64.hip,
// dda_passes_f32.hip).
//
// A = the interaction matrix of Draine (1988) plus the diagonal 1/alpha
// ("Dipole Polarizabilities"); the product is a convolution on a zero-padded
// grid (Goodman, Draine & Flatau 1990; "Choice of FFT Algorithm"), evaluated
// in five pruned passes over three interleaved component grids:
//   1. scatter + forward FFT along x of the occupied (y < ny, z < nz) lines
//   2. forward FFT along y of the z < nz planes (inputs y < ny only)
//   3. along z for every (x, y): forward FFT of the z < nz inputs, product
//      with the symmetric 3x3 tensor FFT, inverse FFT, keep z < nz
//   4. inverse FFT along y of the z < nz planes, keep y < ny
//   5. inverse FFT along x, gather the occupied sites, add 1/alpha x.
// Passes 1 and 5 also carry the BiCGSTAB vector updates and the partial sums
// of the inner products that touch the same sites.
//
// Each kernel has two forms.  For the FFT lengths in CT_LENGTHS the length,
// the tile shape and the radix plan are compile-time constants (index
// arithmetic folds to shifts and multiplies); the x passes then run one
// x-line (three components) per workgroup of one or two wavefronts.  Other lengths use the
// runtime plan with twiddles staged in LDS.
#pragma once

#include <stdexcept>
#include <type_traits>

#include "dda_kernels.h"

namespace dda {
namespace passes {

// lengths with compile-time kernels
#define DDA_CT_LENGTHS(X) X(32) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(384) X(512)

// x columns per workgroup of a compile-time strided pass: a tile of about
// 1536 complex values (three components per column)
constexpr int ct_cols(int L) {
    if (L <= 0) return 1;
    int tx = 1536 / (3 * L);
    int p = 1;
    while (p * 2 <= tx && p * 2 <= 16) p *= 2;
    return p;
}
// threads of a compile-time x-pass workgroup: one wavefront up to length
// 128, two beyond (a line of 3 x 256 values gives one wavefront 12 elements
// per thread, which serialises its dependent map and site loads)
constexpr int xthr(int L) { return L > 128 ? 128 : 64; }

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

__device__ __forceinline__ bool skip_rhs(const RhsState* st, int chk) {
    return chk != CHK_NONE && st->status != ST_ACTIVE;
}

// g_a X + g_b Y + g_c Z for one row of the symmetric tensor product, each
// part one expression so that it contracts to a multiply and five fused
// multiply-adds (every pass-3 form uses this, so all stay bitwise identical)
template <typename C>
__device__ __forceinline__ C trow(const C& ga, const C& gb, const C& gc, const C& X, const C& Y, const C& Z) {
    C r;
    r.x = ga.x * X.x - ga.y * X.y + gb.x * Y.x - gb.y * Y.y + gc.x * Z.x - gc.y * Z.y;
    r.y = ga.x * X.y + ga.y * X.x + gb.x * Y.y + gb.y * Y.x + gc.x * Z.y + gc.y * Z.x;
    return r;
}

inline __host__ __device__ int pad_len(int L) { return L | 1; }
inline __host__ __device__ int even_up(int L) { return (L + 1) & ~1; }

// LDS of a runtime-length kernel: [twiddles (L)][tile (nlines * Lp)][scratch];
// of a compile-time kernel: [tile][scratch].
template <typename C> inline size_t smem_rt(int L, int nlines) {
    return ((size_t)even_up(L) + (size_t)nlines * pad_len(L)) * sizeof(C) + 8 * (NT / 64) * sizeof(double) + 64;
}
template <typename C> inline size_t smem_ct(int L, int nlines) {
    return (size_t)nlines * pad_len(L) * sizeof(C) + 8 * (NT / 64) * sizeof(double) + 64;
}

// ------------------------------------------------------------------ pass 1

template <typename T, int MODE, int LC, int NTHR>
__global__ __launch_bounds__(NTHR) void k_scatter_x(Geo g, SiteArgs a, typename V2<T>::t* grid, const double2* tw64,
                                                   int XLrt, int chk) {
    using C = typename V2<T>::t;
    constexpr bool CT = LC > 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int q = blockIdx.z;
    const RhsState* st = a.st + q;
    if (skip_rhs(st, chk)) return;
    int nx = g.n[0], ny = g.n[1];
    const int* map = a.map;
    const int Mx = CT ? LC : g.M[0];
    const int My = g.M[1];
    const int XL = CT ? 1 : XLrt;
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * XL;
    // the workgroups of one right-hand side along y, and its partial-sum index
    int bx = gridDim.x;
    if (a.rg) {   // ragged batch: this right-hand side's target
        const RhsGeo& r = a.rg[q];
        if (z >= r.n[2] || y0 >= r.n[1]) return;
        nx = r.n[0];
        ny = r.n[1];
        map += r.map_off;
        bx = (ny + XL - 1) / XL;
    }
    const int nl = CT ? 1 : min(XL, ny - y0);
    const int nlines = 3 * nl;
    const int Lp = pad_len(Mx);
    C* lds;
    C* tws = nullptr;
    if constexpr (CT) {
        lds = (C*)smem;
    } else {
        tws = (C*)smem;
        lds = tws + even_up(Mx);
        load_twiddles<T, NTHR>(tws, tw64, g.ax[0]);
    }
    double2 beta = {0, 0}, omega = {0, 0}, alpha = {0, 0};
    double w_old = 0.0, w_new = 0.0;
    int pend = 0;
    if (MODE == SC_P) { beta = st->beta; omega = st->omega; alpha = st->alpha; pend = st->pend; }
    if (MODE == SC_S) alpha = st->alpha;
    if (MODE == SC_Q) { beta = st->beta; w_old = st->w_old; w_new = st->w_new; }
    if (MODE == SC_B0 || MODE == SC_B2) beta = st->beta;
    if (MODE == SC_B1 || MODE == SC_B3) alpha = st->alpha;
    const long long vb = (long long)q * a.n3;
    const int* mrow = map + ((long long)z * ny + y0) * nx;
    double ss[3] = {0.0, 0.0, 0.0};
    // forward transform of a line that is zero beyond nx: with 2 nx <= Mx the
    // first radix pass never reads the upper half, which is then not filled
    // (always so at the compile-time lengths, which are even and >= 2 nx - 1)
    bool hin = false;
    if constexpr (CT) hin = ct_half_in_ok(LC) && 2 * nx <= Mx;
    const int ext = hin ? Mx / 2 : Mx;
    const int tin = nl * ext * 3;
    // the site-vector values this mode reads at element i (all of them are
    // loaded before any update is stored, so that the loads of every element
    // a thread fills are in flight together)
    struct Ops {
        double2 o[6];
    };
    auto load_ops = [&](long long i) {
        Ops v;
        if (MODE == SC_PLAIN || MODE == SC_CONJ) {
            v.o[0] = a.in[i];
        } else if (MODE == SC_P) {
            v.o[0] = a.r[i]; v.o[1] = a.p[i]; v.o[2] = a.v[i]; v.o[3] = a.x[i]; v.o[4] = a.t[i];
        } else if (MODE == SC_B0) {
            v.o[0] = a.r[i]; v.o[1] = a.p[i];
        } else if (MODE == SC_B1) {
            v.o[0] = a.r[i]; v.o[1] = a.v[i]; v.o[2] = a.x[i]; v.o[3] = a.p[i];
        } else if (MODE == SC_B2) {
            v.o[0] = a.r[i]; v.o[1] = a.p[i]; v.o[2] = a.t[i]; v.o[3] = a.v[i];
        } else if (MODE == SC_B3) {
            v.o[0] = a.r[i]; v.o[1] = a.v[i]; v.o[2] = a.t[i]; v.o[3] = a.u2[i]; v.o[4] = a.x[i]; v.o[5] = a.p[i];
        } else if (MODE == SC_Q) {
            v.o[0] = a.r[i]; v.o[1] = a.p[i]; v.o[2] = a.rhat[i]; v.o[3] = a.t[i]; v.o[4] = a.x[i];
        } else {   // SC_S
            v.o[0] = a.r[i]; v.o[1] = a.v[i]; v.o[2] = a.rhat[i];
        }
        return v;
    };
    // the product's input at element i after this mode's vector update from
    // the loaded values v, the update stored back (and summed) only where
    // `live` (a site of this line; elsewhere the value is unused)
    auto update = [&](long long i, const Ops& v, bool live) -> double2 {
        double2 u;
        if (MODE == SC_PLAIN) {
            u = v.o[0];
        } else if (MODE == SC_CONJ) {
            u = cconj(v.o[0]);
        } else if (MODE == SC_P) {
            // the previous iteration's end, if pending: x += alpha p + omega
            // s, r = s - omega t (s is held in r); then p = r + beta (p -
            // omega v)
            double2 rr = v.o[0];
            const double2 pp = v.o[1];
            if (pend) {
                const double2 xx = cadd(cadd(v.o[3], cmul(alpha, pp)), cmul(omega, rr));
                rr = csub(rr, cmul(omega, v.o[4]));
                if (live) {
                    a.x[i] = xx;
                    a.r[i] = rr;
                }
            }
            u = cadd(rr, cmul(beta, csub(pp, cmul(omega, v.o[2]))));
            if (live) a.p[i] = u;
        } else if (MODE == SC_B0) {
            // BiCGstab(2), first BiCG step: u_0 = r_0 - beta u_0
            u = csub(v.o[0], cmul(beta, v.o[1]));
            if (live) a.p[i] = u;
        } else if (MODE == SC_B1) {
            // r_0 -= alpha u_1, x += alpha u_0; product of r_0
            u = csub(v.o[0], cmul(alpha, v.o[1]));
            if (live) {
                a.r[i] = u;
                a.x[i] = cadd(v.o[2], cmul(alpha, v.o[3]));
            }
        } else if (MODE == SC_B2) {
            // second BiCG step: u_0 = r_0 - beta u_0, u_1 = r_1 - beta u_1; product of u_1
            u = csub(v.o[2], cmul(beta, v.o[3]));
            if (live) {
                a.p[i] = csub(v.o[0], cmul(beta, v.o[1]));
                a.v[i] = u;
            }
        } else if (MODE == SC_B3) {
            // r_0 -= alpha u_1, r_1 -= alpha u_2, x += alpha u_0; product of r_1
            u = csub(v.o[2], cmul(alpha, v.o[3]));
            if (live) {
                a.r[i] = csub(v.o[0], cmul(alpha, v.o[1]));
                a.t[i] = u;
                a.x[i] = cadd(v.o[4], cmul(alpha, v.o[5]));
            }
        } else if (MODE == SC_Q) {
            // QMR: p = r + beta p, and the pending smoothing step
            // (y, s) <- w_old (y, s) + w_new (x, r)
            const double2 rr = v.o[0];
            u = cadd(rr, cmul(beta, v.o[1]));
            if (live) {
                const double2 sm = v.o[2], ym = v.o[3], xx = v.o[4];
                a.p[i] = u;
                a.rhat[i] = double2{w_old * sm.x + w_new * rr.x, w_old * sm.y + w_new * rr.y};
                a.t[i] = double2{w_old * ym.x + w_new * xx.x, w_old * ym.y + w_new * xx.y};
            }
        } else {
            // s = r - alpha v, stored over r; |s|^2 and <rhat, s>
            u = csub(v.o[0], cmul(alpha, v.o[1]));
            if (live) {
                const double2 w = cdotc(v.o[2], u);
                a.r[i] = u;
                ss[0] += u.x * u.x + u.y * u.y;
                ss[1] += w.x;
                ss[2] += w.y;
            }
        }
        return u;
    };
    if constexpr (CT) {
        // one line: the site indices of every element this thread fills are
        // loaded first, then every operand (clamped to site 0 where there is
        // no site), so that the loads of all elements are in flight together
        constexpr int EXT = ct_half_in_ok(LC) ? LC / 2 : LC;
        constexpr int NPT = (3 * EXT + NTHR - 1) / NTHR;
        int sk[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            const int e = idx / 3;
            sk[k] = (idx < tin && e < nx) ? mrow[e] : -1;
        }
        Ops ok[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            ok[k] = load_ops(vb + (long long)(sk[k] >= 0 ? sk[k] : 0) * 3 + idx % 3);
        }
        double2 uk[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            const bool live = sk[k] >= 0;
            uk[k] = update(vb + (long long)(live ? sk[k] : 0) * 3 + idx % 3, ok[k], live);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            if (idx < tin) {
                C val;
                val.x = 0;
                val.y = 0;
                if (sk[k] >= 0) val = to_c<C>(uk[k]);
                lds[(idx % 3) * Lp + idx / 3] = val;
            }
        }
        // (a full-length input, never the case at these even lengths: zeros
        // beyond the half)
        for (int idx = 3 * EXT + threadIdx.x; idx < tin; idx += NTHR) {
            C val;
            val.x = 0;
            val.y = 0;
            lds[(idx % 3) * Lp + idx / 3] = val;
        }
    } else {
        for (int idx = threadIdx.x; idx < tin; idx += NTHR) {
            const int c = idx % 3;
            const int rest = idx / 3;
            const int e = rest % ext;
            const int yo = rest / ext;
            C val;
            val.x = 0;
            val.y = 0;
            if (e < nx) {
                const int s = mrow[yo * nx + e];
                if (s >= 0) {
                    const long long i = vb + (long long)s * 3 + c;
                    val = to_c<C>(update(i, load_ops(i), true));
                }
            }
            lds[(yo * 3 + c) * Lp + e] = val;
        }
    }
    __syncthreads();
    if constexpr (CT) {
        if (hin) fft_lines_ct<T, -1, LC, 3, NTHR, true, false>(lds, tw64 + g.ax[0].tw);
        else fft_lines_ct<T, -1, LC, 3, NTHR>(lds, tw64 + g.ax[0].tw);
    } else {
        fft_lines<T, -1, NTHR>(lds, tws, nlines, Lp, g.ax[0]);
    }
    C* gq = grid + ((long long)q * g.npts + ((long long)z * My + y0) * Mx) * 3;
    if constexpr (CT) {
        constexpr int NPT = (3 * LC + NTHR - 1) / NTHR;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            if ((3 * LC) % NTHR == 0 || idx < 3 * LC) gq[idx] = lds[(idx % 3) * Lp + idx / 3];
        }
    } else {
        const int tot = nl * Mx * 3;
        for (int idx = threadIdx.x; idx < tot; idx += NTHR) {
            const int c = idx % 3;
            const int rest = idx / 3;
            const int e = rest % Mx;
            const int yo = rest / Mx;
            gq[idx] = lds[(yo * 3 + c) * Lp + e];
        }
    }
    if (MODE == SC_S) {
        // slots 5-7 of the block's entry; the gather of t (same grid) fills
        // slots 0-4 and one finalize reads both
        double* sh = (double*)(lds + nlines * Lp);
        const int blk = blockIdx.y * bx + blockIdx.x;
        publish_partial<3, NTHR, 5>(ss, a.partials + (long long)q * a.maxblk * PSTRIDE, blk, a.maxblk, sh);
    }
}

// ------------------------------------------------------------------ pass 5

// PRE (compile-time lengths): each element's site operands are loaded
// before the inverse transform, so their latency overlaps it, at the price
// of the registers that hold them (fewer waves per SIMD); else after it.
template <typename T, int MODE, int LC, int NTHR, bool PRE = false>
__global__ __launch_bounds__(NTHR) void k_gather_x(Geo g, SiteArgs a, const typename V2<T>::t* grid,
                                                  const double2* tw64, int XLrt, int chk) {
    using C = typename V2<T>::t;
    constexpr bool CT = LC > 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const int q = blockIdx.z;
    const RhsState* st = a.st + q;
    if (skip_rhs(st, chk)) return;
    int nx = g.n[0], ny = g.n[1];
    const int* map = a.map;
    const int* mat = a.mat;
    const int Mx = CT ? LC : g.M[0];
    const int My = g.M[1];
    const int XL = CT ? 1 : XLrt;
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * XL;
    int bx = gridDim.x;
    if (a.rg) {   // ragged batch: this right-hand side's target
        const RhsGeo& r = a.rg[q];
        if (z >= r.n[2] || y0 >= r.n[1]) return;
        nx = r.n[0];
        ny = r.n[1];
        map += r.map_off;
        mat += r.site_off;
        bx = (ny + XL - 1) / XL;
    }
    const int nl = CT ? 1 : min(XL, ny - y0);
    const int nlines = 3 * nl;
    const int Lp = pad_len(Mx);
    C* lds;
    C* tws = nullptr;
    if constexpr (CT) {
        lds = (C*)smem;
    } else {
        tws = (C*)smem;
        lds = tws + even_up(Mx);
        load_twiddles<T, NTHR>(tws, tw64, g.ax[0]);
    }
    const int* mrow = map + ((long long)z * ny + y0) * nx;
    const int tout = nl * nx * 3;
    // compile-time lengths (one line per workgroup): the site index and
    // material of each element this thread gathers are loaded before the
    // transform, so only the operand loads follow it (e < nx <= (L + 1) / 2
    // since L >= 2 nx - 1)
    constexpr int PF = CT ? (3 * ((LC + 1) / 2) + NTHR - 1) / NTHR : 1;
    int ps[PF], pm[PF];
    if constexpr (CT) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            ps[k] = idx < tout ? mrow[idx / 3] : -1;
        }
    }
    const C* gq = grid + ((long long)q * g.npts + ((long long)z * My + y0) * Mx) * 3;
    if constexpr (CT) {
        // the line's 3 LC values: every load in flight before the LDS stores
        // (unrolled: the loads need not wait for one another)
        constexpr int NPT = (3 * LC + NTHR - 1) / NTHR;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            if ((3 * LC) % NTHR == 0 || idx < 3 * LC) lds[(idx % 3) * Lp + idx / 3] = gq[idx];
        }
    } else {
        const int tot = nl * Mx * 3;
        for (int idx = threadIdx.x; idx < tot; idx += NTHR) {
            const int c = idx % 3;
            const int rest = idx / 3;
            const int e = rest % Mx;
            const int yo = rest / Mx;
            lds[(yo * 3 + c) * Lp + e] = gq[idx];
        }
    }
    // the site operands of the gathered elements (what each mode reads
    // besides the product), loaded before the transform so that their
    // latency overlaps it
    const long long vb = (long long)q * a.n3;
    auto operand = [&](long long i) -> double2 {
        if (MODE == GA_PLAIN || MODE == GA_CONJ) return a.in[i];
        if (MODE == GA_V || MODE == GA_Q) return a.p[i];
        if (MODE == GA_T || MODE == GA_B1) return a.r[i];
        if (MODE == GA_RES) return a.x[i];
        if (MODE == GA_B2) return a.v[i];
        return a.t[i];   // GA_B3
    };
    constexpr bool HAS_AUX = MODE == GA_V || MODE == GA_T || MODE == GA_B1 || MODE == GA_B2 || MODE == GA_B3 ||
                             MODE == GA_RES;
    auto auxiliary = [&](long long i) -> double2 {
        if (MODE == GA_RES) return a.b[i];
        if (MODE == GA_B3) return a.r[i];
        return a.rhat[i];
    };
    double2 px[PF], pa[PF];
    if constexpr (CT && PRE) {
        // (clamped to site 0 where there is no site: the value is unused)
#pragma unroll
        for (int k = 0; k < PF; ++k) pm[k] = mat[ps[k] >= 0 ? ps[k] : 0];
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            const long long i = vb + (long long)(ps[k] >= 0 ? ps[k] : 0) * 3 + idx % 3;
            px[k] = operand(i);
            pa[k] = HAS_AUX ? auxiliary(i) : double2{0.0, 0.0};
        }
    }
    __syncthreads();
    if constexpr (CT) {
        // only e < nx is gathered: with 2 nx <= Mx the last pass skips the upper half
        if (ct_half_out_ok(LC) && 2 * nx <= Mx) fft_lines_ct<T, 1, LC, 3, NTHR, false, true>(lds, tw64 + g.ax[0].tw);
        else fft_lines_ct<T, 1, LC, 3, NTHR>(lds, tw64 + g.ax[0].tw);
    } else {
        fft_lines<T, 1, NTHR>(lds, tws, nlines, Lp, g.ax[0]);
    }

    const double2* ai = a.ainv + (long long)q * a.nmat * 3;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // element (line yo, point e, component c) at site s of material mt, with
    // its operand xo and auxiliary vector value xa (as loaded)
    auto site = [&](int c, int e, int yo, int s, int mt, double2 xo, double2 xa) {
        const long long i = vb + (long long)s * 3 + c;
        const double2 gv = to_d(lds[(yo * 3 + c) * Lp + e]);
        const double2 d = ai[mt * 3 + c];
        const double2 xin = MODE == GA_CONJ ? cconj(xo) : xo;
        const double2 y = cadd(gv, cmul(d, xin));
        if (MODE == GA_PLAIN) {
            a.out[i] = y;
        } else if (MODE == GA_CONJ) {
            const double2 yc = cconj(y);
            a.out[i] = yc;
            acc[0] += yc.x * yc.x + yc.y * yc.y;
        } else if (MODE == GA_V) {
            a.v[i] = y;
            const double2 w = cdotc(xa, y);
            acc[0] += w.x;
            acc[1] += w.y;
            acc[2] += y.x * y.x + y.y * y.y;   // |v|^2: bounds <rhat, v> with |rhat|
        } else if (MODE == GA_T) {
            a.t[i] = y;
            const double2 w = cdotc(y, xin);    // <t, s>
            const double2 wr = cdotc(xa, y);    // <rhat, t>
            acc[0] += w.x;
            acc[1] += w.y;
            acc[2] += y.x * y.x + y.y * y.y;
            acc[3] += wr.x;
            acc[4] += wr.y;
        } else if (MODE == GA_Q) {
            a.v[i] = y;
            acc[0] += xin.x * y.x - xin.y * y.y;   // p^T v (bilinear)
            acc[1] += xin.x * y.y + xin.y * y.x;
            acc[2] += y.x * y.x + y.y * y.y;       // |v|^2 and |p|^2 bound |p^T v|
            acc[3] += xin.x * xin.x + xin.y * xin.y;
        } else if (MODE == GA_B1 || MODE == GA_B2) {
            // r_1 = A r_0 or u_2 = A u_1, and <rhat, .>
            if (MODE == GA_B1) a.t[i] = y;
            else a.u2[i] = y;
            const double2 w = cdotc(xa, y);
            acc[0] += w.x;
            acc[1] += w.y;
            acc[2] += y.x * y.x + y.y * y.y;
        } else if (MODE == GA_B3) {
            // r_2 = A r_1 and the minimal-residual sums |r_1|^2, <r_1, r_2>,
            // |r_2|^2, <r_1, r_0>, <r_2, r_0>
            a.r2[i] = y;
            const double2 r0 = xa;
            const double2 w12 = cdotc(xin, y), w10 = cdotc(xin, r0), w20 = cdotc(y, r0);
            acc[0] += xin.x * xin.x + xin.y * xin.y;
            acc[1] += w12.x;
            acc[2] += w12.y;
            acc[3] += y.x * y.x + y.y * y.y;
            acc[4] += w10.x;
            acc[5] += w10.y;
            acc[6] += w20.x;
            acc[7] += w20.y;
        } else {
            const double2 rr = csub(xa, y);
            a.r[i] = rr;
            acc[0] += rr.x * rr.x + rr.y * rr.y;
        }
    };
    if constexpr (CT) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int idx = threadIdx.x + k * NTHR;
            if (idx < tout && ps[k] >= 0) {
                if constexpr (PRE) {
                    site(idx % 3, idx / 3, 0, ps[k], pm[k], px[k], pa[k]);
                } else {
                    const long long i = vb + (long long)ps[k] * 3 + idx % 3;
                    site(idx % 3, idx / 3, 0, ps[k], pm[k], operand(i),
                         HAS_AUX ? auxiliary(i) : double2{0.0, 0.0});
                }
            }
        }
    } else {
        for (int idx = threadIdx.x; idx < tout; idx += NTHR) {
            const int c = idx % 3;
            const int rest = idx / 3;
            const int e = rest % nx;
            const int yo = rest / nx;
            const int s = mrow[yo * nx + e];
            if (s >= 0) {
                const long long i = vb + (long long)s * 3 + c;
                site(c, e, yo, s, mat[s], operand(i), HAS_AUX ? auxiliary(i) : double2{0.0, 0.0});
            }
        }
    }
    if (MODE != GA_PLAIN) {
        double* sh = (double*)(lds + nlines * Lp);
        const int blk = blockIdx.y * bx + blockIdx.x;
        if constexpr (MODE == GA_B3) {
            publish_partial<8, NTHR>(acc, a.partials + (long long)q * a.maxblk * PSTRIDE, blk, a.maxblk, sh);
        } else if constexpr (MODE == GA_T) {
            double a5[5] = {acc[0], acc[1], acc[2], acc[3], acc[4]};
            publish_partial<5, NTHR>(a5, a.partials + (long long)q * a.maxblk * PSTRIDE, blk, a.maxblk, sh);
        } else if constexpr (MODE == GA_Q) {
            double a4[4] = {acc[0], acc[1], acc[2], acc[3]};
            publish_partial<4, NTHR>(a4, a.partials + (long long)q * a.maxblk * PSTRIDE, blk, a.maxblk, sh);
        } else {
            double a3[3] = {acc[0], acc[1], acc[2]};
            publish_partial<3, NTHR>(a3, a.partials + (long long)q * a.maxblk * PSTRIDE, blk, a.maxblk, sh);
        }
    }
}

// ------------------------------------------------------------------ passes 2-4

// Right-hand side q of a strided pass in a ragged batch (g.rg): the y passes
// (axis 1) cover the planes z < n_z of its target (false beyond) and read its
// y < n_y (forward) or write them (inverse); pass 3 (axis 2) reads and writes
// z < n_z with its target's tensor.  Unchanged for a single target.
template <typename C>
__device__ __forceinline__ bool ragged_lines(const Geo& g, int q, int axis, int dir, int o, int& lin, int& lout,
                                             const C*& gh) {
    if (!g.rg) return true;
    const RhsGeo& r = g.rg[q];
    if (axis == 1) {
        if (o >= r.n[2]) return false;
        if (dir < 0) lin = r.n[1];
        else lout = r.n[1];
    } else {
        lin = lout = r.n[2];
        gh = (const C*)r.ghat[sizeof(C) == sizeof(float2) ? 1 : 0];
    }
    return true;
}

// XCD-grouped workgroup order of pass 3: the grid is one-dimensional and
// ordered so that the workgroups sharing tensor values -- the column tiles x
// and Mx - x, the rows y and My - y, every right-hand side -- run
// consecutively on one XCD (workgroups go to the eight XCDs round-robin),
// so each XCD's L2 serves the repeats and the tensor is read from HBM about
// once per launch.  Returns false for the padding workgroups and for the
// mirror copies of self-mirrored tiles (done by the unmirrored one).
constexpr int N_XCD = 8;
__device__ __forceinline__ bool xcd_tile(int Mx, int My, int TX, int nrhs, int& xt, int& o, int& q) {
    const int ntx = (Mx + TX - 1) / TX;
    const int nxp = (ntx + 1) / 2, nyp = My / 2 + 1;
    const int mg = 4 * nrhs;
    const int w = blockIdx.x;
    const int local = w / N_XCD;
    const int gi = (local / mg) * N_XCD + w % N_XCD;
    const int m = local % mg;
    if (gi >= nxp * nyp) return false;
    const int xi = gi % nxp, yi = gi / nxp;
    const int mir = m / nrhs;
    q = m % nrhs;
    xt = (mir & 1) ? ntx - 1 - xi : xi;
    o = (mir & 2) ? (My - yi) % My : yi;
    return !(((mir & 1) && xt == xi) || ((mir & 2) && o == yi));
}
// XCD-contiguous order of a y pass (one-dimensional launch): XCD j takes
// the tiles [j C, (j + 1) C) of the (right-hand side, plane, x tile)
// row-major order, C the tiles over eight, in that order, so neighbouring x
// tiles -- which share the cache lines at their edges -- run together on one
// XCD and meet in its L2.  False for the padding workgroups.
__device__ __forceinline__ bool xcd_rows(int ntx, int n_outer, int nrhs, int& xt, int& o, int& q) {
    const long long total = (long long)ntx * n_outer * nrhs;
    const long long chunk = (total + N_XCD - 1) / N_XCD;
    const long long t = (long long)(blockIdx.x % N_XCD) * chunk + blockIdx.x / N_XCD;
    if (t >= total) return false;
    xt = (int)(t % ntx);
    o = (int)((t / ntx) % n_outer);
    q = (int)(t / ((long long)ntx * n_outer));
    return true;
}
inline unsigned xcd_rows_grid(int ntx, int n_outer, int nrhs) {
    const long long total = (long long)ntx * n_outer * nrhs;
    return (unsigned)(((total + N_XCD - 1) / N_XCD) * N_XCD);
}
inline unsigned xcd_grid(int Mx, int My, int TX, int nrhs) {
    const long long groups = (long long)(((Mx + TX - 1) / TX + 1) / 2) * (My / 2 + 1);
    return (unsigned)(((groups + N_XCD - 1) / N_XCD) * N_XCD * 4 * nrhs);
}

// Strided FFT along axis 1 (y, outer index = z) or 2 (z, outer index = y)
// over TX adjacent x columns times NC components.  With GH: forward FFT, the
// tensor product, inverse FFT.  Variants of the GH form (VAR):
//   0  the workgroup handles every right-hand side in turn, its tensor values
//      read once and kept in registers;
//   1  every right-hand side in turn, tensor values re-read (cache) each time;
//   2  one right-hand side per workgroup (grid z, or the XCD-grouped order
//      of xcd_tile with XG), tensor values read.
// TXC is the compile-time tile width (x columns).
template <typename T, int NC, int GH, int DIR, int LC, int TXC = 1, int VAR = 0, bool XG = false>
__global__ __launch_bounds__(NT) void k_strided(Geo g, typename V2<T>::t* grid, const double2* tw64,
                                               const typename V2<T>::t* ghat, const RhsState* st, int nrhs,
                                               int axis, int TXrt, int lin, int lout, int chk) {
    using C = typename V2<T>::t;
    constexpr bool CT = LC > 0;
    constexpr bool RHS_LOOP = GH && VAR != 2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mx = g.M[0], My = g.M[1];
    const AxisPlan& pl = g.ax[axis];
    const int L = CT ? LC : pl.L;
    const int TX = CT ? TXC : TXrt;
    const int Lp = pad_len(L);
    int xt = blockIdx.x, o = blockIdx.y, qx = blockIdx.z;
    if constexpr (XG) {
        static_assert(!XG || (GH && VAR == 2 && LC > 0), "XCD order: pass 3, one right-hand side per workgroup");
        if (!xcd_tile(Mx, My, TX, nrhs, xt, o, qx)) return;
    }
    const int x0 = xt * TX;
    const int nxl = min(TX, Mx - x0);
    const int nlines = NC * TX;   // lines beyond nxl hold zeros and are not stored
    const long long estride = (axis == 1) ? (long long)Mx * NC : (long long)My * Mx * NC;
    const long long obase = (axis == 1) ? (long long)o * My * Mx * NC : (long long)o * Mx * NC;
    C* lds;
    C* tws = nullptr;
    if constexpr (CT) {
        lds = (C*)smem;
    } else {
        tws = (C*)smem;
        lds = tws + even_up(L);
        load_twiddles<T>(tws, tw64, pl);
    }
    const int nval = NC * nxl;
    // tensor values of this thread's points (GH, compile-time form)
    constexpr int MAXP = CT ? (TXC * LC + NT - 1) / NT : 1;
    C G[MAXP][6];
    const int Hx = g.H[0], Hy = g.H[1];
    const int Mz = g.M[2];
    const int ky = o;
    const int fy = (ky <= My / 2) ? ky : My - ky;
    const int sy = (ky <= My / 2) ? 1 : -1;
    auto tensor_at = [&](int xo, int kz, C* out6) {
        const int kx = x0 + xo;
        const int fx = (kx <= Mx / 2) ? kx : Mx - kx;
        const int sx = (kx <= Mx / 2) ? 1 : -1;
        const int fz = (kz <= Mz / 2) ? kz : Mz - kz;
        const int sz = (kz <= Mz / 2) ? 1 : -1;
        const C* Gp = ghat + (((long long)fz * Hy + fy) * Hx + fx) * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) out6[c] = Gp[c];
        // diagonal components are even in every index, ab is odd in a and b
        if (sx * sy < 0) { out6[1].x = -out6[1].x; out6[1].y = -out6[1].y; }
        if (sx * sz < 0) { out6[2].x = -out6[2].x; out6[2].y = -out6[2].y; }
        if (sy * sz < 0) { out6[4].x = -out6[4].x; out6[4].y = -out6[4].y; }
    };
    if constexpr (GH && CT && VAR == 0) {
#pragma unroll
        for (int i = 0; i < MAXP; ++i) {
            const int p = threadIdx.x + i * NT;
            if (p < TX * L) {
                const int xo = p % TX;
                const int kz = p / TX;
                if (xo < nxl) tensor_at(xo, kz, G[i]);
            }
        }
    }
    const int q0 = RHS_LOOP ? 0 : qx;
    const int q1 = RHS_LOOP ? nrhs : qx + 1;
    // forward transforms with 2 lin <= L never read the upper half of a line;
    // inverse transforms with 2 lout <= L never write it
    if constexpr (!RHS_LOOP) {
        if (!ragged_lines(g, qx, axis, DIR, o, lin, lout, ghat)) return;
    }
    bool hin = false, hout = false;
    if constexpr (CT) {
        hin = (GH || DIR < 0) && ct_half_in_ok(LC) && 2 * lin <= L;
        hout = (GH || DIR > 0) && ct_half_out_ok(LC) && 2 * lout <= L;
    }
    for (int q = q0; q < q1; ++q) {
        if (skip_rhs(st + q, chk)) continue;
        C* gq = grid + (long long)q * g.npts * NC + obase + (long long)x0 * NC;
        const int tin = nlines * (hin ? L / 2 : L);
        for (int idx = threadIdx.x; idx < tin; idx += NT) {
            const int inner = idx % nlines;
            const int e = idx / nlines;
            C v;
            if (e < lin && inner < nval) {
                v = gq[e * estride + inner];
            } else {
                v.x = 0;
                v.y = 0;
            }
            lds[inner * Lp + e] = v;
        }
        __syncthreads();
        if constexpr (GH) {
            if constexpr (CT) {
                if (hin) fft_lines_ct<T, -1, LC, NC * TXC, NT, true, false>(lds, tw64 + pl.tw);
                else fft_lines_ct<T, -1, LC, NC * TXC, NT>(lds, tw64 + pl.tw);
            } else {
                fft_lines<T, -1>(lds, tws, nlines, Lp, pl);
            }
            // y_a = sum_b Ghat_ab x_b at (kx, ky = o, kz)
            if constexpr (CT && VAR != 0) {
                // kz and L - kz share the stored tensor entry; the xz and yz
                // components change sign between them (odd in z).  One
                // thread takes both points of a pair from one read: the
                // pairs (h, L - h) for 0 < h < L / 2, and h = 0 and h = L / 2
                // alone.
                constexpr int UNITS = TXC * (LC / 2 + 1);
#pragma unroll
                for (int i = 0; i < (UNITS + NT - 1) / NT; ++i) {
                    const int u = threadIdx.x + i * NT;
                    const int xo = u % TX;
                    const int h = u / TX;
                    if (u < UNITS && xo < nxl) {
                        C Gl[6];
                        tensor_at(xo, h, Gl);
                        C* px = lds + (xo * 3 + 0) * Lp;
                        C* py = lds + (xo * 3 + 1) * Lp;
                        C* pz = lds + (xo * 3 + 2) * Lp;
                        {
                            const C X = px[h], Y = py[h], Z = pz[h];
                            px[h] = trow(Gl[0], Gl[1], Gl[2], X, Y, Z);
                            py[h] = trow(Gl[1], Gl[3], Gl[4], X, Y, Z);
                            pz[h] = trow(Gl[2], Gl[4], Gl[5], X, Y, Z);
                        }
                        if (h > 0 && 2 * h < LC) {
                            const int m = LC - h;
                            Gl[2].x = -Gl[2].x;
                            Gl[2].y = -Gl[2].y;
                            Gl[4].x = -Gl[4].x;
                            Gl[4].y = -Gl[4].y;
                            const C X = px[m], Y = py[m], Z = pz[m];
                            px[m] = trow(Gl[0], Gl[1], Gl[2], X, Y, Z);
                            py[m] = trow(Gl[1], Gl[3], Gl[4], X, Y, Z);
                            pz[m] = trow(Gl[2], Gl[4], Gl[5], X, Y, Z);
                        }
                    }
                }
            } else if constexpr (CT) {
#pragma unroll
                for (int i = 0; i < MAXP; ++i) {
                    const int p = threadIdx.x + i * NT;
                    if (p < TX * L) {
                        const int xo = p % TX;
                        const int kz = p / TX;
                        if (xo < nxl) {
                            C* px = lds + (xo * 3 + 0) * Lp + kz;
                            C* py = lds + (xo * 3 + 1) * Lp + kz;
                            C* pz = lds + (xo * 3 + 2) * Lp + kz;
                            const C X = *px, Y = *py, Z = *pz;
                            C Gl[6];
                            if constexpr (VAR != 0) tensor_at(xo, kz, Gl);
                            const C* Gi = VAR == 0 ? G[i] : Gl;
                            *px = trow(Gi[0], Gi[1], Gi[2], X, Y, Z);
                            *py = trow(Gi[1], Gi[3], Gi[4], X, Y, Z);
                            *pz = trow(Gi[2], Gi[4], Gi[5], X, Y, Z);
                        }
                    }
                }
            } else {
                for (int p = threadIdx.x; p < nxl * L; p += NT) {
                    const int xo = p % nxl;
                    const int kz = p / nxl;
                    C Gi[6];
                    tensor_at(xo, kz, Gi);
                    C* px = lds + (xo * 3 + 0) * Lp + kz;
                    C* py = lds + (xo * 3 + 1) * Lp + kz;
                    C* pz = lds + (xo * 3 + 2) * Lp + kz;
                    const C X = *px, Y = *py, Z = *pz;
                    *px = trow(Gi[0], Gi[1], Gi[2], X, Y, Z);
                    *py = trow(Gi[1], Gi[3], Gi[4], X, Y, Z);
                    *pz = trow(Gi[2], Gi[4], Gi[5], X, Y, Z);
                }
            }
            __syncthreads();
            if constexpr (CT) {
                if (hout) fft_lines_ct<T, 1, LC, NC * TXC, NT, false, true>(lds, tw64 + pl.tw);
                else fft_lines_ct<T, 1, LC, NC * TXC, NT>(lds, tw64 + pl.tw);
            } else {
                fft_lines<T, 1>(lds, tws, nlines, Lp, pl);
            }
        } else {
            if constexpr (CT) {
                if (hin) fft_lines_ct<T, DIR, LC, NC * TXC, NT, true, false>(lds, tw64 + pl.tw);
                else if (hout) fft_lines_ct<T, DIR, LC, NC * TXC, NT, false, true>(lds, tw64 + pl.tw);
                else fft_lines_ct<T, DIR, LC, NC * TXC, NT>(lds, tw64 + pl.tw);
            } else {
                fft_lines<T, DIR>(lds, tws, nlines, Lp, pl);
            }
        }
        const int tout = nlines * lout;
        for (int idx = threadIdx.x; idx < tout; idx += NT) {
            const int inner = idx % nlines;
            const int e = idx / nlines;
            if (inner < nval) gq[e * estride + inner] = lds[inner * Lp + e];
        }
        if (RHS_LOOP) __syncthreads();   // the next right-hand side refills the tile
    }
}

// Pass 3 with the tensor read once per launch.  The workgroup owns octant
// columns hx0 .. hx0+TX-1 of octant row hy and transforms, for every
// right-hand side, the up to four column sets (hx or Mx-hx) x (hy or My-hy)
// that share those tensor values; the values (with the z parity folded in)
// stay in registers, the x and y parities are applied per column set.
template <typename T, int LC, int TXC>
__global__ __launch_bounds__(NT) void k_zfold(Geo g, typename V2<T>::t* grid, const double2* tw64,
                                             const typename V2<T>::t* ghat, const RhsState* st, int nrhs, int lin,
                                             int lout, int chk) {
    using C = typename V2<T>::t;
    constexpr int L = LC;
    constexpr int TX = TXC;
    constexpr int NL = 3 * TX;
    constexpr int LP = L | 1;
    constexpr int MAXP = (TX * L + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = (C*)smem;
    const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
    const int Hx = g.H[0], Hy = g.H[1];
    const int hx0 = blockIdx.x * TX;
    const int hy = blockIdx.y;
    const double2* tw = tw64 + g.ax[2].tw;
    C G[MAXP][6];
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
        const int p = threadIdx.x + i * NT;
        if (p < TX * L) {
            const int xo = p % TX;
            const int kz = p / TX;
            const int hx = hx0 + xo;
            if (hx < Hx) {
                const int fz = (kz <= Mz / 2) ? kz : Mz - kz;
                const C* Gp = ghat + (((long long)fz * Hy + hy) * Hx + hx) * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) G[i][c] = Gp[c];
                if (kz > Mz / 2) {   // xz and yz are odd in z
                    G[i][2].x = -G[i][2].x; G[i][2].y = -G[i][2].y;
                    G[i][4].x = -G[i][4].x; G[i][4].y = -G[i][4].y;
                }
            }
        }
    }
    const bool hin = ct_half_in_ok(LC) && 2 * lin <= L;
    const bool hout = ct_half_out_ok(LC) && 2 * lout <= L;
    const long long plane = (long long)My * Mx * 3;
    for (int combo = 0; combo < 4; ++combo) {
        const int mxf = combo & 1, myf = combo >> 1;
        if (myf && !(hy >= 1 && 2 * hy != My)) continue;
        const int ky = myf ? My - hy : hy;
        auto col_ok = [&](int xo) {
            const int hx = hx0 + xo;
            return hx < Hx && (!mxf || (hx >= 1 && 2 * hx != Mx));
        };
        auto kx_of = [&](int xo) { return mxf ? Mx - (hx0 + xo) : hx0 + xo; };
        bool any = false;
#pragma unroll
        for (int xo = 0; xo < TX; ++xo) any |= col_ok(xo);
        if (!any) continue;
        for (int q = 0; q < nrhs; ++q) {
            if (skip_rhs(st + q, chk)) continue;
            C* gq = grid + (long long)q * g.npts * 3 + (long long)ky * Mx * 3;
            const int tin = NL * (hin ? L / 2 : L);
            for (int idx = threadIdx.x; idx < tin; idx += NT) {
                const int inner = idx % NL;
                const int e = idx / NL;
                const int xo = inner / 3, c = inner % 3;
                C v;
                if (e < lin && col_ok(xo)) {
                    v = gq[e * plane + (long long)kx_of(xo) * 3 + c];
                } else {
                    v.x = 0;
                    v.y = 0;
                }
                lds[inner * LP + e] = v;
            }
            __syncthreads();
            if (hin) fft_lines_ct<T, -1, LC, NL, NT, true, false>(lds, tw);
            else fft_lines_ct<T, -1, LC, NL, NT>(lds, tw);
#pragma unroll
            for (int i = 0; i < MAXP; ++i) {
                const int p = threadIdx.x + i * NT;
                if (p < TX * L) {
                    const int xo = p % TX;
                    const int kz = p / TX;
                    if (col_ok(xo)) {
                        C gxy = G[i][1], gxz = G[i][2], gyz = G[i][4];
                        if (mxf != myf) { gxy.x = -gxy.x; gxy.y = -gxy.y; }
                        if (mxf) { gxz.x = -gxz.x; gxz.y = -gxz.y; }
                        if (myf) { gyz.x = -gyz.x; gyz.y = -gyz.y; }
                        C* px = lds + (xo * 3 + 0) * LP + kz;
                        C* py = lds + (xo * 3 + 1) * LP + kz;
                        C* pz = lds + (xo * 3 + 2) * LP + kz;
                        const C X = *px, Y = *py, Z = *pz;
                        *px = trow(G[i][0], gxy, gxz, X, Y, Z);
                        *py = trow(gxy, G[i][3], gyz, X, Y, Z);
                        *pz = trow(gxz, gyz, G[i][5], X, Y, Z);
                    }
                }
            }
            __syncthreads();
            if (hout) fft_lines_ct<T, 1, LC, NL, NT, false, true>(lds, tw);
            else fft_lines_ct<T, 1, LC, NL, NT>(lds, tw);
            const int tout = NL * lout;
            for (int idx = threadIdx.x; idx < tout; idx += NT) {
                const int inner = idx % NL;
                const int e = idx / NL;
                const int xo = inner / 3, c = inner % 3;
                if (col_ok(xo)) gq[e * plane + (long long)kx_of(xo) * 3 + c] = lds[inner * LP + e];
            }
            __syncthreads();
        }
    }
}

// Passes 2-4 in register-resident form.  Each line is handled by Q = L/P
// threads: thread t loads the subsequence e = t + Q m (m < P) of its lines,
// runs the first pass group in registers, the tile is exchanged once through
// LDS, and the thread then runs the remaining passes on its residue classes
// and stores X[kappa + P g] directly.  With GH the three components of a
// column stay in one thread, so the tensor product is applied in registers,
// and the thread's frequencies are already its subsequence for the inverse
// transform (a renumbering of its registers, no exchange).  The passes are those of fft_lines_ct (bitwise-identical
// results to k_strided); only the data movement differs.  One right-hand
// side per workgroup (grid z).  XR: the exchange runs in XR rounds over the
// tile's lines (LDS of 3 TX / XR lines).  HIN / HOUT: the half-line pruning
// of the forward input / inverse output (the host launches this kernel only
// where the pass allows it).
// nct: component lines per thread (3: pass 3 with the product in registers)
constexpr int rf_threads(int L, int TX, int nct) { return (nct == 3 ? TX : 3 * TX) * (L / ct_split(L)); }
template <int L> constexpr int rf_line_stride() { return ((L / ct_split(L)) * (ct_split(L) + 1)) | 1; }
template <typename T, int L, int TX, int XR> constexpr size_t rf_smem() {
    return (size_t)(3 * TX / XR) * rf_line_stride<L>() * sizeof(typename V2<T>::t);
}

// XG: the XCD-grouped workgroup order of xcd_tile (pass 3) or of xcd_rows
// (y passes; n_outer planes).
// Occupancy asked of the compiler for passes 2 and 4 (one line per thread):
// four waves per SIMD (128 VGPRs) when the line data take at most 32 VGPRs,
// three (168) up to 64, two (256) for the four-pass length 256 -- none of
// which spills.  For pass 3 the occupancy is a tuning choice (WV).
template <typename T> constexpr int rf_waves(int L) {
    const int d = ct_split(L) * (int)(2 * sizeof(T) / 4);
    if (L == 256) return 2;
    return d <= 32 ? 4 : (d <= 64 ? 3 : 1);
}
template <typename T, int GH, int DIR, int L, int TX, int XR, bool HIN, bool HOUT, bool XG, int WV>
__global__ __launch_bounds__(rf_threads(L, TX, GH ? 3 : 1))
__attribute__((amdgpu_waves_per_eu(GH ? WV : rf_waves<T>(L)))) void k_strided_rf(Geo g, typename V2<T>::t* grid,
                                                                       const double2* tw64,
                                                                       const typename V2<T>::t* ghat,
                                                                       const RhsState* st, int axis, int lin,
                                                                       int lout, int chk, int nrhs,
                                                                       int n_outer) {
    using C = typename V2<T>::t;
    constexpr int P = ct_split(L);
    constexpr int Q = L / P;
    constexpr int NCT = GH ? 3 : 1;               // component lines per thread
    constexpr int NIN = NCT == 3 ? TX : 3 * TX;   // threads across the tile's lines
    constexpr int LS = rf_line_stride<L>();
    static_assert((3 * TX) % XR == 0, "exchange rounds must split the tile's lines");
    // exchange round and LDS row of line ln
    auto round_of = [](int ln) { return ln % XR; };
    auto slot_of = [](int ln) { return ln / XR; };
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = (C*)smem;
    const int Mx = g.M[0], My = g.M[1];
    int q, o, xt;
    if constexpr (XG && GH) {
        if (!xcd_tile(Mx, My, TX, nrhs, xt, o, q)) return;
    } else if constexpr (XG) {
        if (!xcd_rows((Mx + TX - 1) / TX, n_outer, nrhs, xt, o, q)) return;
    } else {
        q = blockIdx.z;
        o = blockIdx.y;
        xt = blockIdx.x;
    }
    if (skip_rhs(st + q, chk)) return;
    if (!ragged_lines(g, q, axis, DIR, o, lin, lout, ghat)) return;
    const int in = threadIdx.x % NIN;
    const int t = threadIdx.x / NIN;
    const int x0 = xt * TX;
    const double2* tw = tw64 + g.ax[axis].tw;
    const long long estride = (axis == 1) ? (long long)Mx * 3 : (long long)My * Mx * 3;
    const long long obase = (axis == 1) ? (long long)o * My * Mx * 3 : (long long)o * Mx * 3;
    C* gq = grid + (long long)q * g.npts * 3 + obase + (long long)x0 * 3;
    const int nval = 3 * min(TX, Mx - x0);
    // line (column * 3 + component) of this thread's component a
    auto line_of = [&](int a) { return NCT == 3 ? in * 3 + a : in; };

    C v[NCT][P];
#pragma unroll
    for (int a = 0; a < NCT; ++a) {
        const int ln = line_of(a);
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int e = t + Q * m;
            if ((!HIN || 2 * m < P) && e < lin && ln < nval) {
                v[a][m] = gq[(long long)e * estride + ln];
            } else {
                v[a][m].x = 0;
                v[a][m].y = 0;
            }
        }
    }
    // first group -> exchange -> second group (one transform of every line)
    auto transform = [&](auto dir_tag, auto hin_tag, auto hout_tag) {
        constexpr int D = decltype(dir_tag)::value;
        constexpr bool HI = decltype(hin_tag)::value;
        constexpr bool HO = decltype(hout_tag)::value;
        rf_group_a<T, D, L, HI, NCT>(v, tw);
#pragma unroll
        for (int rd = 0; rd < XR; ++rd) {
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NCT; ++a) {
                const int ln = line_of(a);
                if (round_of(ln) == rd) {
                    C* row = lds + slot_of(ln) * LS + t * (P + 1);
#pragma unroll
                    for (int f = 0; f < P; ++f) row[f] = v[a][f];
                }
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NCT; ++a) {
                const int ln = line_of(a);
                if (round_of(ln) == rd) {
                    const C* row = lds + slot_of(ln) * LS;
#pragma unroll
                    for (int c = 0; c < P / Q; ++c) {
#pragma unroll
                        for (int jj = 0; jj < Q; ++jj) v[a][c * Q + jj] = row[jj * (P + 1) + t + Q * c];
                    }
                }
            }
        }
        rf_group_b<T, D, L, HO, NCT>(v, t, tw);
    };
    using Fwd = std::integral_constant<int, GH ? -1 : DIR>;
    transform(Fwd{}, std::integral_constant<bool, HIN>{},
              std::integral_constant<bool, GH ? false : HOUT>{});
    if constexpr (GH) {
        // y_a = sum_b Ghat_ab x_b at (kx = x0 + in, ky = o, kz = kappa + P g)
        const int Mz = g.M[2];
        const int Hx = g.H[0], Hy = g.H[1];
        const int kx = x0 + in;
        if (3 * in < nval) {
            const int fx = (kx <= Mx / 2) ? kx : Mx - kx;
            const int sx = (kx <= Mx / 2) ? 1 : -1;
            const int fy = (o <= My / 2) ? o : My - o;
            const int sy = (o <= My / 2) ? 1 : -1;
#pragma unroll
            for (int c = 0; c < P / Q; ++c) {
#pragma unroll
                for (int gg = 0; gg < Q; ++gg) {
                    const int kz = t + Q * c + P * gg;
                    const int fz = (kz <= Mz / 2) ? kz : Mz - kz;
                    const int sz = (kz <= Mz / 2) ? 1 : -1;
                    const C* Gp = ghat + (((long long)fz * Hy + fy) * Hx + fx) * 6;
                    C G6[6];
#pragma unroll
                    for (int k = 0; k < 6; ++k) G6[k] = Gp[k];
                    // parity flips as selects (no branches)
                    const bool f1 = sx * sy < 0, f2 = sx * sz < 0, f4 = sy * sz < 0;
                    G6[1].x = f1 ? -G6[1].x : G6[1].x;
                    G6[1].y = f1 ? -G6[1].y : G6[1].y;
                    G6[2].x = f2 ? -G6[2].x : G6[2].x;
                    G6[2].y = f2 ? -G6[2].y : G6[2].y;
                    G6[4].x = f4 ? -G6[4].x : G6[4].x;
                    G6[4].y = f4 ? -G6[4].y : G6[4].y;
                    const int sl = c * Q + gg;
                    const C X = v[0][sl], Y = v[NCT > 1 ? 1 : 0][sl], Z = v[NCT > 2 ? 2 : 0][sl];
                    v[0][sl] = trow(G6[0], G6[1], G6[2], X, Y, Z);
                    v[NCT > 1 ? 1 : 0][sl] = trow(G6[1], G6[3], G6[4], X, Y, Z);
                    v[NCT > 2 ? 2 : 0][sl] = trow(G6[2], G6[4], G6[5], X, Y, Z);
                }
            }
        }
        // back to subsequences: thread t holds X[kappa_c + P g] = X[t + Q m]
        // with m = c + (P / Q) g, every element of its subsequence, so the
        // inverse transform's input is a renumbering of its own registers
        C w[NCT][P];
#pragma unroll
        for (int a = 0; a < NCT; ++a) {
#pragma unroll
            for (int c = 0; c < P / Q; ++c) {
#pragma unroll
                for (int gg = 0; gg < Q; ++gg) w[a][c + (P / Q) * gg] = v[a][c * Q + gg];
            }
        }
#pragma unroll
        for (int a = 0; a < NCT; ++a) {
#pragma unroll
            for (int m = 0; m < P; ++m) v[a][m] = w[a][m];
        }
        transform(std::integral_constant<int, 1>{}, std::integral_constant<bool, false>{},
                  std::integral_constant<bool, HOUT>{});
    }
#pragma unroll
    for (int a = 0; a < NCT; ++a) {
        const int ln = line_of(a);
        if (ln < nval) {
#pragma unroll
            for (int c = 0; c < P / Q; ++c) {
#pragma unroll
                for (int gg = 0; gg < (HOUT ? Q / 2 : Q); ++gg) {
                    const int e = t + Q * c + P * gg;
                    if (e < lout) gq[(long long)e * estride + ln] = v[a][c * Q + gg];
                }
            }
        }
    }
}

// Pass 3 for the square lengths L = P^2 (64 = 8 x 8, 256 = 16 x 16) in
// register-resident form.  With P = Q the forward transform's second pass
// group leaves thread t with the frequencies kz = t + P g (g < P), in the
// very order in which the inverse transform's first group reads its
// subsequence t + Q m (k_strided_rf renumbers its registers there).  The
// same passes and twiddles as every other form, so bitwise-identical
// results.  Beyond k_strided_rf: the twiddles come from the table in the
// grid's precision (no FP64 -> FP32 conversion), the z extent is the
// compile-time L so the z parities and the octant rows of the tensor are
// compile-time for all but one frequency per thread, and each thread keeps
// one base address per column.  TX columns per
// workgroup, Q threads per column (thread t = threadIdx.x / TX); one
// right-hand side per workgroup; XR exchange rounds; XG: the XCD-grouped
// order of xcd_tile; WV: occupancy asked of the compiler; PD: how many
// points ahead the tensor values are loaded (0: where the compiler puts
// them, which is all sixteen at once).
template <typename T> __device__ __forceinline__ const typename V2<T>::t* tw_table(const Geo& g, const double2* tw64);
template <> __device__ __forceinline__ const double2* tw_table<double>(const Geo&, const double2* tw64) { return tw64; }
template <> __device__ __forceinline__ const float2* tw_table<float>(const Geo& g, const double2*) { return g.tw32; }

constexpr bool zsq_length(int L) { return L == 64 || L == 256; }

template <typename T, int L, int TX, int XR, bool XG, int WV, int PD = 0>
__global__ __launch_bounds__(TX * (L / ct_split(L))) __attribute__((amdgpu_waves_per_eu(WV)))
void k_zsq(Geo g, typename V2<T>::t* grid, const double2* tw64, const typename V2<T>::t* ghat, const RhsState* st,
           int lin, int lout, int chk, int nrhs) {
    using C = typename V2<T>::t;
    constexpr int P = ct_split(L);
    constexpr int Q = L / P;
    static_assert(P == Q, "square lengths only");
    constexpr int LS = rf_line_stride<L>();
    static_assert((3 * TX) % XR == 0, "exchange rounds must split the tile's lines");
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = (C*)smem;
    const int Mx = g.M[0], My = g.M[1];
    int q, o, xt;
    if constexpr (XG) {
        if (!xcd_tile(Mx, My, TX, nrhs, xt, o, q)) return;
    } else {
        q = blockIdx.z;
        o = blockIdx.y;
        xt = blockIdx.x;
    }
    if (skip_rhs(st + q, chk)) return;
    if (!ragged_lines(g, q, 2, -1, o, lin, lout, ghat)) return;
    const int in = threadIdx.x % TX;
    const int t = threadIdx.x / TX;
    const int kx = xt * TX + in;
    const bool col = kx < Mx;
    const C* tw = tw_table<T>(g, tw64) + g.ax[2].tw;
    const long long zs = (long long)My * Mx * 3;   // z stride of the grid
    // this thread's column at z = t; element m of its subsequence is z = t + Q m
    C* gc = grid + (long long)q * g.npts * 3 + (long long)o * Mx * 3 + (long long)kx * 3 + (long long)t * zs;
    C v[3][P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (2 * m < P && col && t + Q * m < lin) {
                v[a][m] = gc[(long long)m * Q * zs + a];
            } else {
                v[a][m].x = 0;
                v[a][m].y = 0;
            }
        }
    }
    // residue classes <-> subsequences through LDS, one component of XR per round
    auto exchange = [&]() {
#pragma unroll
        for (int rd = 0; rd < XR; ++rd) {
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int ln = in * 3 + a;
                if (ln % XR == rd) {
                    C* row = lds + (ln / XR) * LS + t * (P + 1);
#pragma unroll
                    for (int f = 0; f < P; ++f) row[f] = v[a][f];
                }
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int ln = in * 3 + a;
                if (ln % XR == rd) {
                    const C* row = lds + (ln / XR) * LS + t;
#pragma unroll
                    for (int jj = 0; jj < Q; ++jj) v[a][jj] = row[jj * (P + 1)];
                }
            }
        }
    };
    rf_group_a<T, -1, L, true, 3>(v, tw);
    exchange();
    rf_group_b<T, -1, L, false, 3>(v, t, tw);
    // y_a = sum_b Ghat_ab x_b at (kx, ky = o, kz = t + P gg); the stored
    // octant and the parities (diagonal even, ab odd in a and b)
    if (col) {
        const int Hx = g.H[0], Hy = g.H[1];
        const int fx = (kx <= Mx / 2) ? kx : Mx - kx;
        const int fy = (o <= My / 2) ? o : My - o;
        const bool fxy = (kx <= Mx / 2) != (o <= My / 2);   // sx sy < 0
        const bool nx = kx > Mx / 2, ny = o > My / 2;       // sx < 0, sy < 0
        const long long hz = (long long)Hy * Hx * 6;        // octant z stride
        const C* gl = ghat + ((long long)fy * Hx + fx) * 6 + (long long)t * hz;        // fz = t + P gg
        const C* gu = ghat + ((long long)fy * Hx + fx) * 6 + (long long)(L - t) * hz;  // fz = L - t - P gg
        // kz = t + P gg <= L/2 for gg < P/2, > L/2 for gg > P/2; at gg = P/2
        // only t = 0 (kz = L/2) is in the lower half
        auto gptr = [&](int gg) {
            const bool up = 2 * gg > P || (2 * gg == P && t != 0);
            return up ? gu - (long long)P * gg * hz : gl + (long long)P * gg * hz;
        };
        // PD > 0: the tensor values of point gg + PD are loaded while point gg
        // is formed, and not earlier (their address is tied to point gg's
        // result), which bounds the registers the loads hold
        C Gb[PD > 0 ? PD : 1][6];
        if constexpr (PD > 0) {
#pragma unroll
            for (int d = 0; d < PD; ++d) {
                const C* Gp = gptr(d);
#pragma unroll
                for (int k = 0; k < 6; ++k) Gb[d][k] = Gp[k];
            }
        }
#pragma unroll
        for (int gg = 0; gg < P; ++gg) {
            const bool up = 2 * gg > P || (2 * gg == P && t != 0);   // sz < 0
            C G6[6];
            if constexpr (PD > 0) {
#pragma unroll
                for (int k = 0; k < 6; ++k) G6[k] = Gb[gg % PD][k];
            } else {
                const C* Gp = gptr(gg);
#pragma unroll
                for (int k = 0; k < 6; ++k) G6[k] = Gp[k];
            }
            const bool f2 = nx != up, f4 = ny != up;   // sx sz < 0, sy sz < 0
            G6[1].x = fxy ? -G6[1].x : G6[1].x;
            G6[1].y = fxy ? -G6[1].y : G6[1].y;
            G6[2].x = f2 ? -G6[2].x : G6[2].x;
            G6[2].y = f2 ? -G6[2].y : G6[2].y;
            G6[4].x = f4 ? -G6[4].x : G6[4].x;
            G6[4].y = f4 ? -G6[4].y : G6[4].y;
            const C X = v[0][gg], Y = v[1][gg], Z = v[2][gg];
            v[0][gg] = trow(G6[0], G6[1], G6[2], X, Y, Z);
            v[1][gg] = trow(G6[1], G6[3], G6[4], X, Y, Z);
            v[2][gg] = trow(G6[2], G6[4], G6[5], X, Y, Z);
            if constexpr (PD > 0) {
                if (gg + PD < P) {
                    const C* Gp = gptr(gg + PD);
                    asm volatile("" : "+v"(Gp) : "v"(v[2][gg].x));
#pragma unroll
                    for (int k = 0; k < 6; ++k) Gb[gg % PD][k] = Gp[k];
                }
            }
        }
    }
    rf_group_a<T, 1, L, false, 3>(v, tw);
    exchange();
    rf_group_b<T, 1, L, true, 3>(v, t, tw);
    if (col) {
#pragma unroll
        for (int gg = 0; gg < Q / 2; ++gg) {
            if (t + P * gg < lout) {
#pragma unroll
                for (int a = 0; a < 3; ++a) gc[(long long)gg * P * zs + a] = v[a][gg];
            }
        }
    }
}

// ------------------------------------------------------------------ launchers

template <typename T, int MODE>
void scatter_dispatch(int chk, const Geo& g, const SiteArgs& a, typename V2<T>::t* grid, const double2* tw,
                      hipStream_t s) {
    using C = typename V2<T>::t;
    const int L = g.M[0];
    const int XL = x_lines_per_tile(g, a.nrhs, sizeof(T) == 4);
    dim3 grd((g.n[1] + XL - 1) / XL, g.n[2], a.nrhs);
    switch (L) {
#define DDA_CASE(LL)                                                                                            \
    case LL:                                                                                                   \
        DDA_LAUNCH((k_scatter_x<T, MODE, LL, xthr(LL)>), grd, dim3(xthr(LL)), smem_ct<C>(LL, 3), s, g, a, grid, \
                           tw, 1, chk);                                                                        \
        return;
        DDA_CT_LENGTHS(DDA_CASE)
#undef DDA_CASE
        default:
            DDA_LAUNCH((k_scatter_x<T, MODE, 0, NT>), grd, dim3(NT), smem_rt<C>(L, 3 * XL), s, g, a, grid,
                               tw, XL, chk);
    }
}

template <typename T, int MODE>
void gather_dispatch(int chk, const Geo& g, const SiteArgs& a, const typename V2<T>::t* grid, const double2* tw,
                     hipStream_t s) {
    using C = typename V2<T>::t;
    const int L = g.M[0];
    const int XL = x_lines_per_tile(g, a.nrhs, sizeof(T) == 4);
    dim3 grd((g.n[1] + XL - 1) / XL, g.n[2], a.nrhs);
    // operands before the transform pay in launches of few right-hand sides
    // (latency-bound workgroups); with many, the launch is bandwidth-bound
    // and the registers they take cost more occupancy than they save
    // (measured: 2-RHS solves gain, the 128-RHS brick loses 10%)
    const bool pre = a.nrhs <= 16;
    switch (L) {
#define DDA_CASE(LL)                                                                                            \
    case LL:                                                                                                   \
        if (pre)                                                                                               \
            DDA_LAUNCH((k_gather_x<T, MODE, LL, xthr(LL), true>), grd, dim3(xthr(LL)), smem_ct<C>(LL, 3), s, g, \
                       a, grid, tw, 1, chk);                                                                   \
        else                                                                                                   \
            DDA_LAUNCH((k_gather_x<T, MODE, LL, xthr(LL), false>), grd, dim3(xthr(LL)), smem_ct<C>(LL, 3), s,   \
                       g, a, grid, tw, 1, chk);                                                                \
        return;
        DDA_CT_LENGTHS(DDA_CASE)
#undef DDA_CASE
        default:
            DDA_LAUNCH((k_gather_x<T, MODE, 0, NT>), grd, dim3(NT), smem_rt<C>(L, 3 * XL), s, g, a, grid,
                               tw, XL, chk);
    }
}

// Compile-time variants of a strided pass.  LDS form (k_strided, k_zfold):
// (tile width, VAR, XCD order), indices 0 .. n_lds_variants - 1, index 0 the
// default.
// Register-resident form (k_strided_rf): (tile width, exchange rounds),
// the following rf_variants indices.  The autotuner of the C ABI picks among
// them by timing; all give bitwise-identical results.  Wider tiles give
// longer contiguous runs per plane (what large grids need); LDS tiles are
// bounded by 48 KB per workgroup.
constexpr int n_lds_variants(int gh) { return gh ? 12 : 4; }
constexpr int rf_variants(int gh) { return gh ? 12 : 8; }
// pass 3 at the square lengths: k_zsq variants after the register-resident
// ones (elsewhere they fall back to variant 0)
constexpr int zsq_variants(int gh) { return gh ? 4 : 0; }
constexpr int n_strided_variants(int gh) { return n_lds_variants(gh) + rf_variants(gh) + zsq_variants(gh); }
// k_zsq variant r: (tile width, tensor prefetch distance), all in the
// XCD-grouped order, three exchange rounds and the occupancy the line data
// allow: r = 0 (16, 2), 1 (8, 4), 2 (8, 2), 3 (16, none); each exists where
// its LDS tile fits 64 KB
constexpr int zsq_tx(int r) { return (r == 1 || r == 2) ? 8 : 16; }
constexpr int zsq_xr(int) { return 3; }
constexpr bool zsq_xg(int) { return true; }
constexpr int zsq_pd(int r) { return r == 1 ? 4 : (r == 3 ? 0 : 2); }
template <typename T> constexpr bool zsq_feasible(int L, int r) {
    const int P = ct_split(L);
    return (size_t)(3 * zsq_tx(r) / zsq_xr(r)) * (((L / P) * (P + 1)) | 1) * 2 * sizeof(T) <= 65536;
}
template <typename T> constexpr int zsq_wv(int L, int) {
    const int d = 3 * ct_split(L) * (int)(2 * sizeof(T) / 4);   // VGPRs of line data
    return d <= 48 ? 4 : (d <= 96 ? 2 : 1);
}
template <typename T> constexpr int ct_budget() { return sizeof(T) == 4 ? 6144 : 3072; }
template <typename T> constexpr int variant_tx(int L, int gh, int v) {
    const int base = ct_cols(L);
    const int half = base > 1 ? base / 2 : 1;
    const int dbl = (2 * base <= 32 && 3 * 2 * base * L <= ct_budget<T>()) ? 2 * base : base;
    const int quad = (4 * base <= 32 && 3 * 4 * base * L <= ct_budget<T>()) ? 4 * base : dbl;
    if (gh) {
        switch (v) {
            case 2: case 4: case 8: case 11: return half;
            case 5: return dbl;
            case 6: return quad;
            case 9: return half > 1 ? half / 2 : 1;
            default: return base;
        }
    }
    switch (v) {
        case 1: return half;
        case 2: return dbl;
        case 3: return quad;
        default: return base;
    }
}
// VAR 3: the octant-folded kernel k_zfold; variants 10 and 11: VAR 2 in the
// XCD-grouped order
constexpr int variant_var(int gh, int v) {
    if (!gh) return 0;
    if (v >= 10) return 2;
    if (v >= 7) return 3;
    return v == 0 ? 0 : (v <= 2 ? 1 : 2);
}
constexpr bool variant_xg(int gh, int v) { return gh && v >= 10; }
// register-resident variant r (0 .. rf_variants-1): tile width and rounds,
// and the XCD-grouped workgroup order for r >= 4 (y passes: r - 4's tiling);
// for pass 3 also an occupancy of three waves per SIMD asked of the compiler
// (r >= 8, where the line data take at most 96 VGPRs; a few spilled
// registers are the price)
constexpr int rf_tx(int gh, int r) {
    return gh ? (r % 2 == 0 ? 16 : 8) : (r % 4 == 1 ? 16 : (r % 4 == 3 ? 4 : 8));
}
constexpr int rf_xr(int gh, int r) { return gh ? (r % 4 < 2 ? 3 : 1) : (r % 4 == 2 ? 3 : 1); }
constexpr bool rf_xg(int, int r) { return r >= 4; }
template <typename T> constexpr int rf_wv(int L, int gh, int r) {
    return (gh && r >= 8 && 3 * ct_split(L) * (int)(2 * sizeof(T) / 4) <= 96) ? 3 : 1;
}
constexpr int rf_nct(int gh) { return gh ? 3 : 1; }
// a register-resident variant exists where its data fit: at most 192 VGPRs
// of line data per thread, 512 threads and 64 KB of LDS per workgroup
template <typename T> constexpr bool rf_feasible(int L, int gh, int r) {
    const int P = ct_split(L);
    const int vgpr = rf_nct(gh) * P * (int)(2 * sizeof(T) / 4);
    const int thr = rf_threads(L, rf_tx(gh, r), rf_nct(gh));
    const size_t lds = (size_t)(3 * rf_tx(gh, r) / rf_xr(gh, r)) * (((L / P) * (P + 1)) | 1) * 2 * sizeof(T);
    return P > 0 && vgpr <= 192 && thr <= 512 && lds <= 65536;
}

constexpr int RAGGED_FALLBACK = 3;

template <typename T, int NC, int GH, int DIR, int LL, int V>
void strided_ct_launch(int axis, int chk, const Geo& g, int nrhs, int n_outer, int lin, int lout,
                       typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat,
                       const RhsState* st, hipStream_t s);

// the default variant, or for a ragged batch's pass 3 the default among the
// one-right-hand-side-per-workgroup variants
template <typename T, int NC, int GH, int DIR, int LL>
void strided_ct_fallback(int axis, int chk, const Geo& g, int nrhs, int n_outer, int lin, int lout,
                         typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat,
                         const RhsState* st, hipStream_t s) {
    static_assert(ragged_variant(1, RAGGED_FALLBACK) && RAGGED_FALLBACK < n_lds_variants(1), "fallback");
    if (GH && g.rg)
        strided_ct_launch<T, NC, GH, DIR, LL, RAGGED_FALLBACK>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw,
                                                              ghat, st, s);
    else
        strided_ct_launch<T, NC, GH, DIR, LL, 0>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
}

template <typename T, int NC, int GH, int DIR, int LL, int V>
void strided_ct_launch(int axis, int chk, const Geo& g, int nrhs, int n_outer, int lin, int lout,
                       typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat,
                       const RhsState* st, hipStream_t s) {
    using C = typename V2<T>::t;
    if constexpr (V >= n_lds_variants(GH) + rf_variants(GH)) {
        constexpr int R = V - n_lds_variants(GH) - rf_variants(GH);
        if constexpr (NC == 3 && GH && zsq_length(LL) && zsq_feasible<T>(LL, R)) {
            constexpr int TX = zsq_tx(R), XR = zsq_xr(R);
            constexpr bool XG = zsq_xg(R);
            constexpr int WV = zsq_wv<T>(LL, R);
            if (2 * lin <= LL && 2 * lout <= LL) {
                constexpr int Q = LL / ct_split(LL);
                dim3 grd((g.M[0] + TX - 1) / TX, n_outer, nrhs);
                if (XG) grd = dim3(xcd_grid(g.M[0], g.M[1], TX, nrhs));
                const size_t shm = (size_t)(3 * TX / XR) * rf_line_stride<LL>() * sizeof(C);
                DDA_LAUNCH((k_zsq<T, LL, TX, XR, XG, WV, zsq_pd(R)>), grd, dim3(TX * Q), shm, s, g, grid, tw, ghat, st,
                           lin, lout, chk, nrhs);
                return;
            }
        }
        strided_ct_fallback<T, NC, GH, DIR, LL>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
    } else if constexpr (V >= n_lds_variants(GH)) {
        constexpr int R = V - n_lds_variants(GH);
        constexpr int TX = rf_tx(GH, R), XR = rf_xr(GH, R);
        constexpr bool XG = rf_xg(GH, R);
        constexpr int WV = rf_wv<T>(LL, GH, R);
        const bool hin = (GH || DIR < 0) && 2 * lin <= LL;
        const bool hout = (GH || DIR > 0) && 2 * lout <= LL;
        // the instantiated pruning: both halves for pass 3, the input half of
        // a forward and the output half of an inverse y pass
        const bool pruned = GH ? (hin && hout) : (DIR < 0 ? hin : hout);
        if constexpr (NC == 3 && rf_feasible<T>(LL, GH, R)) {
            if (pruned) {
                constexpr bool HI = GH || DIR < 0, HO = GH || DIR > 0;
                const int ntx = (g.M[0] + TX - 1) / TX;
                dim3 grd(ntx, n_outer, nrhs);
                if (XG) grd = dim3(GH ? xcd_grid(g.M[0], g.M[1], TX, nrhs) : xcd_rows_grid(ntx, n_outer, nrhs));
                const dim3 blk(rf_threads(LL, TX, rf_nct(GH)));
                const size_t shm = rf_smem<T, LL, TX, XR>();
                DDA_LAUNCH((k_strided_rf<T, GH, DIR, LL, TX, XR, HI, HO, XG, WV>), grd, blk, shm, s, g, grid, tw,
                           ghat, st, axis, lin, lout, chk, nrhs, n_outer);
                return;
            }
        }
        strided_ct_fallback<T, NC, GH, DIR, LL>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
    } else {
        constexpr int TX = variant_tx<T>(LL, GH, V);
        constexpr int VR = variant_var(GH, V);
        if constexpr (VR == 3) {
            dim3 grd((g.H[0] + TX - 1) / TX, g.H[1], 1);
            DDA_LAUNCH((k_zfold<T, LL, TX>), grd, dim3(NT), smem_ct<C>(LL, 3 * TX), s, g, grid, tw, ghat, st, nrhs,
                       lin, lout, chk);
        } else if constexpr (variant_xg(GH, V)) {
            const dim3 grd(xcd_grid(g.M[0], g.M[1], TX, nrhs));
            DDA_LAUNCH((k_strided<T, NC, GH, DIR, LL, TX, VR, true>), grd, dim3(NT), smem_ct<C>(LL, NC * TX), s, g,
                       grid, tw, ghat, st, nrhs, axis, TX, lin, lout, chk);
        } else {
            const int gz = (GH && VR != 2) ? 1 : nrhs;
            dim3 grd((g.M[0] + TX - 1) / TX, n_outer, gz);
            DDA_LAUNCH((k_strided<T, NC, GH, DIR, LL, TX, VR>), grd, dim3(NT), smem_ct<C>(LL, NC * TX), s, g, grid,
                       tw, ghat, st, nrhs, axis, TX, lin, lout, chk);
        }
    }
}

template <typename T, int NC, int GH, int DIR, int LL>
void strided_ct_variant(int v, int axis, int chk, const Geo& g, int nrhs, int n_outer, int lin, int lout,
                        typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat,
                        const RhsState* st, hipStream_t s) {
    if (g.rg && !ragged_variant(GH, v)) v = -1;
    switch (v) {
#define DDA_V(VV)                                                                                             \
    case VV:                                                                                                 \
        if constexpr (VV < n_strided_variants(GH)) {                                                         \
            strided_ct_launch<T, NC, GH, DIR, LL, VV>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s); \
            return;                                                                                          \
        }                                                                                                    \
        break;
        DDA_V(1) DDA_V(2) DDA_V(3) DDA_V(4) DDA_V(5) DDA_V(6) DDA_V(7) DDA_V(8) DDA_V(9) DDA_V(10) DDA_V(11)
        DDA_V(12) DDA_V(13) DDA_V(14) DDA_V(15) DDA_V(16) DDA_V(17) DDA_V(18) DDA_V(19) DDA_V(20) DDA_V(21)
        DDA_V(22) DDA_V(23) DDA_V(24) DDA_V(25) DDA_V(26) DDA_V(27)
#undef DDA_V
        default:
            break;
    }
    strided_ct_fallback<T, NC, GH, DIR, LL>(axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
}

template <typename T, int NC, int GH, int DIR>
void strided_dispatch(int variant, int axis, int chk, const Geo& g, int nrhs, int n_outer, int lin, int lout,
                      typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat, const RhsState* st,
                      hipStream_t s) {
    using C = typename V2<T>::t;
    const int L = g.M[axis];
    if constexpr (NC == 3) {
        switch (L) {
#define DDA_CASE(LL)                                                                                       \
    case LL:                                                                                              \
        strided_ct_variant<T, NC, GH, DIR, LL>(variant, axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, \
                                               ghat, st, s);                                              \
        return;
            DDA_CT_LENGTHS(DDA_CASE)
#undef DDA_CASE
            default:
                break;
        }
    }
    if (g.rg) throw std::invalid_argument("a ragged batch needs compile-time FFT lengths");
    const int TX = strided_cols_per_tile(L, NC, sizeof(T) == 4);
    dim3 grd((g.M[0] + TX - 1) / TX, n_outer, GH ? 1 : nrhs);
    DDA_LAUNCH((k_strided<T, NC, GH, DIR, 0>), grd, dim3(NT), smem_rt<C>(L, NC * TX), s, g, grid, tw, ghat,
                       st, nrhs, axis, TX, lin, lout, chk);
}

}  // namespace passes

// ------------------------------------------------------------------ entry points

template <typename T>
void launch_scatter_x(int mode, int chk, const Geo& g, const SiteArgs& a, typename V2<T>::t* grid, const double2* tw,
                      hipStream_t s) {
    using namespace passes;
    switch (mode) {
        case SC_PLAIN: scatter_dispatch<T, SC_PLAIN>(chk, g, a, grid, tw, s); break;
        case SC_CONJ: scatter_dispatch<T, SC_CONJ>(chk, g, a, grid, tw, s); break;
        case SC_P: scatter_dispatch<T, SC_P>(chk, g, a, grid, tw, s); break;
        case SC_Q: scatter_dispatch<T, SC_Q>(chk, g, a, grid, tw, s); break;
        case SC_B0: scatter_dispatch<T, SC_B0>(chk, g, a, grid, tw, s); break;
        case SC_B1: scatter_dispatch<T, SC_B1>(chk, g, a, grid, tw, s); break;
        case SC_B2: scatter_dispatch<T, SC_B2>(chk, g, a, grid, tw, s); break;
        case SC_B3: scatter_dispatch<T, SC_B3>(chk, g, a, grid, tw, s); break;
        default: scatter_dispatch<T, SC_S>(chk, g, a, grid, tw, s); break;
    }
}

template <typename T>
void launch_gather_x(int mode, int chk, const Geo& g, const SiteArgs& a, const typename V2<T>::t* grid,
                     const double2* tw, hipStream_t s) {
    using namespace passes;
    switch (mode) {
        case GA_PLAIN: gather_dispatch<T, GA_PLAIN>(chk, g, a, grid, tw, s); break;
        case GA_CONJ: gather_dispatch<T, GA_CONJ>(chk, g, a, grid, tw, s); break;
        case GA_V: gather_dispatch<T, GA_V>(chk, g, a, grid, tw, s); break;
        case GA_T: gather_dispatch<T, GA_T>(chk, g, a, grid, tw, s); break;
        case GA_Q: gather_dispatch<T, GA_Q>(chk, g, a, grid, tw, s); break;
        case GA_B1: gather_dispatch<T, GA_B1>(chk, g, a, grid, tw, s); break;
        case GA_B2: gather_dispatch<T, GA_B2>(chk, g, a, grid, tw, s); break;
        case GA_B3: gather_dispatch<T, GA_B3>(chk, g, a, grid, tw, s); break;
        default: gather_dispatch<T, GA_RES>(chk, g, a, grid, tw, s); break;
    }
}

template <typename T>
void launch_strided(int axis, int dir, int chk, const Geo& g, int nrhs, int nc, int n_outer, int lin, int lout,
                    typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat, const RhsState* st,
                    hipStream_t s, int variant) {
    using namespace passes;
    if (nc != 3) throw std::invalid_argument("strided passes take three-component lines");
    if (ghat) {
        strided_dispatch<T, 3, 1, -1>(variant, axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
    } else if (dir < 0) {
        strided_dispatch<T, 3, 0, -1>(variant, axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
    } else {
        strided_dispatch<T, 3, 0, 1>(variant, axis, chk, g, nrhs, n_outer, lin, lout, grid, tw, ghat, st, s);
    }
}

static_assert(passes::n_strided_variants(1) == 28 && passes::n_strided_variants(0) == 12,
              "strided_variants() in dda_kernels.h counts these variants");

#define DDA_INSTANTIATE_PASSES(T)                                                                                 \
    template void launch_scatter_x<T>(int, int, const Geo&, const SiteArgs&, V2<T>::t*, const double2*,           \
                                      hipStream_t);                                                              \
    template void launch_gather_x<T>(int, int, const Geo&, const SiteArgs&, const V2<T>::t*, const double2*,      \
                                     hipStream_t);                                                               \
    template void launch_strided<T>(int, int, int, const Geo&, int, int, int, int, int, V2<T>::t*, const double2*, \
                                    const V2<T>::t*, const RhsState*, hipStream_t, int);

}  // namespace dda
