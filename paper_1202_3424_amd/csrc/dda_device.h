// Device-side building blocks of the DDA solver for gfx950 (CDNA4):
// complex helpers, the mixed-radix Stockham FFT over lines held in LDS, and
// deterministic workgroup / grid reductions.
//
// The FFT follows the autosort (Stockham) formulation: a line of length
// L = R_1 R_2 ... R_s is transformed in s passes; in the pass with radix R,
// after the radices already applied multiply to Ns, butterfly j (0 <= j < L/R)
// reads x[j + r L/R], multiplies input r by W_{Ns R}^{r (j mod Ns)}, takes a
// length-R DFT and writes output q to ((j - j mod Ns) R + j mod Ns + q Ns).
// The result is in natural order.  Twiddles W_L^t are FP64 tables computed
// on the host and staged in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dda {

constexpr int NT = 256;      // threads per workgroup, every kernel
constexpr int MAXST = 12;    // radix stages per line

// One FFT axis: length, radix sequence, offset of its W_L^t table.
struct AxisPlan {
    int L;
    int nst;
    int R[MAXST];
    int tw;
};

enum RhsStatus : int {
    ST_ACTIVE = 0,
    ST_CONVERGED = 1,
    ST_MAXITER = 2,
    ST_BREAKDOWN = 3,
    ST_NONFINITE = 4
};

// Per right-hand-side solver state, device resident.  Scalars of BiCGSTAB
// (van der Vorst 1992), BiCGstab(2) (Sleijpen & Fokkema 1993) or QMR for
// complex-symmetric A (COCG with quasi-minimal-residual smoothing) and the
// reductions that produce them.
struct RhsState {
    double2 rho;     // <rhat, r> (BiCGSTAB, BiCGstab(2): rho_0) or r^T r (QMR)
    double2 alpha;
    double2 omega;
    double2 beta;
    double bnorm2;   // |E|^2
    double rnorm2;   // |r|^2 of the latest residual
    double snorm2;   // |s|^2 of the latest half step (BiCGSTAB) or smoothed residual (QMR)
    double tol2;     // tol^2
    double tau2;     // QMR: squared quasi-residual norm
    double w_old;    // QMR: weights of the pending smoothing step (y, s) <- w_old (y, s) + w_new (x, r)
    double w_new;
    double2 g1;      // BiCGstab(2): minimal-residual coefficients of r_1 and r_2
    double2 g2;
    double2 rs;      // BiCGSTAB: <rhat, s> of the latest half step
    double rhat2;    // |rhat|^2 (BiCGSTAB, BiCGstab(2)): bounds the inner products with rhat
    double red[8];   // end-of-solve reductions (see kernels)
    int status;
    int iters;
    int matvecs;
    int sconv;       // converged at the half step of the current iteration
    int max_iter;
    int restarts;
    int pad0;        // FP64 residual refinements taken (FP32-matvec mode)
    // QMR: the smoothing step (w_old, w_new) has not been applied yet.
    // BiCGSTAB: the end of the latest iteration has not been applied to x
    // and r yet (1: x += alpha p + omega s, r = s - omega t; 2: x += alpha p,
    // after a half-step convergence)
    int pend;
    // FP32-matvec mode: an FP64 residual of the current x has confirmed its
    // convergence (later refinement checks leave it alone)
    int checked;
};

template <typename T> struct V2;
template <> struct V2<double> { using t = double2; };
template <> struct V2<float> { using t = float2; };

template <typename C> __device__ __forceinline__ C mk(double re, double im) {
    C c;
    c.x = re;
    c.y = im;
    return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C c;
    c.x = a.x * b.x - a.y * b.y;
    c.y = a.x * b.y + a.y * b.x;
    return c;
}
template <typename C> __device__ __forceinline__ C cconj(C a) { C c; c.x = a.x; c.y = -a.y; return c; }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { C c; c.x = a.x * s; c.y = a.y * s; return c; }
// conj(a) * b
template <typename C> __device__ __forceinline__ C cdotc(C a, C b) {
    C c;
    c.x = a.x * b.x + a.y * b.y;
    c.y = a.x * b.y - a.y * b.x;
    return c;
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    double2 c;
    c.x = (a.x * b.x + a.y * b.y) / d;
    c.y = (a.y * b.x - a.x * b.y) / d;
    return c;
}
// multiply by exp(DIR i pi/2): -i for the forward transform, +i for the inverse
template <int DIR, typename C> __device__ __forceinline__ C rot(C a) {
    C c;
    if (DIR < 0) { c.x = a.y; c.y = -a.x; } else { c.x = -a.y; c.y = a.x; }
    return c;
}

// ---------------------------------------------------------------- small DFTs
// y_q = sum_r v_r exp(DIR 2 pi i q r / R), in place.

template <int R, int DIR, typename C> struct Dft;

template <int DIR, typename C> struct Dft<2, DIR, C> {
    static __device__ __forceinline__ void run(C* v) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int DIR, typename C> struct Dft<4, DIR, C> {
    static __device__ __forceinline__ void run(C* v) {
        C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        C s13 = cadd(v[1], v[3]), d13 = rot<DIR>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    }
};

template <int DIR, typename C> struct Dft<8, DIR, C> {
    static __device__ __forceinline__ void run(C* v) {
        using S = decltype(v[0].x);
        const S h = (S)0.70710678118654752440;
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, DIR, C>::run(e);
        Dft<4, DIR, C>::run(o);
        // o[q] *= exp(DIR 2 pi i q / 8)
        C t1, t3;
        t1.x = (o[1].x - DIR * o[1].y) * h;
        t1.y = (o[1].y + DIR * o[1].x) * h;
        t3.x = (-o[3].x - DIR * o[3].y) * h;
        t3.y = (-o[3].y + DIR * o[3].x) * h;
        C t2 = rot<DIR>(o[2]);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], t1);
        v[5] = csub(e[1], t1);
        v[2] = cadd(e[2], t2);
        v[6] = csub(e[2], t2);
        v[3] = cadd(e[3], t3);
        v[7] = csub(e[3], t3);
    }
};

template <int DIR, typename C> struct Dft<3, DIR, C> {
    static __device__ __forceinline__ void run(C* v) {
        using S = decltype(v[0].x);
        const S s = (S)0.86602540378443864676;
        C t1 = cadd(v[1], v[2]);
        C t2 = cscale(rot<DIR>(csub(v[1], v[2])), s);
        C m = csub(v[0], cscale(t1, (S)0.5));
        v[0] = cadd(v[0], t1);
        v[1] = cadd(m, t2);
        v[2] = csub(m, t2);
    }
};

template <int DIR, typename C> struct Dft<5, DIR, C> {
    static __device__ __forceinline__ void run(C* v) {
        using S = decltype(v[0].x);
        const S c1 = (S)0.30901699437494742410, c2 = (S)-0.80901699437494742410;
        const S s1 = (S)0.95105651629515357212, s2 = (S)0.58778525229247312917;
        C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        C p1 = cadd(v[0], cadd(cscale(a1, c1), cscale(a2, c2)));
        C p2 = cadd(v[0], cadd(cscale(a1, c2), cscale(a2, c1)));
        C q1 = rot<DIR>(cadd(cscale(b1, s1), cscale(b2, s2)));
        C q2 = rot<DIR>(csub(cscale(b1, s2), cscale(b2, s1)));
        v[0] = cadd(v[0], cadd(a1, a2));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

// ---------------------------------------------------------------- LDS FFT

// Elements of one FFT tile (lines x line length) held in LDS: 32 KB.
template <typename T> struct Tile { static constexpr int EMAX = 32768 / (int)sizeof(typename V2<T>::t); };

// One Stockham pass of radix R over `nlines` lines of length L stored at
// lds[line * Lp + e].  Every thread holds up to MAXB butterflies in registers
// between the two barriers, so the pass is in place.
template <typename T, int R, int DIR, int NTHR = NT>
__device__ __forceinline__ void fft_pass(typename V2<T>::t* lds, const typename V2<T>::t* tw, int nlines, int Lp,
                                         int L, int Ns) {
    using C = typename V2<T>::t;
    constexpr int MAXB = (Tile<T>::EMAX + R * NTHR - 1) / (R * NTHR);
    const int LR = L / R;
    const int B = nlines * LR;
    const int tstep = L / (Ns * R);
    C v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * NTHR;
        if (b < B) {
            const int line = b % nlines;
            const int j = b / nlines;
            const C* src = lds + line * Lp + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[r * LR];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * NTHR;
        if (b < B) {
            const int line = b % nlines;
            const int j = b / nlines;
            const int k = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[r * k * tstep];
                    if (DIR > 0) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            Dft<R, DIR, C>::run(v[i]);
            C* dst = lds + line * Lp + (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[q * Ns] = v[i][q];
        }
    }
    __syncthreads();
}

// Full transform of every line in the tile (direction DIR: -1 forward, +1
// inverse, unnormalised).  Caller has synchronised after filling the tile.
template <typename T, int DIR, int NTHR = NT>
__device__ void fft_lines(typename V2<T>::t* lds, const typename V2<T>::t* tw, int nlines, int Lp, const AxisPlan& pl) {
    int Ns = 1;
    for (int s = 0; s < pl.nst; ++s) {
        const int R = pl.R[s];
        switch (R) {
            case 8: fft_pass<T, 8, DIR, NTHR>(lds, tw, nlines, Lp, pl.L, Ns); break;
            case 4: fft_pass<T, 4, DIR, NTHR>(lds, tw, nlines, Lp, pl.L, Ns); break;
            case 2: fft_pass<T, 2, DIR, NTHR>(lds, tw, nlines, Lp, pl.L, Ns); break;
            case 3: fft_pass<T, 3, DIR, NTHR>(lds, tw, nlines, Lp, pl.L, Ns); break;
            default: fft_pass<T, 5, DIR, NTHR>(lds, tw, nlines, Lp, pl.L, Ns); break;
        }
        Ns *= R;
    }
}

// ------------------------------------------------ compile-time FFT lengths
// Radix sequence of each compile-time length: ct_plan(L, -1) is the number
// of passes, ct_plan(L, s) the radix of pass s.  The passes fall into two
// groups, the first with radix product P = ct_split(L) >= Q = L / P and Q
// dividing P: the register-resident transform runs the first group on a
// thread's own subsequence x[t + Q m] and the second on a thread's own
// residue classes of the first group's output (see rf_group_a/rf_group_b).
// Every form of the transform (LDS and register-resident) runs exactly these
// passes, so they give bitwise-identical results.
constexpr int ct_plan(int L, int s) {
    int r[6] = {};
    int n = 0;
    switch (L) {
        case 32: r[0] = 8; r[1] = 4; n = 2; break;
        case 48: r[0] = 4; r[1] = 3; r[2] = 4; n = 3; break;
        case 64: r[0] = 8; r[1] = 8; n = 2; break;
        case 80: r[0] = 4; r[1] = 5; r[2] = 4; n = 3; break;
        case 96: r[0] = 8; r[1] = 3; r[2] = 4; n = 3; break;
        case 128: r[0] = 4; r[1] = 4; r[2] = 8; n = 3; break;
        case 160: r[0] = 8; r[1] = 5; r[2] = 4; n = 3; break;
        case 192: r[0] = 8; r[1] = 3; r[2] = 8; n = 3; break;
        case 256: r[0] = 4; r[1] = 4; r[2] = 4; r[3] = 4; n = 4; break;
        case 384: r[0] = 4; r[1] = 3; r[2] = 4; r[3] = 8; n = 4; break;
        case 512: r[0] = 8; r[1] = 4; r[2] = 4; r[3] = 4; n = 4; break;
        default: break;
    }
    return s < 0 ? n : r[s];
}
constexpr int ct_split(int L) {
    switch (L) {
        case 32: return 8;
        case 48: return 12;
        case 64: return 8;
        case 80: return 20;
        case 96: return 24;
        case 128: return 16;
        case 160: return 40;
        case 192: return 24;
        case 256: return 16;
        case 384: return 48;
        case 512: return 32;
        default: return 0;
    }
}
// passes in the first group
constexpr int ct_split_passes(int L) {
    int p = 1, s = 0;
    while (p < ct_split(L)) p *= ct_plan(L, s++);
    return s;
}
constexpr bool ct_plan_ok(int L) {
    int p = 1;
    for (int s = 0; s < ct_plan(L, -1); ++s) p *= ct_plan(L, s);
    int pa = 1;
    for (int s = 0; s < ct_split_passes(L); ++s) pa *= ct_plan(L, s);
    return p == L && pa == ct_split(L) && ct_split(L) % (L / ct_split(L)) == 0;
}
static_assert(ct_plan_ok(32) && ct_plan_ok(48) && ct_plan_ok(64) && ct_plan_ok(80) && ct_plan_ok(96) &&
                  ct_plan_ok(128) && ct_plan_ok(160) && ct_plan_ok(192) && ct_plan_ok(256) && ct_plan_ok(384) &&
                  ct_plan_ok(512),
              "radix plans must factor L with the split P >= Q, Q | P");

// One radix-R pass over NL lines of compile-time length L (same in-place
// scheme as fft_pass; the twiddles W_L^t are read from the FP64 table in
// global memory, which stays cache resident, before the first barrier).
// HALF_IN: the upper half of every line is zero (the first pass of a forward
// transform of zero-padded data; R even), so inputs r >= R/2 are not read.
// HALF_OUT: only the lower half of every line is wanted (the last pass of an
// inverse transform; R even), so outputs q >= R/2 are not written.
template <typename T, int R, int DIR, int L, int NL, int NS, int NTHR, bool HALF_IN = false, bool HALF_OUT = false>
__device__ __forceinline__ void fft_pass_ct(typename V2<T>::t* lds, const double2* tw) {
    static_assert(!(HALF_IN || HALF_OUT) || R % 2 == 0, "half-line pruning needs an even radix");
    constexpr int RIN = HALF_IN ? R / 2 : R;
    constexpr int ROUT = HALF_OUT ? R / 2 : R;
    using C = typename V2<T>::t;
    constexpr int LR = L / R;
    constexpr int B = NL * LR;
    constexpr int MAXB = (B + NTHR - 1) / NTHR;
    constexpr int LP = L | 1;
    constexpr int TSTEP = L / (NS * R);
    C v[MAXB][R];
    C w[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * NTHR;
        if ((B % NTHR) == 0 || b < B) {
            const int line = b % NL;
            const int j = b / NL;
            const C* src = lds + line * LP + j;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r < RIN) {
                    v[i][r] = src[r * LR];
                } else {
                    v[i][r].x = 0;
                    v[i][r].y = 0;
                }
            }
            if (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const double2 t = tw[r * k * TSTEP];
                    w[i][r].x = (decltype(w[i][r].x))t.x;
                    w[i][r].y = (decltype(w[i][r].y))(DIR > 0 ? -t.y : t.y);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * NTHR;
        if ((B % NTHR) == 0 || b < B) {
            const int line = b % NL;
            const int j = b / NL;
            const int k = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[i][r]);
            }
            Dft<R, DIR, C>::run(v[i]);
            C* dst = lds + line * LP + (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < ROUT; ++q) dst[q * NS] = v[i][q];
        }
    }
    __syncthreads();
}

// Every pass of a compile-time length.  HALF_IN / HALF_OUT (see fft_pass_ct)
// apply to the first / last pass; the caller sets them only when the data
// allow it (inputs e >= L/2 zero, outputs e >= L/2 unused).
template <typename T, int DIR, int L, int NL, int NTHR, bool HALF_IN = false, bool HALF_OUT = false, int S = 0,
          int NS = 1>
__device__ __forceinline__ void fft_lines_ct(typename V2<T>::t* lds, const double2* tw) {
    constexpr int NST = ct_plan(L, -1);
    if constexpr (S < NST) {
        constexpr int R = ct_plan(L, S);
        constexpr bool HI = HALF_IN && S == 0 && R % 2 == 0;
        constexpr bool HO = HALF_OUT && S == NST - 1 && R % 2 == 0;
        fft_pass_ct<T, R, DIR, L, NL, NS, NTHR, HI, HO>(lds, tw);
        fft_lines_ct<T, DIR, L, NL, NTHR, HALF_IN, HALF_OUT, S + 1, NS * R>(lds, tw);
    }
}

// L/2 pruning is exact for this length when the first pass (forward) or the
// last pass (inverse) has an even radix.
constexpr bool ct_half_in_ok(int L) { return ct_plan(L, 0) % 2 == 0; }
constexpr bool ct_half_out_ok(int L) { return ct_plan(L, ct_plan(L, -1) - 1) % 2 == 0; }

// ------------------------------------------------ register-resident passes
// The passes of ct_plan(L) on data held in registers.  Stockham indices: after
// the passes with radix product NS, element j*NS + f is frequency f of the
// NS-point transform of the subsequence x[j + (L/NS) m].  A pass only combines
// elements whose subsequence index agrees modulo Q = L/P (first group) or
// whose frequency agrees modulo P (second group), which is what lets a thread
// run a whole group on its own registers.

// The twiddle table TW is the host's FP64 W_L^t (double2) or its values
// rounded to FP32 (float2); either way the factors used equal those of the
// LDS form, which rounds the FP64 table the same way.
// First group on NCL lines of one subsequence each (the lines share the
// twiddles), thread index t: on entry v[a][m] = x_a[t + Q m]; on exit
// v[a][f] = element t*P + f of line a.  HIN: x[e] = 0 for e >= L/2 (the
// first pass reads only its lower inputs, as fft_pass_ct does).
template <typename T, int DIR, int L, bool HIN, int NCL, int S = 0, int NS = 1, typename TW>
__device__ __forceinline__ void rf_group_a(typename V2<T>::t (&v)[NCL][ct_split(L)], const TW* tw) {
    using C = typename V2<T>::t;
    constexpr int P = ct_split(L);
    if constexpr (NS < P) {
        constexpr int R = ct_plan(L, S);
        constexpr int TSTEP = L / (NS * R);
        constexpr bool HI = HIN && S == 0;
        C o[NCL][P];
#pragma unroll
        for (int u0 = 0; u0 < P / (NS * R); ++u0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                C w[R];
                if constexpr (NS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        const TW t = tw[r * k * TSTEP];
                        w[r].x = (decltype(w[r].x))t.x;
                        w[r].y = (decltype(w[r].y))(DIR > 0 ? -t.y : t.y);
                    }
                }
#pragma unroll
                for (int a = 0; a < NCL; ++a) {
                    C b[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (HI && 2 * r >= R) {
                            b[r].x = 0;
                            b[r].y = 0;
                        } else {
                            b[r] = v[a][u0 * NS + k + r * (P / R)];
                        }
                    }
                    if constexpr (NS > 1) {
#pragma unroll
                        for (int r = 1; r < R; ++r) b[r] = cmul(b[r], w[r]);
                    }
                    Dft<R, DIR, C>::run(b);
#pragma unroll
                    for (int q = 0; q < R; ++q) o[a][u0 * NS * R + k + q * NS] = b[q];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < NCL; ++a) {
#pragma unroll
            for (int i = 0; i < P; ++i) v[a][i] = o[a][i];
        }
        rf_group_a<T, DIR, L, HIN, NCL, S + 1, NS * R>(v, tw);
    }
}

// Second group on residue classes kappa_c = t + Q c (c < P/Q) of the first
// group's frequency, NCL lines sharing the twiddles: on entry
// v[a][c*Q + jj] = element jj*P + kappa_c of line a; on exit
// v[a][c*Q + g] = X_a[kappa_c + P g].  HOUT: only X[e], e < L/2, is wanted
// (the last pass computes only its lower outputs, as fft_pass_ct does).
template <typename T, int DIR, int L, bool HOUT, int NCL, int S = ct_split_passes(L), int NS = ct_split(L),
          typename TW>
__device__ __forceinline__ void rf_group_b(typename V2<T>::t (&v)[NCL][ct_split(L)], int t, const TW* tw) {
    using C = typename V2<T>::t;
    constexpr int P = ct_split(L);
    constexpr int Q = L / P;
    constexpr int NST = ct_plan(L, -1);
    if constexpr (S < NST) {
        constexpr int R = ct_plan(L, S);
        constexpr int TSTEP = L / (NS * R);
        constexpr bool HO = HOUT && S == NST - 1;
        constexpr int G = NS / P;
        C o[NCL][P];
#pragma unroll
        for (int c = 0; c < P / Q; ++c) {
            const int kappa = t + Q * c;
#pragma unroll
            for (int jh = 0; jh < L / (NS * R); ++jh) {
#pragma unroll
                for (int gk = 0; gk < G; ++gk) {
                    const int ks = kappa + P * gk;
                    C w[R];
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        const TW tt = tw[r * ks * TSTEP];
                        w[r].x = (decltype(w[r].x))tt.x;
                        w[r].y = (decltype(w[r].y))(DIR > 0 ? -tt.y : tt.y);
                    }
#pragma unroll
                    for (int a = 0; a < NCL; ++a) {
                        C b[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) b[r] = v[a][c * Q + (jh + r * (L / (R * NS))) * G + gk];
#pragma unroll
                        for (int r = 1; r < R; ++r) b[r] = cmul(b[r], w[r]);
                        Dft<R, DIR, C>::run(b);
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            if (!HO || 2 * q < R) o[a][c * Q + jh * G * R + gk + q * G] = b[q];
                            else o[a][c * Q + jh * G * R + gk + q * G] = b[0];   // never stored
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < NCL; ++a) {
#pragma unroll
            for (int i = 0; i < P; ++i) v[a][i] = o[a][i];
        }
        rf_group_b<T, DIR, L, HOUT, NCL, S + 1, NS * R>(v, t, tw);
    }
}

// Stage the W_L^t table of an axis into LDS (FP64 table converted to T).
template <typename T, int NTHR = NT>
__device__ __forceinline__ void load_twiddles(typename V2<T>::t* dst, const double2* tw64, const AxisPlan& pl) {
    using C = typename V2<T>::t;
    for (int i = threadIdx.x; i < pl.L; i += NTHR) {
        double2 w = tw64[pl.tw + i];
        C c;
        c.x = (T)w.x;
        c.y = (T)w.y;
        dst[i] = c;
    }
}

// ---------------------------------------------------------------- reductions

// Sum NV doubles over the workgroup; the result is valid in thread 0.
// Fixed order: xor-butterfly inside each 64-lane wavefront, then the four
// wavefront sums in index order.
template <int NV, int NTHR = NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
    }
    if constexpr (NTHR == 64) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wid * NV + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = sh[i];
            for (int w = 1; w < NTHR / 64; ++w) s += sh[w * NV + i];
            v[i] = s;
        }
    }
    __syncthreads();
}

// Doubles of partial sums per workgroup and right-hand side.
constexpr int PSTRIDE = 8;

// This workgroup's sums go to partials[(OFF + i) * stride + blk], stride the
// workgroups reserved per right-hand side: slot-major, so a finalize's loads
// of one slot over consecutive workgroups are contiguous (no atomics, no
// fences: the consumer is a later kernel on the same stream).  Two kernels
// with the same grid may fill disjoint slots of one workgroup.
template <int NV, int NTHR = NT, int OFF = 0>
__device__ __forceinline__ void publish_partial(double (&v)[NV], double* partials, int blk, int stride, double* sh) {
    static_assert(OFF + NV <= PSTRIDE, "partial slots");
    block_sum<NV, NTHR>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) partials[(long)(OFF + i) * stride + blk] = v[i];
    }
}

// Sum the partials of nblk workgroups in block order; result in thread 0.
// The loop is unrolled so that several blocks' loads are in flight before
// the first add (the adds keep their order).
template <int NV>
__device__ __forceinline__ void sum_partials(double (&acc)[NV], const double* partials, int nblk, int stride,
                                             double* sh) {
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblk; b += NT) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += partials[(long)i * stride + b];
    }
    block_sum<NV>(acc, sh);
}

}  // namespace dda
