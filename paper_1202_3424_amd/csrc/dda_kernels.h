// Host-visible declarations of the DDA kernels' launchers and the argument
// blocks they take.  Included by the kernels file and by the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "dda_device.h"

namespace dda {

// Start/stop events for the next matvec-pass launch on this thread: when
// set, DDA_LAUNCH issues it with hipExtLaunchKernelGGL so that the events
// carry the kernel's own execution timestamps, then clears them.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
LaunchEvents& launch_events();

#define DDA_LAUNCH(kernel, grid, block, shmem, stream, ...)                                               \
    do {                                                                                                \
        ::dda::LaunchEvents& ev_ = ::dda::launch_events();                                              \
        if (ev_.start) {                                                                                \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0, __VA_ARGS__); \
            ev_ = ::dda::LaunchEvents{};                                                                \
        } else {                                                                                        \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                        \
        }                                                                                               \
    } while (0)

// One right-hand side of a launch over several targets that share the
// padded grid (a ragged batch): its target's bounding box and site count, kd,
// where that target's occupancy map, materials, coordinates and permutation
// start in the batch's concatenated arrays, its tensor octants (FP64 and FP32),
// and the workgroup counts its own single-target solve uses for
// the x passes and for the site kernels (a right-hand side reduces over
// exactly those blocks, so its results equal that solve's bitwise).
struct RhsGeo {
    int n[3];
    int nsites;
    long long map_off;
    int site_off;
    int pass_blocks;
    int site_blocks;
    int pad;
    double kd;
    const void* ghat[2];   // tensor FFT: FP64 (double2), FP32 (float2)
};

// Geometry of one target's FFT grid.
//   n[a]  occupied bounding-box extent on axis a (x = first ijk index); in a
//         ragged batch the largest over its targets
//   M[a]  padded FFT extent (>= 2n-1)
//   H[a]  M[a]/2 + 1: extent of the stored octant of the tensor FFT
// Grids hold NC complex components interleaved per point, point index
// (z * My + y) * Mx + x, right-hand side outermost.
//   tw32  the twiddle tables W_L^t rounded to FP32 (the FP64 tables' offsets)
//   rg    per right-hand side geometry of a ragged batch, or null (one target)
struct Geo {
    int n[3];
    int M[3];
    int H[3];
    long long npts;
    AxisPlan ax[3];
    const float2* tw32;
    const RhsGeo* rg;
};

// Site-indexed FP64 vectors of one batched solve, each [nrhs][n3] with
// n3 = 3 * nsites, sites in box-scan order (x fastest, then y, then z).
struct SiteArgs {
    int nsites;
    long long n3;
    int nrhs;
    int nmat;
    const int* map;        // [nz][ny][nx] -> sorted site index or -1
    const int* mat;        // [nsites] material index
    const double2* ainv;   // [nrhs][nmat][3] diagonal of 1/alpha
    double2* x;
    double2* r;
    double2* rhat;
    double2* p;
    double2* v;
    double2* t;
    double2* b;
    double2* u2;           // BiCGstab(2): third search vector
    double2* r2;           // BiCGstab(2): third residual
    const double2* in;     // input of the plain / conjugated product
    double2* out;          // output of the plain / conjugated product
    RhsState* st;          // [nrhs]
    double* partials;      // [nrhs][PSTRIDE][maxblk] per-workgroup sums of the last reducing kernel
    double* chains;        // [nrhs][PSTRIDE][NT] k_finalize's per-thread sums of them, or null
    int maxblk;
    int slot;              // RhsState::red slot written by the conjugated product
    double kd;
    // ragged batch (else null): per right-hand side geometry; n3 and nmat
    // are then the strides (largest target) of the site vectors and of 1/alpha
    const RhsGeo* rg;
};

// Sites of right-hand side q, its kd, and where its target's sites start in
// the map / material / coordinate arrays.
__device__ __forceinline__ long long rhs_n3(const SiteArgs& a, int q) { return a.rg ? 3LL * a.rg[q].nsites : a.n3; }
__device__ __forceinline__ double rhs_kd(const SiteArgs& a, int q) { return a.rg ? a.rg[q].kd : a.kd; }
__device__ __forceinline__ int rhs_site_off(const SiteArgs& a, int q) { return a.rg ? a.rg[q].site_off : 0; }
// workgroups of the site kernels for right-hand side q (a ragged batch
// launches the largest count; the extra workgroups of smaller targets exit)
__device__ __forceinline__ int rhs_site_blocks(const SiteArgs& a, int q) {
    return a.rg ? a.rg[q].site_blocks : (int)gridDim.x;
}

// SC_Q / GA_Q: the QMR iteration (p = r + beta p with the pending smoothing
// step; v = A p with p^T v).  SC_B0..SC_B3 / GA_B1..GA_B3: the four products
// of a BiCGstab(2) iteration (vectors: r_0 = r, r_1 = t, r_2 = r2, u_0 = p,
// u_1 = v, u_2 = u2, shadow residual rhat; GA_V serves the first product).
enum ScatterMode { SC_PLAIN = 0, SC_CONJ = 1, SC_P = 2, SC_S = 3, SC_Q = 4, SC_B0 = 5, SC_B1 = 6, SC_B2 = 7, SC_B3 = 8 };
enum GatherMode { GA_PLAIN = 0, GA_CONJ = 1, GA_V = 2, GA_T = 3, GA_RES = 4, GA_Q = 5, GA_B1 = 6, GA_B2 = 7, GA_B3 = 8 };
// which right-hand sides a pass skips
enum Check { CHK_NONE = 0, CHK_ACTIVE = 1 };
// what k_finalize makes of the partial sums of the kernel before it
enum FinKind {
    // BiCGSTAB: alpha after the first product; the half-step check, omega,
    // rho, beta and the status after the second; the pending flag cleared
    // after k_bicg_flush
    FIN_V = 0, FIN_T, FIN_FLUSH, FIN_COLD, FIN_WARM, FIN_RESTART, FIN_QSUM, FIN_RES, FIN_CONJ, FIN_REFINE,
    // QMR: after the product (alpha), after the update (smoothing, beta,
    // status), after the cold / warm start, after an FP64 refinement residual
    // and after k_qmr_final (clears the pending smoothing step)
    FIN_QV, FIN_QUPD, FIN_QCOLD, FIN_QWARM, FIN_QREFINE, FIN_QFINAL,
    // BiCGstab(2): beta after the second product, the minimal-residual
    // coefficients after the fourth, status and beta after the update
    FIN_B_BETA, FIN_B_MR, FIN_B_UPD
};

// partial-sum slots k_finalize reads for a kind
__host__ __device__ constexpr int fin_slots(int kind) {
    return (kind == FIN_B_MR || kind == FIN_T) ? 8
           : (kind == FIN_QUPD || kind == FIN_QCOLD || kind == FIN_QWARM || kind == FIN_QREFINE || kind == FIN_QV)
               ? 4
               : 3;
}

// FFT lengths with compile-time kernels (dda_passes.h)
inline bool ct_length(int L) {
    return L == 32 || L == 48 || L == 64 || L == 80 || L == 96 || L == 128 || L == 160 || L == 192 || L == 256 ||
           L == 384 || L == 512;
}

// tile sizes chosen by the host: x-lines (along y) per workgroup of the x
// passes, x columns per workgroup of the strided passes
int x_lines_per_tile(const Geo& g, int nrhs, bool fp32);
int strided_cols_per_tile(int L, int nc, bool fp32);
// workgroups of the x passes and of the site-level kernels, per right-hand side
int x_pass_blocks(const Geo& g, int nrhs, bool fp32);
int site_blocks_for(long long n3, int nrhs);

template <typename T>
void launch_scatter_x(int mode, int chk, const Geo& g, const SiteArgs& a, typename V2<T>::t* grid, const double2* tw,
                      hipStream_t s);
template <typename T>
void launch_gather_x(int mode, int chk, const Geo& g, const SiteArgs& a, const typename V2<T>::t* grid,
                     const double2* tw, hipStream_t s);
// strided FFT along axis 1 (y) or 2 (z) over lines whose other coordinates
// are x in [0, Mx) and outer in [0, n_outer); loads e < lin (zero beyond),
// stores e < lout; ghat != null fuses forward FFT, tensor product, inverse.
// variant: one of strided_variants(L, ghat != null) compile-time tilings
// (all give bitwise-identical results; the autotuner picks the fastest)
template <typename T>
void launch_strided(int axis, int dir, int chk, const Geo& g, int nrhs, int nc, int n_outer, int lin, int lout,
                    typename V2<T>::t* grid, const double2* tw, const typename V2<T>::t* ghat, const RhsState* st,
                    hipStream_t s, int variant = 0);
inline int strided_variants(int L, bool gh) { return ct_length(L) ? (gh ? 28 : 12) : 1; }
// the variants a ragged batch runs: every y-pass variant, and the pass-3
// variants that take one right-hand side per workgroup (each right-hand side
// reads its own tensor and extent); the others run as variant 3 there
constexpr bool ragged_variant(int gh, int v) {
    return !gh || !(v == 0 || v == 1 || v == 2 || v == 7 || v == 8 || v == 9);
}
// The interaction tensor on the padded grid is held as two three-component
// slabs [2][npts][3]: (xx, xy, xz) and (yy, yz, zz), so that its transforms
// run as the three-component passes with two right-hand sides.
void launch_xgrid3(const Geo& g, double2* grid, const double2* tw, hipStream_t s);

void launch_green_sample(const Geo& g, double kd, double2* G, hipStream_t s);
void launch_green_octant(const Geo& g, const double2* G, double2* gh64, float2* gh32, hipStream_t s);
// 1/alpha (scheme + 2: its derivative in eps) per (right-hand side, material)
// from the target's distinct refractive indices mats [nmat] and the ambient
// medium's index
void launch_alpha(int nrhs, int nmat, const double2* mats, double m_medium, const double* khat, const double2* e0,
                  double kd, int scheme, double2* ainv, hipStream_t s, int ostride = 0);
void launch_einc(const SiteArgs& a, const int* coords, const double* khat, const double2* e0, hipStream_t s);
void launch_init_cold(const SiteArgs& a, int site_blocks, hipStream_t s);
void launch_init_warm(const SiteArgs& a, int site_blocks, hipStream_t s);
// BiCGSTAB: apply the pending end of the latest iteration to x and r
void launch_bicg_flush(const SiteArgs& a, int site_blocks, hipStream_t s);
void launch_restart(const SiteArgs& a, int site_blocks, hipStream_t s);
// QMR: start (cold: r = b, x = 0; warm: r holds b - A x), update, and the
// pending smoothing step applied to x (x <- the smoothed iterate)
void launch_qmr_init(const SiteArgs& a, bool cold, int site_blocks, hipStream_t s);
void launch_qmr_update(const SiteArgs& a, int site_blocks, hipStream_t s);
void launch_qmr_final(const SiteArgs& a, int site_blocks, hipStream_t s);
// BiCGstab(2): x += g1 r + g2 t, r -= g1 t + g2 r2, p -= g1 v + g2 u2
void launch_b2_update(const SiteArgs& a, int site_blocks, hipStream_t s);
void launch_qsum(const SiteArgs& a, int site_blocks, hipStream_t s);
// far-field amplitudes: P sorted [nrhs][nsites][3], dirs [ndir][9] (n, theta,
// phi), f [nrhs][ndir][2], dcs [nrhs][ndir]; every site coordinate lies in the
// box lo .. lo + n - 1
void launch_farfield(int nsites, const int* coords, const double2* P, int nrhs, const double* dirs, int ndir,
                     double k, const int lo[3], const int n[3], double2* f, double* dcs, hipStream_t s);
// the direction sets of the angular averages for ng right-hand sides
// (incidence directions kh [ng][3], Gauss-Legendre nodes mu [n_theta]):
// dirs [ng][n_theta][n_phi][9]
void launch_avg_dirs(int ng, const double* kh, const double* mu, int n_theta, int n_phi, double* dirs,
                     hipStream_t s);
// the same with a set of per directions for each right-hand side: dirs
// [nrhs * per][9], f [nrhs * per][2], dcs [nrhs * per]
void launch_farfield_sets(int nsites, const int* coords, const double2* P, int nrhs, const double* dirs, int per,
                          double k, const int lo[3], const int n[3], double2* f, double* dcs, hipStream_t s);
// near field on an extended lattice box (first point org, extents dims):
// P (caller order) into the box-scan site vector x at the target's sites;
// E_sca = -v and E_inc at every point (either output may be null); the
// trilinear line a..b of n points through E [nrhs][box][3]
void launch_nf_place(int nsites, const int* perm, const int* coords, const double2* P, int nrhs, const int org[3],
                     const int dims[3], double2* x, hipStream_t s);
void launch_nf_out(int nrhs, const int org[3], const int dims[3], const double* khat, const double2* e0, double kd,
                   const double2* v, double2* einc, double2* esca, hipStream_t s);
void launch_field_line(int nrhs, const int org[3], const int dims[3], const double2* E, const double a[3],
                       const double b[3], int n, double2* out, hipStream_t s);
// nblk: the producer's workgroups per right-hand side; in a ragged batch
// NBLK_PASS / NBLK_SITE take each right-hand side's own count from a.rg
constexpr int NBLK_PASS = -1, NBLK_SITE = -2;
// Where a right-hand side has at least FIN_CHAIN_MIN workgroups of partial
// sums (and a.chains is set), k_chain_sums first forms each k_finalize
// thread's sum of them, one workgroup per slot and right-hand side, with the
// same additions in the same order; k_finalize then only forms the
// workgroup's tree, so the results are bitwise those of one workgroup.
constexpr int FIN_CHAIN_MIN = 2048;
void launch_finalize(const SiteArgs& a, int kind, int nblk, hipStream_t s);
// width complex values per site; to_sorted: dst[sorted] = src[caller], else dst[caller] = src[sorted]
void launch_permute(int nrhs, int nsites, int width, const int* perm, const double2* src, double2* dst,
                    bool to_sorted, hipStream_t s);
void launch_fill(double2* p, long long n, hipStream_t s);
void launch_set_state(RhsState* st, int nrhs, double tol, int max_iter, hipStream_t s);
void launch_grad(const SiteArgs& a, const double2* dainv, double w_qabs, double2* grad, hipStream_t s);
void launch_adjoint_rhs(const SiteArgs& a, const double2* P_sorted, double w_qabs, double w_qext, hipStream_t s);

}  // namespace dda
