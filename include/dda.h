/*
 * dda.h -- C ABI of the MI355X (gfx950) discrete-dipole-approximation solver.
 *
 * The library solves A P = E for the 3N complex dipole polarizations P of a
 * target made of N point dipoles on a cubic lattice, and returns P together
 * with the efficiency factors Q_ext, Q_abs, Q_sca and Q_pha.  The problem
 * statement follows the DDSCAT 7.2 User Guide (Draine & Flatau,
 * arXiv:1202.3424):
 *   - A P = E and the error measure: section "Choice of Iterative Algorithm"
 *     (eq. AP=E and eq. err_tol);
 *   - occupied lattice sites and per-site composition: "Target Generation:
 *     Isolated Finite Targets" (the IXYZ/ICOMP site lists of FROM_FILE);
 *   - refractive index per material and the ambient medium: "Dielectric
 *     Functions" and "Application to Targets in Dielectric Media";
 *   - wavelength and effective radius: "Vacuum Wavelengths", "Target Size
 *     a_eff" and "Applicability of the DDA" (a_eff = (3N/4pi)^(1/3) d);
 *   - incident direction and polarization in the target frame: "Target
 *     Orientation" and "Incident Polarization State";
 *   - TOL and MXITER: "Error Tolerance", "Maximum Number of Iterations";
 *   - polarizability prescriptions LATTDR / GKDLDR: "Dipole Polarizabilities";
 *   - Q_ext, Q_abs, Q_sca, Q_pha: "What Does It Calculate?";
 *   - P and 1/alpha as stored for post-processing: appendix ".pol Files".
 * The interaction matrix is applied as an FFT convolution on a zero-padded
 * grid ("Choice of FFT Algorithm"), inside BiCGSTAB, QMR for complex-symmetric
 * A or BiCGstab(2) (the PBCGST, QMRCCG and PBCGS2 options).  From P the
 * library also gives the far-field amplitudes, the Mueller matrix and the
 * averages over scattering directions, the electric field in and around the
 * target ("Near-Field Calculations"), and the adjoint gradient of Q_abs and
 * Q_ext in the per-site permittivity.
 *
 * Conventions
 *   - Lengths are in units of the lattice spacing d internally; E0 has unit
 *     amplitude; the phase of E_inc is referred to lattice index (0,0,0).
 *   - Complex numbers are {re, im} pairs of doubles (dda_c64).
 *   - Site-indexed device arrays are [n_rhs][n_sites][3] dda_c64, row-major,
 *     in the caller's site order (the order of ijk passed to
 *     dda_target_create).
 *   - Every function returns a dda_status; nothing throws or exits across
 *     the ABI.  After a non-OK status, dda_last_error() describes it.
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied.  Device arrays are owned by the caller and never freed by the
 *     library.  Handles are owned by the library until *_destroy.
 *   - Work is enqueued on the context's HIP stream; functions that return
 *     results on the host synchronise that stream before returning.
 *   - A context and the targets created from it must be used from one host
 *     thread at a time.
 */
#ifndef DDA_H
#define DDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } dda_c64;

typedef enum {
    DDA_OK = 0,
    DDA_E_INVALID = 1,        /* bad argument (see dda_last_error) */
    DDA_E_NOMEM = 2,          /* device or host allocation failed */
    DDA_E_DEVICE = 3,         /* a HIP call failed */
    DDA_E_NOT_CONVERGED = 4,  /* max_iter reached; best iterate returned */
    DDA_E_BREAKDOWN = 5,      /* Krylov breakdown (BiCGSTAB, BiCGstab(2): after one restart) */
    DDA_E_NONFINITE = 6       /* NaN or Inf met in the iteration */
} dda_status;

/* Polarizability prescription ("Dipole Polarizabilities"). */
typedef enum { DDA_LATTDR = 0, DDA_GKDLDR = 1 } dda_polarizability;

/* Iterative method ("Choice of Iterative Algorithm"):
 *   DDA_BICGSTAB  PBCGST: BiCGSTAB (van der Vorst 1992), two products per
 *                 iteration; stops when the recursive residual satisfies
 *                 |r| / |E| < tol, checked after the half step (|s|) and
 *                 after the iteration (|r|^2 = |s|^2 - |<t,s>|^2 / |t|^2, the
 *                 norm of s - omega t).
 *   DDA_QMR_SYM   QMRCCG: QMR for complex-symmetric A, read as COCG (van der
 *                 Vorst & Melissen 1990) with quasi-minimal-residual smoothing
 *                 (Zhou & Walker 1994); one product per iteration; stops on
 *                 the smoothed residual |E - A P| / |E| < tol and returns the
 *                 smoothed iterate.  A breakdown (p^T A p or r^T r vanishing)
 *                 ends the solve with DDA_E_BREAKDOWN and that iterate (no
 *                 restart).
 *   DDA_BICGSTAB2 PBCGS2: BiCGstab(l) with l = 2 (Sleijpen & Fokkema 1993), four
 *                 products per iteration (iters counts these iterations);
 *                 stops on |E - A P| / |E| < tol after an iteration.
 * Breakdown: an inner product that divides (<rhat, A p>, <rhat, r>, <t, s>;
 * p^T A p, r^T r for QMR) is taken as zero when its modulus is at most 1e-12
 * times the product of the norms of its two vectors (FP64 rounding level).
 * BiCGSTAB and BiCGstab(2) then restart once from the current iterate with
 * the shadow residual conj(r) in place of r (for A = A^T the form <conj(r),
 * A r> = r^T A r is independent of <r, A r>, so a breakdown in the first
 * step after a start is not repeated); a second breakdown ends the solve
 * with DDA_E_BREAKDOWN. */
typedef enum { DDA_BICGSTAB = 0, DDA_QMR_SYM = 1, DDA_BICGSTAB2 = 2 } dda_solver;

/* Arithmetic of the FFT matrix-vector product.  The Krylov recurrences,
 * inner products, diagonal term and residual checks are FP64 in both modes
 * ("Single vs. Double Precision" offers whole-program single or double). */
typedef enum { DDA_FP64 = 0, DDA_FP32_MATVEC = 1 } dda_precision;

typedef struct dda_ctx dda_ctx;
typedef struct dda_target dda_target;

/* One right-hand side: propagation direction khat (unit vector) and complex
 * polarization e0 (normalised by the library; must be transverse to khat),
 * both in the target frame. */
typedef struct {
    double khat[3];
    dda_c64 e0[3];
} dda_incidence;

/* dda_opts.flags */
#define DDA_FLAG_RECOMPUTE_GREEN 1u  /* rebuild the FFT of the Green tensor even if cached */
#define DDA_FLAG_NO_FINAL_CHECKS 2u  /* skip the true-residual and eq. err_tol matvecs */
#define DDA_FLAG_NO_AUTOTUNE 4u      /* use the default kernel tiling instead of timing the
                                        variants once per grid shape (results are identical) */
#define DDA_FLAG_NO_GRAPH 8u         /* dda_solve_batched: launch the Krylov iterations one kernel at
                                        a time instead of replaying a captured HIP graph of each
                                        chunk of iterations (with several targets in flight the
                                        host's launch rate is the limit; single-target calls always
                                        launch directly; with kernel timing on, one chunk in the
                                        timing sample period runs as direct launches) */
#define DDA_FLAG_SEPARATE_TARGETS 16u /* dda_solve_batched: give this target launches of its own
                                         instead of sharing them with the other targets on the
                                         same padded grid (results are identical) */

typedef struct {
    double wavelength;   /* vacuum wavelength (any physical unit) > 0 */
    double aeff;         /* effective radius, same unit > 0 */
    double m_medium;     /* real refractive index of the ambient medium > 0 (1 = vacuum) */
    double tol;          /* stop when |E - A P| / |E| < tol; > 0 */
    int32_t max_iter;    /* iteration cap >= 1 (matvecs per iteration: BiCGSTAB 2, QMR 1,
                            BiCGstab(2) 4) */
    int32_t polarizability;  /* dda_polarizability */
    int32_t solver;          /* dda_solver */
    int32_t precision;       /* dda_precision */
    uint32_t flags;          /* DDA_FLAG_* */
    int32_t kernel_variant;  /* 0: automatic; v > 0 forces tiling variant v-1 of the
                                strided FFT passes where it exists (for testing; every
                                variant computes bitwise-identical results) */
} dda_opts;

typedef struct {
    double qext, qabs, qsca, qpha;   /* efficiency factors; qsca = qext - qabs */
    double rel_residual;             /* true |E - A P| / |E| at the returned P */
    double normal_eq_residual;       /* |A^H A P - A^H E| / |A^H E| (eq. err_tol) */
    double kd;                       /* k d in the ambient medium */
    double aeff_d;                   /* a_eff / d */
    int32_t iters;                   /* iterations of the chosen solver taken */
    int32_t matvecs;                 /* FFT matrix-vector products in the iteration */
    int32_t status;                  /* dda_status of this right-hand side */
    int32_t restarts;                /* breakdown restarts taken (0 or 1) */
    int32_t refinements;             /* FP64 residual refinements (DDA_FP32_MATVEC) */
    int32_t reserved;
} dda_result;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
dda_status dda_ctx_create(int device, void* hip_stream, dda_ctx** out);
dda_status dda_ctx_destroy(dda_ctx* ctx);

/* Upload a target.
 *   ijk    host int32 [n_sites][3]: lattice indices of the occupied sites
 *          (any integers; duplicates are an error).
 *   m_site host dda_c64 [n_sites]: complex refractive index of each site
 *          (equal values share one material).
 * The library keeps sorted device copies, the occupancy map of the bounding
 * box and, lazily, the FFT of the interaction tensor per (kd, precision).
 * Errors: DDA_E_INVALID for n_sites < 1, duplicate sites, a box extent above
 * 256 on an axis (a padded FFT extent above 512), more than 65535 distinct
 * materials, a vacuum site (m = 1) or non-finite m; DDA_E_NOMEM. */
dda_status dda_target_create(dda_ctx* ctx, int64_t n_sites, const int32_t* ijk,
                             const dda_c64* m_site, dda_target** out);
dda_status dda_target_destroy(dda_target* t);

/* Geometry of a target: box[3] = bounding-box extents n, grid[3] = padded
 * FFT extents M >= 2n - 1 (every separation -(n-1)..n-1 its own slot, so the
 * circulant product is exactly the Toeplitz one).  With m the smooth extent
 * (2n when 2,3,5-smooth, else the smallest 2,3,5-smooth value >= 2n - 1), M is
 * the smallest of the compile-time lengths 32, 48, 64, 80, 96, 128, 160, 192,
 * 256, 384, 512 that is >= 2n - 1, when 5 M <= 7 m; else m. */
dda_status dda_target_geometry(const dda_target* t, int32_t box[3], int32_t grid[3]);

/* y = A x for n_rhs right-hand sides (A depends on the incidence through
 * 1/alpha).  x, y: device [n_rhs][n_sites][3], caller order; x and y may not
 * alias.  Enqueued on the context stream; returns without synchronising. */
dda_status dda_apply(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs,
                     const dda_incidence* inc, const dda_c64* x, dda_c64* y);

/* dda_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same product (the same kernels: results are bitwise those of dda_apply),
 * with every work buffer -- the incidences, 1/alpha, the sorted input and
 * output site vectors and the padded FFT grid -- taken from one fixed
 * 128 MiB (134217728-byte) device array that the library holds on each GPU it
 * runs on until the process ends; the call makes no hipMalloc or hipFree.
 *   Needs, rounded up to 256 bytes per part: n_rhs * (72 + 48 n_materials
 *   + 96 n_sites + 24 c M) bytes, c = 2 (DDA_FP64) or 1 (DDA_FP32_MATVEC),
 *   M = the padded grid's point count; E_INVALID above the 128 MiB, or for
 *   n_rhs outside 1..256.
 *   The FFT of the interaction tensor at this kd and precision must already
 *   be built on the target (by a dda_apply or dda_solve call with the same
 *   wavelength, aeff, m_medium and precision), else E_INVALID; so must not
 *   DDA_FLAG_RECOMPUTE_GREEN be set.  The strided-pass tiling is the one the
 *   autotuner chose for this shape, if any, else the default (or
 *   opts->kernel_variant); no timing events are recorded.
 * x, y, inc and the errors otherwise as dda_apply.  The work array keeps the
 * last call's contents and nothing in it needs to start at zero; every call
 * on one GPU shares it, so calls that overlap on one GPU (several streams or
 * host threads) race and must be serialised by the caller.  Enqueued on the
 * context's stream; returns without synchronising. */
dda_status dda_apply_noalloc(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs,
                             const dda_incidence* inc, const dda_c64* x, dda_c64* y);

/* Solve A P = E for n_rhs incidences on one target (batched in every kernel;
 * the right-hand sides share the interaction-tensor FFT).
 *   P   device [n_rhs][n_sites][3] output (may be NULL: Q only);
 *   P0  device warm start of the same shape, or NULL for P = 0;
 *   res host [n_rhs] results.
 * Returns the worst per-right-hand-side status (DDA_OK if all converged);
 * the best iterate and its residuals are returned in every case. */
dda_status dda_solve(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs,
                     const dda_incidence* inc, dda_c64* P, const dda_c64* P0, dda_result* res);

/* Solve A x = b for caller-given right-hand sides (the system of "Choice of
 * Iterative Algorithm" with any b, e.g. the localized right-hand side of a
 * perturbed site).  A is the matrix of the given incidences (1/alpha depends
 * on them through LATTDR/GKDLDR).
 *   b   device [n_rhs][n_sites][3], caller order (not modified);
 *   x   device output of the same shape;
 *   x0  device warm start or NULL;
 *   res host [n_rhs]: residuals, iterations and status; the efficiency fields
 *       are zero (b is not an incident field).
 * Returns the worst per-right-hand-side status, as dda_solve. */
dda_status dda_solve_rhs(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs,
                         const dda_incidence* inc, const dda_c64* b, dda_c64* x, const dda_c64* x0,
                         dda_result* res);

/* Solve several targets, each with its own right-hand sides, in one call.
 *   targets[n_targets], opts[n_targets];
 *   rhs_target[n_rhs] gives the target index of each right-hand side,
 *   inc[n_rhs], P[n_rhs] (per right-hand side device pointer of
 *   [n_sites(target)][3], or NULL), res[n_rhs].
 * Targets whose padded grids are equal, with compile-time FFT lengths on every
 * axis (32, 48, 64, 80, 96, 128, 160, 192, 256), and whose options agree in
 * solver, precision, flags and kernel_variant share every launch: one kernel
 * per step covers all their right-hand sides, each reading its own target's
 * box, sites, materials, kd and tensor.  Other targets run as their own
 * batches on up to four streams: the first calls of a batch shape (the jobs'
 * grids, right-hand sides, solver and precision) try 4, 2 and 1 jobs in
 * flight, and later calls of that shape use the fastest (not with
 * DDA_FLAG_NO_AUTOTUNE: 4).  Every right-hand side's result is bitwise the
 * one dda_solve gives for its target and its right-hand sides alone, whatever
 * the schedule.
 * A target may appear under several indices only with one kd (equal
 * wavelength and aeff); E_INVALID otherwise. */
dda_status dda_solve_batched(dda_ctx* ctx, int32_t n_targets, dda_target* const* targets,
                             const dda_opts* opts, int32_t n_rhs, const int32_t* rhs_target,
                             const dda_incidence* inc, dda_c64* const* P, dda_result* res);

/* Gradient of w_qabs*Q_abs + w_qext*Q_ext with respect to the permittivity
 * eps_j = m_j^2 of every site, for one incidence, by the adjoint method (A is
 * complex symmetric, so the adjoint system reuses the forward matvec).
 *   P     device [n_sites][3] converged solution from dda_solve (caller order);
 *   grad  device [n_sites] output, dQ/dRe(eps_j) + i dQ/dIm(eps_j);
 *   adj   host result of the adjoint solve (iterations, residual, status). */
dda_status dda_grad_eps(dda_ctx* ctx, dda_target* t, const dda_opts* opts, const dda_incidence* inc,
                        const dda_c64* P, double w_qabs, double w_qext, dda_c64* grad,
                        dda_result* adj);

/* Near field ("Near-Field Calculations"; the volume of "Additional
 * Nearfield Calculation?").  The volume is the target's bounding box grown by
 * round(r_i * n_a) lattice points on each side, ext = (r1, r2, r3, r4, r5, r6)
 * for -x, +x, -y, +y, -z, +z and n_a the box's extent in sites on axis a;
 * 0 <= r_i <= 16, and each grown extent must allow a padded FFT extent of at
 * most 512, i.e. at most 256 points (E_INVALID otherwise).  dda_nearfield_volume writes the lattice
 * coordinates of the volume's first point (origin) and its extents (dims). */
dda_status dda_nearfield_volume(const dda_target* t, const double ext[6], int32_t origin[3], int32_t dims[3]);

/* At every point j of that volume: the incident field E_inc,j = e exp(i kd
 * khat . r_j) (phase origin at lattice index (0, 0, 0), as in dda_solve) and
 * the field of the target's dipoles, the dipole at j itself excluded:
 *   E_sca,j = - sum_{l != j} A_jl P_l
 * (the guide's E_sca; the total field is E_inc + E_sca, and at a target site
 * P_j = alpha_j (E_inc,j + E_sca,j) holds to the solve's tolerance).  It is
 * one FFT product on the volume with a zero diagonal, in the precision of
 * opts (FP32_MATVEC: FP32 product).  kd is the target's (opts and its site
 * count).
 *   inc    host [n_rhs] incidences (for E_inc)
 *   P      device [n_rhs][n_sites][3], caller order (as dda_solve writes it)
 *   E_inc  device [n_rhs][dims z][dims y][dims x][3] output, or NULL
 *   E_sca  device, same shape, output
 * Enqueued on the context's stream (no host synchronisation).  The volume's
 * site map and tensor FFT are built on the first call for an extension and
 * kept with the target until another extension is asked for or the target is
 * destroyed. */
dda_status dda_nearfield(dda_ctx* ctx, dda_target* t, const dda_opts* opts, const double ext[6], int32_t n_rhs,
                         const dda_incidence* inc, const dda_c64* P, dda_c64* E_inc, dda_c64* E_sca);

/* Values of a lattice field along a line (the guide's readnf program, section
 * "The Program readnf"): n_points equally spaced points from a to b inclusive
 * (lattice coordinates; a alone when n_points = 1), each the trilinear
 * interpolation of the 8 surrounding lattice points (the guide does not state
 * readnf's interpolation; trilinear reproduces its printed track).
 *   E    device [n_rhs][dims z][dims y][dims x][3], first point at origin
 *   out  device [n_rhs][n_points][3] output
 * E_INVALID if a or b lies outside the box [origin, origin + dims - 1].
 * Enqueued on the context's stream. */
dda_status dda_field_line(dda_ctx* ctx, int32_t n_rhs, const int32_t origin[3], const int32_t dims[3],
                          const dda_c64* E, const double a[3], const double b[3], int32_t n_points, dda_c64* out);

/* Far-field scattering amplitudes ("Scattering by Finite Targets: The Mueller
 * Matrix"; Draine 1988).  For each right-hand side q and direction d:
 *   A = k^3 sum_j P_qj exp(-i k n_d . r_j)  (lattice units, r_j = the ijk of
 *   dda_target_create, k = kd of opts),
 *   f[q][d][0] = theta_d . A, f[q][d][1] = phi_d . A  (the guide's f_ml with
 *   m = 1, 2 for the scattered polarizations theta_d, phi_d),
 *   dcs[q][d] = (|f_0|^2 + |f_1|^2) / k^2  (differential scattering cross
 *   section per steradian, in units of d^2; over pi a_eff^2 at theta = 180
 *   deg this is Q_bk).
 * P: device [n_rhs][n_sites][3] in the caller's site order (as dda_solve
 * writes it).  n_hat, theta_hat, phi_hat: host [n_dir][3] orthonormal unit
 * vectors in the target frame.  f: host [n_rhs][n_dir][2], dcs: host
 * [n_rhs][n_dir]; either may be NULL.  E_INVALID for NULL inputs, counts
 * outside 1..65535, or direction vectors that are not unit (1e-6) and
 * mutually orthogonal (1e-6). */
dda_status dda_far_field(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs, const dda_c64* P,
                         int32_t n_dir, const double* n_hat, const double* theta_hat, const double* phi_hat,
                         dda_c64* f, double* dcs);

/* Averages over scattering directions ("Averaging over Scattering
 * Directions"): for each right-hand side q, with theta the angle between the
 * scattering direction and khat of inc[q],
 *   out[q][0] = Q_sca = (1 / pi a_eff^2) int dC_sca/dOmega dOmega,
 *   out[q][1] = g = <cos theta>,  out[q][2] = <cos^2 theta>,
 * the cross section dC_sca/dOmega being dda_far_field's dcs, integrated with
 * n_theta Gauss-Legendre nodes in cos theta times n_phi equally spaced
 * azimuths (the far field is band limited, so the rule converges quickly;
 * 48 x 64 is ample for targets of size parameter up to about 5).  P: device
 * [n_rhs][n_sites][3], caller order.  out: host [n_rhs][3].  E_INVALID for
 * NULL arguments, bad incidences, n_theta < 2, n_phi < 1 or
 * n_theta * n_phi > 65535. */
dda_status dda_scattering_averages(dda_ctx* ctx, dda_target* t, const dda_opts* opts, int32_t n_rhs,
                                   const dda_incidence* inc, const dda_c64* P, int32_t n_theta, int32_t n_phi,
                                   double* out);

/* The 4x4 Mueller matrix ("Scattering by Finite Targets: The Mueller
 * Matrix") in the Lab Frame (incidence along x_LF) from the amplitudes of
 * the two incident polarizations e01, e02 (Lab Frame, as solved): f1, f2
 * host [n_dir][2] (dda_far_field's f of each, with theta_d, phi_d the
 * Lab-Frame unit vectors of direction d), phi_deg host [n_dir] the
 * scattering-plane angle of direction d (phi = 0: the x-y plane).  Builds the
 * amplitude matrix (S2 S3; S4 S1) of Bohren & Huffman (1983) from f by the
 * guide's relation and returns its 16 Mueller elements, row-major
 * S[d][4 (i-1) + (j-1)] = S_ij (host).  Host computation; no device use. */
dda_status dda_mueller(int32_t n_dir, const dda_c64* f1, const dda_c64* f2, const dda_c64* e01, const dda_c64* e02,
                       const double* phi_deg, double* S);

/* Kernel timing on the context stream (HIP events around every launch of
 * the solver's kernels, read back at the stream synchronisations the calls
 * already make).  Categories (index into dda_timing arrays):
 *   0 scatter + forward FFT along x      1 forward FFT along y
 *   2 FFT along z with the tensor product 3 inverse FFT along y
 *   4 inverse FFT along x + gather        5 Krylov updates and reductions
 *   6 interaction-tensor sampling + FFT   7 other setup (E_inc, 1/alpha, permutes)
 * dda_ctx_set_timing(ctx, mask) clears the totals and records the
 * categories whose bit (1 << category) is set in mask (0xff: all; 0: stop).
 * dda_ctx_get_timing copies the totals accumulated so far. */
#define DDA_TIMING_CATEGORIES 8
typedef struct {
    double ms[DDA_TIMING_CATEGORIES];            /* summed kernel time of the timed launches */
    int64_t launches[DDA_TIMING_CATEGORIES];     /* kernel launches timed */
    int64_t all_launches[DDA_TIMING_CATEGORIES]; /* launches of the category, timed or not */
} dda_timing;
dda_status dda_ctx_set_timing(dda_ctx* ctx, int mask);
dda_status dda_ctx_get_timing(dda_ctx* ctx, dda_timing* out);
/* Record events on every `every`-th launch of each recorded category only (a
 * systematic sample that keeps the event overhead off most launches);
 * every = 1 (the default) times every launch.  In batched solves that replay
 * graphs, one chunk of iterations in `every` runs as direct launches (and is
 * sampled as above); all_launches still counts every launch.  E_INVALID for
 * every < 1. */
dda_status dda_ctx_set_timing_sample(dda_ctx* ctx, int every);

/* The strided-pass variants the autotuner chose for this context, target,
 * right-hand-side count and precision: variants[0] forward y pass,
 * variants[1] z pass with the tensor product, variants[2] inverse y pass
 * (each the value opts->kernel_variant - 1 would force).  All three are -1
 * when no solve with these parameters has been tuned yet.
 * E_INVALID for NULL arguments, n_rhs < 1 or an unknown precision. */
dda_status dda_ctx_tuned_variants(dda_ctx* ctx, const dda_target* t, int32_t n_rhs, dda_precision precision,
                                  int32_t variants[3]);

/* Description of the last error or warning on this thread ("" if none).
 * Valid until the next library call on the thread.  |m|kd >= 1 (the validity
 * bound of "Applicability of the DDA") is reported here as a warning. */
const char* dda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDA_H */
