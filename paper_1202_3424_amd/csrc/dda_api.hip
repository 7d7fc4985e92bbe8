// C ABI of the DDA solver (include/dda.h): contexts, targets, the
// FFT-matvec plan, the cached FFT of the interaction tensor, and the batched
// BiCGSTAB driver.  Every arithmetic step runs in the kernels of
// dda_kernels.hip; this file validates, plans, allocates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <complex>
#include <cstring>
#include <array>
#include <chrono>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dda.h"
#include "dda_kernels.h"

using namespace dda;

namespace {

thread_local std::string g_err;

void set_err(const std::string& m) { g_err = m; }

struct Fail {
    dda_status st;
};

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_err(std::string(#expr) + " failed: " + hipGetErrorString(e_));            \
            throw Fail{e_ == hipErrorOutOfMemory ? DDA_E_NOMEM : DDA_E_DEVICE};           \
        }                                                                                 \
    } while (0)

[[noreturn]] void invalid(const std::string& m) {
    set_err(m);
    throw Fail{DDA_E_INVALID};
}

// Device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void* ensure(size_t need) {
        if (need <= bytes) return p;
        if (p) HIPCHK(hipFree(p));
        p = nullptr;
        bytes = 0;
        HIPCHK(hipMalloc(&p, need));
        bytes = need;
        return p;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

bool smooth235(int m) {
    for (int f : {2, 3, 5})
        while (m % f == 0) m /= f;
    return m == 1;
}

// Any padded extent M >= 2n - 1 gives every separation -(n-1)..(n-1) its own
// slot, so the circulant product equals the Toeplitz one exactly.  The
// smooth extent: 2n when 2,3,5-smooth, else the smallest smooth one >=
// 2n - 1.  The padded extent: the smallest FFT length with compile-time
// kernels >= 2n - 1 when that is at most 1.4 times the smooth extent (those
// kernels are several times faster than the runtime-planned ones, and
// targets of similar size then share a grid, which lets a batched solve run
// them in the same launches), else the smooth extent.
int smooth_extent(int n) {
    if (smooth235(2 * n)) return 2 * n;
    int m = std::max(2 * n - 1, 1);
    while (!smooth235(m)) ++m;
    return m;
}
int padded_extent(int n) {
    const int m = smooth_extent(n);
    for (int L : {32, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512})
        if (L >= 2 * n - 1) return 5 * L <= 7 * m ? L : m;
    return m;
}
// Largest padded extent on an axis: the FP64 LDS tile holds three
// components of a line up to 682 points, and the compile-time kernels stop
// at 512.  Every box extent up to 256 pads to at most 512.
constexpr int MAX_PADDED = 512;

// Radix sequence: powers of two as 8s and 4s (a single 2 only for L = 2^1 or
// 2^(3j+1) with j = 0), then 3s, then 5s.
AxisPlan make_plan(int L) {
    AxisPlan pl{};
    pl.L = L;
    int m = L, e2 = 0;
    while (m % 2 == 0) { m /= 2; ++e2; }
    std::vector<int> r;
    if (e2 % 3 == 1 && e2 >= 4) { r.push_back(4); r.push_back(4); e2 -= 4; }
    if (e2 % 3 == 2) { r.push_back(4); e2 -= 2; }
    if (e2 % 3 == 1) { r.push_back(2); e2 -= 1; }
    while (e2 >= 3) { r.push_back(8); e2 -= 3; }
    while (m % 3 == 0) { r.push_back(3); m /= 3; }
    while (m % 5 == 0) { r.push_back(5); m /= 5; }
    if (m != 1 || (int)r.size() > MAXST) invalid("unsupported FFT length " + std::to_string(L));
    pl.nst = (int)r.size();
    for (int i = 0; i < pl.nst; ++i) pl.R[i] = r[i];
    return pl;
}

}  // namespace

// Device buffers and pinned status copy of one in-flight solve, with the
// stream it runs on.  The context's own workspace uses the context stream;
// dda_solve_batched adds workspaces with their own (default-priority) streams
// so that several targets iterate concurrently.
struct Workspace {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevBuf grid, vecs, state, partials, chains, inc, ainv;
    RhsState* host_state = nullptr;
    int host_state_cap = 0;
    hipEvent_t ready = nullptr;   // recorded after the last asynchronous status copy
    // captured chunks of Krylov iterations, keyed by every value their kernel
    // arguments hold; replayed on `stream`, or on the side stream `gstream`
    // when `stream` is the null stream (which cannot be captured)
    struct Graph {
        hipGraphExec_t exec;
        long long launches[DDA_TIMING_CATEGORIES];   // launches per category in the chunk
    };
    std::map<std::string, Graph> graphs;
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second.exec);
        graphs.clear();
    }
    void release() {
        drop_graphs();
        if (gstream) (void)hipStreamDestroy(gstream);
        gstream = nullptr;
        for (hipEvent_t& e : gev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        for (DevBuf* b : {&grid, &vecs, &state, &partials, &chains, &inc, &ainv}) b->release();
        if (host_state) (void)hipHostFree(host_state);
        host_state = nullptr;
        host_state_cap = 0;
        if (ready) (void)hipEventDestroy(ready);
        ready = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

struct dda_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Workspace main;
    std::vector<Workspace*> extra;
    DevBuf dainv, aux, gtmp;
    DevBuf ffbuf;   // far-field amplitudes: sorted P, directions, results
    // kernel timing (dda_ctx_set_timing)
    int timing = 0;   // bit mask of recorded categories
    int tsample = 1;  // events on every tsample-th launch of a category (dda_ctx_set_timing_sample)
    long long tall[DDA_TIMING_CATEGORIES] = {};   // every launch of each recorded category
    bool tsuppress = false;   // inside a graph capture: count launches (tcap), record no events
    long long tcap[DDA_TIMING_CATEGORIES] = {};
    long long tchunk = 0;     // Krylov chunks run while timing (graph replays sample chunks)
    struct Pending {
        int cat;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> evpool;
    std::vector<Pending> pending;
    double tms[DDA_TIMING_CATEGORIES] = {};
    long long tlaunch[DDA_TIMING_CATEGORIES] = {};
    // autotuned strided-pass variants per (grid, box, right-hand sides, precision)
    std::map<std::tuple<int, int, int, int, int, int, int, int>, std::array<int, 3>> tuned;
    // batched calls: seconds taken with 4, 2 and 1 jobs in flight (< 0: not
    // tried yet), per batch shape (the jobs' grids and right-hand sides)
    std::map<std::string, std::array<double, 3>> sched;
    long long captures = 0;   // iteration chunks captured into graphs so far
};

struct dda_target {
    dda_ctx* ctx = nullptr;
    int nsites = 0;
    int nmat = 0;
    Geo geo{};
    std::vector<double2> mats;       // distinct refractive indices (and their device copy mdev)
    DevBuf map, mat, coords, perm, tw, tw32, mdev;
    // cached FFT of the interaction tensor
    double green_kd = -1.0;
    bool have64 = false, have32 = false;
    DevBuf gh64, gh32;
    int lo[3] = {0, 0, 0};             // lattice coordinates of the bounding box's first point
    // near field: the last extended volume (every point a site), keyed by the
    // points added below and above the box on each axis
    dda_target* nf = nullptr;
    int nf_key[6] = {0, 0, 0, 0, 0, 0};
};

namespace {

// Work memory of dda_apply_noalloc: one fixed device array, a copy of it on
// every GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy: its device address on each
// GPU comes from hipGetSymbolAddress, taken once per device when a context is
// created there (scratch_setup) and kept in g_scratch.
constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
constexpr int NOALLOC_MAX_RHS = 256;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch[SCRATCH_MAX_DEVICES] = {};

// With the context's device current: look up this device's copy of the
// work array once.
void scratch_setup(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_err(std::string("hipGetSymbolAddress of the work array failed: ") + hipGetErrorString(e));
        throw Fail{DDA_E_DEVICE};
    }
    g_scratch[device] = p;
}
void* scratch_of(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

// Layout of the work memory of dda_apply_noalloc (byte offsets, 256-byte
// aligned): incidences, 1/alpha, the sorted input and output site vectors
// and the padded grid of the product's precision.
struct Carve {
    size_t kh, e0, ainv, xs, ys, grid, total;
};
Carve carve_layout(const dda_target* t, int nrhs, bool fp32) {
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t n3 = 3 * (size_t)t->nsites;
    Carve L{};
    size_t off = 0;
    L.kh = off;
    off = up(off + (size_t)nrhs * 3 * sizeof(double));
    L.e0 = off;
    off = up(off + (size_t)nrhs * 3 * sizeof(double2));
    L.ainv = off;
    off = up(off + (size_t)nrhs * t->nmat * 3 * sizeof(double2));
    L.xs = off;
    off = up(off + (size_t)nrhs * n3 * sizeof(double2));
    L.ys = off;
    off = up(off + (size_t)nrhs * n3 * sizeof(double2));
    L.grid = off;
    off = up(off + (size_t)nrhs * (size_t)t->geo.npts * 3 * (fp32 ? sizeof(float2) : sizeof(double2)));
    L.total = off;
    return L;
}

struct Scope {  // make the context's device current for the duration of a call
    int prev = 0;
    explicit Scope(const dda_ctx* c) {
        (void)hipGetDevice(&prev);
        if (c && c->device != prev) HIPCHK(hipSetDevice(c->device));
    }
    ~Scope() { (void)hipSetDevice(prev); }
};

double aeff_over_d(int n) { return std::cbrt(3.0 * n / (4.0 * M_PI)); }

enum TimingCat { T_SCATTER = 0, T_FFTY_FWD = 1, T_FFTZ_G = 2, T_FFTY_INV = 3, T_GATHER = 4, T_KRYLOV = 5,
                 T_GREEN = 6, T_SETUP = 7 };

hipEvent_t take_event(dda_ctx* c) {
    if (!c->evpool.empty()) {
        hipEvent_t e = c->evpool.back();
        c->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreate(&e));
    return e;
}

// Events around the launches issued in this scope, when timing is enabled.
// The matvec-pass categories time their single kernel with the events of
// hipExtLaunchKernelGGL (the kernel's own execution interval); the others
// record the events on the stream around every launch in the scope.
struct Timed {
    dda_ctx* c;
    int cat;
    bool ext;
    hipStream_t st;
    hipEvent_t a = nullptr;
    hipEvent_t b = nullptr;
    Timed(dda_ctx* c_, int cat_, hipStream_t st_) : c(c_), cat(cat_), ext(cat_ <= T_GATHER), st(st_) {
        if (c->tsuppress) {   // captured into a graph: counted, never timed
            ++c->tcap[cat];
            return;
        }
        if (!(c->timing & (1 << cat))) return;
        const long long n = c->tall[cat]++;
        // systematic sample: events on every tsample-th launch of the category
        if (n % c->tsample != 0) return;
        a = take_event(c);
        if (ext) {
            b = take_event(c);
            launch_events() = LaunchEvents{a, b};
        } else {
            HIPCHK(hipEventRecord(a, st));
        }
    }
    ~Timed() {
        if (!a) return;
        if (ext) {
            launch_events() = LaunchEvents{};
        } else {
            if (!c->evpool.empty()) {
                b = c->evpool.back();
                c->evpool.pop_back();
            } else if (hipEventCreate(&b) != hipSuccess) {
                c->evpool.push_back(a);
                return;
            }
            (void)hipEventRecord(b, st);
        }
        c->pending.push_back({cat, a, b});
    }
};

// Accumulate the timed launches that have completed.
void flush_timing(dda_ctx* c) {
    std::vector<dda_ctx::Pending> keep;
    for (const auto& p : c->pending) {
        if (hipEventQuery(p.b) == hipErrorNotReady) {
            keep.push_back(p);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->tms[p.cat] += ms;
            c->tlaunch[p.cat] += 1;
        }
        c->evpool.push_back(p.a);
        c->evpool.push_back(p.b);
    }
    c->pending.swap(keep);
}

double kd_of(const dda_opts* o, int nsites) {
    const double d = o->aeff / aeff_over_d(nsites);
    return 2.0 * M_PI * o->m_medium / o->wavelength * d;
}

void check_opts(const dda_opts* o) {
    if (!o) invalid("opts is NULL");
    if (!(o->wavelength > 0) || !std::isfinite(o->wavelength)) invalid("wavelength must be > 0");
    if (!(o->aeff > 0) || !std::isfinite(o->aeff)) invalid("aeff must be > 0");
    if (!(o->m_medium > 0) || !std::isfinite(o->m_medium)) invalid("m_medium must be > 0");
    if (!(o->tol > 0) || !std::isfinite(o->tol)) invalid("tol must be > 0");
    if (o->max_iter < 1) invalid("max_iter must be >= 1");
    if (o->polarizability != DDA_LATTDR && o->polarizability != DDA_GKDLDR) invalid("unknown polarizability");
    if (o->solver != DDA_BICGSTAB && o->solver != DDA_QMR_SYM && o->solver != DDA_BICGSTAB2)
        invalid("unknown solver");
    if (o->precision != DDA_FP64 && o->precision != DDA_FP32_MATVEC) invalid("unknown precision");
    if (o->kernel_variant < 0) invalid("kernel_variant must be >= 0");
}

// Normalised incidences packed for the device: khat [n][3], e0 [n][3].
void pack_incidence(int n, const dda_incidence* inc, double* kh, double2* e0) {
    if (!inc) invalid("incidence array is NULL");
    for (int q = 0; q < n; ++q) {
        const dda_incidence& I = inc[q];
        double kn = 0, en = 0;
        for (int m = 0; m < 3; ++m) {
            if (!std::isfinite(I.khat[m]) || !std::isfinite(I.e0[m].re) || !std::isfinite(I.e0[m].im))
                invalid("non-finite incidence " + std::to_string(q));
            kn += I.khat[m] * I.khat[m];
            en += I.e0[m].re * I.e0[m].re + I.e0[m].im * I.e0[m].im;
        }
        kn = std::sqrt(kn);
        en = std::sqrt(en);
        if (std::fabs(kn - 1.0) > 1e-6) invalid("khat of incidence " + std::to_string(q) + " is not a unit vector");
        if (en == 0.0) invalid("e0 of incidence " + std::to_string(q) + " is zero");
        double dre = 0, dim = 0;
        for (int m = 0; m < 3; ++m) {
            dre += I.e0[m].re * I.khat[m] / kn;
            dim += I.e0[m].im * I.khat[m] / kn;
        }
        if (std::sqrt(dre * dre + dim * dim) > 1e-6 * en)
            invalid("e0 of incidence " + std::to_string(q) + " is not transverse to khat");
        for (int m = 0; m < 3; ++m) {
            kh[(size_t)q * 3 + m] = I.khat[m] / kn;
            e0[(size_t)q * 3 + m] = double2{I.e0[m].re / en, I.e0[m].im / en};
        }
    }
}
void pack_incidence(int n, const dda_incidence* inc, std::vector<double>& kh, std::vector<double2>& e0) {
    kh.resize((size_t)n * 3);
    e0.resize((size_t)n * 3);
    pack_incidence(n, inc, kh.data(), e0.data());
}


// Everything one batched solve on one target needs on the device.
// The right-hand sides [first, first + count) of one target in a ragged
// batch, with that target's options and kd.
struct Seg {
    dda_target* t;
    const dda_opts* o;
    int first, count;
    double kd;
};

struct Work {
    dda_ctx* c;
    Workspace& ws;
    hipStream_t s;
    dda_target* t;
    int nrhs;
    double kd;
    bool fp32;
    bool qmr = false;   // QMR for complex-symmetric A instead of BiCGSTAB
    bool b2 = false;    // BiCGstab(2) instead of BiCGSTAB
    bool graphs = false; // replay captured iteration chunks (batched solves, unless DDA_FLAG_NO_GRAPH)
    SiteArgs a{};
    int site_blocks = 1;
    int pass_blocks = 1;
    int var[3] = {0, 0, 0};   // strided-pass variants: y forward, z with tensor, y inverse
    void* grid = nullptr;
    double* kh = nullptr;
    double2* e0 = nullptr;
    // ragged batch (several targets on one padded grid): each target's
    // right-hand sides; empty for one target
    std::vector<Seg> segs;

    Work(dda_ctx* c_, Workspace& ws_, dda_target* t_, int nrhs_, double kd_, bool fp32_)
        : c(c_), ws(ws_), s(ws_.stream), t(t_), nrhs(nrhs_), kd(kd_), fp32(fp32_) {
        const Geo& g = t->geo;
        const long long n3 = 3LL * t->nsites;
        const size_t vbytes = (size_t)nrhs * n3 * sizeof(double2);
        char* v = (char*)ws.vecs.ensure(9 * vbytes);
        a.nsites = t->nsites;
        a.n3 = n3;
        a.nrhs = nrhs;
        a.nmat = t->nmat;
        a.map = (const int*)t->map.p;
        a.mat = (const int*)t->mat.p;
        a.x = (double2*)(v + 0 * vbytes);
        a.r = (double2*)(v + 1 * vbytes);
        a.rhat = (double2*)(v + 2 * vbytes);
        a.p = (double2*)(v + 3 * vbytes);
        a.v = (double2*)(v + 4 * vbytes);
        a.t = (double2*)(v + 5 * vbytes);
        a.b = (double2*)(v + 6 * vbytes);
        a.u2 = (double2*)(v + 7 * vbytes);
        a.r2 = (double2*)(v + 8 * vbytes);
        a.kd = kd;
        // FP64-sized even in the FP32-matvec mode: its residual refinement and
        // final checks use FP64 products
        grid = ws.grid.ensure((size_t)nrhs * g.npts * 3 * sizeof(double2));
        a.st = (RhsState*)ws.state.ensure((size_t)nrhs * sizeof(RhsState));
        // workgroups of every reducing kernel, per right-hand side
        pass_blocks = x_pass_blocks(g, nrhs, fp32);
        site_blocks = site_blocks_for(n3, nrhs);
        a.maxblk = std::max(pass_blocks, site_blocks);
        a.partials = (double*)ws.partials.ensure((size_t)nrhs * a.maxblk * PSTRIDE * sizeof(double));
        a.chains = (double*)ws.chains.ensure((size_t)nrhs * PSTRIDE * NT * sizeof(double));
        a.ainv = (const double2*)ws.ainv.ensure((size_t)nrhs * t->nmat * 3 * sizeof(double2));
        char* ib = (char*)ws.inc.ensure((size_t)nrhs * (3 * sizeof(double) + 3 * sizeof(double2)) + 64);
        kh = (double*)ib;
        e0 = (double2*)(ib + (((size_t)nrhs * 3 * sizeof(double) + 15) & ~(size_t)15));
    }

    // The plain product only, every buffer carved from `base` as laid out by
    // carve_layout (the fixed work memory of dda_apply_noalloc): nothing is
    // allocated.  The product reads a.p and writes a.v; the solver vectors,
    // states and partial sums stay null (a plain product never touches them).
    Work(dda_ctx* c_, Workspace& ws_, dda_target* t_, int nrhs_, double kd_, bool fp32_, char* base, const Carve& L)
        : c(c_), ws(ws_), s(ws_.stream), t(t_), nrhs(nrhs_), kd(kd_), fp32(fp32_) {
        a.nsites = t->nsites;
        a.n3 = 3LL * t->nsites;
        a.nrhs = nrhs;
        a.nmat = t->nmat;
        a.map = (const int*)t->map.p;
        a.mat = (const int*)t->mat.p;
        a.kd = kd;
        a.p = (double2*)(base + L.xs);
        a.v = (double2*)(base + L.ys);
        a.ainv = (const double2*)(base + L.ainv);
        grid = base + L.grid;
        kh = (double*)(base + L.kh);
        e0 = (double2*)(base + L.e0);
    }

    // Make this a ragged batch: t is the batch target (its geometry's rg is
    // the device table rg), the site kernels launch the largest per-target
    // workgroup count sblk, and every reduction reads its own target's
    // block count from the table.
    void set_ragged(const std::vector<Seg>& sg, const RhsGeo* rg, int sblk) {
        segs = sg;
        a.rg = rg;
        site_blocks = sblk;
        a.maxblk = std::max(pass_blocks, site_blocks);
        a.partials = (double*)ws.partials.ensure((size_t)nrhs * a.maxblk * PSTRIDE * sizeof(double));
    }
    // block counts k_finalize sums over: this launch's, or each right-hand
    // side's own in a ragged batch
    int fin_site() const { return a.rg ? NBLK_SITE : site_blocks; }
    int fin_pass() const { return a.rg ? NBLK_PASS : pass_blocks; }
    // the targets and their right-hand sides
    std::vector<Seg> parts() const {
        if (!segs.empty()) return segs;
        return {Seg{t, nullptr, 0, nrhs, kd}};
    }
    // tensor FFT handed to pass 3 (a ragged batch's kernels take each right-
    // hand side's own from the table)
    const void* ghat(bool f32) const {
        const dda_target* src = segs.empty() ? t : segs[0].t;
        return f32 ? src->gh32.p : src->gh64.p;
    }
    // per-right-hand-side tolerance and iteration limit, every status active
    void set_states(const dda_opts* o) {
        if (segs.empty()) {
            launch_set_state(a.st, nrhs, o->tol, o->max_iter, s);
            return;
        }
        for (const Seg& sg : segs) launch_set_state(a.st + sg.first, sg.count, sg.o->tol, sg.o->max_iter, s);
    }

    void upload_incidence(const double* khv, const double2* e0v) {
        HIPCHK(hipMemcpyAsync(kh, khv, (size_t)nrhs * 3 * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(e0, e0v, (size_t)nrhs * 3 * sizeof(double2), hipMemcpyHostToDevice, s));
    }
    void upload_incidence(const std::vector<double>& khv, const std::vector<double2>& e0v) {
        HIPCHK(hipMemcpyAsync(kh, khv.data(), khv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(e0, e0v.data(), e0v.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    }

    // 1/alpha for every (right-hand side, material); scheme + 2 = derivative
    // (a ragged batch: each target's own materials, options and kd, rows of
    // the largest material count)
    void alpha_table(int scheme, double m_medium, double2* out) {
        if (segs.empty()) {
            launch_alpha(nrhs, t->nmat, (const double2*)t->mdev.p, m_medium, kh, e0, kd, scheme, out, s);
            return;
        }
        const int shift = scheme >= 2 ? 2 : 0;
        for (const Seg& sg : segs)
            launch_alpha(sg.count, sg.t->nmat, (const double2*)sg.t->mdev.p, sg.o->m_medium, kh + 3 * sg.first,
                         e0 + 3 * sg.first, sg.kd, sg.o->polarizability + shift,
                         out + (size_t)sg.first * t->nmat * 3, s, t->nmat);
    }

    // the three strided passes: 0 = y forward, 1 = z with the tensor product, 2 = y inverse
    template <typename T>
    void strided_slot(int slot, int chk, int variant) {
        using C = typename V2<T>::t;
        const Geo& g = t->geo;
        C* gr = (C*)grid;
        const C* gh = (const C*)ghat(sizeof(T) == 4);
        const double2* tw = (const double2*)t->tw.p;
        if (slot == 0)
            launch_strided<T>(1, -1, chk, g, nrhs, 3, g.n[2], g.n[1], g.M[1], gr, tw, nullptr, a.st, s, variant);
        else if (slot == 1)
            launch_strided<T>(2, 0, chk, g, nrhs, 3, g.M[1], g.n[2], g.n[2], gr, tw, gh, a.st, s, variant);
        else
            launch_strided<T>(1, 1, chk, g, nrhs, 3, g.n[2], g.M[1], g.n[1], gr, tw, nullptr, a.st, s, variant);
    }

    // Pick, once per (grid, box, right-hand sides, precision), a compile-time
    // variant of each strided pass by timing every candidate on the workspace
    // grid (its contents are scratch at this point; all variants compute
    // bitwise-identical results), one warm-up and twenty timed launches
    // each (fewer on large grids), pass 3 each time behind the forward y
    // pass.  Among the variants
    // within 3% of the fastest it takes the lowest-numbered, so that
    // near-ties resolve the same way from run to run.
    void autotune(bool enabled, int forced = 0) {
        const Geo& g = t->geo;
        if (forced > 0) {
            for (int slot = 0; slot < 3; ++slot) {
                const int nv = strided_variants(g.M[slot == 1 ? 2 : 1], slot == 1);
                var[slot] = forced - 1 < nv ? forced - 1 : 0;
            }
            return;
        }
        auto key = std::make_tuple(g.M[0], g.M[1], g.M[2], g.n[0], g.n[1], g.n[2], nrhs,
                                   (fp32 ? 1 : 0) | (a.rg ? 2 : 0));
        auto it = c->tuned.find(key);
        if (it != c->tuned.end()) {
            for (int i = 0; i < 3; ++i) var[i] = it->second[i];
            return;
        }
        std::array<int, 3> best{0, 0, 0};
        if (enabled) {
            hipEvent_t e0 = take_event(c), e1 = take_event(c);
            for (int slot = 0; slot < 3; ++slot) {
                const int L = g.M[slot == 1 ? 2 : 1];
                const int nv = strided_variants(L, slot == 1);
                std::vector<float> t_ms(nv, 0.f);
                // pass 3 is timed behind the chosen forward y pass, which
                // writes its input in the solve, less the time of that y pass
                // alone: back-to-back launches of pass 3 alone find its grid
                // and tensor in the caches, and there the variants that
                // re-read the tensor look faster than they are in the solve
                auto run_y = [&]() {
                    if (fp32) strided_slot<float>(0, CHK_NONE, best[0]);
                    else strided_slot<double>(0, CHK_NONE, best[0]);
                };
                auto run_v = [&](int v) {
                    if (fp32) strided_slot<float>(slot, CHK_NONE, v);
                    else strided_slot<double>(slot, CHK_NONE, v);
                };
                auto candidate = [&](int v) { return !a.rg || ragged_variant(slot == 1, v); };
                int first = 0;
                while (!candidate(first)) ++first;
                // the first candidate's warm-up launch, timed: twenty timed
                // launches per candidate, fewer (at least three, about 40 ms
                // of launches) where one launch is long
                int reps = 20;
                {
                    HIPCHK(hipEventRecord(e0, s));
                    run_v(first);
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    float t1 = 0.f;
                    HIPCHK(hipEventElapsedTime(&t1, e0, e1));
                    if (t1 > 2.f) reps = std::max(3, std::min(20, (int)(40.f / t1)));
                }
                float t_y = 0.f;
                if (slot == 1) {
                    run_y();
                    HIPCHK(hipEventRecord(e0, s));
                    for (int k = 0; k < reps; ++k) run_y();
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    HIPCHK(hipEventElapsedTime(&t_y, e0, e1));
                }
                for (int v = 0; v < nv; ++v) {
                    if (!candidate(v)) {
                        t_ms[v] = std::numeric_limits<float>::infinity();
                        continue;
                    }
                    if (v != first) run_v(v);   // warm-up
                    HIPCHK(hipEventRecord(e0, s));
                    for (int k = 0; k < reps; ++k) {
                        if (slot == 1) run_y();
                        run_v(v);
                    }
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    HIPCHK(hipEventElapsedTime(&t_ms[v], e0, e1));
                    t_ms[v] -= t_y;
                }
                const float fastest = *std::min_element(t_ms.begin(), t_ms.end());
                for (int v = nv - 1; v >= 0; --v)
                    if (t_ms[v] <= 1.03f * fastest) best[slot] = v;
            }
            HIPCHK(hipGetLastError());
            c->evpool.push_back(e0);
            c->evpool.push_back(e1);
            c->tuned[key] = best;
        }
        for (int i = 0; i < 3; ++i) var[i] = best[i];
    }

    template <typename T>
    void matvec_t(int sc, int ga, int chk_sc, int chk_rest, const int* vars) {
        using C = typename V2<T>::t;
        const Geo& g = t->geo;
        C* gr = (C*)grid;
        const double2* tw = (const double2*)t->tw.p;
        {
            Timed tm(c, T_SCATTER, s);
            launch_scatter_x<T>(sc, chk_sc, g, a, gr, tw, s);
        }
        {
            Timed tm(c, T_FFTY_FWD, s);
            strided_slot<T>(0, chk_rest, vars[0]);
        }
        {
            Timed tm(c, T_FFTZ_G, s);
            strided_slot<T>(1, chk_rest, vars[1]);
        }
        {
            Timed tm(c, T_FFTY_INV, s);
            strided_slot<T>(2, chk_rest, vars[2]);
        }
        {
            Timed tm(c, T_GATHER, s);
            launch_gather_x<T>(ga, chk_rest, g, a, gr, tw, s);
        }
        if (ga != GA_PLAIN) {
            static const int kind_of[] = {-1, FIN_CONJ, FIN_V, FIN_T, FIN_RES, FIN_QV, FIN_B_BETA, FIN_V, FIN_B_MR};
            Timed tm(c, T_KRYLOV, s);
            launch_finalize(a, kind_of[ga], fin_pass(), s);
        }
    }
    // fp64: force an FP64 product in the FP32-matvec mode (refinement, checks)
    void matvec(int sc, int ga, int chk_sc, int chk_rest, bool fp64 = false) {
        static const int defaults[3] = {0, 0, 0};
        if (fp32 && !fp64) matvec_t<float>(sc, ga, chk_sc, chk_rest, var);
        else matvec_t<double>(sc, ga, chk_sc, chk_rest, fp32 ? defaults : var);
        HIPCHK(hipGetLastError());
    }
};

// Build (or reuse) the octant FFT of the interaction tensor for this kd.
void ensure_green(dda_ctx* c, dda_target* t, double kd, bool fp32, bool force) {
    const bool fresh = force || t->green_kd != kd;
    if (!fresh && (fp32 ? t->have32 : t->have64)) return;
    const Geo& g = t->geo;
    double2* G = (double2*)c->gtmp.ensure((size_t)g.npts * 6 * sizeof(double2));
    const double2* tw = (const double2*)t->tw.p;
    Timed tm(c, T_GREEN, c->stream);
    launch_green_sample(g, kd, G, c->stream);
    launch_xgrid3(g, G, tw, c->stream);
    launch_strided<double>(1, -1, CHK_NONE, g, 2, 3, g.M[2], g.M[1], g.M[1], G, tw, nullptr, nullptr, c->stream);
    launch_strided<double>(2, -1, CHK_NONE, g, 2, 3, g.M[1], g.M[2], g.M[2], G, tw, nullptr, nullptr, c->stream);
    const size_t nh = (size_t)g.H[0] * g.H[1] * g.H[2] * 6;
    if (fresh) t->have64 = t->have32 = false;
    double2* g64 = (double2*)t->gh64.ensure(nh * sizeof(double2));
    float2* g32 = fp32 ? (float2*)t->gh32.ensure(nh * sizeof(float2)) : nullptr;
    launch_green_octant(g, G, g64, g32, c->stream);
    HIPCHK(hipGetLastError());
    t->green_kd = kd;
    t->have64 = true;
    if (fp32) t->have32 = true;
}

// Asynchronous copy of every right-hand side's status to pinned host memory;
// ws.ready completes with it.
void post_state(Work& w) {
    Workspace& ws = w.ws;
    if (ws.host_state_cap < w.nrhs) {
        if (ws.host_state) (void)hipHostFree(ws.host_state);
        ws.host_state = nullptr;
        HIPCHK(hipHostMalloc((void**)&ws.host_state, (size_t)w.nrhs * sizeof(RhsState), hipHostMallocDefault));
        ws.host_state_cap = w.nrhs;
    }
    if (!ws.ready) HIPCHK(hipEventCreateWithFlags(&ws.ready, hipEventDisableTiming));
    HIPCHK(hipMemcpyAsync(ws.host_state, w.a.st, (size_t)w.nrhs * sizeof(RhsState), hipMemcpyDeviceToHost, w.s));
    HIPCHK(hipEventRecord(ws.ready, w.s));
}

void fetch_state(dda_ctx* c, Work& w) {
    post_state(w);
    HIPCHK(hipEventSynchronize(w.ws.ready));
    flush_timing(c);
}

// x <- the solution of the iterations so far: QMR's smoothed iterate, or
// BiCGSTAB's x and r with the end of the latest iteration applied
// (idempotent; nothing for BiCGstab(2)).
void settle_solution(Work& w) {
    if (w.b2) return;
    Timed tm(w.c, T_KRYLOV, w.s);
    if (w.qmr) {
        launch_qmr_final(w.a, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_QFINAL, 0, w.s);
    } else {
        launch_bicg_flush(w.a, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_FLUSH, 0, w.s);
    }
}

// BiCGSTAB iterations until no right-hand side is active (the device keeps
// every scalar and status; the host polls once per chunk of iterations).
// After a status copy: restart broken-down right-hand sides (once); true if
// any right-hand side still iterates.
bool any_active_after_restart(Work& w) {
    bool active = false, restart = false;
    for (int q = 0; q < w.nrhs; ++q) {
        const RhsState& st = w.ws.host_state[q];
        if (st.status == ST_ACTIVE) active = true;
        // QMR stops at a breakdown and returns its smoothed iterate
        if (!w.qmr && st.status == ST_BREAKDOWN && st.restarts == 0) restart = true;
    }
    if (restart) {
        settle_solution(w);   // the restart starts from r = s - omega t
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_restart(w.a, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_RESTART, w.fin_site(), w.s);
        active = true;
    }
    return active;
}

// One chunk of BiCGSTAB iterations (every scalar and status stays on the
// device; right-hand sides that have stopped skip the work).
void launch_chunk(Work& w, int chunk) {
    if (w.b2) {
        // BiCGstab(2): two BiCG steps of two products each, then the
        // minimal-residual combination
        for (int k = 0; k < chunk; ++k) {
            w.matvec(SC_B0, GA_V, CHK_ACTIVE, CHK_ACTIVE);    // u_1 = A u_0, alpha
            w.matvec(SC_B1, GA_B1, CHK_ACTIVE, CHK_ACTIVE);   // r_1 = A r_0, beta
            w.matvec(SC_B2, GA_B2, CHK_ACTIVE, CHK_ACTIVE);   // u_2 = A u_1, alpha
            w.matvec(SC_B3, GA_B3, CHK_ACTIVE, CHK_ACTIVE);   // r_2 = A r_1, g1, g2
            Timed tm(w.c, T_KRYLOV, w.s);
            launch_b2_update(w.a, w.site_blocks, w.s);
            launch_finalize(w.a, FIN_B_UPD, w.fin_site(), w.s);
        }
        HIPCHK(hipGetLastError());
        return;
    }
    if (w.qmr) {
        // one product per iteration: p, the pending smoothing step, v = A p
        // and alpha; then x, r and the next smoothing step, beta, status
        for (int k = 0; k < chunk; ++k) {
            w.matvec(SC_Q, GA_Q, CHK_ACTIVE, CHK_ACTIVE);
            Timed tm(w.c, T_KRYLOV, w.s);
            launch_qmr_update(w.a, w.site_blocks, w.s);
            launch_finalize(w.a, FIN_QUPD, w.fin_site(), w.s);
        }
        HIPCHK(hipGetLastError());
        return;
    }
    // BiCGSTAB: the end of each iteration (x and r) is applied by the next
    // iteration's first scatter, or by settle_solution once it has stopped
    for (int k = 0; k < chunk; ++k) {
        w.matvec(SC_P, GA_V, CHK_ACTIVE, CHK_ACTIVE);
        w.matvec(SC_S, GA_T, CHK_ACTIVE, CHK_ACTIVE);
    }
    HIPCHK(hipGetLastError());
}

// A chunk of iterations as a captured graph: the launch sequence of
// launch_chunk depends only on values fixed for a workspace, target and
// solve configuration, so one capture serves every later chunk with the
// same key.  With kernel timing on, one chunk in tsample runs as plain
// launches carrying the timing events and the others replay the graph; the
// launch counts recorded at capture keep the per-category totals exact.
template <typename T> void key_bytes(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}
void run_chunk(Work& w, int chunk) {
    dda_ctx* c = w.c;
    if (!w.graphs || (c->timing != 0 && c->tchunk++ % c->tsample == 0)) {
        launch_chunk(w, chunk);
        return;
    }
    Workspace& ws = w.ws;
    std::string key;
    key_bytes(key, w.a);
    key_bytes(key, w.grid);
    key_bytes(key, w.t->geo);
    key_bytes(key, w.t->gh64.p);
    key_bytes(key, w.t->gh32.p);
    key_bytes(key, w.t->tw.p);
    key_bytes(key, w.var);
    key_bytes(key, w.site_blocks);
    key_bytes(key, w.pass_blocks);
    const int flags[4] = {chunk, w.fp32 ? 1 : 0, w.qmr ? 1 : 0, w.b2 ? 1 : 0};
    key_bytes(key, flags);
    hipStream_t gs = w.s;
    if (!gs) {
        if (!ws.gstream) HIPCHK(hipStreamCreateWithFlags(&ws.gstream, hipStreamNonBlocking));
        gs = ws.gstream;
    }
    for (hipEvent_t& e : ws.gev)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (gs != w.s) {
        HIPCHK(hipEventRecord(ws.gev[0], w.s));
        HIPCHK(hipStreamWaitEvent(gs, ws.gev[0], 0));
    }
    auto it = ws.graphs.find(key);
    if (it == ws.graphs.end()) {
        if (ws.graphs.size() >= 32) ws.drop_graphs();
        Workspace::Graph gr{};
        for (long long& n : c->tcap) n = 0;
        hipGraph_t g = nullptr;
        ++c->captures;
        HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        {
            // the chunk is recorded on gs with timing events off; if a launch
            // throws, the capture is still ended and both settings restored
            struct Capture {
                Work& w;
                hipStream_t gs, keep;
                hipGraph_t* g;
                bool ended = false;
                Capture(Work& w_, hipStream_t gs_, hipGraph_t* g_) : w(w_), gs(gs_), keep(w_.s), g(g_) {
                    w.s = gs;
                    w.c->tsuppress = true;
                }
                hipError_t end() {
                    ended = true;
                    w.c->tsuppress = false;
                    w.s = keep;
                    return hipStreamEndCapture(gs, g);
                }
                ~Capture() {
                    if (ended) return;
                    (void)end();
                    if (*g) (void)hipGraphDestroy(*g);
                    *g = nullptr;
                }
            } cap(w, gs, &g);
            launch_chunk(w, chunk);
            HIPCHK(cap.end());
        }
        for (int i = 0; i < DDA_TIMING_CATEGORIES; ++i) gr.launches[i] = c->tcap[i];
        const hipError_t ie = hipGraphInstantiateWithFlags(&gr.exec, g, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ie);
        it = ws.graphs.emplace(key, gr).first;
    }
    HIPCHK(hipGraphLaunch(it->second.exec, gs));
    for (int i = 0; i < DDA_TIMING_CATEGORIES; ++i)
        if (c->timing & (1 << i)) c->tall[i] += it->second.launches[i];
    if (gs != w.s) {
        HIPCHK(hipEventRecord(ws.gev[1], gs));
        HIPCHK(hipStreamWaitEvent(w.s, ws.gev[1], 0));
    }
}

// Iterations to enqueue before the next status poll, at most cap.  Once
// every right-hand side has stopped, the launches of the rest of a chunk
// only read statuses, but each still costs a launch; so the chunk shrinks to
// what the slowest active right-hand side is predicted to need: its average
// reduction of the squared residual per iteration so far, carried on to the
// tolerance, rounded down, at least one.  Before any iteration (or when the
// residual has not fallen) the chunk is cap.  Results do not depend on it.
int next_chunk(const Work& w, int cap) {
    double need = 0.0;
    for (int q = 0; q < w.nrhs; ++q) {
        const RhsState& st = w.ws.host_state[q];
        if (st.status != ST_ACTIVE) continue;
        const double res2 = w.qmr ? st.snorm2 : st.rnorm2;   // what the solver's stop test reads
        const double target = st.tol2 * st.bnorm2;
        if (st.iters < 1 || !(res2 > 0.0) || !(target > 0.0) || !(st.bnorm2 > res2)) return cap;
        const double per_iter = std::log(st.bnorm2 / res2) / st.iters;
        need = std::max(need, std::log(res2 / target) / per_iter);
    }
    if (!(need < cap)) return cap;
    return std::max(1, (int)std::floor(need));
}

// Iterations until no right-hand side is active.  The statuses are copied
// to the host one iteration before the end of each chunk: the host reads
// them and enqueues the next chunk while the GPU runs that last iteration.
// Only when the slowest right-hand side is predicted to finish within it
// does the host wait for the end of the chunk and decide on fresh statuses.
void iterate_loop(Work& w, const dda_opts* o) {
    dda_ctx* c = w.c;
    int launched = 0;
    const int cap = std::min(8, o->max_iter);
    fetch_state(c, w);
    if (!any_active_after_restart(w)) return;
    int chunk = next_chunk(w, cap);
    while (launched <= o->max_iter + 2 * cap) {
        if (chunk > 1) run_chunk(w, chunk - 1);
        post_state(w);
        run_chunk(w, 1);
        launched += chunk;
        HIPCHK(hipEventSynchronize(w.ws.ready));
        flush_timing(c);
        // statuses as of one iteration before the end of the chunk
        if (!any_active_after_restart(w)) break;
        const int need = next_chunk(w, cap + 1);
        if (need >= 2) {
            chunk = std::min(cap, need - 1);
            continue;
        }
        fetch_state(c, w);
        if (!any_active_after_restart(w)) break;
        chunk = next_chunk(w, cap);
    }
}

// Start of BiCGSTAB: state, then r and rhat from b (cold) or b - A x (warm).
void start_iteration(Work& w, const dda_opts* o, bool warm) {
    w.set_states(o);
    if (w.qmr) {
        if (warm) {
            w.a.in = w.a.x;
            w.matvec(SC_PLAIN, GA_RES, CHK_NONE, CHK_NONE, true);  // r = b - A x0
        }
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_qmr_init(w.a, !warm, w.site_blocks, w.s);
        launch_finalize(w.a, warm ? FIN_QWARM : FIN_QCOLD, w.fin_site(), w.s);
        HIPCHK(hipGetLastError());
        return;
    }
    if (warm) {
        w.a.in = w.a.x;
        w.matvec(SC_PLAIN, GA_RES, CHK_NONE, CHK_NONE, true);  // r = b - A x0
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_init_warm(w.a, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_WARM, w.fin_site(), w.s);
    } else {
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_init_cold(w.a, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_COLD, w.fin_site(), w.s);
    }
    HIPCHK(hipGetLastError());
}

// FP64 residual r = b - A x of every converged right-hand side; those that
// miss the tolerance iterate on from x (FP32-matvec mode).
void launch_refinement(Work& w) {
    settle_solution(w);
    if (w.qmr) {
        w.a.in = w.a.x;
        w.matvec(SC_PLAIN, GA_RES, CHK_NONE, CHK_NONE, true);
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_qmr_init(w.a, false, w.site_blocks, w.s);
        launch_finalize(w.a, FIN_QREFINE, w.fin_site(), w.s);
        return;
    }
    w.a.in = w.a.x;
    w.matvec(SC_PLAIN, GA_RES, CHK_NONE, CHK_NONE, true);
    Timed tm(w.c, T_KRYLOV, w.s);
    launch_init_warm(w.a, w.site_blocks, w.s);
    launch_finalize(w.a, FIN_REFINE, w.fin_site(), w.s);
}

// BiCGSTAB on every right-hand side of w (b, ainv prepared); warm start when
// x already holds P0.  In the FP32-matvec mode the recursive residual drifts
// from the true one, so each converged right-hand side is checked with an
// FP64 product r = b - A x and, if that misses the tolerance, the iteration
// restarts from x with that residual (at most 5 refinements).  Leaves P in x.
void iterate(Work& w, const dda_opts* o, bool warm) {
    start_iteration(w, o, warm);
    iterate_loop(w, o);
    if (w.fp32) {
        for (int k = 0; k < 5; ++k) {
            launch_refinement(w);
            fetch_state(w.c, w);
            bool active = false;
            for (int q = 0; q < w.nrhs; ++q) active |= w.ws.host_state[q].status == ST_ACTIVE;
            if (!active) break;
            iterate_loop(w, o);
        }
    }
    settle_solution(w);
}

// true residual, eq. err_tol and the efficiency sums at x
void final_checks(Work& w, bool normal_eq) {
    SiteArgs& a = w.a;
    a.in = a.x;
    w.matvec(SC_PLAIN, GA_RES, CHK_NONE, CHK_NONE, true);  // r = b - A x, red[0] = |r|^2
    if (normal_eq) {
        // A^H y = conj(A conj(y)) because A = A^T
        a.in = a.r;
        a.out = a.t;
        a.slot = 1;
        w.matvec(SC_CONJ, GA_CONJ, CHK_NONE, CHK_NONE, true);
        a.in = a.b;
        a.out = a.v;
        a.slot = 2;
        w.matvec(SC_CONJ, GA_CONJ, CHK_NONE, CHK_NONE, true);
    }
    {
        Timed tm(w.c, T_KRYLOV, w.s);
        launch_qsum(a, w.site_blocks, w.s);
        launch_finalize(a, FIN_QSUM, w.fin_site(), w.s);
    }
    HIPCHK(hipGetLastError());
}

dda_status to_status(int s) {
    switch (s) {
        case ST_CONVERGED: return DDA_OK;
        case ST_MAXITER: return DDA_E_NOT_CONVERGED;
        case ST_BREAKDOWN: return DDA_E_BREAKDOWN;
        case ST_NONFINITE: return DDA_E_NONFINITE;
        default: return DDA_E_NOT_CONVERGED;
    }
}

dda_status fill_results(const Work& w, bool normal_eq, dda_result* res) {
    dda_status worst = DDA_OK;
    for (const Seg& sg : w.parts()) {
    const double a = aeff_over_d(sg.t->nsites);
    const double cq = 4.0 * M_PI * sg.kd / (M_PI * a * a);
    for (int q = sg.first; q < sg.first + sg.count; ++q) {
        const RhsState& s = w.ws.host_state[q];
        dda_result r{};
        r.qext = cq * s.red[3];
        r.qabs = cq * s.red[4];
        r.qpha = 0.5 * cq * s.red[5];
        r.qsca = r.qext - r.qabs;
        r.rel_residual = std::sqrt(s.red[0] / s.bnorm2);
        r.normal_eq_residual = normal_eq ? std::sqrt(s.red[1] / s.red[2]) : -1.0;
        r.kd = sg.kd;
        r.aeff_d = a;
        r.iters = s.iters;
        r.matvecs = s.matvecs;
        r.restarts = s.restarts;
        r.refinements = s.pad0;
        r.status = to_status(s.status);
        if (r.status != DDA_OK && (worst == DDA_OK || r.status > worst)) worst = (dda_status)r.status;
        if (res) res[q] = r;
    }
    }
    return worst;
}

void warn_validity(const dda_target* t, double kd, double m_medium) {
    double mx = 0;
    for (const double2& m : t->mats) mx = std::max(mx, std::hypot(m.x, m.y) / m_medium);
    if (mx * kd >= 1.0) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "warning: |m|kd = %.3f >= 1, outside the DDA validity bound", mx * kd);
        set_err(buf);
    }
}

template <typename F> dda_status guarded(F&& f) {
    g_err.clear();
    try {
        return f();
    } catch (const Fail& e) {
        return e.st;
    } catch (const std::bad_alloc&) {
        set_err("host allocation failed");
        return DDA_E_NOMEM;
    } catch (...) {
        set_err("unexpected C++ exception");
        return DDA_E_DEVICE;
    }
}

// One batched solve on one target: Q's in res, P (caller order) to P_out
// (contiguous [nrhs][n][3]) or per-right-hand-side pointers.  With b_caller
// the right-hand sides are the caller's b instead of E_inc (no efficiencies).
dda_status solve_one(dda_ctx* c, dda_target* t, const dda_opts* o, int nrhs, const dda_incidence* inc,
                     dda_c64* P, dda_c64* const* Pper, const dda_c64* P0, dda_result* res,
                     const dda_c64* b_caller = nullptr) {
    check_opts(o);
    if (nrhs < 1) invalid("n_rhs must be >= 1");
    std::vector<double> kh;
    std::vector<double2> e0;
    pack_incidence(nrhs, inc, kh, e0);
    const double kd = kd_of(o, t->nsites);
    const bool fp32 = o->precision == DDA_FP32_MATVEC;
    ensure_green(c, t, kd, fp32, (o->flags & DDA_FLAG_RECOMPUTE_GREEN) != 0);
    Work w(c, c->main, t, nrhs, kd, fp32);
    w.qmr = o->solver == DDA_QMR_SYM;
    w.b2 = o->solver == DDA_BICGSTAB2;
    w.graphs = false;   // one stream: replays are slower than launches
    w.autotune((o->flags & DDA_FLAG_NO_AUTOTUNE) == 0, o->kernel_variant);
    w.upload_incidence(kh, e0);
    const bool warm = P0 != nullptr;
    {
        Timed tm(c, T_SETUP, w.s);
        w.alpha_table(o->polarizability, o->m_medium, (double2*)w.a.ainv);
        if (b_caller)
            launch_permute(nrhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)b_caller, w.a.b, true, w.s);
        else
            launch_einc(w.a, (const int*)t->coords.p, w.kh, w.e0, w.s);
        if (warm)
            launch_permute(nrhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)P0, w.a.x, true, w.s);
    }
    w.a.in = w.a.x;
    iterate(w, o, warm);
    const bool ne = (o->flags & DDA_FLAG_NO_FINAL_CHECKS) == 0;
    final_checks(w, ne);
    {
        Timed tm(c, T_SETUP, w.s);
        if (P) launch_permute(nrhs, t->nsites, 3, (const int*)t->perm.p, w.a.x, (double2*)P, false, w.s);
        if (Pper) {
            for (int q = 0; q < nrhs; ++q)
                if (Pper[q])
                    launch_permute(1, t->nsites, 3, (const int*)t->perm.p, w.a.x + (size_t)q * w.a.n3,
                                   (double2*)Pper[q], false, w.s);
        }
    }
    HIPCHK(hipGetLastError());
    fetch_state(c, w);
    dda_status st = fill_results(w, ne, res);
    if (b_caller && res) {
        for (int q = 0; q < nrhs; ++q) res[q].qext = res[q].qabs = res[q].qsca = res[q].qpha = 0.0;
    }
    if (st == DDA_OK) warn_validity(t, kd, o->m_medium);
    return st;
}

// ---------------------------------------------------------------- many targets

// One target of a dda_solve_batched call and its progress.
struct Job {
    enum Phase { PENDING, ITER, REFINE, FINAL, DONE };
    dda_target* t = nullptr;
    const dda_opts* o = nullptr;
    std::vector<int> idx;                 // caller indices of its right-hand sides
    std::vector<double> kh;
    std::vector<double2> e0;
    std::vector<dda_c64*> P;
    double kd = 0;
    bool fp32 = false;
    int max_iter = 0;                     // the largest of its targets' limits
    std::unique_ptr<Work> w;
    Phase phase = PENDING;
    int launched = 0;
    int refines = 0;
    // several targets on one padded grid (else null, segs empty)
    std::unique_ptr<struct Batch> batch;
    std::vector<Seg> segs;
    int batch_site_blocks = 0;
};

// Targets of one dda_solve_batched call that share their padded grid, run as
// one job: each step is one launch per kernel over every right-hand side of
// every member, each reading its own target through the RhsGeo table.  The
// batch target holds the members' occupancy maps, materials and coordinates
// back to back, the twiddles of the shared grid, and as its box the largest
// member extent on each axis (the launch shape).
struct Batch {
    dda_target t;
    DevBuf rg;
    std::vector<RhsGeo> host_rg;
    ~Batch() {
        for (DevBuf* b : {&t.map, &t.mat, &t.coords, &t.tw, &t.tw32, &rg}) b->release();
    }
};

// Merge the jobs `mem` (equal padded grids, tensors built) into one job.
Job make_batch(dda_ctx* c, const std::vector<Job*>& mem) {
    Job m;
    m.batch.reset(new Batch());
    Batch& b = *m.batch;
    dda_target& bt = b.t;
    bt.ctx = c;
    const dda_target* t0 = mem[0]->t;
    Geo g = t0->geo;
    size_t map_tot = 0, site_tot = 0;
    for (const Job* j : mem) {
        for (int a = 0; a < 3; ++a) g.n[a] = std::max(g.n[a], j->t->geo.n[a]);
        map_tot += j->t->map.bytes / sizeof(int);
        site_tot += (size_t)j->t->nsites;
        bt.nsites = std::max(bt.nsites, j->t->nsites);
        bt.nmat = std::max(bt.nmat, j->t->nmat);
    }
    hipStream_t s = c->stream;
    bt.map.ensure(map_tot * sizeof(int));
    bt.mat.ensure(site_tot * sizeof(int));
    bt.coords.ensure(site_tot * 3 * sizeof(int));
    bt.tw.ensure(t0->tw.bytes);
    bt.tw32.ensure(t0->tw32.bytes);
    HIPCHK(hipMemcpyAsync(bt.tw.p, t0->tw.p, t0->tw.bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(bt.tw32.p, t0->tw32.p, t0->tw32.bytes, hipMemcpyDeviceToDevice, s));
    m.t = &bt;
    m.o = mem[0]->o;
    m.kd = mem[0]->kd;
    m.fp32 = mem[0]->fp32;
    size_t map_off = 0, site_off = 0;
    for (Job* j : mem) {
        const dda_target* jt = j->t;
        const size_t nmap = jt->map.bytes / sizeof(int), ns = (size_t)jt->nsites;
        HIPCHK(hipMemcpyAsync((int*)bt.map.p + map_off, jt->map.p, nmap * sizeof(int), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync((int*)bt.mat.p + site_off, jt->mat.p, ns * sizeof(int), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync((int*)bt.coords.p + 3 * site_off, jt->coords.p, 3 * ns * sizeof(int),
                              hipMemcpyDeviceToDevice, s));
        const int count = (int)j->idx.size();
        m.segs.push_back(Seg{j->t, j->o, (int)m.idx.size(), count, j->kd});
        RhsGeo r{};
        for (int a = 0; a < 3; ++a) r.n[a] = jt->geo.n[a];
        r.nsites = jt->nsites;
        r.map_off = (long long)map_off;
        r.site_off = (int)site_off;
        r.pass_blocks = x_pass_blocks(jt->geo, count, j->fp32);
        r.site_blocks = site_blocks_for(3LL * jt->nsites, count);
        r.kd = j->kd;
        r.ghat[0] = jt->gh64.p;
        r.ghat[1] = jt->gh32.p;
        for (int k = 0; k < count; ++k) b.host_rg.push_back(r);
        m.batch_site_blocks = std::max(m.batch_site_blocks, r.site_blocks);
        m.idx.insert(m.idx.end(), j->idx.begin(), j->idx.end());
        m.kh.insert(m.kh.end(), j->kh.begin(), j->kh.end());
        m.e0.insert(m.e0.end(), j->e0.begin(), j->e0.end());
        m.P.insert(m.P.end(), j->P.begin(), j->P.end());
        m.max_iter = std::max(m.max_iter, j->o->max_iter);
        map_off += nmap;
        site_off += ns;
    }
    b.rg.ensure(b.host_rg.size() * sizeof(RhsGeo));
    HIPCHK(hipMemcpyAsync(b.rg.p, b.host_rg.data(), b.host_rg.size() * sizeof(RhsGeo), hipMemcpyHostToDevice, s));
    g.tw32 = (const float2*)bt.tw32.p;
    g.rg = (const RhsGeo*)b.rg.p;
    bt.geo = g;
    return m;
}

// The solver configuration that must agree for targets to share launches.
std::tuple<int, int, int, int, int, unsigned, int> batch_key(const Job& j) {
    const Geo& g = j.t->geo;
    return std::make_tuple(g.M[0], g.M[1], g.M[2], (int)j.o->solver, (int)j.o->precision, j.o->flags,
                           j.o->kernel_variant);
}

// Replace every set of at least two jobs with equal batch_key, whose padded
// grid has a compile-time FFT length on every axis, by one merged job (in the
// position of its first member).
void merge_jobs(dda_ctx* c, std::vector<Job>& jobs) {
    auto mergeable = [](const Job& j) {
        const Geo& g = j.t->geo;
        return !(j.o->flags & DDA_FLAG_SEPARATE_TARGETS) && ct_length(g.M[0]) && ct_length(g.M[1]) &&
               ct_length(g.M[2]);
    };
    std::map<std::tuple<int, int, int, int, int, unsigned, int>, std::vector<size_t>> groups;
    for (size_t i = 0; i < jobs.size(); ++i)
        if (mergeable(jobs[i])) groups[batch_key(jobs[i])].push_back(i);
    std::vector<Job> out;
    std::vector<bool> taken(jobs.size(), false);
    for (size_t i = 0; i < jobs.size(); ++i) {
        if (taken[i]) continue;
        const auto it = mergeable(jobs[i]) ? groups.find(batch_key(jobs[i])) : groups.end();
        if (it == groups.end() || it->second.size() < 2) {
            out.push_back(std::move(jobs[i]));
            continue;
        }
        // i is the group's first member, so none of its members has been moved
        std::vector<Job*> mem;
        for (size_t k : it->second) {
            mem.push_back(&jobs[k]);
            taken[k] = true;
        }
        out.push_back(make_batch(c, mem));
    }
    jobs = std::move(out);
}

// Every job's targets iterate concurrently, one workspace and stream per
// job in flight (at most 4; the hardware runs that many queues at once).
// The host never blocks on one job while another can make progress: after
// each chunk of iterations a job posts an asynchronous status copy and the
// host moves on to the next job whose copy has landed.
dda_status solve_many(dda_ctx* c, std::vector<Job>& jobs, dda_result* res) {
    // one tensor per target: a target listed twice must have one kd
    std::map<const dda_target*, double> kd_of_target;
    for (Job& j : jobs) {
        check_opts(j.o);
        j.kd = kd_of(j.o, j.t->nsites);
        j.fp32 = j.o->precision == DDA_FP32_MATVEC;
        j.max_iter = j.o->max_iter;
        auto ins = kd_of_target.emplace(j.t, j.kd);
        if (!ins.second && ins.first->second != j.kd)
            invalid("a target listed twice with different wavelength or aeff (one tensor per target)");
    }
    // tensors: FP64 for every job, FP32 too where any job of that target asks
    std::map<const dda_target*, bool> want32;
    for (Job& j : jobs) want32[j.t] = want32[j.t] || j.fp32;
    for (Job& j : jobs) {
        const bool f32 = want32[j.t];
        ensure_green(c, j.t, j.kd, f32, (j.o->flags & DDA_FLAG_RECOMPUTE_GREEN) != 0);
    }
    merge_jobs(c, jobs);
    // every job's pass tilings are tuned here, on the context stream alone,
    // before any job iterates (candidates timed while other streams run
    // would be skewed); start() then finds them in the context's table
    const auto t_start = std::chrono::steady_clock::now();
    const size_t n_tuned = c->tuned.size();
    for (Job& j : jobs) {
        if ((j.o->flags & DDA_FLAG_NO_AUTOTUNE) || j.o->kernel_variant > 0) continue;
        Work w(c, c->main, j.t, (int)j.idx.size(), j.kd, j.fp32);
        if (j.batch) w.set_ragged(j.segs, j.t->geo.rg, j.batch_site_blocks);
        w.autotune(true);
    }
    // Jobs in flight (each on its own stream): the first calls of a batch
    // shape try 4, 2 and 1 in turn, timing each whole call (not a call that
    // tuned tilings or captured iteration graphs: that work would count), and
    // later calls take the fastest.  Results do not depend on it; with
    // autotuning off, 4.
    static const int kSlots[3] = {4, 2, 1};
    bool explore = jobs.size() > 1 && (jobs[0].o->flags & DDA_FLAG_NO_AUTOTUNE) == 0;
    std::string skey;
    for (const Job& j : jobs) {
        key_bytes(skey, j.t->geo.M);
        key_bytes(skey, (int)j.idx.size());
        key_bytes(skey, j.o->solver);
        key_bytes(skey, j.o->precision);
    }
    int pick = 0;
    if (explore) {
        auto ins = c->sched.emplace(skey, std::array<double, 3>{-1.0, -1.0, -1.0});
        const std::array<double, 3>& sec = ins.first->second;
        pick = -1;
        for (int i = 0; i < 3 && pick < 0; ++i)
            if (sec[i] < 0.0) pick = i;
        if (pick < 0) {
            pick = 0;
            for (int i = 1; i < 3; ++i)
                if (sec[i] < sec[pick]) pick = i;
            explore = false;
        }
    }
    const bool tuned_here = c->tuned.size() != n_tuned;
    const long long captures0 = c->captures;
    const int nslot = (int)std::min<size_t>(kSlots[pick], jobs.size());
    while ((int)c->extra.size() < nslot - 1) {
        auto* ws = new Workspace();
        c->extra.push_back(ws);
        HIPCHK(hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking));
        ws->own_stream = true;
    }
    std::vector<Workspace*> slots{&c->main};
    for (int i = 0; i < nslot - 1; ++i) slots.push_back(c->extra[i]);
    // the other streams start after the tensor FFTs built on the context stream
    hipEvent_t green_done = take_event(c);
    HIPCHK(hipEventRecord(green_done, c->stream));
    for (int i = 1; i < nslot; ++i) HIPCHK(hipStreamWaitEvent(slots[i]->stream, green_done, 0));
    c->evpool.push_back(green_done);

    std::vector<Job*> in_slot(nslot, nullptr);
    size_t next = 0;
    dda_status worst = DDA_OK;
    auto start = [&](Job& j, Workspace& ws) {
        const int nrhs = (int)j.idx.size();
        j.w.reset(new Work(c, ws, j.t, nrhs, j.kd, j.fp32));
        Work& w = *j.w;
        if (j.batch) w.set_ragged(j.segs, j.t->geo.rg, j.batch_site_blocks);
        w.qmr = j.o->solver == DDA_QMR_SYM;
        w.b2 = j.o->solver == DDA_BICGSTAB2;
        w.graphs = (j.o->flags & DDA_FLAG_NO_GRAPH) == 0;
        w.autotune((j.o->flags & DDA_FLAG_NO_AUTOTUNE) == 0, j.o->kernel_variant);
        w.upload_incidence(j.kh, j.e0);
        {
            Timed tm(c, T_SETUP, w.s);
            w.alpha_table(j.o->polarizability, j.o->m_medium, (double2*)w.a.ainv);
            launch_einc(w.a, (const int*)j.t->coords.p, w.kh, w.e0, w.s);
        }
        w.a.in = w.a.x;
        start_iteration(w, j.o, false);
        post_state(w);
        j.phase = Job::ITER;
    };
    auto finish = [&](Job& j) {
        Work& w = *j.w;
        settle_solution(w);
        final_checks(w, (j.o->flags & DDA_FLAG_NO_FINAL_CHECKS) == 0);
        {
            Timed tm(c, T_SETUP, w.s);
            for (const Seg& sg : w.parts())
                for (int q = sg.first; q < sg.first + sg.count; ++q)
                    if (j.P[q])
                        launch_permute(1, sg.t->nsites, 3, (const int*)sg.t->perm.p, w.a.x + (size_t)q * w.a.n3,
                                       (double2*)j.P[q], false, w.s);
        }
        HIPCHK(hipGetLastError());
        post_state(w);
        j.phase = Job::FINAL;
    };
    int live = 0;
    while (true) {
        for (int sl = 0; sl < nslot; ++sl) {
            if (!in_slot[sl] && next < jobs.size()) {
                in_slot[sl] = &jobs[next++];
                start(*in_slot[sl], *slots[sl]);
                ++live;
            }
        }
        if (live == 0) break;
        bool progress = false;
        for (int sl = 0; sl < nslot; ++sl) {
            Job* jp = in_slot[sl];
            if (!jp) continue;
            Job& j = *jp;
            Work& w = *j.w;
            const hipError_t q = hipEventQuery(w.ws.ready);
            if (q == hipErrorNotReady) continue;
            HIPCHK(q);
            progress = true;
            const int cap = std::min(8, j.max_iter);
            if (j.phase == Job::ITER || j.phase == Job::REFINE) {
                const bool active = any_active_after_restart(w);
                if (active && j.launched <= j.max_iter + 2 * cap) {
                    const int chunk = next_chunk(w, cap);
                    run_chunk(w, chunk);
                    j.launched += chunk;
                    j.phase = Job::ITER;
                    post_state(w);
                } else if (j.phase == Job::ITER && j.fp32 && j.refines < 5) {
                    launch_refinement(w);
                    ++j.refines;
                    j.phase = Job::REFINE;
                    post_state(w);
                } else {
                    finish(j);
                }
            } else if (j.phase == Job::FINAL) {
                std::vector<dda_result> r(j.idx.size());
                const dda_status st = fill_results(w, (j.o->flags & DDA_FLAG_NO_FINAL_CHECKS) == 0, r.data());
                for (size_t k = 0; k < j.idx.size(); ++k)
                    if (res) res[j.idx[k]] = r[k];
                if (st != DDA_OK && (worst == DDA_OK || st > worst)) worst = st;
                j.phase = Job::DONE;
                j.w.reset();
                in_slot[sl] = nullptr;
                --live;
            }
        }
        if (!progress) {
            // wait for the first in-flight job instead of spinning
            for (int sl = 0; sl < nslot; ++sl)
                if (in_slot[sl]) {
                    HIPCHK(hipEventSynchronize(in_slot[sl]->w->ws.ready));
                    break;
                }
        }
    }
    for (int i = 1; i < nslot; ++i) HIPCHK(hipStreamSynchronize(slots[i]->stream));
    flush_timing(c);
    if (explore && !tuned_here && c->captures == captures0)
        c->sched[skey][pick] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return worst;
}

// Sorted device copies of a target's sites (throws on invalid input; the
// caller has made the context's device current).
dda_target* create_target(dda_ctx* c, int64_t n_sites, const int32_t* ijk, const dda_c64* m_site) {
    if (n_sites < 1 || n_sites > (int64_t)1 << 30) invalid("n_sites out of range");
    if (!ijk || !m_site) invalid("ijk or m_site is NULL");
    const int n = (int)n_sites;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = ijk[a]; hi[a] = ijk[a]; }
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], ijk[3 * j + a]);
            hi[a] = std::max(hi[a], ijk[3 * j + a]);
        }
    Geo g{};
    for (int a = 0; a < 3; ++a) {
        const long long ext = (long long)hi[a] - lo[a] + 1;
        if (ext > 4096) invalid("target extent above 4096 sites on an axis");
        g.n[a] = (int)ext;
        g.M[a] = padded_extent(g.n[a]);
        g.H[a] = g.M[a] / 2 + 1;
    }
    for (int a = 0; a < 3; ++a)
        if (g.M[a] > MAX_PADDED || 3 * g.M[a] > Tile<double>::EMAX)
            invalid("box extent " + std::to_string(g.n[a]) + " needs a padded FFT extent " +
                    std::to_string(g.M[a]) + " above the supported 512");
    g.npts = (long long)g.M[0] * g.M[1] * g.M[2];
    const long long boxv = (long long)g.n[0] * g.n[1] * g.n[2];
    if (boxv > ((long long)1 << 31) - 1) invalid("bounding box too large");
    // sort sites in box-scan order (x fastest), reject duplicates
    std::vector<std::pair<long long, int>> key(n);
    for (int j = 0; j < n; ++j) {
        const long long x = ijk[3 * j] - lo[0], y = ijk[3 * j + 1] - lo[1], z = ijk[3 * j + 2] - lo[2];
        key[j] = {(z * g.n[1] + y) * g.n[0] + x, j};
    }
    std::sort(key.begin(), key.end());
    for (int j = 1; j < n; ++j)
        if (key[j].first == key[j - 1].first)
            invalid("duplicate lattice site (" + std::to_string(ijk[3 * key[j].second]) + "," +
                    std::to_string(ijk[3 * key[j].second + 1]) + "," + std::to_string(ijk[3 * key[j].second + 2]) +
                    ")");
    auto* t = new dda_target();
    t->ctx = c;
    t->nsites = n;
    std::vector<int> map((size_t)boxv, -1), perm(n), mat(n), coords((size_t)n * 3);
    std::map<std::pair<double, double>, int> mid;
    try {
        for (int s = 0; s < n; ++s) {
            const int j = key[s].second;
            map[(size_t)key[s].first] = s;
            perm[s] = j;
            for (int a = 0; a < 3; ++a) coords[(size_t)s * 3 + a] = ijk[3 * j + a];
            const dda_c64 m = m_site[j];
            if (!std::isfinite(m.re) || !std::isfinite(m.im)) invalid("non-finite refractive index");
            if (m.re == 1.0 && m.im == 0.0) invalid("refractive index 1 (vacuum) on an occupied site");
            auto it = mid.find({m.re, m.im});
            if (it == mid.end()) {
                if (mid.size() >= 65535) invalid("more than 65535 distinct materials");
                it = mid.emplace(std::make_pair(m.re, m.im), (int)mid.size()).first;
                t->mats.push_back(double2{m.re, m.im});
            }
            mat[s] = it->second;
        }
        t->nmat = (int)t->mats.size();
        // FFT plans and their twiddle tables W_L^t = exp(-2 pi i t / L)
        std::vector<double2> tw;
        std::map<int, int> twoff;
        for (int a = 0; a < 3; ++a) {
            g.ax[a] = make_plan(g.M[a]);
            auto it = twoff.find(g.M[a]);
            if (it == twoff.end()) {
                const int off = (int)tw.size();
                for (int i = 0; i < g.M[a]; ++i) {
                    const double ang = -2.0 * M_PI * (double)i / (double)g.M[a];
                    tw.push_back(double2{std::cos(ang), std::sin(ang)});
                }
                it = twoff.emplace(g.M[a], off).first;
            }
            g.ax[a].tw = it->second;
        }
        t->geo = g;
        auto up = [&](DevBuf& b, const void* src, size_t bytes) {
            b.ensure(bytes);
            HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(t->map, map.data(), map.size() * sizeof(int));
        up(t->perm, perm.data(), perm.size() * sizeof(int));
        up(t->mat, mat.data(), mat.size() * sizeof(int));
        up(t->coords, coords.data(), coords.size() * sizeof(int));
        up(t->tw, tw.data(), tw.size() * sizeof(double2));
        std::vector<float2> tw32(tw.size());
        for (size_t i = 0; i < tw.size(); ++i) tw32[i] = float2{(float)tw[i].x, (float)tw[i].y};
        up(t->tw32, tw32.data(), tw32.size() * sizeof(float2));
        t->geo.tw32 = (const float2*)t->tw32.p;
        up(t->mdev, t->mats.data(), t->mats.size() * sizeof(double2));
        for (int a = 0; a < 3; ++a) t->lo[a] = lo[a];
    } catch (...) {
        for (DevBuf* b : {&t->map, &t->perm, &t->mat, &t->coords, &t->tw, &t->tw32, &t->mdev}) b->release();
        delete t;
        throw;
    }
    return t;
}

// Release a target's device memory (and its extended near-field volume).
void free_target(dda_target* t) {
    if (!t) return;
    free_target(t->nf);
    t->nf = nullptr;
    for (DevBuf* b : {&t->map, &t->perm, &t->mat, &t->coords, &t->tw, &t->tw32, &t->mdev, &t->gh64, &t->gh32})
        b->release();
    delete t;
}

// Points the near-field volume adds below (e[2a]) and above (e[2a+1]) the
// bounding box on axis a: round(r * n) for the fractions r1..r6 of the box
// extents n ("Additional Nearfield Calculation?").
void nf_extension(const dda_target* t, const double* r, int e[6], int org[3], int dims[3]) {
    if (!r) invalid("ext is NULL");
    for (int i = 0; i < 6; ++i) {
        if (!std::isfinite(r[i]) || r[i] < 0.0 || r[i] > 16.0) invalid("ext fractions must lie in [0, 16]");
        e[i] = (int)std::floor(r[i] * t->geo.n[i / 2] + 0.5);
    }
    for (int a = 0; a < 3; ++a) {
        org[a] = t->lo[a] - e[2 * a];
        dims[a] = t->geo.n[a] + e[2 * a] + e[2 * a + 1];
        if (padded_extent(dims[a]) > MAX_PADDED)
            invalid("near-field volume of " + std::to_string(dims[a]) + " points on axis " + std::to_string(a) +
                    " needs a padded FFT extent above the supported 512");
    }
}

// The extended volume as a target whose sites are all of its points, in
// box-scan order (cached on t for the last extension asked for).
dda_target* nf_target(dda_ctx* c, dda_target* t, const int e[6], const int org[3], const int dims[3]) {
    if (t->nf && std::equal(e, e + 6, t->nf_key)) return t->nf;
    HIPCHK(hipStreamSynchronize(c->stream));
    free_target(t->nf);
    t->nf = nullptr;
    const long long n = (long long)dims[0] * dims[1] * dims[2];
    std::vector<int32_t> ijk((size_t)n * 3);
    long long i = 0;
    for (int z = 0; z < dims[2]; ++z)
        for (int y = 0; y < dims[1]; ++y)
            for (int x = 0; x < dims[0]; ++x, ++i) {
                ijk[(size_t)i * 3 + 0] = org[0] + x;
                ijk[(size_t)i * 3 + 1] = org[1] + y;
                ijk[(size_t)i * 3 + 2] = org[2] + z;
            }
    // one placeholder material: the product runs with a zero diagonal
    const std::vector<dda_c64> m((size_t)n, dda_c64{2.0, 0.0});
    t->nf = create_target(c, n, ijk.data(), m.data());
    std::copy(e, e + 6, t->nf_key);
    return t->nf;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

dda_status dda_ctx_create(int device, void* hip_stream, dda_ctx** out) {
    return guarded([&]() -> dda_status {
        if (!out) invalid("out is NULL");
        *out = nullptr;
        int n = 0;
        HIPCHK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) invalid("no HIP device " + std::to_string(device));
        std::unique_ptr<dda_ctx> c(new dda_ctx());
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        c->main.stream = c->stream;
        {
            Scope sc(c.get());
            scratch_setup(device);
        }
        *out = c.release();
        return DDA_OK;
    });
}

dda_status dda_ctx_destroy(dda_ctx* c) {
    return guarded([&]() -> dda_status {
        if (!c) return DDA_OK;
        {
            Scope sc(c);
            (void)hipStreamSynchronize(c->stream);
            for (Workspace* ws : c->extra) {
                if (ws->stream) (void)hipStreamSynchronize(ws->stream);
                ws->release();
                delete ws;
            }
            c->main.release();
            for (DevBuf* b : {&c->dainv, &c->aux, &c->gtmp}) b->release();
            for (const auto& p : c->pending) {
                (void)hipEventDestroy(p.a);
                (void)hipEventDestroy(p.b);
            }
            for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
        }
        delete c;
        return DDA_OK;
    });
}

dda_status dda_target_create(dda_ctx* c, int64_t n_sites, const int32_t* ijk, const dda_c64* m_site,
                             dda_target** out) {
    return guarded([&]() -> dda_status {
        if (!c || !out) invalid("ctx or out is NULL");
        *out = nullptr;
        Scope sc(c);
        *out = create_target(c, n_sites, ijk, m_site);
        return DDA_OK;
    });
}

dda_status dda_target_destroy(dda_target* t) {
    return guarded([&]() -> dda_status {
        if (!t) return DDA_OK;
        {
            Scope sc(t->ctx);
            (void)hipStreamSynchronize(t->ctx->stream);
            free_target(t);
        }
        return DDA_OK;
    });
}

dda_status dda_target_geometry(const dda_target* t, int32_t box[3], int32_t grid[3]) {
    return guarded([&]() -> dda_status {
        if (!t || !box || !grid) invalid("NULL argument");
        for (int a = 0; a < 3; ++a) {
            box[a] = t->geo.n[a];
            grid[a] = t->geo.M[a];
        }
        return DDA_OK;
    });
}

dda_status dda_apply(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs, const dda_incidence* inc,
                     const dda_c64* x, dda_c64* y) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !x || !y) invalid("NULL argument");
        if (x == y) invalid("x and y alias");
        if (n_rhs < 1) invalid("n_rhs must be >= 1");
        check_opts(o);
        Scope sc(c);
        std::vector<double> kh;
        std::vector<double2> e0;
        pack_incidence(n_rhs, inc, kh, e0);
        const double kd = kd_of(o, t->nsites);
        const bool fp32 = o->precision == DDA_FP32_MATVEC;
        ensure_green(c, t, kd, fp32, (o->flags & DDA_FLAG_RECOMPUTE_GREEN) != 0);
        Work w(c, c->main, t, n_rhs, kd, fp32);
        w.qmr = o->solver == DDA_QMR_SYM;
        w.b2 = o->solver == DDA_BICGSTAB2;
        w.graphs = false;   // one stream: replays are slower than launches
        w.autotune((o->flags & DDA_FLAG_NO_AUTOTUNE) == 0, o->kernel_variant);
        w.upload_incidence(kh, e0);
        w.alpha_table(o->polarizability, o->m_medium, (double2*)w.a.ainv);
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)x, w.a.p, true, c->stream);
        w.a.in = w.a.p;
        w.a.out = w.a.v;
        w.matvec(SC_PLAIN, GA_PLAIN, CHK_NONE, CHK_NONE);
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, w.a.v, (double2*)y, false, c->stream);
        HIPCHK(hipGetLastError());
        return DDA_OK;
    });
}

dda_status dda_apply_noalloc(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs,
                             const dda_incidence* inc, const dda_c64* x, dda_c64* y) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !x || !y) invalid("NULL argument");
        if (x == y) invalid("x and y alias");
        if (n_rhs < 1 || n_rhs > NOALLOC_MAX_RHS) invalid("n_rhs must lie in 1..256");
        check_opts(o);
        Scope sc(c);
        double khv[3 * NOALLOC_MAX_RHS];
        double2 e0v[3 * NOALLOC_MAX_RHS];
        pack_incidence(n_rhs, inc, khv, e0v);
        const double kd = kd_of(o, t->nsites);
        const bool fp32 = o->precision == DDA_FP32_MATVEC;
        if ((o->flags & DDA_FLAG_RECOMPUTE_GREEN) || t->green_kd != kd || !(fp32 ? t->have32 : t->have64))
            invalid("the interaction-tensor FFT of this target at this kd and precision is not built (a dda_apply "
                    "or dda_solve call with the same options builds it)");
        char* base = (char*)scratch_of(c->device);
        if (!base) invalid("no work memory on this device");
        const Carve L = carve_layout(t, n_rhs, fp32);
        if (L.total > SCRATCH_BYTES)
            invalid("the product needs " + std::to_string(L.total) + " bytes of work memory, above the fixed " +
                    std::to_string(SCRATCH_BYTES));
        // no timing events (they would be created on first use)
        struct NoEvents {
            dda_ctx* c;
            bool keep;
            explicit NoEvents(dda_ctx* c_) : c(c_), keep(c_->tsuppress) { c->tsuppress = true; }
            ~NoEvents() { c->tsuppress = keep; }
        } ne(c);
        Work w(c, c->main, t, n_rhs, kd, fp32, base, L);
        w.autotune(false, o->kernel_variant);   // the tiling tuned for this shape, else the default
        w.upload_incidence(khv, e0v);
        w.alpha_table(o->polarizability, o->m_medium, (double2*)w.a.ainv);
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)x, w.a.p, true, w.s);
        w.a.in = w.a.p;
        w.a.out = w.a.v;
        w.matvec(SC_PLAIN, GA_PLAIN, CHK_NONE, CHK_NONE);
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, w.a.v, (double2*)y, false, w.s);
        HIPCHK(hipGetLastError());
        return DDA_OK;
    });
}

dda_status dda_solve(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs, const dda_incidence* inc,
                     dda_c64* P, const dda_c64* P0, dda_result* res) {
    return guarded([&]() -> dda_status {
        if (!c || !t) invalid("NULL ctx or target");
        Scope sc(c);
        return solve_one(c, t, o, n_rhs, inc, P, nullptr, P0, res);
    });
}

dda_status dda_solve_rhs(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs, const dda_incidence* inc,
                         const dda_c64* b, dda_c64* x, const dda_c64* x0, dda_result* res) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !b || !x) invalid("NULL argument");
        if ((const void*)b == (const void*)x) invalid("b and x alias");
        Scope sc(c);
        return solve_one(c, t, o, n_rhs, inc, x, nullptr, x0, res, b);
    });
}

dda_status dda_solve_batched(dda_ctx* c, int32_t n_targets, dda_target* const* targets, const dda_opts* opts,
                             int32_t n_rhs, const int32_t* rhs_target, const dda_incidence* inc, dda_c64* const* P,
                             dda_result* res) {
    return guarded([&]() -> dda_status {
        if (!c || !targets || !opts || !rhs_target || !inc) invalid("NULL argument");
        if (n_targets < 1 || n_rhs < 1) invalid("n_targets and n_rhs must be >= 1");
        Scope sc(c);
        for (int q = 0; q < n_rhs; ++q)
            if (rhs_target[q] < 0 || rhs_target[q] >= n_targets) invalid("rhs_target out of range");
        std::vector<Job> jobs;
        for (int ti = 0; ti < n_targets; ++ti) {
            Job j;
            for (int q = 0; q < n_rhs; ++q)
                if (rhs_target[q] == ti) j.idx.push_back(q);
            if (j.idx.empty()) continue;
            if (!targets[ti]) invalid("NULL target");
            j.t = targets[ti];
            j.o = &opts[ti];
            std::vector<dda_incidence> sub(j.idx.size());
            for (size_t i = 0; i < j.idx.size(); ++i) {
                sub[i] = inc[j.idx[i]];
                j.P.push_back(P ? P[j.idx[i]] : nullptr);
            }
            pack_incidence((int)sub.size(), sub.data(), j.kh, j.e0);
            jobs.push_back(std::move(j));
        }
        return solve_many(c, jobs, res);
    });
}

dda_status dda_grad_eps(dda_ctx* c, dda_target* t, const dda_opts* o, const dda_incidence* inc, const dda_c64* P,
                        double w_qabs, double w_qext, dda_c64* grad, dda_result* adj) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !P || !grad) invalid("NULL argument");
        if (!std::isfinite(w_qabs) || !std::isfinite(w_qext)) invalid("non-finite weights");
        check_opts(o);
        Scope sc(c);
        std::vector<double> kh;
        std::vector<double2> e0;
        pack_incidence(1, inc, kh, e0);
        const double kd = kd_of(o, t->nsites);
        const bool fp32 = o->precision == DDA_FP32_MATVEC;
        ensure_green(c, t, kd, fp32, (o->flags & DDA_FLAG_RECOMPUTE_GREEN) != 0);
        Work w(c, c->main, t, 1, kd, fp32);
        w.qmr = o->solver == DDA_QMR_SYM;
        w.b2 = o->solver == DDA_BICGSTAB2;
        w.graphs = false;   // one stream: replays are slower than launches
        w.autotune((o->flags & DDA_FLAG_NO_AUTOTUNE) == 0, o->kernel_variant);
        w.upload_incidence(kh, e0);
        w.alpha_table(o->polarizability, o->m_medium, (double2*)w.a.ainv);
        double2* dainv = (double2*)c->dainv.ensure((size_t)t->nmat * 3 * sizeof(double2));
        w.alpha_table(o->polarizability + 2, o->m_medium, dainv);
        // P in sorted order, kept for the gradient
        double2* Ps = (double2*)c->aux.ensure((size_t)w.a.n3 * sizeof(double2) + (size_t)t->nsites * sizeof(double2));
        double2* gs = Ps + w.a.n3;
        launch_permute(1, t->nsites, 3, (const int*)t->perm.p, (const double2*)P, Ps, true, c->stream);
        launch_einc(w.a, (const int*)t->coords.p, w.kh, w.e0, c->stream);
        launch_adjoint_rhs(w.a, Ps, w_qabs, w_qext, c->stream);
        w.a.in = w.a.x;
        iterate(w, o, false);
        final_checks(w, false);
        w.a.in = Ps;
        launch_grad(w.a, dainv, w_qabs, gs, c->stream);
        launch_permute(1, t->nsites, 1, (const int*)t->perm.p, gs, (double2*)grad, false, c->stream);
        HIPCHK(hipGetLastError());
        fetch_state(c, w);
        dda_result r{};
        const dda_status st = fill_results(w, false, &r);
        // the efficiency fields of an adjoint solve carry no physical meaning
        r.qext = r.qabs = r.qsca = r.qpha = 0.0;
        if (adj) *adj = r;
        return st;
    });
}

dda_status dda_ctx_set_timing(dda_ctx* c, int mask) {
    return guarded([&]() -> dda_status {
        if (!c) invalid("ctx is NULL");
        Scope sc(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        flush_timing(c);
        if (mask) {
            for (int i = 0; i < DDA_TIMING_CATEGORIES; ++i) {
                c->tms[i] = 0.0;
                c->tlaunch[i] = 0;
                c->tall[i] = 0;
            }
            c->tchunk = 0;
        }
        c->timing = mask & ((1 << DDA_TIMING_CATEGORIES) - 1);
        return DDA_OK;
    });
}

dda_status dda_ctx_get_timing(dda_ctx* c, dda_timing* out) {
    return guarded([&]() -> dda_status {
        if (!c || !out) invalid("NULL argument");
        Scope sc(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        flush_timing(c);
        for (int i = 0; i < DDA_TIMING_CATEGORIES; ++i) {
            out->ms[i] = c->tms[i];
            out->launches[i] = c->tlaunch[i];
            out->all_launches[i] = c->tall[i];
        }
        return DDA_OK;
    });
}

dda_status dda_ctx_set_timing_sample(dda_ctx* c, int every) {
    return guarded([&]() -> dda_status {
        if (!c) invalid("ctx is NULL");
        if (every < 1) invalid("every must be >= 1");
        c->tsample = every;
        return DDA_OK;
    });
}

dda_status dda_ctx_tuned_variants(dda_ctx* c, const dda_target* t, int32_t n_rhs, dda_precision precision,
                                  int32_t variants[3]) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !variants) invalid("NULL argument");
        if (n_rhs < 1) invalid("n_rhs must be >= 1");
        if (precision != DDA_FP64 && precision != DDA_FP32_MATVEC) invalid("unknown precision");
        const Geo& g = t->geo;
        auto key = std::make_tuple(g.M[0], g.M[1], g.M[2], g.n[0], g.n[1], g.n[2], (int)n_rhs,
                                   precision == DDA_FP32_MATVEC ? 1 : 0);
        auto it = c->tuned.find(key);
        for (int i = 0; i < 3; ++i) variants[i] = it == c->tuned.end() ? -1 : it->second[i];
        return DDA_OK;
    });
}

dda_status dda_far_field(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs, const dda_c64* P,
                         int32_t n_dir, const double* n_hat, const double* theta_hat, const double* phi_hat,
                         dda_c64* f, double* dcs) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !P || !n_hat || !theta_hat || !phi_hat) invalid("NULL argument");
        if (n_rhs < 1 || n_dir < 1) invalid("n_rhs and n_dir must be >= 1");
        if (n_dir > 65535 || n_rhs > 65535) invalid("n_rhs and n_dir must be <= 65535");
        check_opts(o);
        std::vector<double> dirs((size_t)n_dir * 9);
        for (int d = 0; d < n_dir; ++d) {
            const double* v[3] = {n_hat + 3 * d, theta_hat + 3 * d, phi_hat + 3 * d};
            for (int i = 0; i < 3; ++i) {
                double nn = 0.0;
                for (int m = 0; m < 3; ++m) {
                    if (!std::isfinite(v[i][m])) invalid("non-finite direction " + std::to_string(d));
                    nn += v[i][m] * v[i][m];
                    dirs[(size_t)d * 9 + 3 * i + m] = v[i][m];
                }
                if (std::fabs(nn - 1.0) > 1e-6) invalid("direction vectors must be unit vectors (" + std::to_string(d) + ")");
            }
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j) {
                    const double dot = v[i][0] * v[j][0] + v[i][1] * v[j][1] + v[i][2] * v[j][2];
                    if (std::fabs(dot) > 1e-6) invalid("n, theta, phi must be orthogonal (" + std::to_string(d) + ")");
                }
        }
        Scope sc(c);
        const double kd = kd_of(o, t->nsites);
        const size_t n3 = 3 * (size_t)t->nsites;
        const size_t pb = (size_t)n_rhs * n3 * sizeof(double2), db = dirs.size() * sizeof(double);
        const size_t fb = (size_t)n_rhs * n_dir * 2 * sizeof(double2), cb = (size_t)n_rhs * n_dir * sizeof(double);
        char* buf = (char*)c->ffbuf.ensure(pb + db + fb + cb + 256);
        double2* Ps = (double2*)buf;
        double* ddev = (double*)(buf + pb);
        double2* fdev = (double2*)(buf + pb + db);
        double* cdev = (double*)(buf + pb + db + fb);
        HIPCHK(hipMemcpyAsync(ddev, dirs.data(), db, hipMemcpyHostToDevice, c->stream));
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)P, Ps, true, c->stream);
        launch_farfield(t->nsites, (const int*)t->coords.p, Ps, n_rhs, ddev, n_dir, kd, t->lo, t->geo.n, fdev, cdev,
                        c->stream);
        HIPCHK(hipGetLastError());
        if (f) HIPCHK(hipMemcpyAsync(f, fdev, fb, hipMemcpyDeviceToHost, c->stream));
        if (dcs) HIPCHK(hipMemcpyAsync(dcs, cdev, cb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return DDA_OK;
    });
}

}  // extern "C"

namespace {
// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n from
// the Chebyshev-like first guess, P_n and P_n' by the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}
}  // namespace

extern "C" {

dda_status dda_scattering_averages(dda_ctx* c, dda_target* t, const dda_opts* o, int32_t n_rhs,
                                   const dda_incidence* inc, const dda_c64* P, int32_t n_theta, int32_t n_phi,
                                   double* out) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !inc || !P || !out) invalid("NULL argument");
        if (n_rhs < 1 || n_rhs > 65535) invalid("n_rhs must be in 1..65535");
        if (n_theta < 2 || n_phi < 1 || (long long)n_theta * n_phi > 65535) invalid("need n_theta >= 2, n_phi >= 1 and n_theta * n_phi <= 65535");
        check_opts(o);
        std::vector<double> kh;
        std::vector<double2> e0;
        pack_incidence(n_rhs, inc, kh, e0);
        Scope sc(c);
        const double kd = kd_of(o, t->nsites);
        const double a = aeff_over_d(t->nsites);
        std::vector<double> mu, wmu;
        gauss_legendre(n_theta, mu, wmu);
        const int nd = n_theta * n_phi;
        // right-hand sides in groups of at most 4M directions, each group one launch
        const int qg = std::max(1, std::min(n_rhs, (1 << 22) / nd));
        const long long ndt = (long long)nd * qg;
        const size_t n3 = 3 * (size_t)t->nsites;
        const size_t pb = (size_t)n_rhs * n3 * sizeof(double2), db = (size_t)ndt * 9 * sizeof(double);
        const size_t fb = (size_t)ndt * 2 * sizeof(double2), cb = (size_t)ndt * sizeof(double);
        const size_t kb = (size_t)n_rhs * 3 * sizeof(double), mb = (size_t)n_theta * sizeof(double);
        char* buf = (char*)c->ffbuf.ensure(pb + db + fb + cb + kb + mb + 256);
        double2* Ps = (double2*)buf;
        double* ddev = (double*)(buf + pb);
        double2* fdev = (double2*)(buf + pb + db);
        double* cdev = (double*)(buf + pb + db + fb);
        double* kdev = (double*)(buf + pb + db + fb + cb);
        double* mdev = (double*)(buf + pb + db + fb + cb + kb);
        launch_permute(n_rhs, t->nsites, 3, (const int*)t->perm.p, (const double2*)P, Ps, true, c->stream);
        HIPCHK(hipMemcpyAsync(kdev, kh.data(), kb, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(mdev, mu.data(), mb, hipMemcpyHostToDevice, c->stream));
        std::vector<double> dcs((size_t)ndt);
        for (int g0 = 0; g0 < n_rhs; g0 += qg) {
            const int ng = std::min(qg, n_rhs - g0);
            // the directions about each right-hand side's incidence direction,
            // formed on the device
            launch_avg_dirs(ng, kdev + 3 * (size_t)g0, mdev, n_theta, n_phi, ddev, c->stream);
            launch_farfield_sets(t->nsites, (const int*)t->coords.p, Ps + (size_t)g0 * n3, ng, ddev, nd, kd, t->lo,
                                 t->geo.n, fdev, cdev, c->stream);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(dcs.data(), cdev, (size_t)ng * nd * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            for (int q = g0; q < g0 + ng; ++q) {
                const double* dq = dcs.data() + (size_t)(q - g0) * nd;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
                for (int i = 0; i < n_theta; ++i)
                    for (int j = 0; j < n_phi; ++j) {
                        const double wgt = wmu[i] * (2.0 * M_PI / n_phi) * dq[(size_t)i * n_phi + j];
                        s0 += wgt;
                        s1 += wgt * mu[i];
                        s2 += wgt * mu[i] * mu[i];
                    }
                out[3 * q + 0] = s0 / (M_PI * a * a);
                out[3 * q + 1] = s0 > 0 ? s1 / s0 : 0.0;
                out[3 * q + 2] = s0 > 0 ? s2 / s0 : 0.0;
            }
        }
        return DDA_OK;
    });
}

dda_status dda_mueller(int32_t n_dir, const dda_c64* f1, const dda_c64* f2, const dda_c64* e01, const dda_c64* e02,
                       const double* phi_deg, double* S) {
    return guarded([&]() -> dda_status {
        if (!f1 || !f2 || !e01 || !e02 || !phi_deg || !S) invalid("NULL argument");
        if (n_dir < 1) invalid("n_dir must be >= 1");
        typedef std::complex<double> cd;
        auto C = [](const dda_c64& z) { return cd(z.re, z.im); };
        // rows: incident e01, e02 projected on y and z of the Lab Frame
        const cd a = std::conj(C(e01[1])), b = std::conj(C(e01[2]));
        const cd cc = std::conj(C(e02[1])), d = std::conj(C(e02[2]));
        const cd mi(0.0, -1.0);
        for (int k = 0; k < n_dir; ++k) {
            const double p = phi_deg[k] * (M_PI / 180.0);
            const double cp = std::cos(p), sp = std::sin(p);
            // F = (f11 f12; -f21 -f22), then F (a b; c d) R with R = (cp sp; sp -cp)
            const cd F11 = C(f1[2 * k + 0]), F12 = C(f2[2 * k + 0]);
            const cd F21 = -C(f1[2 * k + 1]), F22 = -C(f2[2 * k + 1]);
            const cd G11 = F11 * a + F12 * cc, G12 = F11 * b + F12 * d;
            const cd G21 = F21 * a + F22 * cc, G22 = F21 * b + F22 * d;
            const cd S2 = mi * (G11 * cp + G12 * sp), S3 = mi * (G11 * sp - G12 * cp);
            const cd S4 = mi * (G21 * cp + G22 * sp), S1 = mi * (G21 * sp - G22 * cp);
            const double a1 = std::norm(S1), a2 = std::norm(S2), a3 = std::norm(S3), a4 = std::norm(S4);
            double* M = S + (size_t)k * 16;
            M[0] = 0.5 * (a2 + a3 + a4 + a1);
            M[1] = 0.5 * (a2 - a3 + a4 - a1);
            M[2] = std::real(S2 * std::conj(S3) + S1 * std::conj(S4));
            M[3] = std::imag(S2 * std::conj(S3) - S1 * std::conj(S4));
            M[4] = 0.5 * (a2 + a3 - a4 - a1);
            M[5] = 0.5 * (a2 - a3 - a4 + a1);
            M[6] = std::real(S2 * std::conj(S3) - S1 * std::conj(S4));
            M[7] = std::imag(S2 * std::conj(S3) + S1 * std::conj(S4));
            M[8] = std::real(S2 * std::conj(S4) + S1 * std::conj(S3));
            M[9] = std::real(S2 * std::conj(S4) - S1 * std::conj(S3));
            M[10] = std::real(S1 * std::conj(S2) + S3 * std::conj(S4));
            M[11] = std::imag(S2 * std::conj(S1) + S4 * std::conj(S3));
            M[12] = std::imag(S4 * std::conj(S2) + S1 * std::conj(S3));
            M[13] = std::imag(S4 * std::conj(S2) - S1 * std::conj(S3));
            M[14] = std::imag(S1 * std::conj(S2) - S3 * std::conj(S4));
            M[15] = std::real(S1 * std::conj(S2) - S3 * std::conj(S4));
        }
        return DDA_OK;
    });
}

dda_status dda_nearfield_volume(const dda_target* t, const double ext[6], int32_t origin[3], int32_t dims[3]) {
    return guarded([&]() -> dda_status {
        if (!t || !origin || !dims) invalid("NULL argument");
        int e[6], org[3], dm[3];
        nf_extension(t, ext, e, org, dm);
        for (int a = 0; a < 3; ++a) {
            origin[a] = org[a];
            dims[a] = dm[a];
        }
        return DDA_OK;
    });
}

dda_status dda_nearfield(dda_ctx* c, dda_target* t, const dda_opts* o, const double ext[6], int32_t n_rhs,
                         const dda_incidence* inc, const dda_c64* P, dda_c64* E_inc, dda_c64* E_sca) {
    return guarded([&]() -> dda_status {
        if (!c || !t || !P || !E_sca) invalid("NULL argument");
        if (n_rhs < 1 || n_rhs > 65535) invalid("n_rhs must lie in 1..65535");
        check_opts(o);
        int e[6], org[3], dims[3];
        nf_extension(t, ext, e, org, dims);
        Scope sc(c);
        std::vector<double> kh;
        std::vector<double2> e0;
        pack_incidence(n_rhs, inc, kh, e0);
        // k d of the target itself (a_eff counts its sites, not the volume's)
        const double kd = kd_of(o, t->nsites);
        const bool fp32 = o->precision == DDA_FP32_MATVEC;
        dda_target* x = nf_target(c, t, e, org, dims);
        ensure_green(c, x, kd, fp32, (o->flags & DDA_FLAG_RECOMPUTE_GREEN) != 0);
        Work w(c, c->main, x, n_rhs, kd, fp32);
        w.autotune((o->flags & DDA_FLAG_NO_AUTOTUNE) == 0, o->kernel_variant);
        w.upload_incidence(kh, e0);
        launch_fill((double2*)w.a.ainv, (long long)n_rhs * x->nmat * 3, w.s);
        launch_fill(w.a.p, (long long)n_rhs * w.a.n3, w.s);
        launch_nf_place(t->nsites, (const int*)t->perm.p, (const int*)t->coords.p, (const double2*)P, n_rhs, org,
                        dims, w.a.p, w.s);
        w.a.in = w.a.p;
        w.a.out = w.a.v;
        w.matvec(SC_PLAIN, GA_PLAIN, CHK_NONE, CHK_NONE);
        launch_nf_out(n_rhs, org, dims, w.kh, w.e0, kd, w.a.v, (double2*)E_inc, (double2*)E_sca, w.s);
        HIPCHK(hipGetLastError());
        return DDA_OK;
    });
}

dda_status dda_field_line(dda_ctx* c, int32_t n_rhs, const int32_t origin[3], const int32_t dims[3],
                          const dda_c64* E, const double a[3], const double b[3], int32_t n_points, dda_c64* out) {
    return guarded([&]() -> dda_status {
        if (!c || !origin || !dims || !E || !a || !b || !out) invalid("NULL argument");
        if (n_rhs < 1 || n_rhs > 65535) invalid("n_rhs must lie in 1..65535");
        if (n_points < 1) invalid("n_points must be >= 1");
        for (int d = 0; d < 3; ++d) {
            if (dims[d] < 1) invalid("dims must be >= 1");
            if (!std::isfinite(a[d]) || !std::isfinite(b[d])) invalid("non-finite line end point");
            const double lo = origin[d], hi = (double)origin[d] + dims[d] - 1;
            if (a[d] < lo || a[d] > hi || b[d] < lo || b[d] > hi)
                invalid("line end points must lie inside the lattice box");
        }
        if ((long long)dims[0] * dims[1] * dims[2] > ((long long)1 << 31) - 1) invalid("lattice box too large");
        Scope sc(c);
        const int org[3] = {origin[0], origin[1], origin[2]};
        const int dm[3] = {dims[0], dims[1], dims[2]};
        launch_field_line(n_rhs, org, dm, (const double2*)E, a, b, n_points, (double2*)out, c->stream);
        HIPCHK(hipGetLastError());
        return DDA_OK;
    });
}

const char* dda_last_error(void) { return g_err.c_str(); }

}  // extern "C"
