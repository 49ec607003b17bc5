// C-ABI of libdect: argument validation, physics constants, workspace plans
// and the launch sequence of Algorithm 1 (sinogram form) on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dect_internal.h"

namespace dect {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static double corner_pitch(const dect_geometry& g) {
    const double R = 0.5 * g.pixel_mm * std::hypot((double)g.n_x, (double)g.n_y);
    return 2.0 * g.sdd_mm * std::tan(std::asin(R / g.sid_mm)) / g.n_det;
}

int resolve_geometry(const dect_geometry* in, Geom* out) {
    if (!in) return fail(DECT_EINVAL, "geometry is NULL");
    const dect_geometry& g = *in;
    if (g.n_x < 1 || g.n_y < 1 || g.n_views < 1 || g.n_det < 1)
        return fail(DECT_EINVAL, "geometry sizes must be >= 1 (n_x=%d n_y=%d n_views=%d n_det=%d)",
                    g.n_x, g.n_y, g.n_views, g.n_det);
    if (g.n_x > 16384 || g.n_y > 16384 || g.n_det > 65536 || g.n_views > 65536)
        return fail(DECT_EINVAL, "geometry sizes too large");
    if (!(g.pixel_mm > 0) || !(g.sid_mm > 0) || !(g.sdd_mm > g.sid_mm))
        return fail(DECT_EINVAL, "need pixel_mm > 0 and sdd_mm > sid_mm > 0");
    if (!std::isfinite(g.angle0_rad) || !std::isfinite(g.arc_rad) || g.arc_rad == 0.0 ||
        !std::isfinite(g.det_offset_mm) || !(g.det_pitch_mm >= 0))
        return fail(DECT_EINVAL, "non-finite angle, zero arc, or negative pitch");
    const double R = 0.5 * g.pixel_mm * std::hypot((double)g.n_x, (double)g.n_y);
    if (!(R < g.sid_mm) || !(R < g.sdd_mm - g.sid_mm))
        return fail(DECT_EINVAL,
                    "image half-diagonal %.3f mm must lie strictly between source (%.3f) and "
                    "detector (%.3f)",
                    R, g.sid_mm, g.sdd_mm - g.sid_mm);
    out->nx = g.n_x;
    out->ny = g.n_y;
    out->nv = g.n_views;
    out->nd = g.n_det;
    out->dx = g.pixel_mm;
    out->angle0 = g.angle0_rad;
    out->arc = g.arc_rad;
    out->pitch = g.det_pitch_mm > 0 ? g.det_pitch_mm : corner_pitch(g);
    out->offset = g.det_offset_mm;
    out->sid = g.sid_mm;
    out->sdd = g.sdd_mm;
    return DECT_OK;
}

// ---------------------------------------------------------------------------
// physics (Section II-B), FP64
// ---------------------------------------------------------------------------
static const double kR0 = 2.818e-13;          // cm
static const double kMe = 510.975;            // keV
static const double kNeWater = 6.02214076e23 * 10.0 / 18.01528;   // electrons / cm^3
static const double kMPrinted = 3.8;

static double kn(double E) {
    const double g = E / kMe;
    const double l = std::log1p(2.0 * g);
    const double c0 = 2.0 * M_PI * kR0 * kR0;
    return c0 * ((1.0 + g) / (g * g) * (2.0 * (1.0 + g) / (1.0 + 2.0 * g) - l / g) + l / (2.0 * g) -
                 (1.0 + 3.0 * g) / ((1.0 + 2.0 * g) * (1.0 + 2.0 * g)));
}

static double sigma(const dect_params& p, double Z, double E) {
    return p.Cp * std::pow(p.Z_w, kMPrinted - p.m) * std::pow(Z, p.m) / std::pow(E, p.n) + kn(E);
}

static double mu_of(const dect_params& p, double Z, double rho, double E) {
    return 0.1 * kNeWater * rho * sigma(p, Z, E);
}

static int check_params(const dect_params* p) {
    if (!p) return fail(DECT_EINVAL, "params is NULL");
    const double e[4] = {p->E_lo_keV, p->E_hi_keV, p->E1_keV, p->E2_keV};
    for (double v : e)
        if (!(v > 0) || !std::isfinite(v)) return fail(DECT_EINVAL, "energies must be > 0");
    if (!(p->m > 0) || !(p->n > 0) || !(p->Cp > 0) || !(p->Z_w > 0))
        return fail(DECT_EINVAL, "m, n, Cp, Z_w must be > 0");
    for (int i = 0; i < 2; ++i)
        if (!(p->basis_Z[i] > 0) || !(p->basis_rho[i] > 0))
            return fail(DECT_EINVAL, "basis materials need Z > 0 and rho_e > 0");
    if (!(p->lambda >= 0) || !(p->beta0 >= 0) || !(p->beta_max > 0) || !(p->kappa >= 0) ||
        !(p->eta >= 0) || !(p->xi >= 0))
        return fail(DECT_EINVAL, "lambda, beta0, kappa, eta, xi must be >= 0 and beta_max > 0");
    if (p->n_iter < 1) return fail(DECT_EINVAL, "n_iter must be >= 1");
    if (p->f_inner != 1)
        return fail(DECT_EUNSUPPORTED, "f_inner = %d: the library runs one f-step per iteration",
                    p->f_inner);
    if (!(p->t_tol > 0) || p->t_maxit < 1) return fail(DECT_EINVAL, "t_tol > 0 and t_maxit >= 1");
    if (!(p->t_min > 0)) return fail(DECT_EINVAL, "t_min must be > 0");
    if (p->t_precond < DECT_PRECOND_AUTO || p->t_precond > DECT_PRECOND_MULTIGRID)
        return fail(DECT_EINVAL, "t_precond = %d: must be one of the DECT_PRECOND_* values",
                    p->t_precond);
    if (p->storage < DECT_STORAGE_FP32 || p->storage > DECT_STORAGE_BF16_STATE)
        return fail(DECT_EINVAL, "storage = %d: must be one of the DECT_STORAGE_* values", p->storage);
    return DECT_OK;
}

int build_model(const dect_params& p, Model* M) {
    const double El[2] = {p.E_lo_keV, p.E_hi_keV};
    const double Es[2] = {p.E1_keV, p.E2_keV};
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 2; ++i) M->C[k][i] = mu_of(p, p.basis_Z[i], p.basis_rho[i], El[k]);
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) M->Ms[j][i] = p.basis_rho[i] * sigma(p, p.basis_Z[i], Es[j]) * 1e24;
    for (int j = 0; j < 2; ++j) M->psi[j] = kn(Es[j]) * 1e24;
    M->cpb = p.Cp * std::pow(p.Z_w, kMPrinted - p.m) * 1e24;
    M->Zw = p.Z_w;
    M->m = p.m;
    M->e1n = std::pow(p.E1_keV, p.n);
    M->e2n = std::pow(p.E2_keV, p.n);
    const double zwm = std::pow(p.Z_w, p.m);
    M->a[0] = M->cpb * zwm / M->e1n;
    M->a[1] = M->cpb * zwm / M->e2n;
    M->crho = M->psi[0] * M->e1n - M->psi[1] * M->e2n;
    M->Ww = M->cpb * zwm * (M->psi[0] / M->e2n - M->psi[1] / M->e1n);
    const double det = M->C[0][0] * M->C[1][1] - M->C[1][0] * M->C[0][1];
    if (!(std::fabs(det) > 0) || !(std::fabs(M->crho) > 0) || !(std::fabs(M->Ww) > 0))
        return fail(DECT_EINVAL, "degenerate basis or energies (singular decomposition)");
    return DECT_OK;
}

// resolved copy of the parameters (defaults filled in)
struct Resolved {
    dect_params p;
    double eta, xi, beta0, kappa;
};

// projection-data weight eta for geometry g (the explicit value if given)
static double eta_of(const dect_params* in, const Geom& g) {
    if (in->eta > 0) return in->eta;
    const double mwl = mu_of(*in, in->Z_w, 1.0, in->E_lo_keV);
    const double mwh = mu_of(*in, in->Z_w, 1.0, in->E_hi_keV);
    return g.pitch * g.sid / (g.nv * g.dx * g.dx * g.dx * g.sdd * (mwl * mwl + mwh * mwh));
}

// image-domain data weight: unit water curvature in f2, 1 / (mu_w(E_lo)^2 + mu_w(E_hi)^2)
static double eta_image(const dect_params* in) {
    if (in->eta > 0) return in->eta;
    const double mwl = mu_of(*in, in->Z_w, 1.0, in->E_lo_keV);
    const double mwh = mu_of(*in, in->Z_w, 1.0, in->E_hi_keV);
    return 1.0 / (mwl * mwl + mwh * mwh);
}

// g == nullptr: the image-domain form (no projector)
static int resolve_params(const dect_params* in, const Geom* g, const Model& M, Resolved* r) {
    r->p = *in;
    r->beta0 = in->beta0 > 0 ? in->beta0 : 2.0 * in->lambda;
    if (!(r->beta0 > 0)) return fail(DECT_EINVAL, "beta0 = 0 needs lambda > 0");
    r->kappa = in->kappa > 0 ? in->kappa : std::pow(in->beta_max / r->beta0, 1.0 / in->n_iter);
    r->eta = g ? eta_of(in, *g) : eta_image(in);
    if (in->xi > 0) {
        r->xi = in->xi;
    } else {
        const double s1 = sigma(*in, in->Z_w, in->E1_keV) * 1e24;
        const double s2 = sigma(*in, in->Z_w, in->E2_keV) * 1e24;
        r->xi = 1.0 / (s1 * s1 + s2 * s2);
    }
    (void)M;
    return DECT_OK;
}

// ---------------------------------------------------------------------------
// per-geometry ray tables for the stand-alone operators
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct TableEntry {
    Geom g;
    int device;
    void* mem;
    RayTable t;   // one shared descriptor; pair z's sinograms at z * nv * nd
};
static std::mutex g_tab_mu;
static std::vector<TableEntry> g_tabs;

static bool same_geom(const Geom& a, const Geom& b) {
    return a.nx == b.nx && a.ny == b.ny && a.nv == b.nv && a.nd == b.nd && a.dx == b.dx &&
           a.angle0 == b.angle0 && a.arc == b.arc && a.pitch == b.pitch && a.offset == b.offset &&
           a.sid == b.sid && a.sdd == b.sdd;
}

// the layout ray_table_bytes(g) sizes: table_views(g) views (a quarter of
// them for quarter-turn symmetric geometries)
static void carve_table(const Geom& g, void* mem, RayTable* t) {
    char* p = static_cast<char*>(mem);
    const size_t nr = (size_t)table_views(g) * g.nd;
    t->fix = reinterpret_cast<int4*>(p);
    p += nr * sizeof(int4);
    t->flt = reinterpret_cast<float2*>(p);
    p += nr * sizeof(float2);
    t->span = reinterpret_cast<int2*>(p);
    p += nr * sizeof(int2);
    t->view = reinterpret_cast<float4*>(p);
}

static int get_table(const Geom& g, hipStream_t st, RayTable* out) {
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tab_mu);
    for (auto& e : g_tabs)
        if (e.device == dev && same_geom(e.g, g)) {
            *out = e.t;
            return DECT_OK;
        }
    if (g_tabs.size() >= 16) {
        DECT_HIP(hipDeviceSynchronize());
        DECT_HIP(hipFree(g_tabs.front().mem));
        g_tabs.erase(g_tabs.begin());
    }
    TableEntry e;
    e.g = g;
    e.device = dev;
    const size_t tb = align256(ray_table_bytes(g));
    if (hipMalloc(&e.mem, tb + sizeof(SliceDesc)) != hipSuccess)
        return fail(DECT_ENOMEM, "could not allocate the ray table (%zu bytes)", ray_table_bytes(g));
    carve_table(g, e.mem, &e.t);
    SliceDesc* dd = reinterpret_cast<SliceDesc*>(static_cast<char*>(e.mem) + tb);
    const SliceDesc hd = make_slice_desc(g, 0, 0, 0, 1.0);
    e.t.desc = dd;
    e.t.desc_stride = 0;
    e.t.sino_zstride = (long long)g.nv * g.nd;
    e.t.nv_max = g.nv;
    e.t.nd_max = g.nd;
    launch_build_ray_table(g, e.t, st);
    DECT_HIP(hipMemcpyAsync(dd, &hd, sizeof(SliceDesc), hipMemcpyHostToDevice, st));
    DECT_HIP(hipGetLastError());
    DECT_HIP(hipStreamSynchronize(st));   // the table may be used from other streams
    g_tabs.push_back(e);
    *out = e.t;
    return DECT_OK;
}

// Device allocation on a stream: stream-ordered when the runtime supports it
// for this stream, otherwise a plain hipMalloc (freed with hipFree, which
// waits for the device).
struct DevAlloc {
    void* p = nullptr;
    hipStream_t st = nullptr;
    bool async = false;
};
static int dev_alloc(DevAlloc* a, size_t bytes, hipStream_t st) {
    a->st = st;
    a->async = false;
    a->p = nullptr;
    hipError_t e = hipMallocAsync(&a->p, bytes, st);
    if (e == hipSuccess) {
        a->async = true;
        return DECT_OK;
    }
    (void)hipGetLastError();
    a->p = nullptr;
    e = hipMalloc(&a->p, bytes);
    if (e != hipSuccess) {
        a->p = nullptr;
        (void)hipGetLastError();
        return fail(DECT_ENOMEM, "could not allocate %zu bytes on the device: %s", bytes,
                    hipGetErrorString(e));
    }
    return DECT_OK;
}
static void dev_free(DevAlloc* a) {
    if (!a->p) return;
    if (a->async)
        (void)hipFreeAsync(a->p, a->st);
    else
        (void)hipFree(a->p);
    a->p = nullptr;
}

// scope-bound temporary buffer
struct TempBuf {
    DevAlloc a;
    void* p = nullptr;
    ~TempBuf() { dev_free(&a); }
};
static int temp_alloc(TempBuf* b, size_t bytes, hipStream_t st) {
    const int rc = dev_alloc(&b->a, bytes, st);
    b->p = b->a.p;
    return rc;
}


// ---------------------------------------------------------------------------
// workspace of the L0 step and the solver
// ---------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t n) {
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += align256(n * sizeof(T));
        return p;
    }
};

struct PcgBufs {
    float *r, *z, *p0, *p1, *q, *w2;
    float *r2, *p1b;    // pipelined PCG: second r and s buffers
    double* parts;
    PcgState* st;
    PcgParts L;
    MgPlan mg_plan;     // multigrid levels (mg_plan.ok: the sizes admit them)
    float* mg;          // level buffers, [batch][mg_plan.zstride]
};

static void carve_pcg(Carver& c, int ny, int nx, int batch, PcgBufs* b) {
    const size_t n = (size_t)ny * nx * batch;
    b->L = pcg_parts(ny, nx);
    b->r = c.take<float>(n);
    b->z = c.take<float>(n);
    b->p0 = c.take<float>(n);
    b->p1 = c.take<float>(n);
    b->q = c.take<float>(n);
    b->w2 = c.take<float>(n);
    b->r2 = c.take<float>(n);
    b->p1b = c.take<float>(n);
    b->parts = c.take<double>((size_t)batch * b->L.zstride);
    b->st = c.take<PcgState>((size_t)batch);
    b->mg_plan = mg_plan(ny, nx);
    b->mg = b->mg_plan.ok ? c.take<float>((size_t)batch * b->mg_plan.zstride) : nullptr;
}

static void fill_pcg_args(PcgArgs* a, const PcgBufs& b, int ny, int nx, int batch, float* x) {
    a->ny = ny;
    a->nx = nx;
    a->batch = batch;
    a->x = x;
    a->r = b.r;
    a->z = b.z;
    a->p0 = b.p0;
    a->p1 = b.p1;
    a->q = b.q;
    a->w2 = b.w2;
    a->r2 = b.r2;
    a->p1b = b.p1b;
    a->parts = b.parts;
    a->L = b.L;
    a->st = b.st;
}

static const double kJacobiBelow = 1.5;   // beta below which Jacobi PCG beats scaled-FFT PCG

// Preconditioner of the t' PCG.  Automatic: the multigrid V-cycle where the
// image sizes admit it (it needs 7-10 iterations at every beta of the
// schedule), else Jacobi at small beta and the scaled FFT inverse above.
static int choose_prec(int want, const PcgBufs& b, double beta, PcgArgs* a) {
    int prec = want;
    if (prec == DECT_PRECOND_AUTO)
        prec = b.mg_plan.ok ? PREC_MG : (beta < kJacobiBelow ? PREC_JACOBI : PREC_FFT);
    if (prec == PREC_MG && !b.mg_plan.ok)
        return fail(DECT_EUNSUPPORTED,
                    "multigrid preconditioner: n_x=%d n_y=%d unsupported (sides above 64 must be "
                    "multiples of 16 down to 64, and the coarsest grid at most 64 pixels)",
                    a->nx, a->ny);
    a->prec = prec;
    a->nrz_used = prec == PREC_JACOBI ? a->L.nblk : (prec == PREC_FFT ? a->ny : b.mg_plan.nrz);
    return DECT_OK;
}

static void apply_prec(const PcgArgs& a, int it, const PcgBufs& b, float2* fft_scratch,
                       hipStream_t st) {
    if (a.prec == PREC_FFT) launch_pcg_fft_prec(a, it, fft_scratch, st);
    if (a.prec == PREC_MG) launch_pcg_mg_prec(a, it, b.mg_plan, b.mg, st);
}

// A PCG solve in two halves: pcg_enqueue puts the set-up and a first chunk of
// iterations on the stream and returns at once; pcg_finish waits for the
// host-visible stopping flags and enqueues further chunks until every slice
// stopped (or max_iter).  The host checks once per chunk.  The first chunk is
// as long as the previous solve of the same solver took (successive t' steps
// need about the same count, and an iteration enqueued past the stop still
// costs its launches), further chunks kPcgMoreChunk iterations, doubling up
// to kPcgMaxChunk.
constexpr int kPcgMoreChunk = 2;
constexpr int kPcgMaxChunk = 64;

struct PcgRun {
    PcgArgs a;
    int it = 0, max_iter = 0;
    bool piped = false;        // pipelined form (multigrid with the fused last kernel)
    bool early = false;        // piped, and each iteration tests its own new residual
    PcgState* hs = nullptr;    // host copy of the flags (pinned when the caller has it)
    std::vector<PcgState> own;
};

static void pcg_chunk(PcgRun& R, const PcgBufs& b, float2* fft_scratch, hipStream_t st, int chunk) {
    PcgArgs& a = R.a;
    for (int c = 0; c < chunk && R.it < R.max_iter; ++c, ++R.it) {
        if (R.piped) {
            launch_pcg_mg_prec_w_upd(a, R.it, b.mg_plan, b.mg, st);
            continue;
        }
        launch_pcg_matvec(a, R.it, st);
        launch_pcg_update(a, R.it, st);
        apply_prec(a, R.it, b, fft_scratch, st);
    }
    // with the early test the chunk's last V-cycle has already tested the
    // last residual; a slice left running then counts the host's iterations
    if (!R.early) launch_pcg_check(a, R.it, st);
}

// set-up: preconditioner data and the first preconditioner application
static void pcg_setup(PcgRun& R, const PcgBufs& b, float2* fft_scratch, hipStream_t st) {
    PcgArgs& a = R.a;
    if (a.prec == PREC_MG)
        launch_mg_setup(b.mg_plan, a.w2, b.mg, a.batch, a.beta, a.beta_z, &a.st[0].done,
                        sizeof(PcgState) / sizeof(int), st);
    // with the multigrid preconditioner on sizes whose finest V-cycle kernel
    // can also apply A, the pipelined form: one reduction per iteration
    R.piped = a.prec == PREC_MG && mg_pipelined_ok(b.mg_plan);
    R.early = R.piped && mg_early_stop(b.mg_plan);
    if (R.piped)
        launch_pcg_mg_prec_w(a, 0, b.mg_plan, b.mg, st);
    else
        apply_prec(a, -1, b, fft_scratch, st);
    R.it = 0;
}

// the first chunk of iterations and the read-back of the stopping flags
static int pcg_first_chunk(PcgRun& R, const PcgBufs& b, float2* fft_scratch, hipStream_t st,
                           int first_chunk, PcgState* pinned) {
    PcgArgs& a = R.a;
    if (pinned) {
        R.hs = pinned;
    } else {
        R.own.resize(a.batch);
        R.hs = R.own.data();
    }
    pcg_chunk(R, b, fft_scratch, st, std::max(2, first_chunk));
    DECT_HIP(hipGetLastError());
    DECT_HIP(hipMemcpyAsync(R.hs, a.st, sizeof(PcgState) * a.batch, hipMemcpyDeviceToHost, st));
    return DECT_OK;
}

static int pcg_enqueue(PcgRun& R, const PcgBufs& b, float2* fft_scratch, hipStream_t st,
                       int first_chunk, PcgState* pinned) {
    pcg_setup(R, b, fft_scratch, st);
    return pcg_first_chunk(R, b, fft_scratch, st, first_chunk, pinned);
}

static int pcg_finish(PcgRun& R, const PcgBufs& b, float2* fft_scratch, hipStream_t st,
                      int* iters_out, hipEvent_t after_chunk = nullptr) {
    const int batch = R.a.batch;
    int more = kPcgMoreChunk;
    while (true) {
        DECT_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int z = 0; z < batch; ++z) all = all && R.hs[z].done;
        if (all || R.it >= R.max_iter) break;
        pcg_chunk(R, b, fft_scratch, st, more);
        more = std::min(2 * more, kPcgMaxChunk);
        DECT_HIP(hipGetLastError());
        DECT_HIP(hipMemcpyAsync(R.hs, R.a.st, sizeof(PcgState) * batch, hipMemcpyDeviceToHost, st));
        if (after_chunk) DECT_HIP(hipEventRecord(after_chunk, st));
    }
    int mx = 0;
    for (int z = 0; z < batch; ++z) mx = std::max(mx, R.hs[z].done ? R.hs[z].iters : R.it);
    if (iters_out) *iters_out = mx;
    return DECT_OK;
}

static int run_pcg(PcgArgs& a, const PcgBufs& b, int max_iter, int first_chunk,
                   float2* fft_scratch, hipStream_t st, int* iters_out) {
    PcgRun R;
    R.a = a;
    R.max_iter = max_iter;
    if (int rc = pcg_enqueue(R, b, fft_scratch, st, first_chunk, nullptr)) return rc;
    return pcg_finish(R, b, fft_scratch, st, iters_out);
}

int l0_fft_step(const float* g_tilde, float* g, float* h_out, float* v_out, int n_y, int n_x,
                int batch, double lambda, double beta, float2* fft, hipStream_t st) {
    FftArgs a;
    a.src = FFT_SRC_L0;
    a.in = g_tilde;
    a.base = g;
    a.h_out = h_out;
    a.v_out = v_out;
    a.beta = (float)beta;
    a.thr = (float)(lambda / beta);
    a.c = 1.0;
    a.out = g;
    launch_fft_solve(n_y, n_x, batch, a, fft, st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

}  // namespace dect

using namespace dect;

// ===========================================================================
// C-ABI
// ===========================================================================
// Slices of one image grid with their own fan geometries: distinct
// geometries get one ray table each, back to back; slice z's sinograms start
// at sino0[z] in the concatenated inputs and residuals.
struct BatchGeo {
    std::vector<Geom> g;            // per slice
    std::vector<int> uniq;          // slice -> distinct geometry
    std::vector<Geom> distinct;
    std::vector<int> ray0, view0;   // per distinct geometry
    std::vector<long long> sino0;   // per slice
    size_t rays = 0, views = 0;
    long long sino_total = 0;
    int nv_max = 0, nd_max = 0;
    bool rev = false;   // pair blocks carry the reversed layouts (some slice may be quarter-turn symmetric)
    int kinds = kSlicePlain;   // kSlice* bits of the slices (which back-projectors run)
};

// dedupe = false: every slice gets a table of its own (slots that change
// geometry over time)
static int make_batch(const dect_geometry* gin, int batch, BatchGeo* B, bool dedupe = true) {
    if (!gin) return fail(DECT_EINVAL, "geometry is NULL");
    if (batch < 1) return fail(DECT_EINVAL, "batch must be >= 1");
    B->g.resize(batch);
    B->uniq.resize(batch);
    B->sino0.resize(batch);
    for (int z = 0; z < batch; ++z) {
        if (int rc = resolve_geometry(&gin[z], &B->g[z])) return rc;
        const Geom& a = B->g[z];
        const Geom& b = B->g[0];
        if (a.nx != b.nx || a.ny != b.ny || a.dx != b.dx)
            return fail(DECT_EINVAL, "slice %d: image %dx%d at %g mm differs from slice 0 (%dx%d at %g mm)",
                        z, a.nx, a.ny, a.dx, b.nx, b.ny, b.dx);
        if (a.nd > 4096) return fail(DECT_EINVAL, "slice %d: n_det > 4096 is not supported by the FBP start", z);
        int u = -1;
        if (dedupe)
            for (size_t d = 0; d < B->distinct.size(); ++d)
                if (same_geom(B->distinct[d], a)) u = (int)d;
        if (u < 0) {
            u = (int)B->distinct.size();
            B->distinct.push_back(a);
            B->ray0.push_back((int)B->rays);
            B->view0.push_back((int)B->views);
            // slots (no dedupe) reserve the full table: a later geometry may lack the symmetry
            const int tv = dedupe ? table_views(a) : a.nv;
            B->rays += (size_t)tv * a.nd;
            B->views += (size_t)tv;
        }
        B->uniq[z] = u;
        B->sino0[z] = B->sino_total;
        B->sino_total += (long long)a.nv * a.nd;
        B->nv_max = std::max(B->nv_max, a.nv);
        B->nd_max = std::max(B->nd_max, a.nd);
    }
    if (B->rays > (size_t)INT32_MAX) return fail(DECT_EINVAL, "batch ray tables exceed 2^31 rays");
    int kinds = 0;
    for (const Geom& a : B->g) kinds |= slice_kind(a);
    if (!dedupe) {   // slots: any admitted geometry may be symmetric
        B->rev = grid_sym4(B->g[0]);
        B->kinds = B->rev ? (kSlicePlain | kSliceQuarter | kSliceOcto) : kSlicePlain;
    } else {
        B->rev = (kinds & ~kSlicePlain) != 0;
        B->kinds = kinds;
    }
    return DECT_OK;
}

struct dect_solver {
    Geom g;                          // image grid (and slice 0's fan geometry)
    BatchGeo geo;
    std::vector<SliceDesc> hdesc;    // host copy of the device descriptors
    Resolved rp;
    Model M;
    int batch;
    hipStream_t st;
    void* ws;
    bool owns_ws;
    DevAlloc own;
    RayTable tab;
    float2 *f, *B, *dpad, *S, *zq, *fft;   // dpad: search direction in projector pair blocks
    float *rho, *t, *muL, *muH, *fbpq;
    double *part_img, *part_proj, *alpha;
    double *beta_d, *kappa_d;        // per-slice beta and its growth rate (device)
    int* active_d = nullptr;         // per-slice activity (engine slots); null: all active
    int storage = DECT_STORAGE_FP32;
    unsigned* dpad16 = nullptr;      // BF16 storage: the direction's pair blocks, one word per entry
    bool image = false;              // image-domain form: inputs are mu_lo, mu_hi in muL, muH;
                                     // B holds f^(k+1) during an iteration
    PcgBufs pcg;
    // Concurrency within an iteration: the f-step runs on `side` and the
    // rho_e step on `rst` (or on `side`) while the t' PCG runs on pst (all
    // read iterate k only); t' is double-buffered (the PCG writes t_next) and
    // the rho_e step has its own FFT scratch.  side == nullptr: everything on st.
    hipStream_t side = nullptr;
    hipStream_t pst = nullptr;   // the t' PCG's stream while an iterate call runs
    // sinogram form: the rho_e step on a third stream, concurrent with the
    // forward projection (after the gradient has read rho^(k); the f update
    // and the beta step wait for it); nullptr: on `side`
    hipStream_t rst = nullptr;
    hipEvent_t ev_grad = nullptr, ev_rho = nullptr, ev_rjoin = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_entry = nullptr, ev_mdone = nullptr;
    bool in_pipe = false;        // inside a run of pipelined iterations (pst, side forked)
    // software pipelining of consecutive iterations (see one_iteration)
    hipEvent_t ev_init = nullptr, ev_upd = nullptr, ev_tdone = nullptr;
    bool bp_pending = false;    // this iteration's back-projection is already on `side`
    bool upd_pending = false;   // the last f update ran on `side`, not yet joined
    PcgState* hs_pinned = nullptr;
    PcgRun prun;
    float* t_next = nullptr;
    float2* fft2 = nullptr;
    int k;
    double beta;
    int last_pcg;
    // the t' PCG's first chunk of each outer iteration as one graph launch
    // (dect_solver_set_graphs): instantiated graphs by chunk length and the
    // solution / start buffers they were captured with
    struct ChunkGraph {
        int chunk;
        const float* x;
        const float* x0;
        hipGraphExec_t exec;
    };
    std::vector<ChunkGraph> chunk_graphs;
    dect_schedule sched{4, 0, 1, 0, 0, 1};   // launch schedule (dect_solver_set_schedule)
    // optional kernel timing: event pairs in launch order
    bool timing = false;
    bool timing_fp = false;  // the forward projections too (not with bit 2)
    bool timeline = false;   // iteration timeline (dect_solver_enable_timing bit 1)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_bp, ev_fp;
    // optional iteration timeline (sinogram form): per outer iteration, events
    // at the kTl* points below, and the iteration's index
    std::vector<std::array<hipEvent_t, 5>> tl;
    std::vector<int> tl_k;
    size_t tl_n = 0;
};

// iteration timeline points: the f-step's stream reaches the gradient (its
// back-projection done, t'^(k) available), the forward projection done, the
// update done; the PCG's stream done with the set-up, done with the solve
enum { kTlGrad = 0, kTlFp = 1, kTlUpd = 2, kTlPcgSetup = 3, kTlPcgDone = 4 };
constexpr size_t kTimelineMax = 4096;   // iterations recorded between two reads

static void drop_chunk_graphs(dect_solver* s);

static hipEvent_t take_event(dect_solver* s) {
    hipEvent_t e = nullptr;
    if (!s->ev_pool.empty()) {
        e = s->ev_pool.back();
        s->ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// record timeline point `which` of the current outer iteration
static void tl_mark(dect_solver* s, int which, hipStream_t st) {
    if (!s->timeline || s->image || s->tl_n >= kTimelineMax) return;
    if (s->tl.size() <= s->tl_n) {
        std::array<hipEvent_t, 5> ev{};
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                for (auto& f : ev)
                    if (f) (void)hipEventDestroy(f);
                return;
            }
        s->tl.push_back(ev);
        s->tl_k.push_back(-1);
    }
    (void)hipEventRecord(s->tl[s->tl_n][which], st);
    s->tl_k[s->tl_n] = s->k;
}

// record a start event (returns nullptr when timing is off)
static hipEvent_t mark(dect_solver* s, hipStream_t st) {
    if (!s->timing) return nullptr;
    hipEvent_t e = take_event(s);
    if (e) (void)hipEventRecord(e, st);
    return e;
}
static void mark_end(dect_solver* s, hipStream_t st, hipEvent_t start,
                     std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
    if (!start) return;
    hipEvent_t e = take_event(s);
    if (!e) {
        s->ev_pool.push_back(start);
        return;
    }
    (void)hipEventRecord(e, st);
    v.emplace_back(start, e);
}

// second stream and fork/join events (default priority); without them the
// iteration runs on the solver's stream alone
static void make_side(dect_solver* s) {
    if (hipHostMalloc(reinterpret_cast<void**>(&s->hs_pinned), sizeof(PcgState) * s->batch) !=
        hipSuccess) {
        s->hs_pinned = nullptr;
        (void)hipGetLastError();
    }
    if (hipStreamCreateWithFlags(&s->pst, hipStreamNonBlocking) != hipSuccess) {
        s->pst = nullptr;
        (void)hipGetLastError();
        return;
    }
    if (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess) {
        s->side = nullptr;
        (void)hipGetLastError();
        (void)hipStreamDestroy(s->pst);
        s->pst = nullptr;
        return;
    }
    hipEvent_t* evs[7] = {&s->ev_fork,  &s->ev_join,  &s->ev_init, &s->ev_upd,
                          &s->ev_tdone, &s->ev_entry, &s->ev_mdone};
    bool ok = true;
    for (hipEvent_t* e : evs) ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        for (hipEvent_t* e : evs)
            if (*e) (void)hipEventDestroy(*e);
        for (hipEvent_t* e : evs) *e = nullptr;
        (void)hipStreamDestroy(s->side);
        (void)hipStreamDestroy(s->pst);
        s->side = s->pst = nullptr;
        return;
    }
    // optional third stream for the rho_e step
    hipEvent_t* revs[3] = {&s->ev_grad, &s->ev_rho, &s->ev_rjoin};
    bool rok = hipStreamCreateWithFlags(&s->rst, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* e : revs)
        rok = rok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (!rok) {
        (void)hipGetLastError();
        for (hipEvent_t* e : revs)
            if (*e) (void)hipEventDestroy(*e);
        for (hipEvent_t* e : revs) *e = nullptr;
        if (s->rst) (void)hipStreamDestroy(s->rst);
        s->rst = nullptr;
    }
}
static void free_side(dect_solver* s) {
    if (s->rst) {
        (void)hipStreamSynchronize(s->rst);
        for (hipEvent_t e : {s->ev_grad, s->ev_rho, s->ev_rjoin}) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(s->rst);
        s->rst = nullptr;
    }
    if (s->side) {
        (void)hipStreamSynchronize(s->side);
        (void)hipStreamSynchronize(s->pst);
        for (hipEvent_t e : {s->ev_fork, s->ev_join, s->ev_init, s->ev_upd, s->ev_tdone, s->ev_entry,
                             s->ev_mdone})
            (void)hipEventDestroy(e);
        (void)hipStreamDestroy(s->side);
        (void)hipStreamDestroy(s->pst);
        s->side = s->pst = nullptr;
    }
    if (s->hs_pinned) (void)hipHostFree(s->hs_pinned);
    s->hs_pinned = nullptr;
}
// entry of an iterate call: the PCG stream, the side stream and the rho_e
// stream start after the caller's stream; returns the PCG stream (the
// caller's without them)
static hipStream_t enter_iter(dect_solver* s) {
    if (!s->side) return s->st;
    if (!s->in_pipe) {
        (void)hipEventRecord(s->ev_entry, s->st);
        (void)hipStreamWaitEvent(s->pst, s->ev_entry, 0);
        (void)hipStreamWaitEvent(s->side, s->ev_entry, 0);
        if (s->rst) (void)hipStreamWaitEvent(s->rst, s->ev_entry, 0);
        s->in_pipe = true;
    }
    return s->pst;
}
// exit: the caller's stream waits for all of them
static void leave_iter(dect_solver* s) {
    if (!s->side || !s->in_pipe) return;
    (void)hipEventRecord(s->ev_mdone, s->pst);
    (void)hipEventRecord(s->ev_join, s->side);
    (void)hipStreamWaitEvent(s->st, s->ev_mdone, 0);
    (void)hipStreamWaitEvent(s->st, s->ev_join, 0);
    if (s->rst) {
        (void)hipEventRecord(s->ev_rjoin, s->rst);
        (void)hipStreamWaitEvent(s->st, s->ev_rjoin, 0);
    }
    s->in_pipe = false;
}

extern "C" {

void dect_default_params(dect_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->E_lo_keV = 60.0;
    p->E_hi_keV = 90.0;
    p->E1_keV = 50.0;
    p->E2_keV = 200.0;
    p->m = 3.94;
    p->n = 3.2;
    p->Cp = 9.8e-24;
    p->Z_w = 7.42;
    p->basis_Z[0] = 14.14;
    p->basis_rho[0] = 1.69;
    p->basis_Z[1] = 7.42;
    p->basis_rho[1] = 1.00;
    p->lambda = 0.01;
    p->beta0 = 0.0;
    p->beta_max = 1e5;
    p->kappa = 0.0;
    p->eta = 0.0;
    p->xi = 0.0;
    p->n_iter = 50;
    p->f_inner = 1;
    p->t_tol = 1e-7;
    p->t_maxit = 200;
    p->rho_min = 0.1;
    p->t_min = 1e-6;
    p->t_precond = DECT_PRECOND_AUTO;
}

int dect_resolve_geometry(dect_geometry* g) {
    Geom r;
    const int rc = resolve_geometry(g, &r);
    if (rc) return rc;
    g->det_pitch_mm = r.pitch;
    return DECT_OK;
}

int dect_attenuation(const dect_params* p, const double* Z, const double* rho_e, int64_t n,
                     double* mu_lo, double* mu_hi) {
    if (int rc = check_params(p)) return rc;
    if (n < 0 || (n > 0 && (!Z || !rho_e || !mu_lo || !mu_hi)))
        return fail(DECT_EINVAL, "dect_attenuation: bad arrays");
    for (int64_t i = 0; i < n; ++i) {
        mu_lo[i] = mu_of(*p, Z[i], rho_e[i], p->E_lo_keV);
        mu_hi[i] = mu_of(*p, Z[i], rho_e[i], p->E_hi_keV);
    }
    return DECT_OK;
}

int dect_project(const dect_geometry* gin, const float* img, float* sino, int32_t batch,
                 hipStream_t st) {
    Geom g;
    if (int rc = resolve_geometry(gin, &g)) return rc;
    if (batch < 0) return fail(DECT_EINVAL, "batch must be >= 0");
    if (batch == 0) return DECT_OK;
    if (!img || !sino) return fail(DECT_EINVAL, "dect_project: NULL array");
    RayTable t;
    if (int rc = get_table(g, st, &t)) return rc;
    const int np = (batch + 1) / 2;
    const PadLayout P = pad_layout(g, sym4(g));
    TempBuf tmp;
    if (int rc = temp_alloc(&tmp, P.pair * np * sizeof(float2), st)) return rc;
    float2* pad = static_cast<float2*>(tmp.p);
    launch_pack_pairs(g, P, img, batch, pad, st);
    ProjArgs a;
    a.out = sino;
    a.nout = batch;
    a.four_ray = sym4(g);
    launch_project(g, P, t, pad, np, PROJ_PLAIN, a, st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_backproject(const dect_geometry* gin, const float* sino, float* img, int32_t batch,
                     hipStream_t st) {
    Geom g;
    if (int rc = resolve_geometry(gin, &g)) return rc;
    if (batch < 0) return fail(DECT_EINVAL, "batch must be >= 0");
    if (batch == 0) return DECT_OK;
    if (!img || !sino) return fail(DECT_EINVAL, "dect_backproject: NULL array");
    RayTable t;
    if (int rc = get_table(g, st, &t)) return rc;
    const int np = (batch + 1) / 2;
    TempBuf tmp;
    const size_t nray = (size_t)g.nv * g.nd;
    if (int rc = temp_alloc(&tmp, nray * np * sizeof(float2), st)) return rc;
    float2* sp = static_cast<float2*>(tmp.p);
    launch_pair_sinos(g, sino, batch, sp, st);
    launch_backproject(g, t, sp, np, nullptr, img, batch, st, false, slice_kind(g));
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_fbp(const dect_geometry* gin, const float* sino, float* img, int32_t batch,
             hipStream_t st) {
    Geom g;
    if (int rc = resolve_geometry(gin, &g)) return rc;
    if (batch < 0) return fail(DECT_EINVAL, "batch must be >= 0");
    if (batch == 0) return DECT_OK;
    if (!img || !sino) return fail(DECT_EINVAL, "dect_fbp: NULL array");
    if (g.nd > 4096) return fail(DECT_EINVAL, "dect_fbp: n_det > 4096");
    TempBuf tmp;
    if (int rc = temp_alloc(&tmp, (size_t)g.nv * g.nd * batch * sizeof(float), st)) return rc;
    launch_fbp(g, sino, batch, static_cast<float*>(tmp.p), img, st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

size_t dect_l0_step_workspace_bytes(int32_t n_y, int32_t n_x, int32_t batch, int weighted) {
    if (n_y < 1 || n_x < 1 || batch < 1) return 0;
    Carver c{nullptr};
    c.take<float2>(fft_scratch_bytes(n_y, n_x, batch) / sizeof(float2));
    if (weighted) {
        PcgBufs b;
        carve_pcg(c, n_y, n_x, batch, &b);
    }
    return c.off;
}

int dect_l0_step(const float* g_tilde, const float* weight, float* g, float* h_out, float* v_out,
                 int32_t n_y, int32_t n_x, int32_t batch, double lambda, double beta, double tol,
                 int32_t max_iter, void* ws, size_t ws_bytes, hipStream_t st) {
    if (batch < 0) return fail(DECT_EINVAL, "batch must be >= 0");
    if (batch == 0) return DECT_OK;
    if (!g_tilde || !g) return fail(DECT_EINVAL, "dect_l0_step: NULL g_tilde or g");
    if (!fft_size_ok(n_x) || !fft_size_ok(n_y))
        return fail(DECT_EINVAL, "dect_l0_step: n_x=%d n_y=%d must be 2^a*3^b (b<=1) in [8, 1024]",
                    n_x, n_y);
    if (!(lambda >= 0) || !(beta > 0)) return fail(DECT_EINVAL, "need lambda >= 0 and beta > 0");
    if (weight && (!(tol > 0) || max_iter < 1)) return fail(DECT_EINVAL, "need tol > 0, max_iter >= 1");
    const size_t need = dect_l0_step_workspace_bytes(n_y, n_x, batch, weight != nullptr);
    TempBuf tmp;
    if (!ws) {
        if (int rc = temp_alloc(&tmp, need, st)) return rc;
        ws = tmp.p;
    } else if (ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) {
        return fail(DECT_EWORKSPACE, "dect_l0_step: workspace needs %zu bytes, 256-aligned", need);
    }
    Carver c{static_cast<char*>(ws)};
    float2* fft = c.take<float2>(fft_scratch_bytes(n_y, n_x, batch) / sizeof(float2));
    const float thr = (float)(lambda / beta);
    if (!weight) return l0_fft_step(g_tilde, g, h_out, v_out, n_y, n_x, batch, lambda, beta, fft, st);
    PcgBufs b;
    carve_pcg(c, n_y, n_x, batch, &b);
    PcgArgs a;
    fill_pcg_args(&a, b, n_y, n_x, batch, g);
    a.beta = (float)beta;
    a.thr = thr;
    a.tol2 = tol * tol;
    if (int rc = choose_prec(DECT_PRECOND_AUTO, b, beta, &a)) return rc;
    launch_pcg_init_plain(a, weight, g_tilde, h_out, v_out, st);
    int iters = 0;
    return run_pcg(a, b, max_iter, 8, fft, st, &iters);
}

// ---- solver ---------------------------------------------------------------
static size_t solver_layout(const BatchGeo& B, char* base, dect_solver* s, int storage) {
    const Geom& g = B.g[0];
    const int batch = (int)B.g.size();
    Carver c{base};
    const size_t npix = (size_t)g.nx * g.ny * batch;
    const size_t nsino = (size_t)B.sino_total;
    RayTable t;
    t.fix = c.take<int4>(B.rays);
    t.flt = c.take<float2>(B.rays);
    t.span = c.take<int2>(B.rays);
    t.view = c.take<float4>(B.views);
    SliceDesc* desc = c.take<SliceDesc>((size_t)batch);
    float2* f = c.take<float2>(npix);
    float2* Bimg = c.take<float2>(npix);
    float2* dpad = c.take<float2>(pad_elems(g, B.rev) * batch);
    float2* S = c.take<float2>(nsino);
    float2* zq = c.take<float2>(nsino);   // also the FBP filter scratch at init
    float2* fft = c.take<float2>(npix);
    float* rho = c.take<float>(npix);
    float* tt = c.take<float>(npix);
    float* tnext = c.take<float>(npix);
    float2* fft2 = c.take<float2>(npix);
    double* part_img = c.take<double>((size_t)batch * grad_nblocks(g.ny, g.nx) * 3);
    double* part_proj = c.take<double>((size_t)batch * proj_nblocks(B.nv_max, B.nd_max));
    double* alpha = c.take<double>((size_t)batch);
    double* beta_d = c.take<double>((size_t)batch);
    double* kappa_d = c.take<double>((size_t)batch);
    unsigned* dpad16 =
        storage != DECT_STORAGE_FP32 ? c.take<unsigned>(pad_elems(g, B.rev) * batch) : nullptr;
    PcgBufs pb;
    carve_pcg(c, g.ny, g.nx, batch, &pb);
    if (s) {
        s->dpad16 = dpad16;
        s->beta_d = beta_d;
        s->kappa_d = kappa_d;
        t.desc = desc;
        t.desc_stride = 1;
        t.sino_zstride = 0;
        t.nv_max = B.nv_max;
        t.nd_max = B.nd_max;
        s->tab = t;
        s->f = f;
        s->B = Bimg;
        s->dpad = dpad;
        s->S = S;
        s->zq = zq;
        s->fft = fft;
        s->rho = rho;
        s->t = tt;
        s->t_next = tnext;
        s->fft2 = fft2;
        s->muL = pb.r;   // init-time aliases
        s->muH = pb.z;
        s->fbpq = reinterpret_cast<float*>(zq);
        s->part_img = part_img;
        s->part_proj = part_proj;
        s->alpha = alpha;
        s->pcg = pb;
    }
    return c.off;
}

size_t dect_solve_workspace_bytes_multi(const dect_geometry* geoms, const dect_params* p,
                                        int32_t batch) {
    BatchGeo B;
    if (!p || make_batch(geoms, batch, &B)) return 0;
    return solver_layout(B, nullptr, nullptr, p->storage);
}

size_t dect_solve_workspace_bytes(const dect_geometry* gin, const dect_params* p, int32_t batch) {
    if (!gin || batch < 1) return 0;
    std::vector<dect_geometry> gs((size_t)batch, *gin);
    return dect_solve_workspace_bytes_multi(gs.data(), p, batch);
}

static int solver_create(const dect_geometry* geoms, const dect_params* p, int32_t batch,
                         void* ws, size_t ws_bytes, hipStream_t st, dect_solver** out,
                         bool dedupe) {
    if (!out) return fail(DECT_EINVAL, "out is NULL");
    *out = nullptr;
    BatchGeo B;
    if (int rc = make_batch(geoms, batch, &B, dedupe)) return rc;
    const Geom& g = B.g[0];
    if (int rc = check_params(p)) return rc;
    if (!fft_size_ok(g.nx) || !fft_size_ok(g.ny))
        return fail(DECT_EINVAL, "image sizes must be 2^a*3^b (b <= 1) in [8, 1024], got %dx%d", g.nx,
                    g.ny);
    if (p->t_precond == DECT_PRECOND_MULTIGRID && !mg_plan(g.ny, g.nx).ok)
        return fail(DECT_EUNSUPPORTED, "multigrid preconditioner: image %dx%d unsupported", g.nx,
                    g.ny);
    dect_solver* s = new dect_solver();
    s->g = g;
    s->geo = B;
    s->batch = batch;
    s->st = st;
    if (int rc = build_model(*p, &s->M)) {
        delete s;
        return rc;
    }
    if (int rc = resolve_params(p, &g, s->M, &s->rp)) {
        delete s;
        return rc;
    }
    s->storage = p->storage;
    const size_t need = solver_layout(B, nullptr, nullptr, s->storage);
    if (ws) {
        if (ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) {
            delete s;
            return fail(DECT_EWORKSPACE, "solver workspace needs %zu bytes, 256-aligned", need);
        }
        s->ws = ws;
        s->owns_ws = false;
    } else {
        if (int rc = dev_alloc(&s->own, need, st)) {
            delete s;
            return rc;
        }
        s->ws = s->own.p;
        s->owns_ws = true;
    }
    solver_layout(B, static_cast<char*>(s->ws), s, s->storage);
    s->hdesc.resize(batch);
    for (int z = 0; z < batch; ++z) {
        const int u = B.uniq[z];
        s->hdesc[z] = make_slice_desc(B.g[z], B.ray0[u], B.view0[u], B.sino0[z], eta_of(p, B.g[z]));
    }
    // zero borders of the padded direction layouts and the PCG scalars once
    hipError_t e = hipSuccess;
    e = e != hipSuccess ? e : hipMemsetAsync(s->dpad, 0, pad_elems(g, B.rev) * batch * sizeof(float2), st);
    if (s->dpad16)
        e = e != hipSuccess ? e
                            : hipMemsetAsync(s->dpad16, 0, pad_elems(g, B.rev) * batch * sizeof(unsigned), st);
    e = e != hipSuccess ? e : hipMemsetAsync(s->pcg.st, 0, sizeof(PcgState) * batch, st);
    e = e != hipSuccess ? e
                        : hipMemcpyAsync(const_cast<SliceDesc*>(s->tab.desc), s->hdesc.data(),
                                         sizeof(SliceDesc) * batch, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        if (s->owns_ws) dev_free(&s->own);
        delete s;
        return fail(DECT_EDEVICE, "setting up the solver workspace failed: %s", hipGetErrorString(e));
    }
    for (size_t d = 0; d < B.distinct.size(); ++d) {
        RayTable t = s->tab;
        t.fix += B.ray0[d];
        t.flt += B.ray0[d];
        t.span += B.ray0[d];
        t.view += B.view0[d];
        launch_build_ray_table(B.distinct[d], t, st);
    }
    s->k = 0;
    s->beta = s->rp.beta0;
    s->last_pcg = 0;
    make_side(s);
    *out = s;
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_solver_create_multi(const dect_geometry* geoms, const dect_params* p, int32_t batch,
                             void* ws, size_t ws_bytes, hipStream_t st, dect_solver** out) {
    return solver_create(geoms, p, batch, ws, ws_bytes, st, out, true);
}

int dect_solver_create(const dect_geometry* gin, const dect_params* p, int32_t batch, void* ws,
                       size_t ws_bytes, hipStream_t st, dect_solver** out) {
    if (!out) return fail(DECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!gin) return fail(DECT_EINVAL, "geometry is NULL");
    if (batch < 1) return fail(DECT_EINVAL, "batch must be >= 1");
    std::vector<dect_geometry> gs((size_t)batch, *gin);
    return dect_solver_create_multi(gs.data(), p, batch, ws, ws_bytes, st, out);
}

int dect_solver_destroy(dect_solver* s) {
    if (!s) return DECT_OK;
    if (!s->ev_bp.empty() || !s->ev_fp.empty()) (void)hipStreamSynchronize(s->st);
    for (auto& p : s->ev_bp) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (auto& p : s->ev_fp) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    drop_chunk_graphs(s);
    free_side(s);   // (synchronises the solver's streams)
    for (auto& ev : s->tl)
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (s->owns_ws) dev_free(&s->own);
    delete s;
    return DECT_OK;
}

static PadLayout solver_pad(const dect_solver* s) { return pad_layout(s->g, s->geo.rev); }

static void project_residual(dect_solver* s, const float* lo, const float* hi) {
    const PadLayout P = solver_pad(s);
    launch_pack_f2(s->g, P, s->f, s->batch, s->dpad, s->st);
    ProjArgs a;
    a.p_lo = lo;
    a.p_hi = hi;
    a.res = s->S;
    a.c00 = (float)s->M.C[0][0];
    a.c01 = (float)s->M.C[0][1];
    a.c10 = (float)s->M.C[1][0];
    a.c11 = (float)s->M.C[1][1];
    a.res_bf16 = s->storage != DECT_STORAGE_FP32;
    a.four_ray = (s->geo.kinds & ~kSlicePlain) != 0;
    a.has_plain = (s->geo.kinds & kSlicePlain) != 0;
    launch_project(s->g, P, s->tab, s->dpad, s->batch, PROJ_RESID, a, s->st);
}

// BF16 state storage: the state images hold BF16 values from here on
static void round_state(dect_solver* s, int z0, int n, hipStream_t st) {
    if (s->storage != DECT_STORAGE_BF16_STATE || n < 1) return;
    const size_t npix = (size_t)s->g.nx * s->g.ny;
    launch_round_state(npix, n, s->f + z0 * npix, s->rho + z0 * npix, s->t + z0 * npix, s->beta_d + z0, st);
}
static void round_state(dect_solver* s, int z0, int n) { round_state(s, z0, n, s->st); }

int dect_solver_init(dect_solver* s, const float* lo, const float* hi) {
    if (!s || !lo || !hi) return fail(DECT_EINVAL, "dect_solver_init: NULL argument");
    if (s->image) return fail(DECT_EINVAL, "dect_solver_init: image-domain solver (use dect_image_solver_init)");
    const Geom& g = s->g;
    const BatchGeo& B = s->geo;
    const size_t npix = (size_t)g.nx * g.ny;
    for (int z = 0; z < s->batch;) {   // one FBP per run of slices with the same geometry
        int e = z + 1;
        while (e < s->batch && B.uniq[e] == B.uniq[z]) ++e;
        launch_fbp_pair(B.g[z], lo + B.sino0[z], hi + B.sino0[z], e - z, s->fbpq, s->muL + z * npix,
                        s->muH + z * npix, s->st);
        z = e;
    }
    launch_init_state(s->M, g.ny, g.nx, s->batch, s->muL, s->muH, (float)s->rp.p.rho_min, s->f,
                      s->rho, s->t, s->st);
    s->k = 0;
    s->beta = s->rp.beta0;
    launch_set_beta(s->beta_d, s->kappa_d, 0, s->batch, s->beta, s->rp.kappa, s->st);
    round_state(s, 0, s->batch);   // (seeded by beta^(0))
    project_residual(s, lo, hi);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_solver_set_state(dect_solver* s, const float* lo, const float* hi, const float* f1,
                          const float* f2, const float* rho, const float* t, int32_t k) {
    if (!s || !lo || !hi || !f1 || !f2 || !rho || !t || k < 0)
        return fail(DECT_EINVAL, "dect_solver_set_state: NULL argument or k < 0");
    if (s->image)
        return fail(DECT_EINVAL, "dect_solver_set_state: image-domain solver (use dect_image_solver_set_state)");
    const size_t npix = (size_t)s->g.nx * s->g.ny * s->batch;
    launch_join_f2(s->g.nx * s->g.ny, s->batch, f1, f2, s->f, s->st);
    DECT_HIP(hipMemcpyAsync(s->rho, rho, npix * sizeof(float), hipMemcpyDeviceToDevice, s->st));
    DECT_HIP(hipMemcpyAsync(s->t, t, npix * sizeof(float), hipMemcpyDeviceToDevice, s->st));
    s->k = k;
    s->beta = s->rp.beta0;
    for (int i = 0; i < k; ++i) s->beta *= s->rp.kappa;
    launch_set_beta(s->beta_d, s->kappa_d, 0, s->batch, s->beta, s->rp.kappa, s->st);
    round_state(s, 0, s->batch);   // (seeded by beta^(k))
    project_residual(s, lo, hi);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// rho_e step, subproblem (13b) by the FFT closed form (reads f^(k), rho^(k);
// writes rho^(k+1) in place)
static void rho_step(dect_solver* s, hipStream_t st, float2* scratch) {
    const Geom& g = s->g;
    const Resolved& R = s->rp;
    FftArgs fa;
    fa.src = FFT_SRC_RHO;
    fa.f = s->f;
    fa.base = s->rho;
    fa.m00 = s->M.Ms[0][0];
    fa.m01 = s->M.Ms[0][1];
    fa.m10 = s->M.Ms[1][0];
    fa.m11 = s->M.Ms[1][1];
    fa.e1n = s->M.e1n;
    fa.e2n = s->M.e2n;
    fa.inv_crho = 1.0 / s->M.crho;
    fa.beta = (float)s->beta;
    fa.thr = (float)(R.p.lambda / s->beta);
    fa.beta_z = s->beta_d;
    fa.lam = R.p.lambda;
    fa.c = 1.0;
    fa.out = s->rho;
    launch_fft_solve(g.ny, g.nx, s->batch, fa, scratch, st);
}

// t' step, subproblem (13c) by PCG (reads f^(k), t'^(k); in place)
// t' step, first half: the initial residual (reads f^(k) and t'^(k); the
// solution goes to t_next) and the first chunk of PCG iterations on st.
// `after_init`, if given, is recorded on st once f^(k) has been read.
static int t_step_start(dect_solver* s, hipStream_t ms, hipEvent_t after_init) {
    const Geom& g = s->g;
    const Resolved& R = s->rp;
    PcgArgs& pc = s->prun.a;
    pc = PcgArgs{};
    fill_pcg_args(&pc, s->pcg, g.ny, g.nx, s->batch, s->t_next);
    pc.x0 = s->t;   // t'^(k) stays readable for the concurrent f-step
    pc.beta = (float)s->beta;
    pc.thr = (float)(R.p.lambda / s->beta);
    pc.tol2 = R.p.t_tol * R.p.t_tol;
    pc.beta_z = s->beta_d;
    pc.lam = R.p.lambda;
    pc.active = s->active_d;
    if (int rc = choose_prec(R.p.t_precond, s->pcg, s->beta, &pc)) return rc;
    launch_pcg_init_model(s->M, pc, s->f, ms);
    if (after_init) DECT_HIP(hipEventRecord(after_init, ms));
    s->prun.max_iter = R.p.t_maxit;
    pcg_setup(s->prun, s->pcg, s->fft, ms);
    return DECT_OK;
}

constexpr size_t kMaxChunkGraphs = 16;

static void drop_chunk_graphs(dect_solver* s) {
    if (s->chunk_graphs.empty()) return;
    (void)hipStreamSynchronize(s->pst ? s->pst : s->st);   // no replay in flight
    for (auto& c : s->chunk_graphs) (void)hipGraphExecDestroy(c.exec);
    s->chunk_graphs.clear();
}

// The first chunk replayed from a graph.  Within one solver the chunk's
// kernels take the same arguments in every outer iteration except the t'
// buffers (solution and start alternate between two) and the chunk length:
// beta reaches every kernel through the per-slice device array, and the
// stopping test runs on the device (kernels of a finished slice return at
// once).  So one graph per (length, buffers), captured from the eager
// launch sequence, replays exactly the launches that sequence makes.
static int pcg_chunk_graph(dect_solver* s, hipStream_t ms) {
    PcgRun& R = s->prun;
    PcgArgs& a = R.a;
    if (s->hs_pinned) {
        R.hs = s->hs_pinned;
    } else {
        R.own.resize(a.batch);
        R.hs = R.own.data();
    }
    const int it0 = R.it;
    const int chunk = std::min(std::max(2, s->last_pcg + s->sched.pcg_chunk_extra), R.max_iter - it0);
    hipGraphExec_t ex = nullptr;
    for (const auto& c : s->chunk_graphs)
        if (c.chunk == chunk && c.x == a.x && c.x0 == a.x0) ex = c.exec;
    if (!ex) {
        if (s->chunk_graphs.size() >= kMaxChunkGraphs) drop_chunk_graphs(s);
        DECT_HIP(hipStreamBeginCapture(ms, hipStreamCaptureModeThreadLocal));
        pcg_chunk(R, s->pcg, s->fft, ms, chunk);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(ms, &gr);
        R.it = it0;   // captured, not run
        if (e != hipSuccess)
            return fail(DECT_EDEVICE, "PCG chunk capture failed: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e2 != hipSuccess)
            return fail(DECT_EDEVICE, "PCG chunk graph instantiation failed: %s", hipGetErrorString(e2));
        s->chunk_graphs.push_back({chunk, a.x, a.x0, ex});
    }
    DECT_HIP(hipGraphLaunch(ex, ms));
    R.it = it0 + chunk;
    DECT_HIP(hipMemcpyAsync(R.hs, a.st, sizeof(PcgState) * a.batch, hipMemcpyDeviceToHost, ms));
    return DECT_OK;
}

// the first chunk of PCG iterations (after t_step_start; the host enqueues the
// other stream's work in between so that it is not queued behind this chunk)
static int t_step_chunk(dect_solver* s, hipStream_t ms) {
    // graphs for the pipelined multigrid PCG (its whole chunk is kernels), on
    // a stream of the solver's own (the legacy null stream cannot capture)
    int rc;
    if (s->sched.graphs && s->prun.piped && ms == s->pst && ms && s->prun.max_iter > s->prun.it)
        rc = pcg_chunk_graph(s, ms);
    else
        rc = pcg_first_chunk(s->prun, s->pcg, s->fft, ms, s->last_pcg + s->sched.pcg_chunk_extra,
                             s->hs_pinned);
    tl_mark(s, kTlPcgDone, ms);
    return rc;
}

// second half: wait for the stopping flags, more chunks while needed
static int t_step_finish(dect_solver* s, hipStream_t ms) {
    int iters = 0;
    const bool tl = s->timeline && !s->image && s->tl_n < s->tl.size();
    if (int rc = pcg_finish(s->prun, s->pcg, s->fft, ms, &iters,
                            tl ? s->tl[s->tl_n][kTlPcgDone] : nullptr))
        return rc;
    s->last_pcg = iters;
    return DECT_OK;
}

// One outer iteration of the image-domain form: (f1, f2) by the joint
// minimiser of (13a) (a 2x2 solve per frequency that meets both printed
// closed forms at once), then the rho_e and t' steps, all reading iterate k;
// f^(k+1) is built in B and swapped in.
static int one_iteration_image(dect_solver* s, bool more) {
    const Geom& g = s->g;
    const Resolved& R = s->rp;
    const Model& M = s->M;
    // t' step on the PCG stream, enqueued first; f-step and rho_e step on the
    // side stream (all read iterate k; the f-step writes f^(k+1) into B)
    const hipStream_t ms = enter_iter(s);
    const bool two = s->side != nullptr;
    const hipStream_t side = two ? s->side : s->st;
    if (two && s->upd_pending) DECT_HIP(hipStreamWaitEvent(ms, s->ev_upd, 0));     // f^(k)
    if (int rc = t_step_start(s, ms, nullptr)) return rc;
    // the t' PCG is this form's critical path: its first chunk is enqueued
    // before the side stream's f-step
    if (two)
        if (int rc = t_step_chunk(s, ms)) return rc;
    if (two && s->upd_pending) DECT_HIP(hipStreamWaitEvent(side, s->ev_tdone, 0));  // t'^(k), beta^(k)
    float2* scratch = two ? s->fft2 : s->fft;
    hipEvent_t t0 = mark(s, side);
    {
        FftArgs fa;
        fa.src = FFT_SRC_IMGF;
        fa.f = s->f;
        fa.out = reinterpret_cast<float*>(s->B);
        fa.mu_lo = s->muL;
        fa.mu_hi = s->muH;
        fa.rho_in = s->rho;
        fa.t_in = s->t;
        fa.cL0 = M.C[0][0];
        fa.cL1 = M.C[0][1];
        fa.cH0 = M.C[1][0];
        fa.cH1 = M.C[1][1];
        fa.m00 = M.Ms[0][0];
        fa.m01 = M.Ms[0][1];
        fa.m10 = M.Ms[1][0];
        fa.m11 = M.Ms[1][1];
        fa.ta0 = M.a[0];
        fa.ta1 = M.a[1];
        fa.tpsi0 = M.psi[0];
        fa.tpsi1 = M.psi[1];
        fa.eta_img = R.eta;
        fa.xi_img = R.xi;
        // H = eta C^T C + xi Ms^T Ms, the constant matrix of the data and
        // coupling terms of (13a)
        double H[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                H[i][j] = R.eta * (M.C[0][i] * M.C[0][j] + M.C[1][i] * M.C[1][j]) +
                          R.xi * (M.Ms[0][i] * M.Ms[0][j] + M.Ms[1][i] * M.Ms[1][j]);
        fa.c = H[0][0];
        fa.c_b = H[1][1];
        fa.c_o = H[0][1];
        fa.c_det = H[0][0] * H[1][1] - H[0][1] * H[1][0];
        fa.beta = (float)s->beta;
        fa.thr = (float)(R.p.lambda / s->beta);
        fa.beta_z = s->beta_d;
        fa.lam = R.p.lambda;
        launch_fft_solve(g.ny, g.nx, s->batch, fa, scratch, side);
    }
    mark_end(s, side, t0, s->ev_bp);
    rho_step(s, side, scratch);
    if (two) DECT_HIP(hipEventRecord(s->ev_upd, side));
    if (!two)
        if (int rc = t_step_chunk(s, ms)) return rc;
    if (int rc = t_step_finish(s, ms)) return rc;
    if (two) DECT_HIP(hipStreamWaitEvent(ms, s->ev_upd, 0));   // side done with beta^(k), t'^(k)
    std::swap(s->f, s->B);
    std::swap(s->t, s->t_next);
    s->beta *= R.kappa;
    s->k += 1;
    launch_set_beta(s->beta_d, s->kappa_d, 0, s->batch, s->beta, R.kappa, ms);
    if (two) DECT_HIP(hipEventRecord(s->ev_tdone, ms));
    s->upd_pending = two;
    if (!more) {
        leave_iter(s);
        s->upd_pending = false;
    }
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// Outer iteration k of the sinogram form.  With the side stream:
//   st:   t' step (initial residual reads f^(k), t'^(k); PCG writes t_next),
//         then beta <- kappa beta once the side work has read beta^(k);
//   side: back-projection of S^(k), gradient, forward projection and line
//         search, rho_e step; then, once the PCG has read f^(k), the update
//         f^(k+1), S^(k+1) and, when another iteration follows (`more`), its
//         back-projection, which needs S^(k+1) only.
// So the host's wait for the PCG stopping flags overlaps the next
// back-projection.  Events order every hand-over between the streams; the
// iteration after one with `more` starts with its back-projection queued.
// The iteration in two halves: iter_enqueue puts all of its work on the
// streams (the PCG's first chunk included) and returns; iter_complete waits
// for the PCG's stopping flags, enqueues further chunks while needed and
// finishes the iteration.  Several solvers can have their halves interleaved
// (enqueue all, then complete each) so that their work overlaps on the device.
static int iter_enqueue(dect_solver* s, bool more) {
    const Geom& g = s->g;
    const Resolved& R = s->rp;
    const double beta = s->beta;
    ImgArgs a;
    a.ny = g.ny;
    a.nx = g.nx;
    a.nv = s->tab.nv_max;
    a.nd = s->tab.nd_max;
    a.batch = s->batch;
    a.eta2 = 2.0f;   // each slice's eta is carried by its residual sinograms
    a.xi2 = (float)(2.0 * R.xi);
    a.beta2 = (float)(2.0 * beta);
    a.thr = (float)(R.p.lambda / beta);
    a.beta = (float)beta;
    a.beta_z = s->beta_d;   // every kernel takes its slice's beta from here
    a.lam = R.p.lambda;
    a.bf16 = s->storage != DECT_STORAGE_FP32;
    void* dir = a.bf16 ? static_cast<void*>(s->dpad16) : static_cast<void*>(s->dpad);
    const PadLayout P = solver_pad(s);
    const hipStream_t ms = enter_iter(s);   // the PCG's stream
    const bool two = s->side != nullptr;
    const hipStream_t side = two ? s->side : s->st;
    // ms: the t' step first (f^(k) from the previous update on `side`)
    if (two && s->upd_pending) DECT_HIP(hipStreamWaitEvent(ms, s->ev_upd, 0));
    if (int rc = t_step_start(s, ms, two ? s->ev_init : nullptr)) return rc;
    tl_mark(s, kTlPcgSetup, ms);
    // With the next back-projection already queued on `side` (pipelined
    // iterations), the PCG's first chunk is enqueued first: the side stream
    // has that much work ahead while the host enqueues the chunk, and the PCG
    // does not wait behind the host's side enqueues
    const bool chunk_first = two && s->bp_pending && s->sched.pcg_chunk_first;
    if (chunk_first)
        if (int rc = t_step_chunk(s, ms)) return rc;
    // side: f-step and rho_e step (t'^(k), beta^(k) from the previous iteration on ms)
    if (two && s->upd_pending) DECT_HIP(hipStreamWaitEvent(side, s->ev_tdone, 0));
    if (!s->bp_pending) {
        hipEvent_t t0 = mark(s, side);
        launch_backproject(g, s->tab, s->S, s->batch, s->B, nullptr, 0, side, a.bf16, s->geo.kinds,
                           s->sched.bp_cu_percent);
        mark_end(s, side, t0, s->ev_bp);
    }
    tl_mark(s, kTlGrad, side);
    launch_grad(s->M, a, P, s->f, s->B, s->rho, s->t, dir, s->part_img, side);
    // rho_e step on its own stream once the gradient has read rho^(k)
    const hipStream_t rs = two && s->rst && s->sched.rho_stream ? s->rst : nullptr;
    if (rs) {
        DECT_HIP(hipEventRecord(s->ev_grad, side));
        DECT_HIP(hipStreamWaitEvent(rs, s->ev_grad, 0));
        rho_step(s, rs, s->fft2);
        // ev_rho also orders after the PCG's read of f^(k), so the update
        // below waits for one event instead of two
        if (two) DECT_HIP(hipStreamWaitEvent(rs, s->ev_init, 0));
        DECT_HIP(hipEventRecord(s->ev_rho, rs));
    }
    ProjArgs pa;
    pa.res = s->zq;
    pa.c00 = (float)s->M.C[0][0];
    pa.c01 = (float)s->M.C[0][1];
    pa.c10 = (float)s->M.C[1][0];
    pa.c11 = (float)s->M.C[1][1];
    pa.partials = s->part_proj;
    pa.img_partials = s->part_img;
    pa.img_nblocks = grad_nblocks(g.ny, g.nx);
    pa.w_data = 2.0;
    pa.w_coup = 2.0 * R.xi;
    pa.w_reg = 2.0 * beta;
    pa.beta_z = s->beta_d;
    pa.alpha = s->alpha;
    pa.pad_bf16 = pa.res_bf16 = a.bf16;
    pa.four_ray = (s->geo.kinds & ~kSlicePlain) != 0 && s->sched.fp_rays_per_lane == 4;
    pa.has_plain = (s->geo.kinds & kSlicePlain) != 0;
    hipEvent_t t1 = s->timing_fp ? mark(s, side) : nullptr;
    launch_project(g, P, s->tab, dir, s->batch, PROJ_LINESEARCH, pa, side);
    mark_end(s, side, t1, s->ev_fp);
    tl_mark(s, kTlFp, side);
    if (!rs) rho_step(s, side, two ? s->fft2 : s->fft);
    if (two) {
        // f^(k) read by the PCG and by the rho_e step (whose event orders
        // after the PCG's); the next gradient reads rho^(k+1)
        DECT_HIP(hipStreamWaitEvent(side, rs ? s->ev_rho : s->ev_init, 0));
    }
    // f^(k+1), residual sinograms (beta is stepped on st below)
    launch_update(a, P, s->tab, s->alpha, dir, s->f, s->S, s->zq, nullptr, nullptr, side);
    tl_mark(s, kTlUpd, side);
    if (two) DECT_HIP(hipEventRecord(s->ev_upd, side));
    s->bp_pending = false;
    if (two && more) {   // next back-projection while the host waits for the PCG
        hipEvent_t t2 = mark(s, side);
        launch_backproject(g, s->tab, s->S, s->batch, s->B, nullptr, 0, side, a.bf16, s->geo.kinds,
                           s->sched.bp_cu_percent);
        mark_end(s, side, t2, s->ev_bp);
        s->bp_pending = true;
    }
    s->upd_pending = two;
    if (!chunk_first)
        if (int rc = t_step_chunk(s, ms)) return rc;
    return DECT_OK;
}

static int iter_complete(dect_solver* s, bool more) {
    const Resolved& R = s->rp;
    const bool two = s->side != nullptr;
    const hipStream_t ms = two ? s->pst : s->st;
    const hipStream_t rs = two && s->rst && s->sched.rho_stream ? s->rst : nullptr;
    if (int rc = t_step_finish(s, ms)) return rc;
    // ms: beta^(k+1) once the side work (up to its update, recorded in
    // ev_upd) and the rho_e step have read beta^(k)
    if (two) DECT_HIP(hipStreamWaitEvent(ms, s->ev_upd, 0));
    if (rs) DECT_HIP(hipStreamWaitEvent(ms, s->ev_rho, 0));
    launch_step_beta(s->beta_d, s->kappa_d, s->batch, ms);
    std::swap(s->t, s->t_next);
    if (s->storage == DECT_STORAGE_BF16_STATE) {
        if (two) DECT_HIP(hipStreamWaitEvent(ms, s->ev_upd, 0));
        round_state(s, 0, s->batch, ms);
    }
    if (two) DECT_HIP(hipEventRecord(s->ev_tdone, ms));
    if (!more) {   // join: the caller's stream waits for both streams
        leave_iter(s);
        s->upd_pending = false;
        s->bp_pending = false;
    }
    s->beta *= R.kappa;
    s->k += 1;
    if (s->timeline && s->tl_n < s->tl.size() && s->tl_k[s->tl_n] == s->k - 1) ++s->tl_n;
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

static int one_iteration(dect_solver* s, bool more = false) {
    if (s->image) return one_iteration_image(s, more);
    if (int rc = iter_enqueue(s, more)) return rc;
    return iter_complete(s, more);
}

int dect_solver_iterate(dect_solver* s, int32_t n) {
    if (!s || n < 0) return fail(DECT_EINVAL, "dect_solver_iterate: bad arguments");
    for (int i = 0; i < n; ++i) {
        if (int rc = one_iteration(s, i + 1 < n)) {
            leave_iter(s);   // the caller's stream still orders after everything enqueued
            s->upd_pending = s->bp_pending = false;
            return rc;
        }
    }
    return DECT_OK;
}

int dect_solver_get_state(const dect_solver* s, float* f1, float* f2, float* rho, float* t) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    const int npix = s->g.nx * s->g.ny;
    if (f1 || f2) launch_split_f2(npix, s->batch, s->f, f1, f2, s->st);
    const size_t bytes = (size_t)npix * s->batch * sizeof(float);
    if (rho) DECT_HIP(hipMemcpyAsync(rho, s->rho, bytes, hipMemcpyDeviceToDevice, s->st));
    if (t) DECT_HIP(hipMemcpyAsync(t, s->t, bytes, hipMemcpyDeviceToDevice, s->st));
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_solver_finish(dect_solver* s, float* Z, float* rho_e) {
    if (!s || (!Z && !rho_e)) return fail(DECT_EINVAL, "dect_solver_finish: bad arguments");
    launch_finish(s->M, s->g.ny, s->g.nx, s->batch, s->rho, s->t, (float)s->rp.p.rho_min,
                  s->rp.p.t_min, Z, rho_e, s->st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_solver_stats(const dect_solver* s, int32_t* k, int32_t* last_pcg_iters) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    DECT_HIP(hipStreamSynchronize(s->st));
    if (k) *k = s->k;
    if (last_pcg_iters) *last_pcg_iters = s->last_pcg;
    return DECT_OK;
}

int dect_solver_set_graphs(dect_solver* s, int enable) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    if (s->in_pipe) return fail(DECT_EINVAL, "dect_solver_set_graphs: iterations in flight");
    if (!enable) drop_chunk_graphs(s);
    s->sched.graphs = enable != 0;
    return DECT_OK;
}

static bool schedule_ok(const dect_schedule& c) {
    return (c.fp_rays_per_lane == 1 || c.fp_rays_per_lane == 4) &&
           (c.bp_cu_percent == 0 || (c.bp_cu_percent >= 10 && c.bp_cu_percent <= 400)) &&
           (c.rho_stream == 0 || c.rho_stream == 1) && (c.graphs == 0 || c.graphs == 1) &&
           c.pcg_chunk_extra >= 0 && c.pcg_chunk_extra <= 8 &&
           (c.pcg_chunk_first == 0 || c.pcg_chunk_first == 1);
}

int dect_solver_get_schedule(const dect_solver* s, dect_schedule* out) {
    if (!s || !out) return fail(DECT_EINVAL, "dect_solver_get_schedule: NULL argument");
    *out = s->sched;
    return DECT_OK;
}

int dect_solver_set_schedule(dect_solver* s, const dect_schedule* in) {
    if (!s || !in) return fail(DECT_EINVAL, "dect_solver_set_schedule: NULL argument");
    if (!schedule_ok(*in)) return fail(DECT_EINVAL, "dect_solver_set_schedule: value out of range");
    if (s->in_pipe) return fail(DECT_EINVAL, "dect_solver_set_schedule: iterations in flight");
    if (!in->graphs) drop_chunk_graphs(s);
    s->sched = *in;
    return DECT_OK;
}

// one autotuner trial: init, then `iters` outer iterations timed on the
// solver's stream
static int tune_trial(dect_solver* s, const float* lo, const float* hi, int iters, hipEvent_t e0,
                      hipEvent_t e1, float* ms) {
    int rc = s->image ? dect_image_solver_init(s, lo, hi) : dect_solver_init(s, lo, hi);
    if (rc) return rc;
    DECT_HIP(hipEventRecord(e0, s->st));
    if ((rc = dect_solver_iterate(s, iters))) return rc;
    DECT_HIP(hipEventRecord(e1, s->st));
    DECT_HIP(hipEventSynchronize(e1));
    DECT_HIP(hipEventElapsedTime(ms, e0, e1));
    return DECT_OK;
}

int dect_solver_autotune(dect_solver* s, const float* lo, const float* hi, int32_t iters,
                         int32_t reps, dect_schedule* chosen, double* ms_per_iter) {
    if (!s || !lo || !hi) return fail(DECT_EINVAL, "dect_solver_autotune: NULL argument");
    if (iters < 1 || iters > 100 || reps < 1 || reps > 20)
        return fail(DECT_EINVAL, "dect_solver_autotune: iters must be in 1..100, reps in 1..20");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DECT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(DECT_EDEVICE, "dect_solver_autotune: hipEventCreate failed");
    }
    const dect_schedule start = s->sched;
    // median time per iteration of schedule c, after one untimed trial
    // (ray tables, graph capture)
    auto measure = [&](const dect_schedule& c, double* out) -> int {
        s->sched = c;
        if (!c.graphs) drop_chunk_graphs(s);
        std::vector<float> t((size_t)reps + 1);
        for (int r = 0; r <= reps; ++r)
            if (int rc = tune_trial(s, lo, hi, iters, e0, e1, &t[(size_t)r])) return rc;
        std::sort(t.begin() + 1, t.end());
        *out = (double)t[1 + (size_t)reps / 2] / iters;
        return DECT_OK;
    };
    // the knobs that matter for this solver
    std::vector<std::pair<int32_t dect_schedule::*, std::vector<int32_t>>> knobs;
    if (!s->image) {
        if (s->geo.kinds & ~kSlicePlain) knobs.push_back({&dect_schedule::fp_rays_per_lane, {4, 1}});
        if (s->geo.kinds & (kSliceQuarter | kSliceOcto))
            knobs.push_back({&dect_schedule::bp_cu_percent, {0, 25, 50, 75, 100}});
        if (s->rst) knobs.push_back({&dect_schedule::rho_stream, {1, 0}});
    }
    knobs.push_back({&dect_schedule::graphs, {0, 1}});
    knobs.push_back({&dect_schedule::pcg_chunk_extra, {0, 1, 2}});
    if (!s->image) knobs.push_back({&dect_schedule::pcg_chunk_first, {1, 0}});
    dect_schedule best = start;
    double tbest = 0.0;
    int rc = measure(best, &tbest);
    for (size_t k = 0; rc == DECT_OK && k < knobs.size(); ++k) {
        const auto field = knobs[k].first;
        const int32_t base = best.*field;
        for (int32_t v : knobs[k].second) {
            if (v == base) continue;
            dect_schedule c = best;
            c.*field = v;
            double t = 0.0;
            if ((rc = measure(c, &t))) break;
            if (t < 0.98 * tbest) {
                best = c;
                tbest = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        s->sched = start;
        drop_chunk_graphs(s);
        return rc;
    }
    s->sched = best;
    if (!best.graphs) drop_chunk_graphs(s);
    if (chosen) *chosen = best;
    if (ms_per_iter) *ms_per_iter = tbest;
    return DECT_OK;
}

int dect_solver_enable_timing(dect_solver* s, int enable) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    s->timing = (enable & 1) != 0;
    s->timing_fp = s->timing && (enable & 4) == 0;
    s->timeline = (enable & 2) != 0;
    return DECT_OK;
}

int dect_solver_timing(dect_solver* s, double* bp_ms, int32_t* bp_n, double* fp_ms, int32_t* fp_n) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    DECT_HIP(hipStreamSynchronize(s->st));
    auto sum = [s](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double* ms, int32_t* n) -> int {
        double tot = 0.0;
        for (auto& p : v) {
            float e = 0.f;
            DECT_HIP(hipEventElapsedTime(&e, p.first, p.second));
            tot += e;
            s->ev_pool.push_back(p.first);
            s->ev_pool.push_back(p.second);
        }
        if (ms) *ms = tot;
        if (n) *n = (int32_t)v.size();
        v.clear();
        return DECT_OK;
    };
    if (int rc = sum(s->ev_bp, bp_ms, bp_n)) return rc;
    return sum(s->ev_fp, fp_ms, fp_n);
}

int dect_solver_timeline(dect_solver* s, float* out_us, int32_t max_rows, int32_t* rows) {
    if (!s) return fail(DECT_EINVAL, "solver is NULL");
    if (!rows || (max_rows > 0 && !out_us)) return fail(DECT_EINVAL, "dect_solver_timeline: NULL output");
    int32_t n = 0;
    for (size_t i = 1; i < s->tl_n; ++i) {
        if (s->tl_k[i] != s->tl_k[i - 1] + 1) continue;   // a new solve started
        if (n >= max_rows) break;
        const hipEvent_t u0 = s->tl[i - 1][kTlUpd];
        DECT_HIP(hipEventSynchronize(u0));
        for (int j = 0; j < 5; ++j) {
            DECT_HIP(hipEventSynchronize(s->tl[i][j]));
            float ms = 0.f;
            DECT_HIP(hipEventElapsedTime(&ms, u0, s->tl[i][j]));
            out_us[(size_t)n * 5 + j] = 1e3f * ms;
        }
        ++n;
    }
    *rows = n;
    s->tl_n = 0;
    return DECT_OK;
}

int dect_solve_multi(const float* lo, const float* hi, const dect_geometry* geoms,
                     const dect_params* p, float* Z, float* rho, int32_t batch, void* ws,
                     size_t ws_bytes, hipStream_t st) {
    if (!lo || !hi || (!Z && !rho)) return fail(DECT_EINVAL, "dect_solve_multi: NULL array");
    dect_solver* s = nullptr;
    if (int rc = dect_solver_create_multi(geoms, p, batch, ws, ws_bytes, st, &s)) return rc;
    int rc = dect_solver_init(s, lo, hi);
    if (!rc) rc = dect_solver_iterate(s, p->n_iter);
    if (!rc) rc = dect_solver_finish(s, Z, rho);
    dect_solver_destroy(s);
    return rc;
}

// ---- uneven batches of mixed image sizes ------------------------------------
// The slices are grouped by image grid (n_x, n_y, pixel_mm); each group is an
// uneven-batch solver whose launches cover all of its slices.  An iteration
// enqueues every group's work before it waits for any group's PCG stopping
// flags, so the groups' kernels overlap on the device.
struct dect_uneven {
    std::vector<dect_solver*> grp;
    std::vector<std::vector<int>> members;    // per group: slice indices, ascending
    std::vector<long long> sino0, img0;       // per slice: offsets in the caller's arrays
    std::vector<long long> gsino;             // per group: its sinogram elements
    std::vector<size_t> gimg;                 // per group: its image elements
    std::vector<Geom> g;                      // per slice
    hipStream_t st = nullptr;
    int batch = 0;
};

static void uneven_free(dect_uneven* u) {
    if (!u) return;
    for (dect_solver* s : u->grp) dect_solver_destroy(s);
    delete u;
}

int dect_uneven_create(const dect_geometry* geoms, int32_t batch, const dect_params* p, hipStream_t st,
                       dect_uneven** out) {
    if (!out) return fail(DECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!geoms || !p || batch < 1) return fail(DECT_EINVAL, "dect_uneven_create: bad arguments");
    dect_uneven* u = new dect_uneven();
    u->st = st;
    u->batch = batch;
    u->g.resize(batch);
    u->sino0.resize(batch);
    u->img0.resize(batch);
    long long so = 0, io = 0;
    for (int z = 0; z < batch; ++z) {
        if (int rc = resolve_geometry(&geoms[z], &u->g[z])) {
            uneven_free(u);
            return rc;
        }
        u->sino0[z] = so;
        u->img0[z] = io;
        so += (long long)u->g[z].nv * u->g[z].nd;
        io += (long long)u->g[z].nx * u->g[z].ny;
    }
    // groups in order of first appearance
    for (int z = 0; z < batch; ++z) {
        int gi = -1;
        for (size_t q = 0; q < u->members.size() && gi < 0; ++q) {
            const Geom& a = u->g[u->members[q][0]];
            if (a.nx == u->g[z].nx && a.ny == u->g[z].ny && a.dx == u->g[z].dx) gi = (int)q;
        }
        if (gi < 0) {
            gi = (int)u->members.size();
            u->members.emplace_back();
        }
        u->members[gi].push_back(z);
    }
    for (const auto& m : u->members) {
        std::vector<dect_geometry> gs;
        long long ns = 0;
        for (int z : m) {
            gs.push_back(geoms[z]);
            ns += (long long)u->g[z].nv * u->g[z].nd;
        }
        dect_solver* s = nullptr;
        if (int rc = dect_solver_create_multi(gs.data(), p, (int32_t)gs.size(), nullptr, 0, st, &s)) {
            uneven_free(u);
            return rc;
        }
        u->grp.push_back(s);
        u->gsino.push_back(ns);
        u->gimg.push_back((size_t)u->g[m[0]].nx * u->g[m[0]].ny * m.size());
    }
    *out = u;
    return DECT_OK;
}

int dect_uneven_destroy(dect_uneven* u) {
    uneven_free(u);
    return DECT_OK;
}

int dect_uneven_groups(const dect_uneven* u, int32_t* n_groups) {
    if (!u || !n_groups) return fail(DECT_EINVAL, "dect_uneven_groups: bad arguments");
    *n_groups = (int32_t)u->grp.size();
    return DECT_OK;
}

// a group's sinograms back to back (the order dect_solver_init reads)
static int gather_group(dect_uneven* u, size_t q, const float* lo, const float* hi, TempBuf* buf) {
    if (int rc = temp_alloc(buf, 2 * sizeof(float) * (size_t)u->gsino[q], u->st)) return rc;
    float* dlo = static_cast<float*>(buf->p);
    float* dhi = dlo + u->gsino[q];
    long long o = 0;
    for (int z : u->members[q]) {
        const size_t n = (size_t)u->g[z].nv * u->g[z].nd;
        DECT_HIP(hipMemcpyAsync(dlo + o, lo + u->sino0[z], n * sizeof(float), hipMemcpyDeviceToDevice, u->st));
        DECT_HIP(hipMemcpyAsync(dhi + o, hi + u->sino0[z], n * sizeof(float), hipMemcpyDeviceToDevice, u->st));
        o += (long long)n;
    }
    return DECT_OK;
}

int dect_uneven_init(dect_uneven* u, const float* lo, const float* hi) {
    if (!u || !lo || !hi) return fail(DECT_EINVAL, "dect_uneven_init: NULL argument");
    for (size_t q = 0; q < u->grp.size(); ++q) {
        TempBuf buf;   // stream-ordered: freed after the init's enqueued reads
        if (int rc = gather_group(u, q, lo, hi, &buf)) return rc;
        const float* dlo = static_cast<const float*>(buf.p);
        if (int rc = dect_solver_init(u->grp[q], dlo, dlo + u->gsino[q])) return rc;
    }
    return DECT_OK;
}

int dect_uneven_iterate(dect_uneven* u, int32_t n) {
    if (!u || n < 0) return fail(DECT_EINVAL, "dect_uneven_iterate: bad arguments");
    for (int i = 0; i < n; ++i) {
        const bool more = i + 1 < n;
        int rc = DECT_OK;
        for (dect_solver* s : u->grp)
            if (!rc) rc = iter_enqueue(s, more);
        for (dect_solver* s : u->grp)
            if (!rc) rc = iter_complete(s, more);
        if (rc) {
            for (dect_solver* s : u->grp) {
                leave_iter(s);
                s->upd_pending = s->bp_pending = false;
            }
            return rc;
        }
    }
    return DECT_OK;
}

int dect_uneven_finish(dect_uneven* u, float* Z, float* rho_e) {
    if (!u || (!Z && !rho_e)) return fail(DECT_EINVAL, "dect_uneven_finish: bad arguments");
    for (size_t q = 0; q < u->grp.size(); ++q) {
        TempBuf buf;
        if (int rc = temp_alloc(&buf, 2 * sizeof(float) * u->gimg[q], u->st)) return rc;
        float* gz = static_cast<float*>(buf.p);
        float* gr = gz + u->gimg[q];
        if (int rc = dect_solver_finish(u->grp[q], gz, gr)) return rc;
        size_t o = 0;
        for (int z : u->members[q]) {
            const size_t n = (size_t)u->g[z].nx * u->g[z].ny;
            if (Z) DECT_HIP(hipMemcpyAsync(Z + u->img0[z], gz + o, n * sizeof(float), hipMemcpyDeviceToDevice, u->st));
            if (rho_e)
                DECT_HIP(hipMemcpyAsync(rho_e + u->img0[z], gr + o, n * sizeof(float), hipMemcpyDeviceToDevice, u->st));
            o += n;
        }
    }
    return DECT_OK;
}

// one trial of the whole handle: init, then `iters` interleaved outer
// iterations of every group, timed on the handle's stream
static int uneven_trial(dect_uneven* u, const float* lo, const float* hi, int iters, hipEvent_t e0,
                        hipEvent_t e1, float* ms) {
    if (int rc = dect_uneven_init(u, lo, hi)) return rc;
    DECT_HIP(hipEventRecord(e0, u->st));
    if (int rc = dect_uneven_iterate(u, iters)) return rc;
    DECT_HIP(hipEventRecord(e1, u->st));
    DECT_HIP(hipEventSynchronize(e1));
    DECT_HIP(hipEventElapsedTime(ms, e0, e1));
    return DECT_OK;
}

int dect_uneven_autotune(dect_uneven* u, const float* lo, const float* hi, int32_t iters, int32_t reps) {
    if (!u || !lo || !hi) return fail(DECT_EINVAL, "dect_uneven_autotune: NULL argument");
    if (iters < 1 || iters > 100 || reps < 1 || reps > 20)
        return fail(DECT_EINVAL, "dect_uneven_autotune: iters must be in 1..100, reps in 1..20");
    const size_t ng = u->grp.size();
    std::vector<dect_schedule> start(ng), tuned(ng);
    for (size_t q = 0; q < ng; ++q) start[q] = u->grp[q]->sched;
    // each group alone
    for (size_t q = 0; q < ng; ++q) {
        TempBuf buf;
        if (int rc = gather_group(u, q, lo, hi, &buf)) return rc;
        const float* dlo = static_cast<const float*>(buf.p);
        if (int rc = dect_solver_autotune(u->grp[q], dlo, dlo + u->gsino[q], iters, reps, &tuned[q], nullptr))
            return rc;
    }
    // The groups share the device while their iterations interleave, so a
    // group's choice is kept only if the whole handle runs at least 2%
    // faster with it (one group at a time, from the starting schedules).
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DECT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(DECT_EDEVICE, "dect_uneven_autotune: hipEventCreate failed");
    }
    auto apply = [&](const std::vector<dect_schedule>& sc) -> int {
        for (size_t q = 0; q < ng; ++q)
            if (int rc = dect_solver_set_schedule(u->grp[q], &sc[q])) return rc;
        return DECT_OK;
    };
    // median over `reps` trials after one untimed trial
    auto measure = [&](const std::vector<dect_schedule>& sc, double* out) -> int {
        if (int rc = apply(sc)) return rc;
        std::vector<float> t((size_t)reps + 1);
        for (int r = 0; r <= reps; ++r)
            if (int rc = uneven_trial(u, lo, hi, iters, e0, e1, &t[(size_t)r])) return rc;
        std::sort(t.begin() + 1, t.end());
        *out = (double)t[1 + (size_t)reps / 2];
        return DECT_OK;
    };
    std::vector<dect_schedule> best = start;
    double tbest = 0.0;
    int rc = measure(best, &tbest);
    for (size_t q = 0; rc == DECT_OK && q < ng; ++q) {
        if (std::memcmp(&tuned[q], &best[q], sizeof(dect_schedule)) == 0) continue;
        std::vector<dect_schedule> c = best;
        c[q] = tuned[q];
        double t = 0.0;
        if ((rc = measure(c, &t))) break;
        if (t < 0.98 * tbest) {
            best = c;
            tbest = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        (void)apply(start);
        return rc;
    }
    return apply(best);
}

int dect_uneven_get_schedule(const dect_uneven* u, int32_t group, dect_schedule* out) {
    if (!u || group < 0 || group >= (int32_t)u->grp.size())
        return fail(DECT_EINVAL, "dect_uneven_get_schedule: bad group");
    return dect_solver_get_schedule(u->grp[group], out);
}

int dect_solve_uneven(const float* lo, const float* hi, const dect_geometry* geoms, const dect_params* p,
                      float* Z, float* rho_e, int32_t batch, hipStream_t st) {
    if (!lo || !hi || (!Z && !rho_e)) return fail(DECT_EINVAL, "dect_solve_uneven: NULL array");
    dect_uneven* u = nullptr;
    if (int rc = dect_uneven_create(geoms, batch, p, st, &u)) return rc;
    int rc = dect_uneven_init(u, lo, hi);
    if (!rc) rc = dect_uneven_iterate(u, p->n_iter);
    if (!rc) rc = dect_uneven_finish(u, Z, rho_e);
    dect_uneven_destroy(u);
    return rc;
}

int dect_solve(const float* lo, const float* hi, const dect_geometry* g, const dect_params* p,
               float* Z, float* rho, int32_t batch, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!lo || !hi || (!Z && !rho)) return fail(DECT_EINVAL, "dect_solve: NULL array");
    dect_solver* s = nullptr;
    if (int rc = dect_solver_create(g, p, batch, ws, ws_bytes, st, &s)) return rc;
    int rc = dect_solver_init(s, lo, hi);
    if (!rc) rc = dect_solver_iterate(s, p->n_iter);
    if (!rc) rc = dect_solver_finish(s, Z, rho);
    dect_solver_destroy(s);
    return rc;
}

// ---- image-domain form -----------------------------------------------------
static size_t image_layout(int nx, int ny, int batch, char* base, dect_solver* s) {
    Carver c{base};
    const size_t npix = (size_t)nx * ny * batch;
    float2* f = c.take<float2>(npix);
    float2* fnext = c.take<float2>(npix);
    // FFT scratch: two complex planes per slice (the joint f-step carries
    // both bases)
    float2* fft = c.take<float2>(2 * npix);
    float* rho = c.take<float>(npix);
    float* tt = c.take<float>(npix);
    float* tnext = c.take<float>(npix);
    float2* fft2 = c.take<float2>(2 * npix);
    float* muL = c.take<float>(npix);
    float* muH = c.take<float>(npix);
    double* beta_d = c.take<double>((size_t)batch);
    double* kappa_d = c.take<double>((size_t)batch);
    PcgBufs pb;
    carve_pcg(c, ny, nx, batch, &pb);
    if (s) {
        s->f = f;
        s->B = fnext;
        s->fft = fft;
        s->rho = rho;
        s->t = tt;
        s->t_next = tnext;
        s->fft2 = fft2;
        s->muL = muL;
        s->muH = muH;
        s->beta_d = beta_d;
        s->kappa_d = kappa_d;
        s->pcg = pb;
    }
    return c.off;
}

static int check_image_args(int32_t n_x, int32_t n_y, const dect_params* p, int32_t batch) {
    if (batch < 1) return fail(DECT_EINVAL, "batch must be >= 1");
    if (int rc = check_params(p)) return rc;
    if (!fft_size_ok(n_x) || !fft_size_ok(n_y))
        return fail(DECT_EINVAL, "image sizes must be 2^a*3^b (b <= 1) in [8, 1024], got %dx%d", n_x,
                    n_y);
    if (p->t_precond == DECT_PRECOND_MULTIGRID && !mg_plan(n_y, n_x).ok)
        return fail(DECT_EUNSUPPORTED, "multigrid preconditioner: image %dx%d unsupported", n_x, n_y);
    if (p->storage != DECT_STORAGE_FP32)
        return fail(DECT_EUNSUPPORTED, "image-domain form: storage must be DECT_STORAGE_FP32");
    return DECT_OK;
}

size_t dect_image_workspace_bytes(int32_t n_x, int32_t n_y, const dect_params* p, int32_t batch) {
    if (check_image_args(n_x, n_y, p, batch)) return 0;
    return image_layout(n_x, n_y, batch, nullptr, nullptr);
}

int dect_image_solver_create(int32_t n_x, int32_t n_y, const dect_params* p, int32_t batch,
                             void* ws, size_t ws_bytes, hipStream_t st, dect_solver** out) {
    if (!out) return fail(DECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = check_image_args(n_x, n_y, p, batch)) return rc;
    dect_solver* s = new dect_solver();
    s->image = true;
    s->g = Geom{};
    s->g.nx = n_x;
    s->g.ny = n_y;
    s->g.dx = 1.0;
    s->batch = batch;
    s->st = st;
    if (int rc = build_model(*p, &s->M)) {
        delete s;
        return rc;
    }
    if (int rc = resolve_params(p, nullptr, s->M, &s->rp)) {
        delete s;
        return rc;
    }
    const size_t need = image_layout(n_x, n_y, batch, nullptr, nullptr);
    if (ws) {
        if (ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) {
            delete s;
            return fail(DECT_EWORKSPACE, "image solver workspace needs %zu bytes, 256-aligned", need);
        }
        s->ws = ws;
        s->owns_ws = false;
    } else {
        if (int rc = dev_alloc(&s->own, need, st)) {
            delete s;
            return rc;
        }
        s->ws = s->own.p;
        s->owns_ws = true;
    }
    image_layout(n_x, n_y, batch, static_cast<char*>(s->ws), s);
    const hipError_t e = hipMemsetAsync(s->pcg.st, 0, sizeof(PcgState) * batch, st);
    if (e != hipSuccess) {
        if (s->owns_ws) dev_free(&s->own);
        delete s;
        return fail(DECT_EDEVICE, "setting up the solver workspace failed: %s", hipGetErrorString(e));
    }
    s->k = 0;
    s->beta = s->rp.beta0;
    s->last_pcg = 0;
    make_side(s);
    *out = s;
    return DECT_OK;
}

static int load_mu(dect_solver* s, const float* mu_lo, const float* mu_hi) {
    const size_t bytes = (size_t)s->g.nx * s->g.ny * s->batch * sizeof(float);
    DECT_HIP(hipMemcpyAsync(s->muL, mu_lo, bytes, hipMemcpyDeviceToDevice, s->st));
    DECT_HIP(hipMemcpyAsync(s->muH, mu_hi, bytes, hipMemcpyDeviceToDevice, s->st));
    return DECT_OK;
}

int dect_image_solver_init(dect_solver* s, const float* mu_lo, const float* mu_hi) {
    if (!s || !mu_lo || !mu_hi) return fail(DECT_EINVAL, "dect_image_solver_init: NULL argument");
    if (!s->image) return fail(DECT_EINVAL, "dect_image_solver_init: not an image-domain solver");
    if (int rc = load_mu(s, mu_lo, mu_hi)) return rc;
    launch_init_state(s->M, s->g.ny, s->g.nx, s->batch, s->muL, s->muH, (float)s->rp.p.rho_min, s->f,
                      s->rho, s->t, s->st);
    s->k = 0;
    s->beta = s->rp.beta0;
    launch_set_beta(s->beta_d, s->kappa_d, 0, s->batch, s->beta, s->rp.kappa, s->st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_image_solver_set_state(dect_solver* s, const float* mu_lo, const float* mu_hi,
                                const float* f1, const float* f2, const float* rho, const float* t,
                                int32_t k) {
    if (!s || !mu_lo || !mu_hi || !f1 || !f2 || !rho || !t || k < 0)
        return fail(DECT_EINVAL, "dect_image_solver_set_state: NULL argument or k < 0");
    if (!s->image) return fail(DECT_EINVAL, "dect_image_solver_set_state: not an image-domain solver");
    if (int rc = load_mu(s, mu_lo, mu_hi)) return rc;
    const size_t npix = (size_t)s->g.nx * s->g.ny * s->batch;
    launch_join_f2(s->g.nx * s->g.ny, s->batch, f1, f2, s->f, s->st);
    DECT_HIP(hipMemcpyAsync(s->rho, rho, npix * sizeof(float), hipMemcpyDeviceToDevice, s->st));
    DECT_HIP(hipMemcpyAsync(s->t, t, npix * sizeof(float), hipMemcpyDeviceToDevice, s->st));
    s->k = k;
    s->beta = s->rp.beta0;
    for (int i = 0; i < k; ++i) s->beta *= s->rp.kappa;
    launch_set_beta(s->beta_d, s->kappa_d, 0, s->batch, s->beta, s->rp.kappa, s->st);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_solve_image(const float* mu_lo, const float* mu_hi, int32_t n_x, int32_t n_y,
                     const dect_params* p, float* Z, float* rho, int32_t batch, void* ws,
                     size_t ws_bytes, hipStream_t st) {
    if (!mu_lo || !mu_hi || (!Z && !rho)) return fail(DECT_EINVAL, "dect_solve_image: NULL array");
    dect_solver* s = nullptr;
    if (int rc = dect_image_solver_create(n_x, n_y, p, batch, ws, ws_bytes, st, &s)) return rc;
    int rc = dect_image_solver_init(s, mu_lo, mu_hi);
    if (!rc) rc = dect_solver_iterate(s, p->n_iter);
    if (!rc) rc = dect_solver_finish(s, Z, rho);
    dect_solver_destroy(s);
    return rc;
}

const char* dect_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ===========================================================================
// Continuous batching: a pool of slots on one image grid.  Each slot holds one
// request at its own outer iteration (own geometry, beta, iteration budget);
// a step advances every active slot by one iteration in the same launches, and
// a slot that reaches its budget writes its maps and frees itself.
// ===========================================================================
struct dect_engine {
    dect_solver* s = nullptr;
    int slots = 0, cap_views = 0, cap_det = 0;
    size_t cap_rays = 0;
    dect_params p;
    std::vector<int> k, K;
    std::vector<char> busy;
    std::vector<float*> Zout, Rout;
    std::vector<int> done;
    DevAlloc act;
};

static dect_geometry capacity_geometry(int32_t n_x, int32_t n_y, double pixel_mm, int32_t views,
                                       int32_t det) {
    dect_geometry g{};
    g.n_x = n_x;
    g.n_y = n_y;
    g.pixel_mm = pixel_mm;
    g.n_views = views;
    g.arc_rad = 6.283185307179586;   // full circle
    g.n_det = det;
    g.sid_mm = 1000.0;
    g.sdd_mm = 1500.0;
    // keep the placeholder geometry valid for any image: source outside the
    // image's circumcircle with room to the detector
    const double R = 0.5 * pixel_mm * std::hypot((double)n_x, (double)n_y);
    if (R >= 0.9 * g.sid_mm) {
        g.sid_mm = 2.0 * R;
        g.sdd_mm = 4.0 * R;
    }
    return g;
}

size_t dect_engine_workspace_bytes(int32_t n_x, int32_t n_y, double pixel_mm, int32_t slots,
                                   int32_t max_views, int32_t max_det, const dect_params* p) {
    if (slots < 1 || max_views < 1 || max_det < 1 || !p) return 0;
    std::vector<dect_geometry> gs((size_t)slots, capacity_geometry(n_x, n_y, pixel_mm, max_views, max_det));
    BatchGeo B;
    if (make_batch(gs.data(), slots, &B, false)) return 0;
    return solver_layout(B, nullptr, nullptr, p->storage);
}

int dect_engine_create(int32_t n_x, int32_t n_y, double pixel_mm, int32_t slots, int32_t max_views,
                       int32_t max_det, const dect_params* p, void* ws, size_t ws_bytes,
                       hipStream_t st, dect_engine** out) {
    if (!out) return fail(DECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (slots < 1 || max_views < 1 || max_det < 1)
        return fail(DECT_EINVAL, "need slots, max_views, max_det >= 1");
    if (!p) return fail(DECT_EINVAL, "params is NULL");
    if (p->kappa > 0)
        return fail(DECT_EINVAL, "engine: kappa follows each request's iteration budget (set 0)");
    std::vector<dect_geometry> gs((size_t)slots, capacity_geometry(n_x, n_y, pixel_mm, max_views, max_det));
    dect_engine* e = new dect_engine();
    if (int rc = solver_create(gs.data(), p, slots, ws, ws_bytes, st, &e->s, false)) {
        delete e;
        return rc;
    }
    e->slots = slots;
    e->cap_views = max_views;
    e->cap_det = max_det;
    e->cap_rays = (size_t)max_views * max_det;
    e->p = *p;
    e->k.assign(slots, 0);
    e->K.assign(slots, 0);
    e->busy.assign(slots, 0);
    e->Zout.assign(slots, nullptr);
    e->Rout.assign(slots, nullptr);
    dect_solver* s = e->s;
    if (int rc = dev_alloc(&e->act, sizeof(int) * slots, st)) {
        dect_solver_destroy(s);
        delete e;
        return rc;
    }
    s->active_d = static_cast<int*>(e->act.p);
    // every slot starts empty: no views, inactive, zero state
    SliceDesc none = s->hdesc[0];
    none.nv = 0;
    none.nd = 0;
    const size_t npix = (size_t)s->g.nx * s->g.ny;
    hipError_t he = hipSuccess;
    he = he != hipSuccess ? he : hipMemsetAsync(s->f, 0, sizeof(float2) * npix * slots, st);
    he = he != hipSuccess ? he : hipMemsetAsync(s->rho, 0, sizeof(float) * npix * slots, st);
    he = he != hipSuccess ? he : hipMemsetAsync(s->t, 0, sizeof(float) * npix * slots, st);
    if (he != hipSuccess) {
        dev_free(&e->act);
        dect_solver_destroy(s);
        delete e;
        return fail(DECT_EDEVICE, "engine set-up failed: %s", hipGetErrorString(he));
    }
    for (int z = 0; z < slots; ++z) {
        launch_set_desc(const_cast<SliceDesc*>(s->tab.desc), z, none, st);
        launch_set_int(s->active_d + z, 0, st);
    }
    launch_set_beta(s->beta_d, s->kappa_d, 0, slots, s->rp.beta0, 1.0, st);
    *out = e;
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_engine_destroy(dect_engine* e) {
    if (!e) return DECT_OK;
    if (e->s) (void)hipStreamSynchronize(e->s->st);
    dev_free(&e->act);
    dect_solver_destroy(e->s);
    delete e;
    return DECT_OK;
}

int dect_engine_admit(dect_engine* e, const dect_geometry* gin, const float* lo, const float* hi,
                      int32_t n_iter, float* Z, float* rho_e, int32_t* slot_out) {
    if (!e || !gin || !lo || !hi || (!Z && !rho_e) || n_iter < 1)
        return fail(DECT_EINVAL, "dect_engine_admit: bad arguments");
    dect_solver* s = e->s;
    Geom g;
    if (int rc = resolve_geometry(gin, &g)) return rc;
    if (g.nx != s->g.nx || g.ny != s->g.ny || g.dx != s->g.dx)
        return fail(DECT_EINVAL, "dect_engine_admit: image %dx%d at %g mm, engine holds %dx%d at %g mm",
                    g.nx, g.ny, g.dx, s->g.nx, s->g.ny, s->g.dx);
    if (g.nv > e->cap_views || g.nd > e->cap_det)
        return fail(DECT_EINVAL, "dect_engine_admit: %d views x %d bins exceed the slot capacity %d x %d",
                    g.nv, g.nd, e->cap_views, e->cap_det);
    int z = -1;
    for (int q = 0; q < e->slots && z < 0; ++q)
        if (!e->busy[q]) z = q;
    if (z < 0) return fail(DECT_EBUSY, "dect_engine_admit: all %d slots busy", e->slots);
    hipStream_t st = s->st;
    const size_t npix = (size_t)g.nx * g.ny;
    const long long s0 = (long long)z * (long long)e->cap_rays;
    // this slot's ray table and descriptor
    RayTable t = s->tab;
    t.fix += (size_t)z * e->cap_rays;
    t.flt += (size_t)z * e->cap_rays;
    t.span += (size_t)z * e->cap_rays;
    t.view += (size_t)z * e->cap_views;
    launch_build_ray_table(g, t, st);
    const SliceDesc d = make_slice_desc(g, (int)(z * e->cap_rays), z * e->cap_views, s0, eta_of(&e->p, g));
    launch_set_desc(const_cast<SliceDesc*>(s->tab.desc), z, d, st);
    // FBP start and closed forms for this slot only
    float* q = reinterpret_cast<float*>(s->zq + s0);
    launch_fbp_pair(g, lo, hi, 1, q, s->muL + z * npix, s->muH + z * npix, st);
    launch_init_state(s->M, g.ny, g.nx, 1, s->muL + z * npix, s->muH + z * npix,
                      (float)s->rp.p.rho_min, s->f + z * npix, s->rho + z * npix, s->t + z * npix, st);
    // continuation schedule of this request (beta^(0) also seeds the rounding below)
    const double kappa = std::pow(e->p.beta_max / s->rp.beta0, 1.0 / n_iter);
    launch_set_beta(s->beta_d, s->kappa_d, z, 1, s->rp.beta0, kappa, st);
    round_state(s, z, 1);
    // residual sinograms of the start
    const PadLayout P = solver_pad(s);
    launch_pack_f2(g, P, s->f + z * npix, 1, s->dpad + z * P.pair, st);
    RayTable tz = s->tab;
    tz.desc = s->tab.desc + z;
    tz.desc_stride = 0;
    tz.sino_zstride = 0;
    tz.nv_max = g.nv;
    tz.nd_max = g.nd;
    ProjArgs a;
    a.p_lo = lo;
    a.p_hi = hi;
    a.p_base = s0;
    a.res = s->S;
    a.c00 = (float)s->M.C[0][0];
    a.c01 = (float)s->M.C[0][1];
    a.c10 = (float)s->M.C[1][0];
    a.c11 = (float)s->M.C[1][1];
    a.res_bf16 = s->storage != DECT_STORAGE_FP32;
    a.four_ray = sym4(g);
    launch_project(g, P, tz, s->dpad + z * P.pair, 1, PROJ_RESID, a, st);
    launch_set_int(s->active_d + z, 1, st);
    DECT_HIP(hipGetLastError());
    e->busy[z] = 1;
    e->k[z] = 0;
    e->K[z] = n_iter;
    e->Zout[z] = Z;
    e->Rout[z] = rho_e;
    if (slot_out) *slot_out = z;
    return DECT_OK;
}

int dect_engine_step_n(dect_engine* e, int32_t n, int32_t* done_iters) {
    if (!e || n < 1) return fail(DECT_EINVAL, "dect_engine_step_n: engine is NULL or n < 1");
    if (done_iters) *done_iters = 0;
    bool any = false;
    for (int z = 0; z < e->slots; ++z) any = any || e->busy[z];
    if (!any) return DECT_OK;
    dect_solver* s = e->s;
    // launches cover the slots up to the highest occupied one (admission fills
    // the lowest free slot first); at most as many iterations as the first
    // slot to complete still needs
    int hw = 0, m = n;
    for (int z = 0; z < e->slots; ++z)
        if (e->busy[z]) {
            hw = z + 1;
            m = std::min(m, e->K[z] - e->k[z]);
        }
    s->batch = hw;
    int rc = DECT_OK;
    for (int i = 0; i < m && rc == DECT_OK; ++i) rc = one_iteration(s, i + 1 < m);   // pipelined
    s->batch = e->slots;
    if (rc) return rc;
    if (done_iters) *done_iters = m;
    const size_t npix = (size_t)s->g.nx * s->g.ny;
    SliceDesc none = s->hdesc[0];
    none.nv = 0;
    none.nd = 0;
    for (int z = 0; z < e->slots; ++z) {
        if (!e->busy[z]) continue;
        e->k[z] += m;
        if (e->k[z] < e->K[z]) continue;
        launch_finish(s->M, s->g.ny, s->g.nx, 1, s->rho + z * npix, s->t + z * npix,
                      (float)s->rp.p.rho_min, s->rp.p.t_min, e->Zout[z], e->Rout[z], s->st);
        launch_set_desc(const_cast<SliceDesc*>(s->tab.desc), z, none, s->st);
        launch_set_int(s->active_d + z, 0, s->st);
        e->busy[z] = 0;
        e->done.push_back(z);
    }
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int dect_engine_step(dect_engine* e) { return dect_engine_step_n(e, 1, nullptr); }

int dect_engine_cancel(dect_engine* e, int32_t slot) {
    if (!e) return fail(DECT_EINVAL, "dect_engine_cancel: engine is NULL");
    if (slot < 0 || slot >= e->slots || !e->busy[slot])
        return fail(DECT_EINVAL, "dect_engine_cancel: slot %d holds no request", slot);
    dect_solver* s = e->s;
    SliceDesc none = s->hdesc[0];
    none.nv = 0;
    none.nd = 0;
    launch_set_desc(const_cast<SliceDesc*>(s->tab.desc), slot, none, s->st);
    launch_set_int(s->active_d + slot, 0, s->st);
    DECT_HIP(hipGetLastError());
    e->busy[slot] = 0;
    e->Zout[slot] = e->Rout[slot] = nullptr;
    return DECT_OK;
}

int dect_engine_status(const dect_engine* e, int32_t* active, int32_t* free_slots) {
    if (!e) return fail(DECT_EINVAL, "engine is NULL");
    int n = 0;
    for (int z = 0; z < e->slots; ++z) n += e->busy[z] ? 1 : 0;
    if (active) *active = n;
    if (free_slots) *free_slots = e->slots - n;
    return DECT_OK;
}

int dect_engine_completed(dect_engine* e, int32_t* slots, int32_t cap, int32_t* n) {
    if (!e || !n || (cap > 0 && !slots)) return fail(DECT_EINVAL, "dect_engine_completed: bad arguments");
    const int m = std::min<int>(cap, (int)e->done.size());
    for (int i = 0; i < m; ++i) slots[i] = e->done[i];
    e->done.erase(e->done.begin(), e->done.begin() + m);
    *n = m;
    return DECT_OK;
}
