// Internal declarations of the HIP library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../include/dect.h"

namespace dect {

// ---- errors ---------------------------------------------------------------
int fail(int code, const char* fmt, ...);

#define DECT_HIP(expr)                                                                 \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::dect::fail(DECT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---- geometry -------------------------------------------------------------
// Validated geometry with the detector pitch resolved (host, FP64).
struct Geom {
    int nx, ny, nv, nd;
    double dx, angle0, arc, pitch, offset, sid, sdd;
};
int resolve_geometry(const dect_geometry* in, Geom* out);

// Quarter-turn symmetry: on a square grid whose side is a multiple of 32,
// with a multiple of 4 views over a full circle, view v + nv/4 is view v
// turned by 90 degrees about the centre, which maps pixel (i, k) to
// (k, n - 1 - i).  The projector is then defined from the first quarter of
// the views: ray (v + r nv/4, j) takes the weights of ray (v, j) on the pixels
// turned r times.  Its table holds the first nv/4 views only, and the
// back-projector evaluates each weight once for four views.
//
// Not when a ray runs exactly along a grid line: a view at a multiple of 90
// degrees whose detector has a bin centre straight across the isocentre (an
// odd bin count on a centred detector) has its central ray on the grid line
// through the centre (the side is even).  The chord of such a ray goes to one
// pixel by the half-open rule, and a quarter turn does not preserve which
// side of the line that is; those slices take the per-view projector.
inline bool axis_ray_on_grid_line(const Geom& g) {
    const double half_pi = 1.5707963267948966;
    const double dth = g.arc / g.nv;
    bool axis_view = false;
    for (int r = 0; r < 4 && !axis_view; ++r) {
        const double v = (r * half_pi - g.angle0) / dth;
        const double vr = std::floor(v + 0.5);
        axis_view = std::fabs(v - vr) < 1e-9 && vr >= 0.0 && vr < g.nv;
    }
    if (!axis_view) return false;
    const double c = 0.5 * (g.nd - 1) - g.offset / g.pitch;   // bin index at u = 0
    const double cr = std::floor(c + 0.5);
    return std::fabs(c - cr) < 1e-9 && cr >= 0.0 && cr < g.nd;
}
inline bool sym4(const Geom& g) {
    const double two_pi = 6.283185307179586;
    return g.nx == g.ny && g.nx % 32 == 0 && g.nv >= 4 && g.nv % 4 == 0 &&
           g.arc > two_pi * (1.0 - 1e-12) && g.arc < two_pi * (1.0 + 1e-12) &&
           !axis_ray_on_grid_line(g);
}
inline int table_views(const Geom& g) { return sym4(g) ? g.nv / 4 : g.nv; }
// Transpose symmetry on top of the quarter turns: with the detector centred
// and the first view at angle 0, view nv/4 - v is view v reflected about the
// image diagonal with the bins reversed, which maps pixel (i, k) to (k, i).
// The table's views nv/8 < v < nv/4 are then defined as the transposes of
// views nv/4 - v, and the back-projector evaluates each weight once for
// eight views.
inline bool sym8(const Geom& g) {
    return sym4(g) && g.angle0 == 0.0 && g.offset == 0.0;
}
// slice kinds, as bits: which back-projection kernels a batch needs
enum { kSlicePlain = 1, kSliceQuarter = 2, kSliceOcto = 4 };
inline int slice_kind(const Geom& g) {
    return sym8(g) ? kSliceOcto : (sym4(g) ? kSliceQuarter : kSlicePlain);
}

// Per-ray traversal table, built on the device in FP64.
// For ray (v, j) the ray is parametrised along its major axis (the pixel
// axis it advances along by at most one minor pixel per step).  Coordinates
// are in pixel units from the image corner; the minor coordinate is kept in
// 32.32 fixed point so that every major step adds the slope exactly.
//   fix[v*nd + j]  = {A0, S}: minor coordinate at major 0 and slope (minor
//                    per major step, |s| <= 1), both times 2^32, as int64
//                    stored in an int4 (lo, hi, lo, hi);
//   flt[v*nd + j]  = {inv_s, Ls}: 1/s (+inf when s == 0) and the chord length
//                    per major step in mm, its sign giving the axis (> 0:
//                    x-major, < 0: y-major);
//   span[v*nd + j] = {k_lo, k_hi}: major steps that can meet the image
//                    (inclusive, one step of margin; k_lo > k_hi: none);
//   view[v]        = {cos, sin, h*(|cos| + |sin|), 0} for the voxel-driven
//                    footprint (h = half pixel, mm).
// With quarter-turn symmetry (sym4) the table holds views 0 .. nv/4 - 1.
//
// A batch may hold slices of different fan geometry (same image grid): the
// tables of its distinct geometries sit back to back, and a per-slice
// descriptor gives each slice's sizes, table offsets and sinogram offset.
struct SliceDesc {
    int nv, nd;            // views, bins
    int ray0, view0;       // first ray / view of this slice's table
    long long sino0;       // first element of this slice's sinograms and residuals
    float sid, sdd;        // source-isocentre, source-detector distance (mm)
    float u0, inv_pitch;   // detector coordinate of bin 0 (mm), 1 / bin pitch
    double eta;            // projection-data weight of eq. (10) for this geometry
    int sym;               // 1: quarter-turn symmetric (table of nv / 4 views); 2: also
                           // transpose-symmetric (views nv/8 < v < nv/4 derived)
};
struct RayTable {
    int4* fix = nullptr;
    float2* flt = nullptr;
    int2* span = nullptr;
    float4* view = nullptr;
    // device descriptors: slice / pair z uses desc[desc_stride * z], its
    // sinograms start at desc.sino0 + z * sino_zstride
    const SliceDesc* desc = nullptr;
    int desc_stride = 0;
    long long sino_zstride = 0;
    int nv_max = 0, nd_max = 0;   // largest slice (launch grid)
};
SliceDesc make_slice_desc(const Geom& g, int ray0, int view0, long long sino0, double eta);
void launch_set_desc(SliceDesc* desc, int z, const SliceDesc& d, hipStream_t st);
void launch_set_int(int* p, int value, hipStream_t st);
size_t ray_table_bytes(const Geom& g);
void launch_build_ray_table(const Geom& g, RayTable t, hipStream_t st);

// ---- packed image layouts for the projector --------------------------------
// Two images travel together as float2.  The projector reads them from two
// zero-padded layouts, stored back to back for each pair z:
//   padN: [max(nx, ny)][nx + 2*kPad]  (row-major)
//   padT: [max(nx, ny)][ny + 2*kPad]  (transposed)
// with kPad zero entries at both ends of every line, so a ray step whose
// minor coordinate is clamped into [-kPad, n + kPad) reads zeros only, and
// zero lines past the last row (padN) or column (padT) of a non-square
// image, so that every ray of a wavefront can step over the wavefront's
// common major range.  For quarter-turn symmetric projection (square image)
// two more layouts follow, with every line's entries in reverse order:
//   padNR: [n][n + 2*kPad], entry e of row i = image(i, n - 1 - e)
//   padTR: [n][n + 2*kPad], entry e of column k = image(n - 1 - e, k)
constexpr int kPad = 2;
struct PadLayout {
    int ldN, ldT;     // line strides (elements) of padN and padT
    int lines;        // lines of each layout, max(nx, ny)
    size_t offT;      // offset of padT within a pair block
    size_t offNR, offTR;   // offsets of padNR, padTR (rev only)
    bool rev;
    size_t pair;      // elements per pair block
};
inline bool grid_sym4(const Geom& g) { return g.nx == g.ny && g.nx % 32 == 0; }
// rev: with the reversed layouts (needs a square grid, side a multiple of 32)
inline PadLayout pad_layout(const Geom& g, bool rev = false) {
    PadLayout L;
    L.ldN = g.nx + 2 * kPad;
    L.ldT = g.ny + 2 * kPad;
    L.lines = g.nx > g.ny ? g.nx : g.ny;
    L.offT = (size_t)L.lines * L.ldN;
    L.rev = rev && grid_sym4(g);
    L.offNR = L.offT + (size_t)L.lines * L.ldT;
    L.offTR = L.offNR + (L.rev ? (size_t)L.lines * L.ldN : 0);
    L.pair = L.offTR + (L.rev ? (size_t)L.lines * L.ldT : 0);
    if (!L.rev) L.offNR = L.offTR = 0;
    return L;
}
inline size_t pad_elems(const Geom& g, bool rev = false) { return pad_layout(g, rev).pair; }

// pack img[2z], img[2z+1] ([ny][nx] each, f32) into pair blocks z of `pad`
// (every element of the blocks is written, the zero entries included);
// nimg = number of source images (odd: the last pair's second channel is 0).
void launch_pack_pairs(const Geom& g, const PadLayout& P, const float* img, int nimg, float2* pad,
                       hipStream_t st);
// pack a float2 image [ny][nx] (pairs) into pair blocks
void launch_pack_f2(const Geom& g, const PadLayout& P, const float2* src, int npairs, float2* pad,
                    hipStream_t st);
// interleave sinograms s[2z], s[2z+1] into pairs (second channel 0 if missing)
void launch_pair_sinos(const Geom& g, const float* sino, int nsino, float2* out, hipStream_t st);

// ---- projector ----------------------------------------------------------------
enum ProjMode { PROJ_PLAIN = 0, PROJ_RESID = 1, PROJ_LINESEARCH = 2 };
struct ProjArgs {
    // PROJ_PLAIN (one geometry, sino_zstride = nv*nd): channel 0 to out[2z],
    // channel 1 to out[2z+1] (< nout)
    float* out = nullptr;
    int nout = 0;
    // PROJ_RESID: S = eta C^T (C Y - p) from p_lo/p_hi -> res (float2)
    // PROJ_LINESEARCH: zq = eta C^T C Y -> res; block partials of eta ||C Y||^2
    // (eta of the slice's descriptor: the data weight travels with the residual)
    const float* p_lo = nullptr;
    const float* p_hi = nullptr;
    long long p_base = 0;   // p_lo / p_hi hold the slice's sinograms from element desc.sino0 - p_base
    float2* res = nullptr;
    float c00 = 0, c01 = 0, c10 = 0, c11 = 0;   // C[k][i] = mu_i(E_k)
    double* partials = nullptr;                  // [z][nblocks]
    // line-search step (k_alpha, after the rays): alpha[z] = num / den
    const double* img_partials = nullptr;        // [z][img_nblocks][3]
    int img_nblocks = 0;
    double w_data = 0, w_coup = 0, w_reg = 0;    // 2, 2 xi, 2 beta
    const double* beta_z = nullptr;              // per-slice beta (then w_reg = 2 beta_z[z])
    double* alpha = nullptr;                     // [z]
    // BF16 storage: res holds one 32-bit word of two BF16 values per ray
    // (RESID, LINESEARCH); LINESEARCH also reads BF16 pair blocks
    bool res_bf16 = false;
    bool pad_bf16 = false;
    // four_ray: the quarter-turn symmetric slices take the four-ray form
    // (k_project4: one lane per table ray produces its four turned rays);
    // has_plain: the batch also holds slices of neither symmetry, which then
    // take the per-view form (k_project) in a second launch.  Both forms give
    // a slice's rays bit for bit alike.
    bool four_ray = false;
    bool has_plain = false;
    bool plain_only = false;     // (set by launch_project) k_project skips symmetric slices
    size_t part_stride = 0;      // (set by launch_project) partials per slice
};
int proj_nblocks(int nv_max, int nd_max);  // blocks per pair
// pad: float2 pair blocks, or with a.pad_bf16 one 32-bit BF16 pair per entry
void launch_project(const Geom& g, const PadLayout& P, const RayTable& t, const void* pad, int npairs,
                    int mode, const ProjArgs& a, hipStream_t st);

// ---- back-projector -------------------------------------------------------------
// sino pairs [z][nv][nd] (float2, or BF16 pairs in 32-bit words) -> out pairs
// [z][ny][nx] (float2) or split images.
// kinds: the kSlice* bits of the pairs' slices (one kernel per kind present)
// (two launches, each skipping the other kind of slice)
// bp_pct: workgroups of the symmetric kernels as a percentage of the CUs
// (0: half of them up to one orbit per CU, all of them beyond)
void launch_backproject(const Geom& g, const RayTable& t, const void* sino, int npairs,
                        float2* out_pairs, float* out_split, int nout, hipStream_t st,
                        bool sino_bf16 = false, int kinds = kSlicePlain, int bp_pct = 0);

// ---- FBP ---------------------------------------------------------------------
// q = filtered sinograms (scratch, [nsino][nv][nd]); img [nsino][ny][nx]
// both sinograms of nsino slices of one geometry; q: scratch of 2*nsino*nv*nd floats
void launch_fbp_pair(const Geom& g, const float* sino_a, const float* sino_b, int nsino, float* q,
                     float* img_a, float* img_b, hipStream_t st);
void launch_fbp(const Geom& g, const float* sino, int nsino, float* q, float* img,
                hipStream_t st);

// ---- FFT solve of (c + beta*D^T D) x = rhs, periodic ----------------------------
// Sizes n = 2^a * 3^b (b <= 1), 8 <= n <= 1024.
bool fft_size_ok(int n);
enum FftSrc { FFT_SRC_PLAIN = 0, FFT_SRC_RHO = 1, FFT_SRC_L0 = 2, FFT_SRC_IMGF = 3 };
struct FftArgs {
    int src = FFT_SRC_PLAIN;
    // PLAIN: out = (c + beta L)^-1 in.
    // RHO / L0 (correction form): with g = base (the current iterate, also the
    // hard-threshold input) and S its thresholded-away gradients,
    //   (1 + beta L) delta = (target - g) - beta D^T S,   out = g + delta,
    // target = rho_hat(f) (RHO) or in = g_tilde (L0).  Equal to the closed
    // form for (1 + beta L) out = target + beta D^T HT(D g), without the large
    // cancelling terms.
    // IMGF (image-domain f-subproblem (13a), both bases jointly): per frequency
    //   [[c + beta L, c_o], [c_o, c_b + beta L]] delta = r - beta D^T S,
    //   r_i = eta_i sum_k C_k,i (mu_k - (C f)_k) + xi sum_j Ms_j,i (T_j - (Ms f)_j),
    //   T_j = rho (ta_j t' + tpsi_j), c = H_11, c_b = H_22, c_o = H_12,
    //   c_det = c c_b - c_o^2 (FP64 on the host), H = eta_i C^T C + xi Ms^T Ms;
    // f (interleaved f1, f2) at iterate k is the hard-threshold input; out
    // points to the interleaved f^(k+1) = f + delta.  Scratch holds two
    // complex planes per slice.
    const float* in = nullptr;
    const float2* f = nullptr;
    const float* base = nullptr;
    float* h_out = nullptr;           // L0: optional kept (h, v)
    float* v_out = nullptr;
    double m00 = 0, m01 = 0, m10 = 0, m11 = 0;   // synthesis matrix (barn)
    double e1n = 0, e2n = 0, inv_crho = 0;       // E1^n, E2^n, 1/c_rho
    float beta = 0, thr = 0;
    const double* beta_z = nullptr;   // per-slice beta: then beta = beta_z[z], thr = lam / beta_z[z]
    double lam = 0.0;
    double c = 1.0;                   // diagonal shift, or from partial sums:
    const double* c_parts = nullptr;  //   c = c_scale * sum(c_parts[z*c_zstride + 0..c_n))
    // PLAIN: symmetric diagonal scaling s = sqrt((c + 4 beta) / (w2 + 4 beta)),
    // out = s (c + beta L)^-1 (s in): Jacobi-like where beta is small, the
    // plain FFT inverse where it is large
    const float* scale_w2 = nullptr;
    int c_n = 0;
    size_t c_zstride = 0;
    double c_scale = 0.0;
    const int* skip = nullptr;        // skip slice z when skip[z*skip_zstride] != 0
    size_t skip_zstride = 0;
    float* out = nullptr;
    int bstride = 1, ostride = 1;     // element strides of base and out (2: one half of a float2)
    // IMGF inputs
    const float* mu_lo = nullptr;
    const float* mu_hi = nullptr;
    const float* rho_in = nullptr;
    const float* t_in = nullptr;
    double c_b = 0.0, c_o = 0.0, c_det = 0.0;
    double cL0 = 0, cL1 = 0, cH0 = 0, cH1 = 0;   // attenuation matrix rows (E_lo, E_hi)
    double ta0 = 0, ta1 = 0, tpsi0 = 0, tpsi1 = 0;
    double eta_img = 0, xi_img = 0;
    const float* dot_with = nullptr;  // optional: dot_parts[z*dot_zstride + row] = <out, dot_with>
    double* dot_parts = nullptr;
    size_t dot_zstride = 0;
};
size_t fft_scratch_bytes(int ny, int nx, int batch);
void launch_fft_solve(int ny, int nx, int batch, const FftArgs& a, float2* scratch,
                      hipStream_t st);
// Unit-weight gradient-L0 step (eq. (5)-(9), FFT closed form) with the given
// complex scratch of batch*n_y*n_x values; every scratch value is written
// before it is read.  Arguments validated by the caller.
int l0_fft_step(const float* g_tilde, float* g, float* h_out, float* v_out, int n_y, int n_x,
                int batch, double lambda, double beta, float2* fft, hipStream_t st);

// Per-slice relaxation weight: a batch whose slices sit at different outer
// iterations carries beta per slice on the device; kernels take their slice's
// value (the threshold lambda/beta is formed the same way as on the host).
template <typename A>
__device__ __forceinline__ void slice_beta_thr(A& a, int z) {
    if (a.beta_z) {
        const double b = a.beta_z[z];
        a.beta = (float)b;
        a.thr = (float)(a.lam / b);
    }
}

// ---- image-domain kernels of the solver ------------------------------------------
struct Model {      // FP64 constants of the attenuation model (host)
    double C[2][2];     // C[k][i] = mu_i(E_k), 1/mm
    double Ms[2][2];    // Ms[j][i] = basis i per water electron at E_j (barn)
    double psi[2];      // KN at E1, E2 (barn)
    double a[2];        // Cp' * Zw^m / E_j^n (barn)
    double e1n, e2n, crho, Ww, cpb, Zw, m;
};
int build_model(const dect_params& p, Model* out);

struct ImgArgs {
    int ny, nx, nv, nd, batch;
    float eta2, xi2, beta2, thr;   // 2 (the residual carries eta), 2*xi, 2*beta, lambda/beta
    float beta;
    const double* beta_z = nullptr;   // per-slice beta (overrides beta2, thr, beta)
    double lam = 0.0;
    bool bf16 = false;   // direction pair blocks and residual / line-search sinograms in BF16
};
int grad_nblocks(int ny, int nx);
void launch_init_state(const Model& M, int ny, int nx, int batch, const float* muL,
                       const float* muH, float rho_min, float2* f, float* rho, float* t,
                       hipStream_t st);
// the search direction is written into the projector's pair blocks `dpad`
// (float2 entries, or one 32-bit BF16 pair per entry with a.bf16)
void launch_grad(const Model& M, const ImgArgs& a, const PadLayout& P, const float2* f,
                 const float2* B, const float* rho, const float* t, void* dpad,
                 double* partials, hipStream_t st);
// also steps each slice's beta: beta_z[z] *= kappa_z[z] (when beta_z is given);
// with a.bf16, dpad, S and zq hold BF16 pairs
void launch_update(const ImgArgs& a, const PadLayout& P, const RayTable& T, const double* alpha,
                   const void* dpad, float2* f, void* S, const void* zq, double* beta_z,
                   const double* kappa_z, hipStream_t st);
void launch_round_state(size_t npix, int batch, float2* f, float* rho, float* t, const double* beta_z,
                        hipStream_t st);
// continuation: beta_z[z] *= kappa_z[z] for z < n
void launch_step_beta(double* beta_z, const double* kappa_z, int n, hipStream_t st);
// beta_z[z0 .. z0+n) = beta, kappa_z[...] = kappa
void launch_set_beta(double* beta_z, double* kappa_z, int z0, int n, double beta, double kappa,
                     hipStream_t st);
void launch_finish(const Model& M, int ny, int nx, int batch, const float* rho, const float* t,
                   float rho_min, double t_min, float* Z, float* rho_out, hipStream_t st);
void launch_split_f2(int n, int batch, const float2* f, float* a, float* b, hipStream_t st);
void launch_join_f2(int n, int batch, const float* a, const float* b, float2* f,
                    hipStream_t st);

// ---- PCG for (diag(w^2) + beta D^T D) x = w*g + beta D^T HT(D x0) -------------
// Warm start x = x0; the initial residual is formed without cancellation as
// r0 = w*(g - w*x0) - beta*D^T S(x0), S the thresholded-away gradients of x0.
// Scalars are never stored: every block re-reduces the previous kernel's
// per-block partial sums in a fixed order (deterministic, fence-free).
// Stopping rule: ||r_k|| <= tol * ||r_0||.
struct PcgState {   // per slice, read by the host
    int done, iters, pad0, pad1;
};
struct PcgParts {   // per-slice partial-sum layout (doubles)
    int nblk, nrz;  // blocks of the pixel kernels; entries of an rz sum
    size_t init0, init1, pq, rz, rr;   // offsets within a slice
    size_t dl;      // pipelined PCG: <u, w> partials, two parity slots of nrz
    size_t sc;      // pipelined PCG: (gamma, alpha) of the last two iterations
    size_t zstride;
};
PcgParts pcg_parts(int ny, int nx);
enum PcgPrec { PREC_JACOBI = 1, PREC_FFT = 2, PREC_MG = 3 };
struct PcgArgs {
    int ny, nx, batch;
    float beta, thr;
    const double* beta_z = nullptr;   // per-slice beta: then beta = beta_z[z], thr = lam / beta_z[z]
    double lam = 0.0;
    const int* active = nullptr;      // slices with active[z] == 0 start done (no PCG work)
    double tol2;
    int prec;                // PcgPrec
    int nrz_used;            // entries of the <r, z> partial sums this preconditioner writes
    float* x;                // in: x0 (also HT input), out: solution
    const float* x0 = nullptr;   // when set: x0 (and HT input), x only written
    float *r, *z, *p0, *p1, *q, *w2;
    float *r2 = nullptr, *p1b = nullptr;   // pipelined PCG: second r and s buffers
    double* parts;           // [batch][PcgParts::zstride]
    PcgParts L;
    PcgState* st;            // [batch]
};
// initial residual from the model (t' subproblem): w = W/Ww, g = d_t/Ww from f
void launch_pcg_init_model(const Model& M, const PcgArgs& a, const float2* f, hipStream_t st);
// from explicit weight and g_tilde (dect_l0_step); optional kept (h, v) of x0
void launch_pcg_init_plain(const PcgArgs& a, const float* w, const float* g_tilde, float* h_out,
                           float* v_out, hipStream_t st);
void launch_pcg_matvec(const PcgArgs& a, int it, hipStream_t st);
void launch_pcg_update(const PcgArgs& a, int it, hipStream_t st);
// after `done_iters` completed iterations: set done / iters for the host
void launch_pcg_check(const PcgArgs& a, int done_iters, hipStream_t st);
// FFT preconditioner z = (c + beta L)^-1 r, c = mean(w^2), with <r, z> partials
void launch_pcg_fft_prec(const PcgArgs& a, int it, float2* scratch, hipStream_t st);
// Pipelined PCG (one reduction per iteration, Chronopoulos and Gear) with
// the multigrid preconditioner: iteration i takes u_i = M r_i, w_i = A u_i
// and the partial sums of gamma_i = <r_i, u_i>, delta_i = <u_i, w_i> (from
// the V-cycle's last kernel), forms beta_i = gamma_i / gamma_(i-1) and
// alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_(i-1)), then
// p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s.  It first
// stops the slice when ||r_i||^2 <= tol2 ||r_0||^2.  p is p0; r and s
// alternate between (r, r2) and (p1, p1b) by parity.  The update runs inside
// the first kernel of the next V-cycle: launch_pcg_mg_prec_w_upd below.

// ---- multigrid V-cycle preconditioner for diag(c) + beta L -----------------------
constexpr int kMgMaxLevels = 12;
constexpr int kMgDenseMax = 64;      // unknowns of the exactly solved grid, at most
constexpr int kMgExactMax = 16;      //   and the first grid this small is the one
constexpr int kMgCoarseB = 3;        // smoothed levels of the in-LDS part (32 -> 16 -> 8)
struct MgPlan {
    bool ok = false;                 // sizes admit the V-cycle
    int nlev = 0, ngrid = 0, ncoarse = 0;   // all levels; tile-kernel levels; in-LDS levels
    int ncb = 0, ne = 0;             // smoothed in-LDS levels; unknowns of the exact level
    int ny[kMgMaxLevels] = {}, nx[kMgMaxLevels] = {};
    // per-slice offsets (floats) into the level buffer: xs0 = saved iterate of
    // level 0; b, c, xs, e of tile levels 1..ngrid; set-up data of the in-LDS
    // part: omega / diag of its smoothed levels (id), the diagonals of all
    // but the first (cb), the exact level's inverse (gi, ne x ne)
    size_t xs0 = 0, b[kMgMaxLevels] = {}, c[kMgMaxLevels] = {}, xs[kMgMaxLevels] = {},
           e[kMgMaxLevels] = {};
    size_t id[kMgCoarseB] = {}, cb[kMgCoarseB] = {}, gi = 0;
    size_t zstride = 0;              // floats per slice
    int nrz = 0;                     // <r, z> partials one V-cycle writes
    bool pair[kMgMaxLevels] = {};    // tile levels l and l + 1 run in one kernel each way
};
MgPlan mg_plan(int ny, int nx);
struct CgUpd;   // pipelined PCG update fused into a V-cycle (mg.hip)
// once per linear solve: c pyramid from w2 and the in-LDS part's set-up data
// (inverse diagonals, exact-level inverse) for beta (or beta_z[z] per slice)
void launch_mg_setup(const MgPlan& P, const float* w2, float* mg, int batch, float beta,
                     const double* beta_z, const int* skip, size_t skip_zstride, hipStream_t st);
// z = V(r); <r, z> partials into dot[z*dot_zstride + 0..P.nrz)
void launch_mg_vcycle(const MgPlan& P, const float* r, const float* w2, float* z, float* mg,
                      int batch, float beta, const double* beta_z, const int* skip,
                      size_t skip_zstride, double* dot, size_t dot_zstride, hipStream_t st,
                      float* wout = nullptr, double* dot2 = nullptr,
                      const CgUpd* upd = nullptr);
void launch_pcg_mg_prec(const PcgArgs& a, int it, const MgPlan& P, float* mg, hipStream_t st);
// the V-cycle as the pipelined PCG uses it (needs mg_pipelined_ok: level 0 a
// pair level above at least one more tile level)
bool mg_pipelined_ok(const MgPlan& P);
// pipelined iterations test their new residual within their own V-cycle (then
// a chunk needs no separate check kernel)
bool mg_early_stop(const MgPlan& P);
void launch_pcg_mg_prec_w(const PcgArgs& a, int i, const MgPlan& P, float* mg, hipStream_t st);
// iteration i of the pipelined PCG in one V-cycle: the update fused into its
// first kernel, then u, w and the partial sums of iteration i + 1; needs r2
// and p1b
void launch_pcg_mg_prec_w_upd(const PcgArgs& a, int i, const MgPlan& P, float* mg, hipStream_t st);

}  // namespace dect
