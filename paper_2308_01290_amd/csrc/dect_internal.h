// Internal declarations of the HIP library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

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
struct RayTable {
    int4* fix = nullptr;
    float2* flt = nullptr;
    int2* span = nullptr;
    float4* view = nullptr;
};
size_t ray_table_bytes(const Geom& g);
void launch_build_ray_table(const Geom& g, RayTable t, hipStream_t st);

// ---- packed image layouts for the projector --------------------------------
// Two images travel together as float2.  The projector reads them from two
// zero-padded layouts so that every ray step is a coalesced pair of loads:
//   padN: [ny][nx + 2]  (row-major, one zero column on each side)
//   padT: [nx][ny + 2]  (transposed, one zero row-entry on each side)
inline size_t padN_elems(const Geom& g) { return (size_t)g.ny * (g.nx + 2); }
inline size_t padT_elems(const Geom& g) { return (size_t)g.nx * (g.ny + 2); }

// pack img[2z], img[2z+1] ([ny][nx] each, f32) into padN/padT pairs z;
// nimg = number of source images (odd: the last pair's second channel is 0).
void launch_pack_pairs(const Geom& g, const float* img, int nimg, float2* padN, float2* padT,
                       hipStream_t st);
// pack a float2 image [ny][nx] (pairs) into padN/padT
void launch_pack_f2(const Geom& g, const float2* src, int npairs, float2* padN, float2* padT,
                    hipStream_t st);
// interleave sinograms s[2z], s[2z+1] into pairs (second channel 0 if missing)
void launch_pair_sinos(const Geom& g, const float* sino, int nsino, float2* out, hipStream_t st);

// ---- projector ----------------------------------------------------------------
enum ProjMode { PROJ_PLAIN = 0, PROJ_RESID = 1, PROJ_LINESEARCH = 2 };
struct ProjArgs {
    // PROJ_PLAIN: write channel 0 to out[2z], channel 1 to out[2z+1] (< nout)
    float* out = nullptr;
    int nout = 0;
    // PROJ_RESID: S = C^T (C Y - p) from p_lo/p_hi [z][nv][nd] -> res (float2)
    // PROJ_LINESEARCH: zq = C^T C Y -> res; block partials of ||C Y||^2
    const float* p_lo = nullptr;
    const float* p_hi = nullptr;
    float2* res = nullptr;
    float c00 = 0, c01 = 0, c10 = 0, c11 = 0;   // C[k][i] = mu_i(E_k)
    double* partials = nullptr;                  // [z][nblocks]
    // line-search finish (last block): alpha[z] = num / den
    const double* img_partials = nullptr;        // [z][img_nblocks][3]
    int img_nblocks = 0;
    double w_data = 0, w_coup = 0, w_reg = 0;    // 2 eta, 2 xi, 2 beta
    double* alpha = nullptr;                     // [z]
    unsigned* counter = nullptr;                 // [z]
};
int proj_nblocks(const Geom& g);  // blocks per pair
void launch_project(const Geom& g, const RayTable& t, const float2* padN, const float2* padT,
                    int npairs, int mode, const ProjArgs& a, hipStream_t st);

// ---- back-projector -------------------------------------------------------------
// sino pairs [z][nv][nd] -> out pairs [z][ny][nx] (float2) or split images.
void launch_backproject(const Geom& g, const RayTable& t, const float2* sino, int npairs,
                        float2* out_pairs, float* out_split, int nout, hipStream_t st);

// ---- FBP ---------------------------------------------------------------------
// q = filtered sinograms (scratch, [nsino][nv][nd]); img [nsino][ny][nx]
void launch_fbp(const Geom& g, const float* sino, int nsino, float* q, float* img,
                hipStream_t st);

// ---- FFT solve of (c + beta*D^T D) x = rhs, periodic ----------------------------
// Sizes n = 2^a * 3^b (b <= 1), 8 <= n <= 1024.
bool fft_size_ok(int n);
enum FftSrc { FFT_SRC_PLAIN = 0, FFT_SRC_RHO = 1, FFT_SRC_L0 = 2 };
struct FftArgs {
    int src = FFT_SRC_PLAIN;
    const float* in = nullptr;        // PLAIN: rhs image; L0: g_tilde
    // RHO: rhs = rho_hat(f) + beta*D^T HT(D rho)
    const float2* f = nullptr;        // f pairs
    const float* rho = nullptr;       // current rho (HT input)
    const float* g_cur = nullptr;     // L0: current g (HT input)
    float* h_out = nullptr;           // L0: optional h, v outputs
    float* v_out = nullptr;
    double m00 = 0, m01 = 0, m10 = 0, m11 = 0;   // synthesis matrix (barn)
    double e1n = 0, e2n = 0, inv_crho = 0;       // E1^n, E2^n, 1/c_rho
    float beta = 0, thr = 0;
    double c = 1.0;                   // diagonal shift
    const double* c_dev = nullptr;    // device diagonal shift (overrides c)
    const int* skip = nullptr;        // device flag: skip the solve when nonzero
    float* out = nullptr;             // result image
};
size_t fft_scratch_bytes(int ny, int nx, int batch);
void launch_fft_solve(int ny, int nx, int batch, const FftArgs& a, float2* scratch,
                      hipStream_t st);

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
    float eta2, xi2, beta2, thr;   // 2*eta, 2*xi, 2*beta, lambda/beta (FP32)
    float beta;
};
int grad_nblocks(int ny, int nx);
void launch_init_state(const Model& M, int ny, int nx, int batch, const float* muL,
                       const float* muH, float rho_min, float2* f, float* rho, float* t,
                       hipStream_t st);
void launch_grad(const Model& M, const ImgArgs& a, const float2* f, const float2* B,
                 const float* rho, const float* t, float2* dN, float2* dT, double* partials,
                 hipStream_t st);
void launch_update(const ImgArgs& a, const double* alpha, const float2* dN, float2* f,
                   float2* S, const float2* zq, hipStream_t st);
void launch_finish(const Model& M, int ny, int nx, int batch, const float* rho, const float* t,
                   float rho_min, double t_min, float* Z, float* rho_out, hipStream_t st);
void launch_split_f2(int n, int batch, const float2* f, float* a, float* b, hipStream_t st);
void launch_join_f2(int n, int batch, const float* a, const float* b, float2* f,
                    hipStream_t st);

// ---- PCG for (diag(w^2) + beta D^T D) x = w*g + beta D^T HT(D x0) -------------
struct PcgState {   // per-slice device scalars
    double rz, bnorm2, pq, alpha, beta_cg, cshift, rr;
    int done, iters, pad0, pad1;
};
struct PcgArgs {
    int ny, nx, batch;
    float beta, thr;
    double tol2;             // tol^2 on ||r||^2 / ||b||^2
    bool jacobi;
    float* x;                // in: x0 (also HT input), out: solution
    float *r, *z, *p0, *p1, *q, *w2;
    double* partials;        // [batch][nblocks][4]
    unsigned* counter;       // [batch]
    PcgState* st;            // [batch]
};
int pcg_nblocks(int ny, int nx);
// RHS from the model (t' subproblem): w = W/Ww, g = d_t/Ww from f pairs
void launch_pcg_init_model(const Model& M, const PcgArgs& a, const float2* f, hipStream_t st);
// RHS from explicit weight / g_tilde (dect_l0_step)
void launch_pcg_init_plain(const PcgArgs& a, const float* w, const float* g_tilde, float* h_out,
                           float* v_out, hipStream_t st);
// after an FFT preconditioner produced z from r: rz, p = z
void launch_pcg_after_prec_init(const PcgArgs& a, hipStream_t st);
void launch_pcg_matvec(const PcgArgs& a, int parity, bool first, hipStream_t st);
void launch_pcg_update(const PcgArgs& a, int parity, hipStream_t st);
void launch_pcg_after_prec(const PcgArgs& a, hipStream_t st);

}  // namespace dect
