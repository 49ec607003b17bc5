// Image-domain kernels of Algorithm 1 (sinogram form) on gfx950.
//
//   init_state  Algorithm 1 initialisation: per-pixel Cramer's rule for
//               (f1, f2) from the two attenuation images (eq. (1a,b)), synthesis
//               (2a,b) and the closed forms (4a,b) for rho_e and t' = Z^m/Zw^m,
//               all in FP64 per pixel.
//   grad        gradient of the f-subproblem (13a) with projection data terms,
//               fused: periodic forward differences, hard threshold (9), D^T,
//               coupling terms of (10), data gradient 2*eta*A^T(...), and the
//               three line-search partial sums.  The descent direction is
//               written in both padded layouts the projector reads.
//   update      f += alpha*d, combined residual sinograms += alpha*C^T C A d.
//   finish      Z = Zw*max(t', t_min)^(1/m), masked where rho_e < rho_min.
//   pcg_*       preconditioned CG for subproblem (13c):
//               (diag(w^2) + beta D^T D) t' = w*g + beta D^T HT(D t'^(k)).
#include <algorithm>
#include <cmath>

#include "dect_internal.h"
#include "device_util.h"

namespace dect {

// ---------------------------------------------------------------------------
struct ModelF {   // FP32/FP64 constants passed by value to kernels
    double C[2][2], Ms[2][2], psi[2], a[2], e1n, e2n, crho, Ww, cpb, Zw, m;
};

static ModelF to_dev(const Model& M) {
    ModelF r;
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            r.C[i][j] = M.C[i][j];
            r.Ms[i][j] = M.Ms[i][j];
        }
        r.psi[i] = M.psi[i];
        r.a[i] = M.a[i];
    }
    r.e1n = M.e1n;
    r.e2n = M.e2n;
    r.crho = M.crho;
    r.Ww = M.Ww;
    r.cpb = M.cpb;
    r.Zw = M.Zw;
    r.m = M.m;
    return r;
}

__global__ void k_init_state(ModelF M, int npix, const float* __restrict__ muL,
                             const float* __restrict__ muH, float rho_min, float2* __restrict__ f,
                             float* __restrict__ rho, float* __restrict__ t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (p >= npix) return;
    const size_t q = (size_t)z * npix + p;
    const double L = muL[q], H = muH[q];
    const double det = M.C[0][0] * M.C[1][1] - M.C[1][0] * M.C[0][1];
    const double f1 = (M.C[1][1] * L - M.C[0][1] * H) / det;
    const double f2 = (M.C[0][0] * H - M.C[1][0] * L) / det;
    const double M1 = M.Ms[0][0] * f1 + M.Ms[0][1] * f2;
    const double M2 = M.Ms[1][0] * f1 + M.Ms[1][1] * f2;
    const double r = (M1 * M.e1n - M2 * M.e2n) / M.crho;
    const double zwm = pow(M.Zw, M.m);
    const double W = M.cpb * zwm * (M1 / M.e2n - M2 / M.e1n);
    const bool guard = fabs(W) < 1e-6 * fabs(M.Ww) || r < (double)rho_min;
    const double tt = guard ? 1.0 : (M2 * M.psi[0] - M1 * M.psi[1]) / W;
    f[q] = make_float2((float)f1, (float)f2);
    rho[q] = (float)r;
    t[q] = (float)tt;
}

void launch_init_state(const Model& M, int ny, int nx, int batch, const float* muL,
                       const float* muH, float rho_min, float2* f, float* rho, float* t,
                       hipStream_t st) {
    const int npix = nx * ny;
    hipLaunchKernelGGL(k_init_state, dim3((npix + 255) / 256, batch), dim3(256), 0, st, to_dev(M),
                       npix, muL, muH, rho_min, f, rho, t);
}

// ---------------------------------------------------------------------------
// gradient assembly
// ---------------------------------------------------------------------------
int grad_nblocks(int ny, int nx) { return ((nx + 15) / 16) * ((ny + 15) / 16); }

struct GradConst {
    float ms00, ms01, ms10, ms11;   // synthesis matrix (barn)
    float a0, a1, psi0, psi1;       // coupling model T_j = rho (a_j t + psi_j)
};

__device__ __forceinline__ bool keep_grad(float dx, float dy, float thr) {
    return __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)) > thr;
}

__global__ __launch_bounds__(256) void k_grad(ImgArgs a, GradConst gc, PadLayout P,
                                              const float2* __restrict__ f,
                                              const float2* __restrict__ B,
                                              const float* __restrict__ rho,
                                              const float* __restrict__ t, void* __restrict__ dpad_v,
                                              double* __restrict__ partials) {
    float2* dpad = static_cast<float2*>(dpad_v);
    unsigned* dpad16 = static_cast<unsigned*>(dpad_v);
    __shared__ float2 fL[19][19];
    __shared__ float4 eL[18][18];
    __shared__ float2 dL[17][17];
    __shared__ double sh[4];
    const int nx = a.nx, ny = a.ny;
    const int z = blockIdx.z;
    if (a.beta_z) {
        const double b = a.beta_z[z];
        a.beta = (float)b;
        a.beta2 = (float)(2.0 * b);
        a.thr = (float)(a.lam / b);
    }
    const int i0 = blockIdx.y * 16, k0 = blockIdx.x * 16;
    const size_t npix = (size_t)nx * ny;
    const float2* fz = f + z * npix;
    for (int idx = threadIdx.x; idx < 19 * 19; idx += 256) {
        const int r = idx / 19, c = idx % 19;
        fL[r][c] = fz[(size_t)wrap(i0 - 1 + r, ny) * nx + wrap(k0 - 1 + c, nx)];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 18 * 18; idx += 256) {
        const int r = idx / 18, c = idx % 18;
        const float2 p = fL[r][c], pr = fL[r][c + 1], pd = fL[r + 1][c];
        const float dx1 = pr.x - p.x, dy1 = pd.x - p.x;
        const float dx2 = pr.y - p.y, dy2 = pd.y - p.y;
        const bool k1 = keep_grad(dx1, dy1, a.thr), k2 = keep_grad(dx2, dy2, a.thr);
        // D f - h: the thresholded-away gradients
        eL[r][c] = make_float4(k1 ? 0.f : dx1, k1 ? 0.f : dy1, k2 ? 0.f : dx2, k2 ? 0.f : dy2);
    }
    __syncthreads();
    double gg = 0.0, cq = 0.0, rr = 0.0;
    for (int idx = threadIdx.x; idx < 17 * 17; idx += 256) {
        const int r = idx / 17, c = idx % 17;
        const int gi = wrap(i0 + r, ny), gk = wrap(k0 + c, nx);
        const size_t gp = (size_t)gi * nx + gk;
        const float4 e = eL[r + 1][c + 1], el = eL[r + 1][c], eu = eL[r][c + 1];
        const float dte1 = (el.x - e.x) + (eu.y - e.y);
        const float dte2 = (el.z - e.z) + (eu.w - e.w);
        const float2 fp = fL[r + 1][c + 1];
        const float2 bp = B[z * npix + gp];
        const float rp = rho[z * npix + gp], tp = t[z * npix + gp];
        const float T1 = rp * fmaf(gc.a0, tp, gc.psi0);
        const float T2 = rp * fmaf(gc.a1, tp, gc.psi1);
        const float c1 = fmaf(gc.ms00, fp.x, gc.ms01 * fp.y) - T1;
        const float c2 = fmaf(gc.ms10, fp.x, gc.ms11 * fp.y) - T2;
        const float G1 = a.eta2 * bp.x + a.xi2 * fmaf(gc.ms00, c1, gc.ms10 * c2) + a.beta2 * dte1;
        const float G2 = a.eta2 * bp.y + a.xi2 * fmaf(gc.ms01, c1, gc.ms11 * c2) + a.beta2 * dte2;
        // the direction as stored (rounded to BF16 in that mode): the line
        // search and the update both use the stored value
        const float2 d = a.bf16 ? make_float2(bf16_round(-G1), bf16_round(-G2)) : make_float2(-G1, -G2);
        dL[r][c] = d;
        if (r < 16 && c < 16 && i0 + r < ny && k0 + c < nx) {
            gg -= (double)G1 * d.x + (double)G2 * d.y;   // -<grad, d>
            const double e1 = (double)gc.ms00 * d.x + (double)gc.ms01 * d.y;
            const double e2 = (double)gc.ms10 * d.x + (double)gc.ms11 * d.y;
            cq += e1 * e1 + e2 * e2;
            const size_t o = z * P.pair + (size_t)(i0 + r) * P.ldN + (k0 + c) + kPad;
            // reversed row (quarter-turn symmetric projection)
            const size_t orv = z * P.pair + P.offNR + (size_t)(i0 + r) * P.ldN + (nx - 1 - (k0 + c)) + kPad;
            if (a.bf16) {
                const unsigned pk = bf16x2_pack(d.x, d.y);
                dpad16[o] = pk;
                if (P.rev) dpad16[orv] = pk;
            } else {
                dpad[o] = d;
                if (P.rev) dpad[orv] = d;
            }
        }
    }
    __syncthreads();
    {
        const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
        if (i0 + ty < ny && k0 + tx < nx) {
            const float2 d = dL[ty][tx], dr = dL[ty][tx + 1], dd = dL[ty + 1][tx];
            const double ax = dr.x - d.x, ay = dd.x - d.x, bx = dr.y - d.y, by = dd.y - d.y;
            rr = ax * ax + ay * ay + bx * bx + by * by;
        }
        // transposed layout: row k, entries i
        if (k0 + ty < nx && i0 + tx < ny) {
            const size_t o = z * P.pair + P.offT + (size_t)(k0 + ty) * P.ldT + (i0 + tx) + kPad;
            const size_t orv = z * P.pair + P.offTR + (size_t)(k0 + ty) * P.ldT + (ny - 1 - (i0 + tx)) + kPad;
            const float2 d = dL[tx][ty];
            if (a.bf16) {
                const unsigned pk = bf16x2_pack(d.x, d.y);
                dpad16[o] = pk;
                if (P.rev) dpad16[orv] = pk;
            } else {
                dpad[o] = d;
                if (P.rev) dpad[orv] = d;
            }
        }
    }
    const int nblk = gridDim.x * gridDim.y;
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    const double s0 = block_sum<256>(gg, sh);
    const double s1 = block_sum<256>(cq, sh);
    const double s2 = block_sum<256>(rr, sh);
    if (threadIdx.x == 0) {
        double* o = partials + ((size_t)z * nblk + bid) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

void launch_grad(const Model& M, const ImgArgs& a, const PadLayout& P, const float2* f,
                 const float2* B, const float* rho, const float* t, void* dpad,
                 double* partials, hipStream_t st) {
    GradConst gc;
    gc.ms00 = (float)M.Ms[0][0];
    gc.ms01 = (float)M.Ms[0][1];
    gc.ms10 = (float)M.Ms[1][0];
    gc.ms11 = (float)M.Ms[1][1];
    gc.a0 = (float)M.a[0];
    gc.a1 = (float)M.a[1];
    gc.psi0 = (float)M.psi[0];
    gc.psi1 = (float)M.psi[1];
    dim3 grid((a.nx + 15) / 16, (a.ny + 15) / 16, a.batch);
    hipLaunchKernelGGL(k_grad, grid, dim3(256), 0, st, a, gc, P, f, B, rho, t, dpad, partials);
}

// ---------------------------------------------------------------------------
template <bool BF>
__global__ void k_update(int ny, int nx, PadLayout P, RayTable T, const double* __restrict__ alpha,
                         const void* __restrict__ dpad_v, float2* __restrict__ f,
                         void* __restrict__ S_v, const void* __restrict__ zq_v,
                         double* __restrict__ beta_z, const double* __restrict__ kappa_z) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    const size_t npix = (size_t)nx * ny;
    const float al = (float)alpha[z];
    if (idx == 0 && beta_z) beta_z[z] *= kappa_z[z];   // continuation: the slice's next beta
    if (idx < npix) {
        const int i = (int)(idx / nx), k = (int)(idx % nx);
        const size_t o = z * P.pair + (size_t)i * P.ldN + k + kPad;
        const float2 d = BF ? bf16x2_unpack(static_cast<const unsigned*>(dpad_v)[o])
                            : static_cast<const float2*>(dpad_v)[o];
        float2 v = f[z * npix + idx];
        v.x = fmaf(al, d.x, v.x);
        v.y = fmaf(al, d.y, v.y);
        f[z * npix + idx] = v;
        return;
    }
    const SliceDesc D = T.desc[T.desc_stride * z];
    const size_t r = idx - npix;
    if (r < (size_t)D.nv * D.nd) {
        const size_t o = (size_t)(D.sino0 + (long long)z * T.sino_zstride) + r;
        if constexpr (BF) {
            // the residuals accumulate alpha-scaled updates: stochastic
            // rounding, seeded by this slice's step alpha (new every iteration)
            const float2 q = bf16x2_unpack(static_cast<const unsigned*>(zq_v)[o]);
            unsigned* S = static_cast<unsigned*>(S_v);
            const float2 v = bf16x2_unpack(S[o]);
            const unsigned rb = fmix32((unsigned)r ^ seed_of(alpha[z]));
            S[o] = bf16x2_pack_sr(fmaf(al, q.x, v.x), fmaf(al, q.y, v.y), rb);
        } else {
            const float2 q = static_cast<const float2*>(zq_v)[o];
            float2* S = static_cast<float2*>(S_v);
            float2 v = S[o];
            v.x = fmaf(al, q.x, v.x);
            v.y = fmaf(al, q.y, v.y);
            S[o] = v;
        }
    }
}

void launch_update(const ImgArgs& a, const PadLayout& P, const RayTable& T, const double* alpha,
                   const void* dpad, float2* f, void* S, const void* zq, double* beta_z,
                   const double* kappa_z, hipStream_t st) {
    const size_t n = (size_t)a.nx * a.ny + (size_t)T.nv_max * T.nd_max;
    if (a.bf16)
        hipLaunchKernelGGL(k_update<true>, dim3((unsigned)((n + 255) / 256), a.batch), dim3(256), 0, st,
                           a.ny, a.nx, P, T, alpha, dpad, f, S, zq, beta_z, kappa_z);
    else
        hipLaunchKernelGGL(k_update<false>, dim3((unsigned)((n + 255) / 256), a.batch), dim3(256), 0,
                           st, a.ny, a.nx, P, T, alpha, dpad, f, S, zq, beta_z, kappa_z);
}

// state images rounded to BF16 (the values BF16 storage of f1, f2, rho_e, t'
// holds), stochastically: each iteration's small updates survive in
// expectation.  Seeded per slice by its beta (new every iteration).
__global__ void k_round_state(size_t npix, int batch, float2* __restrict__ f, float* __restrict__ rho,
                              float* __restrict__ t, const double* __restrict__ beta_z) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * (size_t)batch) return;
    const int z = (int)(i / npix);
    const unsigned seed = seed_of(beta_z[z]);
    const unsigned r1 = fmix32((unsigned)(2 * (i - z * npix)) ^ seed);
    const unsigned r2 = fmix32((unsigned)(2 * (i - z * npix) + 1) ^ seed);
    const float2 v = f[i];
    f[i] = make_float2(bf16_round_sr(v.x, r1), bf16_round_sr(v.y, r1 >> 16));
    rho[i] = bf16_round_sr(rho[i], r2);
    t[i] = bf16_round_sr(t[i], r2 >> 16);
}

__global__ void k_step_beta(double* beta_z, const double* kappa_z, int n) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z < n) beta_z[z] *= kappa_z[z];
}

void launch_step_beta(double* beta_z, const double* kappa_z, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_step_beta, dim3((n + 63) / 64), dim3(64), 0, st, beta_z, kappa_z, n);
}

void launch_round_state(size_t npix, int batch, float2* f, float* rho, float* t, const double* beta_z,
                        hipStream_t st) {
    const size_t n = npix * (size_t)batch;
    hipLaunchKernelGGL(k_round_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, npix, batch, f,
                       rho, t, beta_z);
}

__global__ void k_set_beta(double* beta_z, double* kappa_z, int z0, int n, double beta, double kappa) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        beta_z[z0 + i] = beta;
        kappa_z[z0 + i] = kappa;
    }
}

void launch_set_beta(double* beta_z, double* kappa_z, int z0, int n, double beta, double kappa,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_set_beta, dim3((n + 255) / 256), dim3(256), 0, st, beta_z, kappa_z, z0, n,
                       beta, kappa);
}

// ---------------------------------------------------------------------------
__global__ void k_finish(double Zw, double inv_m, int npix, const float* __restrict__ rho,
                         const float* __restrict__ t, float rho_min, double t_min,
                         float* __restrict__ Z, float* __restrict__ rho_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (p >= npix) return;
    const size_t q = (size_t)z * npix + p;
    const float r = rho[q];
    const double tt = fmax((double)t[q], t_min);
    const double zz = Zw * pow(tt, inv_m);
    if (Z) Z[q] = (r < rho_min) ? 0.f : (float)zz;
    if (rho_out) rho_out[q] = r;
}

void launch_finish(const Model& M, int ny, int nx, int batch, const float* rho, const float* t,
                   float rho_min, double t_min, float* Z, float* rho_out, hipStream_t st) {
    const int npix = nx * ny;
    hipLaunchKernelGGL(k_finish, dim3((npix + 255) / 256, batch), dim3(256), 0, st, M.Zw, 1.0 / M.m,
                       npix, rho, t, rho_min, t_min, Z, rho_out);
}

__global__ void k_split_f2(size_t n, const float2* __restrict__ f, float* __restrict__ a,
                           float* __restrict__ b) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 v = f[i];
    if (a) a[i] = v.x;
    if (b) b[i] = v.y;
}
__global__ void k_join_f2(size_t n, const float* __restrict__ a, const float* __restrict__ b,
                          float2* __restrict__ f) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    f[i] = make_float2(a[i], b[i]);
}
void launch_split_f2(int n, int batch, const float2* f, float* a, float* b, hipStream_t st) {
    const size_t tot = (size_t)n * batch;
    hipLaunchKernelGGL(k_split_f2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tot, f, a, b);
}
void launch_join_f2(int n, int batch, const float* a, const float* b, float2* f, hipStream_t st) {
    const size_t tot = (size_t)n * batch;
    hipLaunchKernelGGL(k_join_f2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tot, a, b, f);
}

// ---------------------------------------------------------------------------
// PCG for (diag(w^2) + beta L) x = b, L = D^T D (periodic 5-point)
// ---------------------------------------------------------------------------
constexpr int kPcgPix = 4;                     // pixels per thread
constexpr int kPcgBlock = 256 * kPcgPix;       // pixels per block

PcgParts pcg_parts(int ny, int nx) {
    PcgParts L;
    L.nblk = (nx * ny + kPcgBlock - 1) / kPcgBlock;
    const int tiles = ((ny + 15) / 16) * ((nx + 15) / 16);   // multigrid finest-level tiles
    L.nrz = std::max(std::max(L.nblk, ny), tiles);
    L.init0 = 0;
    L.init1 = L.init0 + L.nblk;
    L.pq = L.init1 + L.nblk;
    L.rz = L.pq + L.nblk;              // two parity slots of nrz
    L.rr = L.rz + 2 * (size_t)L.nrz;   // two parity slots of nblk
    L.dl = L.rr + 2 * (size_t)L.nblk;  // two parity slots of nrz
    L.sc = L.dl + 2 * (size_t)L.nrz;   // (gamma, alpha) x two parity slots
    L.zstride = L.sc + 4;
    return L;
}

// Sum of n partials in fixed order, broadcast to every thread of the block.
__device__ __forceinline__ double sum_parts(const double* a, int n, double* sh, double* bc) {
    const double s = block_sum_array<256>(a, n, 1, sh);
    if (threadIdx.x == 0) *bc = s;
    __syncthreads();
    const double r = *bc;
    __syncthreads();
    return r;
}

// D^T S at (i, k), S = thresholded-away gradients of x; `kept` = kept (h, v) at (i, k).
__device__ __forceinline__ float dt_small(const float* x, int i, int k, int ny, int nx, float thr,
                                          float2* kept) {
    const int ip = (i + 1 == ny) ? 0 : i + 1, im = (i == 0) ? ny - 1 : i - 1;
    const int kp = (k + 1 == nx) ? 0 : k + 1, km = (k == 0) ? nx - 1 : k - 1;
    const float c = x[(size_t)i * nx + k];
    const float r = x[(size_t)i * nx + kp], d = x[(size_t)ip * nx + k];
    const float l = x[(size_t)i * nx + km], dl = x[(size_t)ip * nx + km];
    const float u = x[(size_t)im * nx + k], ur = x[(size_t)im * nx + kp];
    float hx = r - c, hy = d - c;          // at (i, k)
    const bool kh = keep_grad(hx, hy, thr);
    if (kept) *kept = kh ? make_float2(hx, hy) : make_float2(0.f, 0.f);
    if (kh) hx = hy = 0.f;
    float lx = c - l, ly = dl - l;         // at (i, k-1)
    if (keep_grad(lx, ly, thr)) lx = ly = 0.f;
    float ux = ur - u, uy = c - u;         // at (i-1, k)
    if (keep_grad(ux, uy, thr)) ux = uy = 0.f;
    return (lx - hx) + (uy - hy);
}

template <bool MODEL>
__global__ __launch_bounds__(256) void k_pcg_init(PcgArgs a, ModelF M, const float2* __restrict__ f,
                                                  const float* __restrict__ w_in,
                                                  const float* __restrict__ g_in,
                                                  float* __restrict__ h_out, float* __restrict__ v_out) {
    __shared__ double sh[4];
    const int nx = a.nx, ny = a.ny, npix = nx * ny;
    const int z = blockIdx.y;
    slice_beta_thr(a, z);
    const size_t zo = (size_t)z * npix;
    double* P = a.parts + (size_t)z * a.L.zstride;
    const float* x = (a.x0 ? a.x0 : a.x) + zo;
    double rz = 0.0, rr = 0.0, ws = 0.0;
    for (int q = 0; q < kPcgPix; ++q) {
        const int p = blockIdx.x * kPcgBlock + q * 256 + threadIdx.x;
        if (p >= npix) break;
        const int i = p / nx, k = p % nx;
        double w, g;
        if (MODEL) {
            const float2 fv = f[zo + p];
            const double M1 = M.Ms[0][0] * fv.x + M.Ms[0][1] * fv.y;
            const double M2 = M.Ms[1][0] * fv.x + M.Ms[1][1] * fv.y;
            const double W = M.cpb * pow(M.Zw, M.m) * (M1 / M.e2n - M2 / M.e1n);
            w = W / M.Ww;
            g = (M2 * M.psi[0] - M1 * M.psi[1]) / M.Ww;
        } else {
            w = w_in[zo + p];
            g = g_in[zo + p];
        }
        float2 kept;
        const float dts = dt_small(x, i, k, ny, nx, a.thr, &kept);
        if (h_out) h_out[zo + p] = kept.x;
        if (v_out) v_out[zo + p] = kept.y;
        // r0 = b - A x0 = w (g - w x0) - beta D^T S(x0)
        const float r = (float)(w * (g - w * (double)x[p])) - a.beta * dts;
        if (a.x0) a.x[zo + p] = x[p];
        const float w2 = (float)(w * w);
        a.w2[zo + p] = w2;
        a.r[zo + p] = r;
        if (a.prec == PREC_JACOBI) {
            const float zz = r / (w2 + 4.f * a.beta);
            a.z[zo + p] = zz;
            rz += (double)r * zz;
        }
        rr += (double)r * r;
        ws += w2;
    }
    const double s_rz = block_sum<256>(rz, sh);
    const double s_rr = block_sum<256>(rr, sh);
    const double s_ws = block_sum<256>(ws, sh);
    if (threadIdx.x == 0) {
        P[a.L.init0 + blockIdx.x] = s_rr;               // ||r0||^2, the reference
        P[a.L.init1 + blockIdx.x] = s_ws;               // sum of w^2 (FFT shift)
        P[a.L.rr + a.L.nblk + blockIdx.x] = s_rr;       // parity slot 1: "previous" rr
        if (a.prec == PREC_JACOBI) P[a.L.rz + a.L.nrz + blockIdx.x] = s_rz;
        if (blockIdx.x == 0) {
            a.st[z].done = (a.active && !a.active[z]) ? 1 : 0;
            a.st[z].iters = 0;
        }
    }
}

void launch_pcg_init_model(const Model& M, const PcgArgs& a, const float2* f, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_init<true>, dim3(a.L.nblk, a.batch), dim3(256), 0, st, a, to_dev(M), f,
                       nullptr, nullptr, nullptr, nullptr);
}

void launch_pcg_init_plain(const PcgArgs& a, const float* w, const float* g_tilde, float* h_out,
                           float* v_out, hipStream_t st) {
    Model dummy{};
    hipLaunchKernelGGL(k_pcg_init<false>, dim3(a.L.nblk, a.batch), dim3(256), 0, st, a,
                       to_dev(dummy), nullptr, w, g_tilde, h_out, v_out);
}

// Iteration it, first half: convergence test, direction p = z + beta_cg p_prev,
// q = A p, <p, q> partials.
__global__ __launch_bounds__(256) void k_pcg_matvec(PcgArgs a, int it) {
    __shared__ double sh[4];
    __shared__ double shn[16];
    const int nx = a.nx, ny = a.ny, npix = nx * ny;
    const int z = blockIdx.y;
    slice_beta_thr(a, z);
    if (a.st[z].done) return;
    double* P = a.parts + (size_t)z * a.L.zstride;
    const int cur = it & 1, prev = cur ^ 1;
    const int nrz = a.nrz_used;
    double v[4] = {0.0, 0.0, 0.0, 0.0};   // rz_new, rr, r0^2, rz_old
    {
        const double* rzn = P + a.L.rz + (size_t)prev * a.L.nrz;
        const double* rzo = P + a.L.rz + (size_t)cur * a.L.nrz;
        const double* rrp = P + a.L.rr + (size_t)prev * a.L.nblk;
        const double* r0p = P + a.L.init0;
        for (int t = threadIdx.x; t < nrz; t += 256) {
            v[0] += rzn[t];
            if (it > 0) v[3] += rzo[t];
        }
        for (int t = threadIdx.x; t < a.L.nblk; t += 256) {
            v[1] += rrp[t];
            v[2] += r0p[t];
        }
    }
    block_sum_n<256, 4>(v, shn);
    const double rz_new = v[0], rr = v[1], r0 = v[2];
    if (rr <= a.tol2 * r0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.st[z].done = 1;
            a.st[z].iters = it;
        }
        return;
    }
    float bcg = 0.f;
    if (it > 0) bcg = v[3] > 0.0 ? (float)(rz_new / v[3]) : 0.f;
    const size_t zo = (size_t)z * npix;
    float* pout = (cur ? a.p1 : a.p0) + zo;
    const float* pin = (cur ? a.p0 : a.p1) + zo;
    const float* zz = a.z + zo;
    // all pixels' loads are issued before any result is used (the loop is
    // unrolled; out-of-range pixels read pixel 0 and are not stored)
    float pv[kPcgPix][5], wv[kPcgPix];
#pragma unroll
    for (int s = 0; s < kPcgPix; ++s) {
        int p = blockIdx.x * kPcgBlock + s * 256 + threadIdx.x;
        p = p < npix ? p : 0;
        const int i = p / nx, k = p % nx;
        const int ip = (i + 1 == ny) ? 0 : i + 1, im = (i == 0) ? ny - 1 : i - 1;
        const int kp = (k + 1 == nx) ? 0 : k + 1, km = (k == 0) ? nx - 1 : k - 1;
        const int nb[5] = {i * nx + k, i * nx + kp, i * nx + km, ip * nx + k, im * nx + k};
#pragma unroll
        for (int q = 0; q < 5; ++q) pv[s][q] = it == 0 ? zz[nb[q]] : fmaf(bcg, pin[nb[q]], zz[nb[q]]);
        wv[s] = a.w2[zo + p];
    }
    double pq = 0.0;
#pragma unroll
    for (int s = 0; s < kPcgPix; ++s) {
        const int p = blockIdx.x * kPcgBlock + s * 256 + threadIdx.x;
        if (p >= npix) continue;
        const float* u = pv[s];
        pout[p] = u[0];
        const float qv = fmaf(wv[s], u[0], a.beta * (4.f * u[0] - u[1] - u[2] - u[3] - u[4]));
        a.q[zo + p] = qv;
        pq += (double)u[0] * qv;
    }
    const double s_pq = block_sum<256>(pq, sh);
    if (threadIdx.x == 0) P[a.L.pq + blockIdx.x] = s_pq;
}

void launch_pcg_matvec(const PcgArgs& a, int it, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_matvec, dim3(a.L.nblk, a.batch), dim3(256), 0, st, a, it);
}

// Iteration it, second half: alpha = rz / <p, q>; x += alpha p; r -= alpha q;
// Jacobi: z = r / (w^2 + 4 beta) and <r, z> partials; <r, r> partials.
__global__ __launch_bounds__(256) void k_pcg_update(PcgArgs a, int it) {
    __shared__ double sh[4];
    __shared__ double shn[8];
    const int npix = a.nx * a.ny;
    const int z = blockIdx.y;
    slice_beta_thr(a, z);
    if (a.st[z].done) return;
    double* P = a.parts + (size_t)z * a.L.zstride;
    const int cur = it & 1, prev = cur ^ 1;
    const int nrz = a.nrz_used;
    double v[2] = {0.0, 0.0};   // rz, <p, q>
    for (int t = threadIdx.x; t < nrz; t += 256) v[0] += P[a.L.rz + (size_t)prev * a.L.nrz + t];
    for (int t = threadIdx.x; t < a.L.nblk; t += 256) v[1] += P[a.L.pq + t];
    block_sum_n<256, 2>(v, shn);
    const float al = v[1] > 0.0 ? (float)(v[0] / v[1]) : 0.f;
    const size_t zo = (size_t)z * npix;
    const float* pd = (cur ? a.p1 : a.p0) + zo;
    float xv[kPcgPix], pv[kPcgPix], qv[kPcgPix], rv[kPcgPix];
#pragma unroll
    for (int s = 0; s < kPcgPix; ++s) {   // loads first (see k_pcg_matvec)
        int p = blockIdx.x * kPcgBlock + s * 256 + threadIdx.x;
        p = p < npix ? p : 0;
        xv[s] = a.x[zo + p];
        pv[s] = pd[p];
        qv[s] = a.q[zo + p];
        rv[s] = a.r[zo + p];
    }
    double rzn = 0.0, rr = 0.0;
#pragma unroll
    for (int s = 0; s < kPcgPix; ++s) {
        const int p = blockIdx.x * kPcgBlock + s * 256 + threadIdx.x;
        if (p >= npix) continue;
        a.x[zo + p] = fmaf(al, pv[s], xv[s]);
        const float r = fmaf(-al, qv[s], rv[s]);
        a.r[zo + p] = r;
        rr += (double)r * r;
        if (a.prec == PREC_JACOBI) {
            const float zv = r / (a.w2[zo + p] + 4.f * a.beta);
            a.z[zo + p] = zv;
            rzn += (double)r * zv;
        }
    }
    const double s_rr = block_sum<256>(rr, sh);
    const double s_rz = block_sum<256>(rzn, sh);
    if (threadIdx.x == 0) {
        P[a.L.rr + (size_t)cur * a.L.nblk + blockIdx.x] = s_rr;
        if (a.prec == PREC_JACOBI) P[a.L.rz + (size_t)cur * a.L.nrz + blockIdx.x] = s_rz;
    }
}

void launch_pcg_update(const PcgArgs& a, int it, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_update, dim3(a.L.nblk, a.batch), dim3(256), 0, st, a, it);
}

__global__ __launch_bounds__(256) void k_pcg_check(PcgArgs a, int n) {
    __shared__ double sh[4];
    __shared__ double bc;
    const int z = blockIdx.y;
    if (a.st[z].done) return;
    const double* P = a.parts + (size_t)z * a.L.zstride;
    const int last = (n + 1) & 1;   // parity slot written by iteration n - 1 (or init for n = 0)
    const double rr = sum_parts(P + a.L.rr + (size_t)last * a.L.nblk, a.L.nblk, sh, &bc);
    const double r0 = sum_parts(P + a.L.init0, a.L.nblk, sh, &bc);
    if (threadIdx.x == 0) {
        a.st[z].iters = n;
        if (rr <= a.tol2 * r0) a.st[z].done = 1;
    }
}

void launch_pcg_check(const PcgArgs& a, int done_iters, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_check, dim3(1, a.batch), dim3(256), 0, st, a, done_iters);
}

void launch_pcg_fft_prec(const PcgArgs& a, int it, float2* scratch, hipStream_t st) {
    // z = (c + beta L)^-1 r with c = mean(w^2); <r, z> per row into the rz slot
    // of iteration it (it = -1: initial residual, slot 1)
    const int slot = it < 0 ? 1 : (it & 1);
    FftArgs fa;
    fa.src = FFT_SRC_PLAIN;
    fa.in = a.r;
    fa.out = a.z;
    fa.beta = a.beta;
    fa.beta_z = a.beta_z;
    fa.lam = a.lam;
    fa.c_parts = a.parts + a.L.init1;
    fa.c_n = a.L.nblk;
    fa.c_zstride = a.L.zstride;
    fa.c_scale = 1.0 / ((double)a.nx * a.ny);
    fa.skip = &a.st[0].done;
    fa.skip_zstride = sizeof(PcgState) / sizeof(int);
    fa.scale_w2 = a.w2;
    fa.dot_with = a.r;
    fa.dot_parts = a.parts + a.L.rz + (size_t)slot * a.L.nrz;
    fa.dot_zstride = a.L.zstride;
    launch_fft_solve(a.ny, a.nx, a.batch, fa, scratch, st);
}

}  // namespace dect
