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

__global__ __launch_bounds__(256) void k_grad(ImgArgs a, GradConst gc, const float2* __restrict__ f,
                                              const float2* __restrict__ B,
                                              const float* __restrict__ rho,
                                              const float* __restrict__ t, float2* __restrict__ dN,
                                              float2* __restrict__ dT, double* __restrict__ partials) {
    __shared__ float2 fL[19][19];
    __shared__ float4 eL[18][18];
    __shared__ float2 dL[17][17];
    __shared__ double sh[4];
    const int nx = a.nx, ny = a.ny;
    const int z = blockIdx.z;
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
        const float2 d = make_float2(-G1, -G2);
        dL[r][c] = d;
        if (r < 16 && c < 16 && i0 + r < ny && k0 + c < nx) {
            gg += (double)G1 * G1 + (double)G2 * G2;
            const double e1 = (double)gc.ms00 * d.x + (double)gc.ms01 * d.y;
            const double e2 = (double)gc.ms10 * d.x + (double)gc.ms11 * d.y;
            cq += e1 * e1 + e2 * e2;
            dN[z * (size_t)ny * (nx + 2) + (size_t)(i0 + r) * (nx + 2) + (k0 + c) + 1] = d;
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
        if (k0 + ty < nx && i0 + tx < ny)
            dT[z * (size_t)nx * (ny + 2) + (size_t)(k0 + ty) * (ny + 2) + (i0 + tx) + 1] = dL[tx][ty];
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

void launch_grad(const Model& M, const ImgArgs& a, const float2* f, const float2* B,
                 const float* rho, const float* t, float2* dN, float2* dT, double* partials,
                 hipStream_t st) {
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
    hipLaunchKernelGGL(k_grad, grid, dim3(256), 0, st, a, gc, f, B, rho, t, dN, dT, partials);
}

// ---------------------------------------------------------------------------
__global__ void k_update(int ny, int nx, size_t nray, const double* __restrict__ alpha,
                         const float2* __restrict__ dN, float2* __restrict__ f,
                         float2* __restrict__ S, const float2* __restrict__ zq) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    const size_t npix = (size_t)nx * ny;
    const float al = (float)alpha[z];
    if (idx < npix) {
        const int i = (int)(idx / nx), k = (int)(idx % nx);
        const float2 d = dN[z * (size_t)ny * (nx + 2) + (size_t)i * (nx + 2) + k + 1];
        float2 v = f[z * npix + idx];
        v.x = fmaf(al, d.x, v.x);
        v.y = fmaf(al, d.y, v.y);
        f[z * npix + idx] = v;
    } else if (idx < npix + nray) {
        const size_t r = idx - npix;
        const float2 q = zq[z * nray + r];
        float2 v = S[z * nray + r];
        v.x = fmaf(al, q.x, v.x);
        v.y = fmaf(al, q.y, v.y);
        S[z * nray + r] = v;
    }
}

void launch_update(const ImgArgs& a, const double* alpha, const float2* dN, float2* f, float2* S,
                   const float2* zq, hipStream_t st) {
    const size_t n = (size_t)a.nx * a.ny + (size_t)a.nv * a.nd;
    hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256), a.batch), dim3(256), 0, st, a.ny,
                       a.nx, (size_t)a.nv * a.nd, alpha, dN, f, S, zq);
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
int pcg_nblocks(int ny, int nx) { return (nx * ny + 255) / 256; }

// D^T HT(D x) at (i, k) from the 7 neighbours the two-sided stencil needs.
__device__ __forceinline__ float dt_ht(const float* x, int i, int k, int ny, int nx, float thr,
                                       float* h_here, float* v_here) {
    const int ip = (i + 1 == ny) ? 0 : i + 1, im = (i == 0) ? ny - 1 : i - 1;
    const int kp = (k + 1 == nx) ? 0 : k + 1, km = (k == 0) ? nx - 1 : k - 1;
    const float c = x[(size_t)i * nx + k];
    const float r = x[(size_t)i * nx + kp], d = x[(size_t)ip * nx + k];
    const float l = x[(size_t)i * nx + km], dl = x[(size_t)ip * nx + km];
    const float u = x[(size_t)im * nx + k], ur = x[(size_t)im * nx + kp];
    // (h, v) at (i, k)
    float hx = r - c, hy = d - c;
    if (!keep_grad(hx, hy, thr)) hx = hy = 0.f;
    // at (i, k-1)
    float lx = c - l, ly = dl - l;
    if (!keep_grad(lx, ly, thr)) lx = ly = 0.f;
    // at (i-1, k)
    float ux = ur - u, uy = c - u;
    if (!keep_grad(ux, uy, thr)) ux = uy = 0.f;
    if (h_here) *h_here = hx;
    if (v_here) *v_here = hy;
    return (lx - hx) + (uy - hy);
}

__device__ __forceinline__ float lap(const float* x, int i, int k, int ny, int nx) {
    const int ip = (i + 1 == ny) ? 0 : i + 1, im = (i == 0) ? ny - 1 : i - 1;
    const int kp = (k + 1 == nx) ? 0 : k + 1, km = (k == 0) ? nx - 1 : k - 1;
    return 4.f * x[(size_t)i * nx + k] - x[(size_t)i * nx + kp] - x[(size_t)i * nx + km] -
           x[(size_t)ip * nx + k] - x[(size_t)im * nx + k];
}

// finish of a PCG reduction in the last block: 4 partial sums per block
__device__ __forceinline__ void pcg_sums(const double* part, int nblk, double* sh, double out[4]) {
    for (int c = 0; c < 4; ++c) out[c] = block_sum_array<256>(part + c, nblk, 4, sh);
}

template <bool MODEL>
__global__ __launch_bounds__(256) void k_pcg_init(PcgArgs a, ModelF M, const float2* __restrict__ f,
                                                  const float* __restrict__ w_in,
                                                  const float* __restrict__ g_in,
                                                  float* __restrict__ h_out, float* __restrict__ v_out) {
    __shared__ double sh[4];
    const int nx = a.nx, ny = a.ny;
    const int npix = nx * ny;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    const size_t zo = (size_t)z * npix;
    double bb = 0.0, rz = 0.0, ws = 0.0, rr = 0.0;
    if (p < npix) {
        const int i = p / nx, k = p % nx;
        float w, wg;
        if (MODEL) {
            const float2 fv = f[zo + p];
            const double M1 = M.Ms[0][0] * fv.x + M.Ms[0][1] * fv.y;
            const double M2 = M.Ms[1][0] * fv.x + M.Ms[1][1] * fv.y;
            const double W = M.cpb * pow(M.Zw, M.m) * (M1 / M.e2n - M2 / M.e1n);
            const double dt = M2 * M.psi[0] - M1 * M.psi[1];
            w = (float)(W / M.Ww);
            wg = (float)((W / M.Ww) * (dt / M.Ww));
        } else {
            w = w_in[zo + p];
            wg = w * g_in[zo + p];
        }
        const float* x = a.x + zo;
        float hh, vv;
        const float b = wg + a.beta * dt_ht(x, i, k, ny, nx, a.thr, &hh, &vv);
        if (h_out) h_out[zo + p] = hh;
        if (v_out) v_out[zo + p] = vv;
        const float w2 = w * w;
        const float ax = fmaf(w2, x[p], a.beta * lap(x, i, k, ny, nx));
        const float r = b - ax;
        const float zz = r / (w2 + 4.f * a.beta);
        a.w2[zo + p] = w2;
        a.r[zo + p] = r;
        a.z[zo + p] = zz;
        a.p0[zo + p] = zz;
        bb = (double)b * b;
        rz = (double)r * zz;
        ws = w2;
        rr = (double)r * r;
    }
    const int nblk = gridDim.x;
    const double s0 = block_sum<256>(bb, sh), s1 = block_sum<256>(rz, sh);
    const double s2 = block_sum<256>(ws, sh), s3 = block_sum<256>(rr, sh);
    double* part = a.partials + (size_t)z * nblk * 4;
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = s0;
        part[blockIdx.x * 4 + 1] = s1;
        part[blockIdx.x * 4 + 2] = s2;
        part[blockIdx.x * 4 + 3] = s3;
    }
    if (last_block_arrive(a.counter + z, (unsigned)nblk)) {
        double s[4];
        pcg_sums(part, nblk, sh, s);
        if (threadIdx.x == 0) {
            PcgState& S = a.st[z];
            S.bnorm2 = s[0];
            S.rz = s[1];
            S.cshift = fmax(s[2] / (double)npix, 1e-12);
            S.rr = s[3];
            S.iters = 0;
            S.done = (s[0] == 0.0 || s[3] <= a.tol2 * s[0]) ? 1 : 0;
            S.alpha = 0.0;
            S.beta_cg = 0.0;
            S.pq = 0.0;
        }
    }
}

void launch_pcg_init_model(const Model& M, const PcgArgs& a, const float2* f, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_init<true>, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a,
                       to_dev(M), f, nullptr, nullptr, nullptr, nullptr);
}

void launch_pcg_init_plain(const PcgArgs& a, const float* w, const float* g_tilde, float* h_out,
                           float* v_out, hipStream_t st) {
    Model dummy{};
    hipLaunchKernelGGL(k_pcg_init<false>, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a,
                       to_dev(dummy), nullptr, w, g_tilde, h_out, v_out);
}

// after z = P^-1 r by the FFT preconditioner at initialisation: rz, p0 = z
__global__ __launch_bounds__(256) void k_pcg_prec_init(PcgArgs a) {
    __shared__ double sh[4];
    const int npix = a.nx * a.ny;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (a.st[z].done) return;
    const size_t zo = (size_t)z * npix;
    double rz = 0.0;
    if (p < npix) {
        const float zz = a.z[zo + p];
        a.p0[zo + p] = zz;
        rz = (double)a.r[zo + p] * zz;
    }
    const int nblk = gridDim.x;
    const double s = block_sum<256>(rz, sh);
    double* part = a.partials + (size_t)z * nblk * 4;
    if (threadIdx.x == 0) part[blockIdx.x * 4] = s;
    if (last_block_arrive(a.counter + z, (unsigned)nblk)) {
        const double t = block_sum_array<256>(part, nblk, 4, sh);
        if (threadIdx.x == 0) a.st[z].rz = t;
    }
}

void launch_pcg_after_prec_init(const PcgArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_prec_init, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a);
}

// q = A p with p = z + beta_cg * p_prev (first: p = p0); <p, q>; alpha = rz / <p, q>
__global__ __launch_bounds__(256) void k_pcg_matvec(PcgArgs a, int parity, int first) {
    __shared__ double sh[4];
    const int nx = a.nx, ny = a.ny, npix = nx * ny;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (a.st[z].done) return;
    const size_t zo = (size_t)z * npix;
    float* pout = (parity ? a.p1 : a.p0) + zo;
    const float* pin = (parity ? a.p0 : a.p1) + zo;
    const float* zz = a.z + zo;
    const float bc = (float)a.st[z].beta_cg;
    double pq = 0.0;
    if (p < npix) {
        const int i = p / nx, k = p % nx;
        const int ip = (i + 1 == ny) ? 0 : i + 1, im = (i == 0) ? ny - 1 : i - 1;
        const int kp = (k + 1 == nx) ? 0 : k + 1, km = (k == 0) ? nx - 1 : k - 1;
        const int nb[5] = {i * nx + k, i * nx + kp, i * nx + km, ip * nx + k, im * nx + k};
        float v[5];
        for (int q = 0; q < 5; ++q)
            v[q] = first ? pout[nb[q]] : fmaf(bc, pin[nb[q]], zz[nb[q]]);
        if (!first) pout[p] = v[0];
        const float qv = fmaf(a.w2[zo + p], v[0], a.beta * (4.f * v[0] - v[1] - v[2] - v[3] - v[4]));
        a.q[zo + p] = qv;
        pq = (double)v[0] * qv;
    }
    const int nblk = gridDim.x;
    const double s = block_sum<256>(pq, sh);
    double* part = a.partials + (size_t)z * nblk * 4;
    if (threadIdx.x == 0) part[blockIdx.x * 4 + 1] = s;
    if (last_block_arrive(a.counter + z, (unsigned)nblk)) {
        const double t = block_sum_array<256>(part + 1, nblk, 4, sh);
        if (threadIdx.x == 0) {
            a.st[z].pq = t;
            a.st[z].alpha = t > 0.0 ? a.st[z].rz / t : 0.0;
        }
    }
}

void launch_pcg_matvec(const PcgArgs& a, int parity, bool first, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_matvec, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a,
                       parity, first ? 1 : 0);
}

__device__ __forceinline__ void pcg_close(PcgArgs& a, int z, double rz_new, double rr) {
    PcgState& S = a.st[z];
    S.beta_cg = S.rz > 0.0 ? rz_new / S.rz : 0.0;
    S.rz = rz_new;
    S.rr = rr;
    S.iters += 1;
    if (rr <= a.tol2 * S.bnorm2) S.done = 1;
}

// x += alpha p; r -= alpha q; Jacobi: z = r / (w^2 + 4 beta), <r, z>, <r, r>
__global__ __launch_bounds__(256) void k_pcg_update(PcgArgs a, int parity) {
    __shared__ double sh[4];
    const int npix = a.nx * a.ny;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (a.st[z].done) return;
    const size_t zo = (size_t)z * npix;
    const float* pd = (parity ? a.p1 : a.p0) + zo;
    const float al = (float)a.st[z].alpha;
    double rz = 0.0, rr = 0.0;
    if (p < npix) {
        a.x[zo + p] = fmaf(al, pd[p], a.x[zo + p]);
        const float r = fmaf(-al, a.q[zo + p], a.r[zo + p]);
        a.r[zo + p] = r;
        rr = (double)r * r;
        if (a.jacobi) {
            const float zz = r / (a.w2[zo + p] + 4.f * a.beta);
            a.z[zo + p] = zz;
            rz = (double)r * zz;
        }
    }
    const int nblk = gridDim.x;
    const double s0 = block_sum<256>(rz, sh), s1 = block_sum<256>(rr, sh);
    double* part = a.partials + (size_t)z * nblk * 4;
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 2] = s0;
        part[blockIdx.x * 4 + 3] = s1;
    }
    if (last_block_arrive(a.counter + z, (unsigned)nblk)) {
        const double t0 = block_sum_array<256>(part + 2, nblk, 4, sh);
        const double t1 = block_sum_array<256>(part + 3, nblk, 4, sh);
        if (threadIdx.x == 0) {
            if (a.jacobi) {
                pcg_close(a, z, t0, t1);
            } else {
                a.st[z].rr = t1;
            }
        }
    }
}

void launch_pcg_update(const PcgArgs& a, int parity, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_update, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a,
                       parity);
}

// after the FFT preconditioner: <r, z> and close the iteration
__global__ __launch_bounds__(256) void k_pcg_after_prec(PcgArgs a) {
    __shared__ double sh[4];
    const int npix = a.nx * a.ny;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (a.st[z].done) return;
    const size_t zo = (size_t)z * npix;
    double rz = 0.0;
    if (p < npix) rz = (double)a.r[zo + p] * a.z[zo + p];
    const int nblk = gridDim.x;
    const double s = block_sum<256>(rz, sh);
    double* part = a.partials + (size_t)z * nblk * 4;
    if (threadIdx.x == 0) part[blockIdx.x * 4 + 2] = s;
    if (last_block_arrive(a.counter + z, (unsigned)nblk)) {
        const double t = block_sum_array<256>(part + 2, nblk, 4, sh);
        if (threadIdx.x == 0) pcg_close(a, z, t, a.st[z].rr);
    }
}

void launch_pcg_after_prec(const PcgArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_after_prec, dim3(pcg_nblocks(a.ny, a.nx), a.batch), dim3(256), 0, st, a);
}

}  // namespace dect
