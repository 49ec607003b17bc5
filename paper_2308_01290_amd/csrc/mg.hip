// Geometric multigrid V-cycle, the preconditioner of the PCG that solves the
// Z^m subproblem (13c): A = diag(c) + beta L, c = w^2, L = D^T D on the
// periodic pixel grid.
//
// Level l is the grid coarsened 2^l times per axis (cell-centred), with the
// operator re-discretised as A_l = diag(c_l) + (beta / 4^l) L and c_l the 2x2
// average of c_(l-1).  Transfers: restriction = 2x2 average, prolongation =
// piecewise constant (R = P^T / 4).  Smoothing: kMgNu damped-Jacobi sweeps
// (omega = 0.8) before the coarse correction, starting from zero, and kMgNu
// after it.  The first grid of at most 16 unknowns (else the coarsest one,
// an odd side, which must have at most 64) is solved exactly with A_l^-1,
// computed once per linear solve (FP64 Gauss-Jordan, symmetrised).  The V-cycle is therefore a fixed symmetric linear map, as
// PCG requires; it has no atomics, so it is deterministic.
//
// Kernels: levels whose larger side exceeds 32 run as tile kernels going
// down (sweeps, residual, restriction) and up (prolongation, sweeps), two
// levels per kernel where the finer one splits into 32 x 32 cores (its halo
// then covers both levels' sweeps, so the coarser level needs no launch of
// its own), else one level on 16 x 16 tiles with a kMgNu-pixel halo; the
// levels of 32 and below run in one workgroup per slice, one thread per
// pixel, neighbours exchanged through LDS.
#include <algorithm>

#include "dect_internal.h"
#include "device_util.h"

namespace dect {

constexpr float kOmega = 0.8f;
constexpr int kMgNu = 3;                  // smoothing sweeps before and after the correction
constexpr int kMgCoarseMax = 32;          // larger side at which the in-LDS kernel takes over
constexpr int kMgCoarseThreads = 1024;    // one thread per pixel of the largest in-LDS level

// one damped-Jacobi sweep at a pixel: x + omega (b - A x) / diag(A)
__device__ __forceinline__ float jac(float x, float b, float c, float beta, float nsum) {
    const float d = c + 4.f * beta;
    return x + kOmega * (b - (c * x + beta * (4.f * x - nsum))) / d;
}

MgPlan mg_plan(int ny, int nx) {
    MgPlan P;
    P.ny[0] = ny;
    P.nx[0] = nx;
    if (ny < 1 || nx < 1) return P;
    int l = 0;
    bool ok = true;
    while (std::max(ny, nx) > kMgCoarseMax) {   // tile levels
        if (ny % 16 || nx % 16 || l + 1 >= kMgMaxLevels) {
            ok = false;
            break;
        }
        ny /= 2;
        nx /= 2;
        ++l;
        ++P.ngrid;
        P.ny[l] = ny;
        P.nx[l] = nx;
    }
    P.ncoarse = 1;
    while (ok && ny % 2 == 0 && nx % 2 == 0 && l + 1 < kMgMaxLevels) {
        ny /= 2;
        nx /= 2;
        ++l;
        ++P.ncoarse;
        P.ny[l] = ny;
        P.nx[l] = nx;
    }
    P.nlev = l + 1;
    const int nc = ny * nx;
    ok = ok && nc <= kMgDenseMax;
    size_t off = 0;
    P.xs0 = off;
    off += (size_t)P.ny[0] * P.nx[0];
    for (int q = 1; q <= P.ngrid; ++q) {
        const size_t n = (size_t)P.ny[q] * P.nx[q];
        P.b[q] = off;
        off += n;
        P.c[q] = off;
        off += n;
        P.xs[q] = off;
        off += n;
        P.e[q] = off;
        off += n;
    }
    // in-LDS part: the first level with at most kMgExactMax unknowns (else the
    // coarsest, at most kMgDenseMax) is solved exactly, the ones above it
    // (at most kMgCoarseB) are smoothed; the set-up data computed once per
    // linear solve follows the tile levels
    const int g0 = P.ngrid;
    int q = 0;
    while (ok && q + 1 < P.ncoarse && P.ny[g0 + q] * P.nx[g0 + q] > kMgExactMax) ++q;
    ok = ok && q <= kMgCoarseB && P.ny[g0 + q] * P.nx[g0 + q] <= kMgDenseMax;
    if (ok) {
        P.ncb = q;
        P.ne = P.ny[g0 + q] * P.nx[g0 + q];
        for (int l = 0; l < P.ncb; ++l) {
            const size_t n = (size_t)P.ny[g0 + l] * P.nx[g0 + l];
            P.id[l] = off;
            off += n;
            P.cb[l] = off;   // (the first level's diagonal is the level buffer's own)
            off += l > 0 ? n : 0;
        }
        P.gi = off;
        off += (size_t)P.ne * P.ne;
    }
    P.zstride = (off + 63) & ~(size_t)63;
    // pair tile levels from the top: l and l + 1 share a kernel when level l
    // splits into 32 x 32 cores
    for (int q = 0; q < P.ngrid;) {
        if (q + 1 < P.ngrid && P.ny[q] % 32 == 0 && P.nx[q] % 32 == 0) {
            P.pair[q] = true;
            q += 2;
        } else {
            q += 1;
        }
    }
    P.nrz = P.ngrid == 0 ? 1 : (P.pair[0] ? (P.ny[0] / 32) * (P.nx[0] / 32)
                                          : (P.ny[0] / 16) * (P.nx[0] / 16));
    P.ok = ok;
    return P;
}

__device__ __forceinline__ bool mg_skip(const int* skip, size_t stride, int z) {
    return skip && skip[(size_t)z * stride];
}

__device__ __forceinline__ int wrap_near(int i, int n) {   // i in [-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// ---------------------------------------------------------------------------
// c_(l+1) = 2x2 average of c_l on the tile levels (once per linear solve)
// ---------------------------------------------------------------------------
__global__ void k_mg_restrict_c(const float* __restrict__ cf, size_t cf_zstride, int nyf, int nxf,
                                float* __restrict__ cc, size_t cc_zstride) {
    const int nyc = nyf / 2, nxc = nxf / 2;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (p >= nyc * nxc) return;
    const int i = p / nxc, k = p % nxc;
    const float* f = cf + (size_t)z * cf_zstride;
    const size_t a = (size_t)(2 * i) * nxf + 2 * k;
    cc[(size_t)z * cc_zstride + p] = 0.25f * (f[a] + f[a + 1] + f[a + nxf] + f[a + nxf + 1]);
}

// All G tile levels of the coefficient pyramid in one pass: a workgroup takes
// a 2^G x 2^G tile of level 0 and writes its cells of levels 1..G, each the
// mean of 2 x 2 cells of the level below, summed in k_mg_restrict_c's order
// (so the pyramid is the same bit for bit).  Needs every level an exact half
// of the one below.
struct MgCOffs {
    size_t c[kMgMaxLevels];   // per-slice offsets of the levels in the level buffer
};
template <int G>
__global__ __launch_bounds__(1 << (2 * G)) void k_mg_restrict_c_all(const float* __restrict__ c0,
                                                                    size_t c0_zstride, int nx0,
                                                                    float* __restrict__ mg,
                                                                    MgCOffs O, size_t zstride) {
    constexpr int T = 1 << G;   // tile side at level 0
    __shared__ float t[2][T * T];
    const int z = blockIdx.z;
    const int i0 = blockIdx.y * T, k0 = blockIdx.x * T;
    const int tid = threadIdx.x;
    t[0][tid] = c0[(size_t)z * c0_zstride + (size_t)(i0 + tid / T) * nx0 + (k0 + tid % T)];
    __syncthreads();
    int src = 0;
#pragma unroll
    for (int l = 1; l <= G; ++l) {
        const int n = T >> (l - 1), m = n >> 1, nxl = nx0 >> l;
        if (tid < m * m) {
            const int a = tid / m, b = tid % m;
            const float* f = t[src] + (2 * a) * n + 2 * b;
            const float v = 0.25f * (f[0] + f[1] + f[n] + f[n + 1]);
            t[src ^ 1][tid] = v;
            mg[O.c[l] + (size_t)z * zstride + (size_t)((i0 >> l) + a) * nxl + ((k0 >> l) + b)] = v;
        }
        __syncthreads();
        src ^= 1;
    }
}

// ---------------------------------------------------------------------------
// tile kernels: 16 x 16 pixels of one level per workgroup, two-pixel halo
// ---------------------------------------------------------------------------
struct MgLevel {
    const float* b;   // right-hand side
    const float* c;   // diagonal
    float* xs;        // saved pre-smoothed iterate (down: written, up: read)
    float* out;       // down: coarse right-hand side; up: this level's correction
    const float* e;   // up: coarse correction
    size_t zs_b, zs_c, zs_xs, zs_out, zs_e;   // per-slice strides (floats)
    int ny, nx;
    float beta;                  // beta of this level, or with beta_z:
    const double* beta_z;        //   beta_z[z] * scale (per-slice beta)
    float scale;
};

constexpr int kTile = 16;
constexpr int kW0 = kTile + 2 * kMgNu;   // tile with halo

// one sweep over the square [off, off + n)^2 of the halo tile: dst = J(src)
__device__ __forceinline__ void tile_sweep(const float (*X)[kW0 + 1], float (*Y)[kW0 + 1],
                                           const float (*B)[kW0 + 1], const float (*C)[kW0 + 1],
                                           int off, int n, float be) {
    for (int t = threadIdx.x; t < n * n; t += 256) {
        const int r = off + t / n, s = off + t % n;
        const float ns = X[r - 1][s] + X[r + 1][s] + X[r][s - 1] + X[r][s + 1];
        Y[r][s] = jac(X[r][s], B[r][s], C[r][s], be, ns);
    }
}

__global__ __launch_bounds__(256) void k_mg_down(MgLevel L, const int* skip, size_t skip_zstride) {
    __shared__ float B[kW0][kW0 + 1], C[kW0][kW0 + 1], X[2][kW0][kW0 + 1], R[kTile][kTile + 1];
    const int z = blockIdx.z;
    if (mg_skip(skip, skip_zstride, z)) return;
    const int i0 = blockIdx.y * kTile, k0 = blockIdx.x * kTile;
    const float* b = L.b + (size_t)z * L.zs_b;
    const float* c = L.c + (size_t)z * L.zs_c;
    const float be = L.beta_z ? (float)L.beta_z[z] * L.scale : L.beta;
    for (int t = threadIdx.x; t < kW0 * kW0; t += 256) {
        const int r = t / kW0, s = t % kW0;
        const size_t g = (size_t)wrap_near(i0 - kMgNu + r, L.ny) * L.nx +
                         wrap_near(k0 - kMgNu + s, L.nx);
        const float bb = b[g], cc = c[g];
        B[r][s] = bb;
        C[r][s] = cc;
        X[0][r][s] = kOmega * bb / (cc + 4.f * be);   // first sweep from zero
    }
    __syncthreads();
    // sweep q (q = 2..nu) reads X[q - 2 mod 2], writes X[q - 1 mod 2], valid on [q - 1, kW0 - q + 1)
#pragma unroll
    for (int q = 2; q <= kMgNu; ++q) {
        tile_sweep(X[(q - 2) & 1], X[(q - 1) & 1], B, C, q - 1, kW0 - 2 * (q - 1), be);
        __syncthreads();
    }
    const float (*Xn)[kW0 + 1] = X[(kMgNu - 1) & 1];   // sweep nu, valid on [nu - 1, kW0 - nu + 1)
    {
        const int r = threadIdx.x / kTile + kMgNu, s = threadIdx.x % kTile + kMgNu;
        const float x = Xn[r][s];
        const float ns = Xn[r - 1][s] + Xn[r + 1][s] + Xn[r][s - 1] + Xn[r][s + 1];
        R[r - kMgNu][s - kMgNu] = B[r][s] - (C[r][s] * x + be * (4.f * x - ns));
        L.xs[(size_t)z * L.zs_xs + (size_t)(i0 + r - kMgNu) * L.nx + (k0 + s - kMgNu)] = x;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int a = threadIdx.x / 8, q = threadIdx.x % 8;
        const float v = 0.25f * (R[2 * a][2 * q] + R[2 * a + 1][2 * q] + R[2 * a][2 * q + 1] +
                                 R[2 * a + 1][2 * q + 1]);
        L.out[(size_t)z * L.zs_out + (size_t)(i0 / 2 + a) * (L.nx / 2) + (k0 / 2 + q)] = v;
    }
}

// y0 = xs + P e; nu sweeps; out = y_nu.  With `dot` (finest level) the tile's
// <b, out> goes to dot[z*dot_zstride + tile].
__global__ __launch_bounds__(256) void k_mg_up(MgLevel L, const int* skip, size_t skip_zstride,
                                               double* dot, size_t dot_zstride) {
    __shared__ float B[kW0][kW0 + 1], C[kW0][kW0 + 1], Y[2][kW0][kW0 + 1];
    __shared__ double sh[4];
    const int z = blockIdx.z;
    if (mg_skip(skip, skip_zstride, z)) return;
    const int i0 = blockIdx.y * kTile, k0 = blockIdx.x * kTile;
    const float* b = L.b + (size_t)z * L.zs_b;
    const float* c = L.c + (size_t)z * L.zs_c;
    const float* xs = L.xs + (size_t)z * L.zs_xs;
    const float* e = L.e + (size_t)z * L.zs_e;
    const int nxc = L.nx / 2;
    const float be = L.beta_z ? (float)L.beta_z[z] * L.scale : L.beta;
    for (int t = threadIdx.x; t < kW0 * kW0; t += 256) {
        const int r = t / kW0, s = t % kW0;
        const int gi = wrap_near(i0 - kMgNu + r, L.ny), gk = wrap_near(k0 - kMgNu + s, L.nx);
        const size_t g = (size_t)gi * L.nx + gk;
        B[r][s] = b[g];
        C[r][s] = c[g];
        Y[0][r][s] = xs[g] + e[(size_t)(gi / 2) * nxc + gk / 2];
    }
    __syncthreads();
    // sweep q (q = 1..nu - 1) is valid on [q, kW0 - q)
#pragma unroll
    for (int q = 1; q < kMgNu; ++q) {
        tile_sweep(Y[(q - 1) & 1], Y[q & 1], B, C, q, kW0 - 2 * q, be);
        __syncthreads();
    }
    const float (*Yp)[kW0 + 1] = Y[(kMgNu - 1) & 1];
    const int r = threadIdx.x / kTile + kMgNu, s = threadIdx.x % kTile + kMgNu;
    const float ns = Yp[r - 1][s] + Yp[r + 1][s] + Yp[r][s - 1] + Yp[r][s + 1];
    const float y = jac(Yp[r][s], B[r][s], C[r][s], be, ns);
    L.out[(size_t)z * L.zs_out + (size_t)(i0 + r - kMgNu) * L.nx + (k0 + s - kMgNu)] = y;
    if (dot) {
        const double v = block_sum<256>((double)y * (double)B[r][s], sh);
        if (threadIdx.x == 0) dot[(size_t)z * dot_zstride + blockIdx.y * gridDim.x + blockIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// two-level tile kernels: 32 x 32 core at level l, 16 x 16 at level l + 1
// ---------------------------------------------------------------------------
constexpr int kCore2 = 32;
constexpr int kPairThreads = 512;
// down: level-l inputs on the core plus 3*nu (level l + 1 needs its residual on
// a nu halo, i.e. 2*nu at level l, whose sweeps need nu more)
constexpr int kD0 = kCore2 + 6 * kMgNu;
constexpr int kD1 = kTile + 2 * kMgNu;
// up: level l needs y0 on a nu halo, i.e. e_(l+1) on a ceil(nu/2) halo, whose
// sweeps need nu more at level l + 1
constexpr int kUh1 = (kMgNu + 1) / 2;
constexpr int kU0 = kCore2 + 2 * kMgNu;
constexpr int kU1 = kTile + 2 * (kUh1 + kMgNu);

template <int W>
__device__ __forceinline__ void pair_sweep(const float (*X)[W + 1], float (*Y)[W + 1],
                                           const float (*B)[W + 1], const float (*C)[W + 1],
                                           int off, int n, float be) {
    for (int t = threadIdx.x; t < n * n; t += kPairThreads) {
        const int r = off + t / n, s = off + t % n;
        const float ns = X[r - 1][s] + X[r + 1][s] + X[r][s - 1] + X[r][s + 1];
        Y[r][s] = jac(X[r][s], B[r][s], C[r][s], be, ns);
    }
}

struct MgPair {
    const float* b0;   // level l: right-hand side, diagonal, saved iterate, correction out
    const float* c0;
    float* xs0;
    float* e0;
    size_t zs_b0, zs_c0, zs_xs0, zs_e0;
    int ny0, nx0;
    float beta0;         // beta of level l, or with beta_z: beta_z[z] * scale
    const double* beta_z;
    float scale;
    float* b1;         // level l + 1 (level buffer): rhs (down writes), diagonal, saved iterate
    const float* c1;
    float* xs1;
    float* b2;         // down: level l + 2 rhs out
    const float* e2;   // up: level l + 2 correction in
    size_t zsm;        // per-slice stride of the level buffer
};

// The update of a pipelined PCG iteration, fused into the first kernel of the
// next V-cycle (UPD): every block reduces the iteration's partial sums to
// alpha and beta (or stops the slice when ||r_i||^2 <= tol2 ||r_0||^2), forms
// r_(i+1) = r_i - alpha (w_i + beta s_(i-1)) on its whole region (the core and
// the halo the sweeps need), uses it as the right-hand side, and writes
// p = u + beta p, s, x += alpha p, r_(i+1) and the ||r_(i+1)||^2 partial for
// its core.  r and s are double-buffered (neighbouring blocks read the old
// ones on their halos).
struct CgUpd {
    const float* r_old;   // r_i
    float* r_new;         // r_(i+1)
    const float* s_old;   // s_(i-1) (not read at i = 0)
    float* s_new;         // s_i
    const float* u;       // u_i = M r_i
    const float* w;       // w_i = A u_i
    float* p;             // in place on the core
    float* x;             // in place on the core
    size_t zs;            // per-slice stride of these images
    int it;
    double* parts;
    PcgParts L;
    int nrz_used;
    double tol2;
    PcgState* st;
    // k_mg_down2<false> only: 1 = first run the stopping test of the residual
    // that iteration `it`'s update wrote (see there)
    int check;
};

template <bool UPD>
__global__ __launch_bounds__(kPairThreads) void k_mg_down2(MgPair A, const int* skip,
                                                           size_t skip_zstride, CgUpd U) {
    __shared__ float B0[kD0][kD0 + 1], C0[kD0][kD0 + 1], X0[2][kD0][kD0 + 1];
    __shared__ float B1[kD1][kD1 + 1], C1[kD1][kD1 + 1], X1[2][kD1][kD1 + 1];
    __shared__ float R1[kTile][kTile + 1];
    __shared__ double shn[4 * (kPairThreads / kWave)];
    const int z = blockIdx.z;
    if (mg_skip(skip, skip_zstride, z)) return;
    if constexpr (!UPD) {
        // Second kernel of a pipelined PCG iteration's V-cycle: the stopping
        // test of r_(it+1), which the iteration's first kernel has just
        // written, reduced exactly as the next iteration's first kernel
        // would (same partial sums, same block reduction), so the decision
        // and the recorded count are the same; a converged slice stops here
        // and the rest of this V-cycle, whose result would go unused, skips.
        if (U.check) {
            const double* P = U.parts + (size_t)z * U.L.zstride;
            const double* rrc = P + U.L.rr + (size_t)(U.it & 1) * U.L.nblk;
            const double* r0p = P + U.L.init0;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int t = threadIdx.x; t < U.L.nblk; t += kPairThreads) {
                v[2] += rrc[t];
                v[3] += r0p[t];
            }
            block_sum_n<kPairThreads, 4>(v, shn);
            if (v[2] <= U.tol2 * v[3]) {   // the same decision in every block
                if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
                    U.st[z].done = 1;
                    U.st[z].iters = U.it + 1;
                }
                return;
            }
        }
    }
    constexpr int H0 = 3 * kMgNu;
    const int ny0 = A.ny0, nx0 = A.nx0, ny1 = ny0 / 2, nx1 = nx0 / 2;
    const int i0 = blockIdx.y * kCore2, k0 = blockIdx.x * kCore2;
    const float be0 = A.beta_z ? (float)A.beta_z[z] * A.scale : A.beta0, be1 = 0.25f * be0;
    const float* b0 = A.b0 + (size_t)z * A.zs_b0;
    const float* c0 = A.c0 + (size_t)z * A.zs_c0;
    // UPD: the region's r_i, w_i, s_(i-1) (and the core's u, p, x) are loaded
    // before the partial sums are reduced, so the two latencies overlap
    constexpr int kReg = (kD0 * kD0 + kPairThreads - 1) / kPairThreads;
    float lr[kReg], lw[kReg], ls[kReg], lu[kReg], lp[kReg], lx[kReg];
    if constexpr (UPD) {
#pragma unroll
        for (int m = 0; m < kReg; ++m) {
            const int t = threadIdx.x + m * kPairThreads;
            lr[m] = lw[m] = ls[m] = lu[m] = lp[m] = lx[m] = 0.f;
            if (t >= kD0 * kD0) continue;
            const int r = t / kD0, s = t % kD0;
            const size_t gz = (size_t)z * U.zs +
                              (size_t)wrap_near(i0 - H0 + r, ny0) * nx0 + wrap_near(k0 - H0 + s, nx0);
            lr[m] = U.r_old[gz];
            lw[m] = U.w[gz];
            if (U.it > 0) ls[m] = U.s_old[gz];
            if (r >= H0 && r < H0 + kCore2 && s >= H0 && s < H0 + kCore2) {
                lu[m] = U.u[gz];
                if (U.it > 0) lp[m] = U.p[gz];
                lx[m] = U.x[gz];
            }
        }
    }
    float af = 0.f, bf = 0.f;
    double* P = nullptr;
    int cur = 0;
    if constexpr (UPD) {
        P = U.parts + (size_t)z * U.L.zstride;
        cur = U.it & 1;
        const int prev = cur ^ 1;
        double v[4] = {0.0, 0.0, 0.0, 0.0};   // gamma_i, delta_i, ||r_i||^2, ||r_0||^2
        const double* g = P + U.L.rz + (size_t)cur * U.L.nrz;
        const double* d = P + U.L.dl + (size_t)cur * U.L.nrz;
        const double* rrp = P + U.L.rr + (size_t)prev * U.L.nblk;
        const double* r0p = P + U.L.init0;
        for (int t = threadIdx.x; t < U.nrz_used; t += kPairThreads) {
            v[0] += g[t];
            v[1] += d[t];
        }
        for (int t = threadIdx.x; t < U.L.nblk; t += kPairThreads) {
            v[2] += rrp[t];
            v[3] += r0p[t];
        }
        block_sum_n<kPairThreads, 4>(v, shn);
        const double gam = v[0], del = v[1];
        if (v[2] <= U.tol2 * v[3]) {   // the same decision in every block
            if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
                U.st[z].done = 1;
                U.st[z].iters = U.it;
            }
            return;
        }
        double beta = 0.0, alpha;
        if (U.it == 0) {
            alpha = del > 0.0 ? gam / del : 0.0;
        } else {
            const double gam_p = P[U.L.sc + 2 * prev], alpha_p = P[U.L.sc + 2 * prev + 1];
            beta = gam_p > 0.0 ? gam / gam_p : 0.0;
            const double den = alpha_p != 0.0 ? del - beta * gam / alpha_p : 0.0;
            alpha = den > 0.0 ? gam / den : 0.0;
        }
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            P[U.L.sc + 2 * cur] = gam;
            P[U.L.sc + 2 * cur + 1] = alpha;
        }
        af = (float)alpha;
        bf = (float)beta;
    }
    double rr = 0.0;
#pragma unroll
    for (int m = 0; m < kReg; ++m) {
        const int t = threadIdx.x + m * kPairThreads;
        if (t >= kD0 * kD0) continue;
        const int r = t / kD0, s = t % kD0;
        const size_t g = (size_t)wrap_near(i0 - H0 + r, ny0) * nx0 + wrap_near(k0 - H0 + s, nx0);
        float bb;
        if constexpr (UPD) {
            const float sn = fmaf(bf, ls[m], lw[m]);
            bb = fmaf(-af, sn, lr[m]);
            if (r >= H0 && r < H0 + kCore2 && s >= H0 && s < H0 + kCore2) {
                const size_t gz = (size_t)z * U.zs + g;
                const float pn = fmaf(bf, lp[m], lu[m]);
                U.p[gz] = pn;
                U.s_new[gz] = sn;
                U.x[gz] = fmaf(af, pn, lx[m]);
                U.r_new[gz] = bb;
                rr += (double)bb * bb;
            }
        } else {
            bb = b0[g];
        }
        const float cc = c0[g];
        B0[r][s] = bb;
        C0[r][s] = cc;
        X0[0][r][s] = kOmega * bb / (cc + 4.f * be0);
    }
    if constexpr (UPD) {
        const double s_rr = block_sum<kPairThreads>(rr, shn);
        if (threadIdx.x == 0) P[U.L.rr + (size_t)cur * U.L.nblk + blockIdx.y * gridDim.x + blockIdx.x] = s_rr;
    }
    const float* c1 = A.c1 + (size_t)z * A.zsm;
    for (int t = threadIdx.x; t < kD1 * kD1; t += kPairThreads) {
        const int r = t / kD1, s = t % kD1;
        C1[r][s] = c1[(size_t)wrap_near(i0 / 2 - kMgNu + r, ny1) * nx1 +
                      wrap_near(k0 / 2 - kMgNu + s, nx1)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 2; q <= kMgNu; ++q) {
        pair_sweep<kD0>(X0[(q - 2) & 1], X0[(q - 1) & 1], B0, C0, q - 1, kD0 - 2 * (q - 1), be0);
        __syncthreads();
    }
    // level-l residual on [nu, kD0 - nu) into the free buffer; saved iterate on the core
    const float (*Xn)[kD0 + 1] = X0[(kMgNu - 1) & 1];
    float (*Rr)[kD0 + 1] = X0[kMgNu & 1];
    constexpr int nr = kD0 - 2 * kMgNu;
    float* xs0 = A.xs0 + (size_t)z * A.zs_xs0;
    for (int t = threadIdx.x; t < nr * nr; t += kPairThreads) {
        const int r = kMgNu + t / nr, s = kMgNu + t % nr;
        const float x = Xn[r][s];
        const float ns = Xn[r - 1][s] + Xn[r + 1][s] + Xn[r][s - 1] + Xn[r][s + 1];
        Rr[r][s] = B0[r][s] - (C0[r][s] * x + be0 * (4.f * x - ns));
        if (r >= H0 && r < H0 + kCore2 && s >= H0 && s < H0 + kCore2)
            xs0[(size_t)(i0 + r - H0) * nx0 + (k0 + s - H0)] = x;
    }
    __syncthreads();
    // level l + 1 on [-nu, 16 + nu): rhs = restricted residual, first sweep from zero
    float* b1 = A.b1 + (size_t)z * A.zsm;
    for (int t = threadIdx.x; t < kD1 * kD1; t += kPairThreads) {
        const int r = t / kD1, s = t % kD1;
        const int a = kMgNu + 2 * r, c = kMgNu + 2 * s;
        const float v = 0.25f * (Rr[a][c] + Rr[a + 1][c] + Rr[a][c + 1] + Rr[a + 1][c + 1]);
        B1[r][s] = v;
        X1[0][r][s] = kOmega * v / (C1[r][s] + 4.f * be1);
        if (r >= kMgNu && r < kMgNu + kTile && s >= kMgNu && s < kMgNu + kTile)
            b1[(size_t)(i0 / 2 + r - kMgNu) * nx1 + (k0 / 2 + s - kMgNu)] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 2; q <= kMgNu; ++q) {
        pair_sweep<kD1>(X1[(q - 2) & 1], X1[(q - 1) & 1], B1, C1, q - 1, kD1 - 2 * (q - 1), be1);
        __syncthreads();
    }
    const float (*Xm)[kD1 + 1] = X1[(kMgNu - 1) & 1];
    float* xs1 = A.xs1 + (size_t)z * A.zsm;
    if (threadIdx.x < kTile * kTile) {
        const int r = threadIdx.x / kTile + kMgNu, s = threadIdx.x % kTile + kMgNu;
        const float x = Xm[r][s];
        const float ns = Xm[r - 1][s] + Xm[r + 1][s] + Xm[r][s - 1] + Xm[r][s + 1];
        R1[r - kMgNu][s - kMgNu] = B1[r][s] - (C1[r][s] * x + be1 * (4.f * x - ns));
        xs1[(size_t)(i0 / 2 + r - kMgNu) * nx1 + (k0 / 2 + s - kMgNu)] = x;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int a = threadIdx.x / 8, q = threadIdx.x % 8;
        const float v = 0.25f * (R1[2 * a][2 * q] + R1[2 * a + 1][2 * q] + R1[2 * a][2 * q + 1] +
                                 R1[2 * a + 1][2 * q + 1]);
        A.b2[(size_t)z * A.zsm + (size_t)(i0 / 4 + a) * (nx1 / 2) + (k0 / 4 + q)] = v;
    }
}

// up: level l + 1 from its saved iterate and e_(l+2), then level l; with `dot`
// (finest level) the block's <b0, out> goes to dot[z*dot_zstride + block].
// W (finest level of a pipelined PCG): the level-l region carries one more
// halo pixel, so the last sweep yields u = out on the core plus one ring and
// the block also writes w = A u on the core (A = diag(c0) + beta L) and the
// partial sum <u, w> to dot2.  u is the same as without W, bit for bit.
template <bool W>
__global__ __launch_bounds__(kPairThreads) void k_mg_up2(MgPair A, const int* skip,
                                                         size_t skip_zstride, double* dot,
                                                         size_t dot_zstride, float* wout,
                                                         double* dot2) {
    constexpr int H0 = W ? kMgNu + 1 : kMgNu;   // level-l halo of the loaded region
    constexpr int U0 = kCore2 + 2 * H0;
    __shared__ float B0[U0][U0 + 1], C0[U0][U0 + 1], Y0[2][U0][U0 + 1];
    __shared__ float B1[kU1][kU1 + 1], C1[kU1][kU1 + 1], Y1[2][kU1][kU1 + 1];
    __shared__ double sh[kPairThreads / kWave];
    static_assert((H0 + 1) / 2 == kUh1, "level l + 1 region covers the parents of the level-l region");
    const int z = blockIdx.z;
    if (mg_skip(skip, skip_zstride, z)) return;
    const int ny0 = A.ny0, nx0 = A.nx0, ny1 = ny0 / 2, nx1 = nx0 / 2, nx2 = nx1 / 2;
    const int i0 = blockIdx.y * kCore2, k0 = blockIdx.x * kCore2;
    const float be0 = A.beta_z ? (float)A.beta_z[z] * A.scale : A.beta0, be1 = 0.25f * be0;
    constexpr int H1 = kUh1 + kMgNu;   // level-(l+1) halo of the loaded region
    {
        const float* b1 = A.b1 + (size_t)z * A.zsm;
        const float* c1 = A.c1 + (size_t)z * A.zsm;
        const float* xs1 = A.xs1 + (size_t)z * A.zsm;
        const float* e2 = A.e2 + (size_t)z * A.zsm;
        for (int t = threadIdx.x; t < kU1 * kU1; t += kPairThreads) {
            const int r = t / kU1, s = t % kU1;
            const int gi = wrap_near(i0 / 2 - H1 + r, ny1), gk = wrap_near(k0 / 2 - H1 + s, nx1);
            const size_t g = (size_t)gi * nx1 + gk;
            B1[r][s] = b1[g];
            C1[r][s] = c1[g];
            Y1[0][r][s] = xs1[g] + e2[(size_t)(gi / 2) * nx2 + gk / 2];
        }
        const float* b0 = A.b0 + (size_t)z * A.zs_b0;
        const float* c0 = A.c0 + (size_t)z * A.zs_c0;
        for (int t = threadIdx.x; t < U0 * U0; t += kPairThreads) {
            const int r = t / U0, s = t % U0;
            const size_t g = (size_t)wrap_near(i0 - H0 + r, ny0) * nx0 + wrap_near(k0 - H0 + s, nx0);
            B0[r][s] = b0[g];
            C0[r][s] = c0[g];
        }
    }
    __syncthreads();
    // level l + 1: nu sweeps; sweep q is valid on [q, kU1 - q)
#pragma unroll
    for (int q = 1; q <= kMgNu; ++q) {
        pair_sweep<kU1>(Y1[(q - 1) & 1], Y1[q & 1], B1, C1, q, kU1 - 2 * q, be1);
        __syncthreads();
    }
    const float (*E1)[kU1 + 1] = Y1[kMgNu & 1];   // e_(l+1), valid on [nu, kU1 - nu)
    // level l: y0 = xs0 + P e_(l+1) on [-H0, 32 + H0)
    const float* xs0 = A.xs0 + (size_t)z * A.zs_xs0;
    for (int t = threadIdx.x; t < U0 * U0; t += kPairThreads) {
        const int r = t / U0, s = t % U0;
        const size_t g = (size_t)wrap_near(i0 - H0 + r, ny0) * nx0 + wrap_near(k0 - H0 + s, nx0);
        // parent of level-l row i0 - H0 + r, relative to i0 / 2, plus the region offset H1
        const int pr = ((r + H0) >> 1) - H0 + H1, ps = ((s + H0) >> 1) - H0 + H1;
        Y0[0][r][s] = xs0[g] + E1[pr][ps];
    }
    __syncthreads();
#pragma unroll
    for (int q = 1; q < kMgNu; ++q) {
        pair_sweep<U0>(Y0[(q - 1) & 1], Y0[q & 1], B0, C0, q, U0 - 2 * q, be0);
        __syncthreads();
    }
    const float (*Yp)[U0 + 1] = Y0[(kMgNu - 1) & 1];
    float* out = A.e0 + (size_t)z * A.zs_e0;
    double part = 0.0, part2 = 0.0;
    if constexpr (!W) {
        for (int t = threadIdx.x; t < kCore2 * kCore2; t += kPairThreads) {
            const int r = kMgNu + t / kCore2, s = kMgNu + t % kCore2;
            const float ns = Yp[r - 1][s] + Yp[r + 1][s] + Yp[r][s - 1] + Yp[r][s + 1];
            const float y = jac(Yp[r][s], B0[r][s], C0[r][s], be0, ns);
            out[(size_t)(i0 + r - kMgNu) * nx0 + (k0 + s - kMgNu)] = y;
            part += (double)y * (double)B0[r][s];
        }
    } else {
        // last sweep on the core and one ring, into the free buffer
        float (*Yu)[U0 + 1] = Y0[kMgNu & 1];
        pair_sweep<U0>(Yp, Yu, B0, C0, kMgNu, U0 - 2 * kMgNu, be0);
        __syncthreads();
        float* wo = wout + (size_t)z * A.zs_e0;
        for (int t = threadIdx.x; t < kCore2 * kCore2; t += kPairThreads) {
            const int r = H0 + t / kCore2, s = H0 + t % kCore2;
            const float u = Yu[r][s];
            // the PCG operator as k_pcg_matvec evaluates it
            const float wv = fmaf(C0[r][s], u,
                                  be0 * (4.f * u - Yu[r][s + 1] - Yu[r][s - 1] - Yu[r + 1][s] - Yu[r - 1][s]));
            const size_t g = (size_t)(i0 + r - H0) * nx0 + (k0 + s - H0);
            out[g] = u;
            wo[g] = wv;
            part += (double)u * (double)B0[r][s];
            part2 += (double)u * (double)wv;
        }
    }
    if (dot) {
        const double v = block_sum<kPairThreads>(part, sh);
        if (threadIdx.x == 0) dot[(size_t)z * dot_zstride + blockIdx.y * gridDim.x + blockIdx.x] = v;
    }
    if (W && dot2) {
        const double v = block_sum<kPairThreads>(part2, sh);
        if (threadIdx.x == 0) dot2[(size_t)z * dot_zstride + blockIdx.y * gridDim.x + blockIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// the in-LDS part: all levels with larger side <= 32, one workgroup per slice.
// The levels above the exact one (at most kMgCoarseB) are smoothed with one
// thread per pixel (pixel values in registers, neighbours exchanged through
// LDS); the exact level is solved with its inverse, computed once per linear
// solve by k_mg_coarse_setup together with the inverse diagonals
// omega / diag(A_l) of the smoothed levels.
// ---------------------------------------------------------------------------
struct MgCoarse {
    const float* b;       // right-hand side of the first in-LDS level
    const float* c;       // its diagonal
    float* e;             // its correction (output)
    size_t zs_b, zs_c, zs_e;
    const float* aux;     // per-slice set-up data (level buffer), stride zs_aux:
    size_t zs_aux;        //   omega / diag and diagonal of smoothed level q at
    size_t o_id[kMgCoarseB], o_c[kMgCoarseB], o_g;   // o_id[q], o_c[q] (q >= 1), inverse at o_g
    float beta;           // beta of the first in-LDS level, or with beta_z:
    const double* beta_z; //   beta_z[z] * scale
    float scale;
    int ncb, ne;          // smoothed levels; unknowns of the exact level
    int ny[kMgCoarseB + 1], nx[kMgCoarseB + 1];   // levels 0..ncb (repeated past ncb)
    double* dot;          // optional <b, e> (when this is the finest level)
    size_t dot_zstride;
};

// one pixel of a smoothed in-LDS level, owned by thread t < ny * nx
struct MgPx {
    bool on;
    int self, nb[4], par;   // own index, periodic neighbours, parent on the next level
    float b, c, id, xs;     // rhs, diagonal, omega / (c + 4 beta), saved pre-smoothed iterate
};

__device__ __forceinline__ MgPx mg_px(int t, int ny, int nx, int nxc) {
    MgPx P;
    P.on = t < ny * nx;
    const int i = P.on ? t / nx : 0, k = P.on ? t - i * nx : 0;
    const int ip = i + 1 == ny ? 0 : i + 1, im = i == 0 ? ny - 1 : i - 1;
    const int kp = k + 1 == nx ? 0 : k + 1, km = k == 0 ? nx - 1 : k - 1;
    P.self = t;
    P.nb[0] = ip * nx + k;
    P.nb[1] = im * nx + k;
    P.nb[2] = i * nx + kp;
    P.nb[3] = i * nx + km;
    P.par = (i / 2) * nxc + k / 2;
    P.b = P.c = P.id = P.xs = 0.f;
    return P;
}

constexpr int kMgLdsPx = kMgCoarseMax * kMgCoarseMax;   // pixels of the largest in-LDS level

// Ping-pong exchange buffers: publish() writes this thread's value into the
// other buffer and waits for the workgroup; every read of a published buffer
// comes before the next publish, so a buffer is rewritten only after the
// barrier that follows all reads of its previous contents.
struct MgX {
    float (*X)[kMgLdsPx];
    int cur;
    __device__ void publish(const MgPx& P, float v) {
        cur ^= 1;
        if (P.on) X[cur][P.self] = v;
        __syncthreads();
    }
    __device__ float nsum(const MgPx& P) const {
        return X[cur][P.nb[0]] + X[cur][P.nb[1]] + X[cur][P.nb[2]] + X[cur][P.nb[3]];
    }
};

__device__ __forceinline__ float mg_apply(const MgPx& P, float x, float beta, float ns) {
    return fmaf(P.c, x, beta * (4.f * x - ns));   // (A x) at the pixel
}

// down at a smoothed level: kMgNu sweeps from zero, then the residual is
// published (the caller restricts it before its next publish)
__device__ __forceinline__ void mg_lds_down(MgPx& P, float beta, MgX& E) {
    float x = P.id * P.b;   // first sweep from zero
#pragma unroll
    for (int q = 2; q <= kMgNu; ++q) {
        E.publish(P, x);
        if (P.on) x = fmaf(P.id, P.b - mg_apply(P, x, beta, E.nsum(P)), x);
    }
    P.xs = x;
    E.publish(P, x);
    const float r = P.on ? P.b - mg_apply(P, x, beta, E.nsum(P)) : 0.f;
    E.publish(P, r);
}

// 2 x 2 average of the published level (row length nxf) at coarse pixel t
__device__ __forceinline__ float mg_lds_restrict(const MgX& E, int t, int nxf, int nxc) {
    const int i = t / nxc, k = t - i * nxc;
    const float* R = E.X[E.cur];
    const int a = (2 * i) * nxf + 2 * k;
    return 0.25f * (R[a] + R[a + 1] + R[a + nxf] + R[a + nxf + 1]);
}

// up at a smoothed level: y0 = xs + P e_c, then kMgNu sweeps; returns y
__device__ __forceinline__ float mg_lds_up(const MgPx& P, float beta, float ec, MgX& E) {
    float y = P.xs + ec;
#pragma unroll
    for (int q = 1; q <= kMgNu; ++q) {
        E.publish(P, y);
        if (P.on) y = fmaf(P.id, P.b - mg_apply(P, y, beta, E.nsum(P)), y);
    }
    return y;
}

__global__ __launch_bounds__(kMgCoarseThreads) void k_mg_coarse(MgCoarse G, const int* skip,
                                                                 size_t skip_zstride) {
    __shared__ float X[2][kMgLdsPx];
    __shared__ float BE[kMgDenseMax], EE[kMgDenseMax];
    __shared__ double sh[kMgCoarseThreads / kWave];
    const int z = blockIdx.x;
    if (mg_skip(skip, skip_zstride, z)) return;
    const int t = threadIdx.x;
    const float beta0 = G.beta_z ? (float)G.beta_z[z] * G.scale : G.beta;
    const float* aux = G.aux + (size_t)z * G.zs_aux;
    const int ncb = G.ncb, ne = G.ne;
    // row t / 16 of the exact level's inverse, columns t % 16 + 16 m
    const int grow = t >> 4, gpart = t & 15;
    float gv[kMgDenseMax / 16];
#pragma unroll
    for (int m = 0; m < kMgDenseMax / 16; ++m) {
        const int j = gpart + 16 * m;
        gv[m] = grow < ne && j < ne ? aux[G.o_g + (size_t)grow * ne + j] : 0.f;
    }
    MgX E{X, 1};
    MgPx P[kMgCoarseB];
    float bl[kMgCoarseB];
#pragma unroll
    for (int q = 0; q < kMgCoarseB; ++q) {
        P[q] = mg_px(t, G.ny[q], G.nx[q], G.nx[q + 1]);
        P[q].on = P[q].on && q < ncb;
        bl[q] = q == 0 ? beta0 : 0.25f * bl[q - 1];
        if (P[q].on) {
            P[q].c = q == 0 ? G.c[(size_t)z * G.zs_c + t] : aux[G.o_c[q] + t];
            P[q].id = aux[G.o_id[q] + t];
        }
    }
    const float b0 = t < G.ny[0] * G.nx[0] ? G.b[(size_t)z * G.zs_b + t] : 0.f;
    P[0].b = b0;
    float be = b0;   // rhs of the exact level at pixel t (t < ne)
#pragma unroll
    for (int q = 0; q < kMgCoarseB; ++q) {
        if (q >= ncb) break;   // uniform
        if (q > 0 && P[q].on) P[q].b = mg_lds_restrict(E, t, G.nx[q - 1], G.nx[q]);
        mg_lds_down(P[q], bl[q], E);
        if (q + 1 == ncb) be = t < ne ? mg_lds_restrict(E, t, G.nx[q], G.nx[q + 1]) : 0.f;
    }
    if (t < kMgDenseMax) BE[t] = t < ne ? be : 0.f;
    __syncthreads();
    {
        // e = A_e^-1 b_e: 16 lanes per row, a fixed reduction order
        float acc = 0.f;
#pragma unroll
        for (int m = 0; m < kMgDenseMax / 16; ++m) acc = fmaf(gv[m], BE[gpart + 16 * m], acc);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (gpart == 0 && grow < kMgDenseMax) EE[grow] = acc;
    }
    __syncthreads();
    float y = t < ne ? EE[t] : 0.f;   // correction at pixel t of the current level
#pragma unroll
    for (int q = kMgCoarseB - 1; q >= 0; --q) {
        if (q >= ncb) continue;   // uniform
        const float ec = P[q].on ? (q + 1 == ncb ? EE[P[q].par] : E.X[E.cur][P[q].par]) : 0.f;
        y = mg_lds_up(P[q], bl[q], ec, E);
        if (q > 0) E.publish(P[q], y);
    }
    double dot = 0.0;
    if (t < G.ny[0] * G.nx[0]) {
        G.e[(size_t)z * G.zs_e + t] = y;
        dot = (double)y * (double)b0;
    }
    if (G.dot) {
        const double v = block_sum<kMgCoarseThreads>(dot, sh);
        if (t == 0) G.dot[(size_t)z * G.dot_zstride] = v;
    }
}

// Once per linear solve: the diagonals of the in-LDS levels (2 x 2 averages
// of the first one), omega / diag(A_l) of the smoothed ones, and the exact
// level's inverse A_e^-1 by Gauss-Jordan elimination in FP64 (A_e is SPD; a
// pivot that has fallen below 1e-12 of its diagonal, a numerically singular
// direction, is dropped from the inverse), symmetrised and stored in FP32.
struct MgCoarseSetup {
    const float* c;       // diagonal of the first in-LDS level
    size_t zs_c;
    float* aux;
    size_t zs_aux, o_id[kMgCoarseB], o_c[kMgCoarseB], o_g;
    float beta;
    const double* beta_z;
    float scale;
    int ncb, ne;
    int ny[kMgCoarseB + 1], nx[kMgCoarseB + 1];
};

__global__ __launch_bounds__(kMgCoarseThreads) void k_mg_coarse_setup(MgCoarseSetup S, const int* skip,
                                                                       size_t skip_zstride) {
    __shared__ float cl[2][kMgLdsPx];
    __shared__ double A[kMgDenseMax][kMgDenseMax + 1];
    __shared__ double dg[kMgDenseMax], fc[2][kMgDenseMax];
    const int z = blockIdx.x;
    if (mg_skip(skip, skip_zstride, z)) return;
    const int t = threadIdx.x;
    float* aux = S.aux + (size_t)z * S.zs_aux;
    float be = S.beta_z ? (float)S.beta_z[z] * S.scale : S.beta;
    int cur = 0;
    if (t < S.ny[0] * S.nx[0]) cl[0][t] = S.c[(size_t)z * S.zs_c + t];
    __syncthreads();
    for (int q = 0; q < S.ncb; ++q) {
        if (t < S.ny[q] * S.nx[q]) {
            aux[S.o_id[q] + t] = kOmega / (cl[cur][t] + 4.f * be);
            if (q > 0) aux[S.o_c[q] + t] = cl[cur][t];
        }
        const int nxf = S.nx[q], nxc = S.nx[q + 1];
        if (t < S.ny[q + 1] * nxc) {
            const int i = t / nxc, k = t - i * nxc;
            const int a = (2 * i) * nxf + 2 * k;
            cl[cur ^ 1][t] = 0.25f * (cl[cur][a] + cl[cur][a + 1] + cl[cur][a + nxf] + cl[cur][a + nxf + 1]);
        }
        __syncthreads();
        cur ^= 1;
        be *= 0.25f;
    }
    // A_e = diag(c_e) + beta_e L on the periodic grid, one row per thread, as
    // the sweeps apply it: c x + beta (4 x - neighbours), a neighbour that
    // wraps onto the pixel itself included
    const int ny = S.ny[S.ncb], nx = S.nx[S.ncb], ne = S.ne;
    if (t < ne) {
        for (int j = 0; j < ne; ++j) A[t][j] = 0.0;
        const int i = t / nx, k = t - i * nx;
        const int ip = i + 1 == ny ? 0 : i + 1, im = i == 0 ? ny - 1 : i - 1;
        const int kp = k + 1 == nx ? 0 : k + 1, km = k == 0 ? nx - 1 : k - 1;
        A[t][t] = (double)cl[cur][t] + 4.0 * (double)be;
        A[t][ip * nx + k] -= (double)be;
        A[t][im * nx + k] -= (double)be;
        A[t][i * nx + kp] -= (double)be;
        A[t][i * nx + km] -= (double)be;
    }
    __syncthreads();
    if (t < ne) {
        dg[t] = A[t][t];
        fc[0][t] = A[t][0];
    }
    __syncthreads();
    // in-place Gauss-Jordan; fc[k & 1] holds column k as it is before step k.
    // Thread t updates row t / 16, columns t % 16 + 16 m.
    const int gi = t >> 4, gj = t & 15;
    for (int k = 0; k < ne; ++k) {
        const double* f = fc[k & 1];
        double* fn = fc[(k + 1) & 1];
        const double p = f[k];
        const double inv = p > 1e-12 * dg[k] ? 1.0 / p : 0.0;
        if (t < ne) {
            const double v = (t == k ? 1.0 : A[k][t]) * inv;
            A[k][t] = v;
            if (t == k + 1) fn[k] = v;
        }
        __syncthreads();
        if (gi < ne && gi != k) {
            const double fi = f[gi];
#pragma unroll
            for (int m = 0; m < kMgDenseMax / 16; ++m) {
                const int j = gj + 16 * m;
                if (j >= ne) break;
                const double v = (j == k ? 0.0 : A[gi][j]) - fi * A[k][j];
                A[gi][j] = v;
                if (j == k + 1) fn[gi] = v;
            }
        }
        __syncthreads();
    }
    if (gi < ne) {
#pragma unroll
        for (int m = 0; m < kMgDenseMax / 16; ++m) {
            const int j = gj + 16 * m;
            if (j >= ne) break;
            aux[S.o_g + (size_t)gi * ne + j] = (float)(0.5 * (A[gi][j] + A[j][gi]));
        }
    }
}

// dimensions of in-LDS levels 0..kMgCoarseB (the exact level repeated past ncb)
static void coarse_dims(const MgPlan& P, int* ny, int* nx) {
    for (int q = 0; q <= kMgCoarseB; ++q) {
        const int l = P.ngrid + std::min(q, P.ncb);
        ny[q] = P.ny[l];
        nx[q] = P.nx[l];
    }
}

void launch_mg_setup(const MgPlan& P, const float* w2, float* mg, int batch, float beta,
                     const double* beta_z, const int* skip, size_t skip_zstride, hipStream_t st) {
    const size_t n0 = (size_t)P.ny[0] * P.nx[0];
    // the tile levels' coefficients: one pass when levels 1..G halve exactly
    // and G <= 4, else one launch per level
    const int G = P.ngrid;
    bool halves = G >= 1 && G <= 4 && P.ny[0] % (1 << G) == 0 && P.nx[0] % (1 << G) == 0;
    for (int l = 1; halves && l <= G; ++l)
        halves = P.ny[l] == P.ny[0] >> l && P.nx[l] == P.nx[0] >> l;
    if (halves) {
        MgCOffs O{};
        for (int l = 1; l <= G; ++l) O.c[l] = P.c[l];
        const dim3 grid(P.nx[0] >> G, P.ny[0] >> G, batch);
        switch (G) {
            case 1:
                hipLaunchKernelGGL(k_mg_restrict_c_all<1>, grid, dim3(4), 0, st, w2, n0, P.nx[0], mg, O,
                                   P.zstride);
                break;
            case 2:
                hipLaunchKernelGGL(k_mg_restrict_c_all<2>, grid, dim3(16), 0, st, w2, n0, P.nx[0], mg, O,
                                   P.zstride);
                break;
            case 3:
                hipLaunchKernelGGL(k_mg_restrict_c_all<3>, grid, dim3(64), 0, st, w2, n0, P.nx[0], mg, O,
                                   P.zstride);
                break;
            default:
                hipLaunchKernelGGL(k_mg_restrict_c_all<4>, grid, dim3(256), 0, st, w2, n0, P.nx[0], mg, O,
                                   P.zstride);
                break;
        }
    } else {
        for (int l = 0; l < P.ngrid; ++l) {
            const float* cf = l == 0 ? w2 : mg + P.c[l];
            const size_t cfz = l == 0 ? n0 : P.zstride;
            const int n = P.ny[l + 1] * P.nx[l + 1];
            hipLaunchKernelGGL(k_mg_restrict_c, dim3((n + 255) / 256, batch), dim3(256), 0, st, cf, cfz,
                               P.ny[l], P.nx[l], mg + P.c[l + 1], P.zstride);
        }
    }
    const int g0 = P.ngrid;
    const float sc = std::ldexp(1.f, -2 * g0);   // beta scale 4^-g0 of the first in-LDS level
    MgCoarseSetup S;
    S.c = g0 == 0 ? w2 : mg + P.c[g0];
    S.zs_c = g0 == 0 ? n0 : P.zstride;
    S.aux = mg;
    S.zs_aux = P.zstride;
    for (int q = 0; q < kMgCoarseB; ++q) {
        S.o_id[q] = P.id[q];
        S.o_c[q] = P.cb[q];
    }
    S.o_g = P.gi;
    S.beta = beta * sc;
    S.beta_z = beta_z;
    S.scale = sc;
    S.ncb = P.ncb;
    S.ne = P.ne;
    coarse_dims(P, S.ny, S.nx);
    hipLaunchKernelGGL(k_mg_coarse_setup, dim3(batch), dim3(kMgCoarseThreads), 0, st, S, skip,
                       skip_zstride);
}

void launch_mg_vcycle(const MgPlan& P, const float* r, const float* w2, float* z, float* mg,
                      int batch, float beta, const double* beta_z, const int* skip,
                      size_t skip_zstride, double* dot, size_t dot_zstride, hipStream_t st,
                      float* wout, double* dot2, const CgUpd* upd) {
    const size_t n0 = (size_t)P.ny[0] * P.nx[0];
    float bl[kMgMaxLevels], sc[kMgMaxLevels];   // level beta; level scale 4^-l
    bl[0] = beta;
    sc[0] = 1.f;
    for (int l = 1; l < kMgMaxLevels; ++l) {
        bl[l] = 0.25f * bl[l - 1];
        sc[l] = 0.25f * sc[l - 1];
    }
    auto level = [&](int l) {
        MgLevel L;
        L.b = l == 0 ? r : mg + P.b[l];
        L.zs_b = l == 0 ? n0 : P.zstride;
        L.c = l == 0 ? w2 : mg + P.c[l];
        L.zs_c = l == 0 ? n0 : P.zstride;
        L.xs = l == 0 ? mg + P.xs0 : mg + P.xs[l];
        L.zs_xs = P.zstride;
        L.out = nullptr;
        L.zs_out = P.zstride;
        L.e = nullptr;
        L.zs_e = P.zstride;
        L.ny = P.ny[l];
        L.nx = P.nx[l];
        L.beta = bl[l];
        L.beta_z = beta_z;
        L.scale = sc[l];
        return L;
    };
    auto pair = [&](int l) {
        MgPair A;
        A.b0 = l == 0 ? r : mg + P.b[l];
        A.zs_b0 = l == 0 ? n0 : P.zstride;
        A.c0 = l == 0 ? w2 : mg + P.c[l];
        A.zs_c0 = l == 0 ? n0 : P.zstride;
        A.xs0 = l == 0 ? mg + P.xs0 : mg + P.xs[l];
        A.zs_xs0 = P.zstride;
        A.e0 = l == 0 ? z : mg + P.e[l];
        A.zs_e0 = l == 0 ? n0 : P.zstride;
        A.ny0 = P.ny[l];
        A.nx0 = P.nx[l];
        A.beta0 = bl[l];
        A.beta_z = beta_z;
        A.scale = sc[l];
        A.b1 = mg + P.b[l + 1];
        A.c1 = mg + P.c[l + 1];
        A.xs1 = mg + P.xs[l + 1];
        A.b2 = mg + P.b[l + 2];
        A.e2 = mg + P.e[l + 2];
        A.zsm = P.zstride;
        return A;
    };
    for (int l = 0; l < P.ngrid;) {
        if (P.pair[l] && l == 0 && upd) {
            hipLaunchKernelGGL(k_mg_down2<true>, dim3(P.nx[l] / kCore2, P.ny[l] / kCore2, batch),
                               dim3(kPairThreads), 0, st, pair(l), skip, skip_zstride, *upd);
            l += 2;
        } else if (P.pair[l]) {
            // after the fused update (level pair 0 with upd): with the early
            // stopping test
            CgUpd c{};
            if (upd && l == 2 && P.pair[0]) {
                c = *upd;
                c.check = 1;
            }
            hipLaunchKernelGGL(k_mg_down2<false>, dim3(P.nx[l] / kCore2, P.ny[l] / kCore2, batch),
                               dim3(kPairThreads), 0, st, pair(l), skip, skip_zstride, c);
            l += 2;
        } else {
            MgLevel L = level(l);
            L.out = mg + P.b[l + 1];
            hipLaunchKernelGGL(k_mg_down, dim3(P.nx[l] / 16, P.ny[l] / 16, batch), dim3(256), 0, st,
                               L, skip, skip_zstride);
            l += 1;
        }
    }
    MgCoarse G;
    const int g0 = P.ngrid;
    G.b = g0 == 0 ? r : mg + P.b[g0];
    G.zs_b = g0 == 0 ? n0 : P.zstride;
    G.c = g0 == 0 ? w2 : mg + P.c[g0];
    G.zs_c = g0 == 0 ? n0 : P.zstride;
    G.e = g0 == 0 ? z : mg + P.e[g0];
    G.zs_e = g0 == 0 ? n0 : P.zstride;
    G.aux = mg;
    G.zs_aux = P.zstride;
    for (int q = 0; q < kMgCoarseB; ++q) {
        G.o_id[q] = P.id[q];
        G.o_c[q] = P.cb[q];
    }
    G.o_g = P.gi;
    G.beta = bl[g0];
    G.beta_z = beta_z;
    G.scale = sc[g0];
    G.ncb = P.ncb;
    G.ne = P.ne;
    coarse_dims(P, G.ny, G.nx);
    G.dot = g0 == 0 ? dot : nullptr;
    G.dot_zstride = dot_zstride;
    hipLaunchKernelGGL(k_mg_coarse, dim3(batch), dim3(kMgCoarseThreads), 0, st, G, skip, skip_zstride);
    // up: walk the same grouping from the bottom
    int top[kMgMaxLevels], ntop = 0;
    for (int l = 0; l < P.ngrid; l += P.pair[l] ? 2 : 1) top[ntop++] = l;
    for (int q = ntop - 1; q >= 0; --q) {
        const int l = top[q];
        double* d = l == 0 ? dot : nullptr;
        if (P.pair[l] && l == 0 && wout) {
            hipLaunchKernelGGL(k_mg_up2<true>, dim3(P.nx[l] / kCore2, P.ny[l] / kCore2, batch),
                               dim3(kPairThreads), 0, st, pair(l), skip, skip_zstride, d,
                               dot_zstride, wout, dot2);
        } else if (P.pair[l]) {
            hipLaunchKernelGGL(k_mg_up2<false>, dim3(P.nx[l] / kCore2, P.ny[l] / kCore2, batch),
                               dim3(kPairThreads), 0, st, pair(l), skip, skip_zstride, d,
                               dot_zstride, nullptr, nullptr);
        } else {
            MgLevel L = level(l);
            L.e = mg + P.e[l + 1];
            L.out = l == 0 ? z : mg + P.e[l];
            L.zs_out = l == 0 ? n0 : P.zstride;
            hipLaunchKernelGGL(k_mg_up, dim3(P.nx[l] / 16, P.ny[l] / 16, batch), dim3(256), 0, st, L,
                               skip, skip_zstride, d, dot_zstride);
        }
    }
}

void launch_pcg_mg_prec(const PcgArgs& a, int it, const MgPlan& P, float* mg, hipStream_t st) {
    // z = V(r); <r, z> partials into the rz slot of iteration it (it = -1:
    // the initial residual, slot 1)
    const int slot = it < 0 ? 1 : (it & 1);
    launch_mg_vcycle(P, a.r, a.w2, a.z, mg, a.batch, a.beta, a.beta_z, &a.st[0].done,
                     sizeof(PcgState) / sizeof(int), a.parts + a.L.rz + (size_t)slot * a.L.nrz,
                     a.L.zstride, st, nullptr, nullptr);
}

bool mg_pipelined_ok(const MgPlan& P) {
    // (the fused update writes one ||r||^2 partial per 32 x 32 core, as many as
    // the PCG's pixel kernels write per 1024 pixels)
    return P.ok && P.ngrid >= 2 && P.pair[0];
}

bool mg_early_stop(const MgPlan& P) {
    // the V-cycle's second kernel is a level pair (k_mg_down2<false>): it runs
    // the stopping test of the residual the iteration's update wrote
    return mg_pipelined_ok(P) && P.ngrid > 2 && P.pair[2];
}

void launch_pcg_mg_prec_w_upd(const PcgArgs& a, int i, const MgPlan& P, float* mg, hipStream_t st) {
    // iteration i's update fused into the V-cycle of r_(i+1): r and s live in
    // (r, r2) and (p1, p1b) by parity
    float* rb[2] = {a.r, a.r2};
    float* sb[2] = {a.p1, a.p1b};
    CgUpd U{};
    U.r_old = rb[i & 1];
    U.r_new = rb[(i + 1) & 1];
    U.s_old = sb[i & 1];
    U.s_new = sb[(i + 1) & 1];
    U.u = a.z;
    U.w = a.q;
    U.p = a.p0;
    U.x = a.x;
    U.zs = (size_t)a.ny * a.nx;
    U.it = i;
    U.parts = a.parts;
    U.L = a.L;
    U.nrz_used = a.nrz_used;
    U.tol2 = a.tol2;
    U.st = a.st;
    const int slot = (i + 1) & 1;
    launch_mg_vcycle(P, U.r_new, a.w2, a.z, mg, a.batch, a.beta, a.beta_z, &a.st[0].done,
                     sizeof(PcgState) / sizeof(int), a.parts + a.L.rz + (size_t)slot * a.L.nrz,
                     a.L.zstride, st, a.q, a.parts + a.L.dl + (size_t)slot * a.L.nrz, &U);
}

void launch_pcg_mg_prec_w(const PcgArgs& a, int i, const MgPlan& P, float* mg, hipStream_t st) {
    // u_i = V(r_i) into z, w_i = A u_i into q; gamma_i = <r_i, u_i> and
    // delta_i = <u_i, w_i> partials into parity slot i & 1
    const int slot = i & 1;
    launch_mg_vcycle(P, a.r, a.w2, a.z, mg, a.batch, a.beta, a.beta_z, &a.st[0].done,
                     sizeof(PcgState) / sizeof(int), a.parts + a.L.rz + (size_t)slot * a.L.nrz,
                     a.L.zstride, st, a.q, a.parts + a.L.dl + (size_t)slot * a.L.nrz);
}

}  // namespace dect
