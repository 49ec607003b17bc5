// Flat-detector fan-beam filtered back-projection (Kak & Slaney, ch. 3,
// equally spaced collinear detectors): the attenuation images that
// Algorithm 1 takes as input, reconstructed from each energy's sinogram.
//   1. weight p_j by sid / sqrt(sid^2 + u'_j^2), u' the bin coordinate on the
//      virtual detector through the isocentre (pitch dp = pitch*sid/sdd);
//   2. Ram-Lak filter as a linear convolution: h(0) = 1/(4 dp^2),
//      h(odd n) = -1/(pi^2 n^2 dp^2), h(even n) = 0, times dp;
//   3. back-project (dtheta/2) * sum_v sid^2/U^2 * q_v(u'(x, y)) with linear
//      interpolation (zero outside the detector), U = sid - (x cos + y sin).
#include "dect_internal.h"
#include "device_util.h"

namespace dect {

// One block per (view, sinogram): the weighted row and the filter taps in LDS,
// FP64 throughout (run once per solve; keeps the initial images, and the
// ill-conditioned closed-form t' computed from them, close to FP64).
__global__ __launch_bounds__(256) void k_fbp_filter(const float* __restrict__ sino, int nv, int nd,
                                                    double pitch, double offset, double sid,
                                                    double sdd, float* __restrict__ q) {
    extern __shared__ double smd[];
    double* pw = smd;          // nd
    double* tap = smd + nd;    // nd: tap[n] = 1/(pi^2 n^2), n odd; 0 otherwise
    const int v = blockIdx.x, b = blockIdx.y;
    const size_t row = ((size_t)b * nv + v) * nd;
    const double mag = sid / sdd;
    for (int j = threadIdx.x; j < nd; j += blockDim.x) {
        const double up = (((double)j - 0.5 * (nd - 1)) * pitch + offset) * mag;
        pw[j] = (double)sino[row + j] * sid / sqrt(sid * sid + up * up);
        tap[j] = (j & 1) ? 1.0 / (M_PI * M_PI * (double)j * (double)j) : 0.0;
    }
    __syncthreads();
    const double inv_dp = 1.0 / (pitch * mag);
    for (int j = threadIdx.x; j < nd; j += blockDim.x) {
        double acc = 0.0;
        const int nmax = max(j, nd - 1 - j);
        for (int n = (nmax & 1) ? nmax : nmax - 1; n >= 1; n -= 2) {
            double t = 0.0;
            if (j - n >= 0) t += pw[j - n];
            if (j + n < nd) t += pw[j + n];
            acc = fma(tap[n], t, acc);
        }
        q[row + j] = (float)((0.25 * pw[j] - acc) * inv_dp);
    }
}

constexpr int kFbpChunk = 1024;

__global__ __launch_bounds__(256) void k_fbp_bp(const float* __restrict__ q, int nx, int ny, int nv,
                                                int nd, double dxmm, double angle0, double arc,
                                                double pitch, double offset, double sid, double sdd,
                                                float* __restrict__ img) {
    __shared__ double2 cs_tab[kFbpChunk];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const bool inside = p < nx * ny;
    const int i = inside ? p / nx : 0, k = inside ? p % nx : 0;
    const double x = ((double)k - 0.5 * (nx - 1)) * dxmm;
    const double y = ((double)i - 0.5 * (ny - 1)) * dxmm;
    const double mag = sid / sdd;
    const double inv_dp = 1.0 / (pitch * mag);
    const double u0 = (-0.5 * (nd - 1) * pitch + offset) * mag;
    const double dth = arc / nv;
    const float* qb = q + (size_t)b * nv * nd;
    double acc = 0.0;
    for (int v0 = 0; v0 < nv; v0 += kFbpChunk) {
        const int nvc = min(kFbpChunk, nv - v0);
        __syncthreads();
        for (int t = threadIdx.x; t < nvc; t += blockDim.x) {
            double sn, cs;
            sincos(angle0 + (double)(v0 + t) * dth, &sn, &cs);
            cs_tab[t] = make_double2(cs, sn);
        }
        __syncthreads();
        if (!inside) continue;
        for (int vv = 0; vv < nvc; ++vv) {
            const double cs = cs_tab[vv].x, sn = cs_tab[vv].y;
            const double U = sid - (x * cs + y * sn);
            const double W = -x * sn + y * cs;
            const double rU = 1.0 / U;
            const double f = (sid * W * rU - u0) * inv_dp;
            const double j0 = floor(f);
            const float t = (float)(f - j0);
            const int a = (int)j0;
            const float* qv = qb + (size_t)(v0 + vv) * nd;
            const float va = (a >= 0 && a < nd) ? qv[a] : 0.f;
            const float vb = (a + 1 >= 0 && a + 1 < nd) ? qv[a + 1] : 0.f;
            const double wgt = sid * sid * rU * rU;
            acc += wgt * (double)fmaf(t, vb - va, va);
        }
    }
    if (inside) img[(size_t)b * nx * ny + p] = (float)(0.5 * dth * acc);
}

// Both energies' back-projections in one pass: the geometry of each (pixel,
// view) pair (U, the detector coordinate, the interpolation weights) is
// computed once and applied to both filtered sinograms; each channel's sum is
// the same as k_fbp_bp's, in the same order.
__global__ __launch_bounds__(256) void k_fbp_bp2(const float* __restrict__ qa, const float* __restrict__ qb,
                                                 int nx, int ny, int nv, int nd, double dxmm, double angle0,
                                                 double arc, double pitch, double offset, double sid,
                                                 double sdd, float* __restrict__ ia, float* __restrict__ ib) {
    __shared__ double2 cs_tab[kFbpChunk];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const bool inside = p < nx * ny;
    const int i = inside ? p / nx : 0, k = inside ? p % nx : 0;
    const double x = ((double)k - 0.5 * (nx - 1)) * dxmm;
    const double y = ((double)i - 0.5 * (ny - 1)) * dxmm;
    const double mag = sid / sdd;
    const double inv_dp = 1.0 / (pitch * mag);
    const double u0 = (-0.5 * (nd - 1) * pitch + offset) * mag;
    const double dth = arc / nv;
    const float* qa_b = qa + (size_t)b * nv * nd;
    const float* qb_b = qb + (size_t)b * nv * nd;
    double acc_a = 0.0, acc_b = 0.0;
    for (int v0 = 0; v0 < nv; v0 += kFbpChunk) {
        const int nvc = min(kFbpChunk, nv - v0);
        __syncthreads();
        for (int t = threadIdx.x; t < nvc; t += blockDim.x) {
            double sn, cs;
            sincos(angle0 + (double)(v0 + t) * dth, &sn, &cs);
            cs_tab[t] = make_double2(cs, sn);
        }
        __syncthreads();
        if (!inside) continue;
        for (int vv = 0; vv < nvc; ++vv) {
            const double cs = cs_tab[vv].x, sn = cs_tab[vv].y;
            const double U = sid - (x * cs + y * sn);
            const double W = -x * sn + y * cs;
            const double rU = 1.0 / U;
            const double f = (sid * W * rU - u0) * inv_dp;
            const double j0 = floor(f);
            const float t = (float)(f - j0);
            const int a = (int)j0;
            const bool ina = a >= 0 && a < nd, inb = a + 1 >= 0 && a + 1 < nd;
            const size_t o = (size_t)(v0 + vv) * nd;
            const float va = ina ? qa_b[o + a] : 0.f, vb = inb ? qa_b[o + a + 1] : 0.f;
            const float wa = ina ? qb_b[o + a] : 0.f, wb = inb ? qb_b[o + a + 1] : 0.f;
            const double wgt = sid * sid * rU * rU;
            acc_a += wgt * (double)fmaf(t, vb - va, va);
            acc_b += wgt * (double)fmaf(t, wb - wa, wa);
        }
    }
    if (inside) {
        ia[(size_t)b * nx * ny + p] = (float)(0.5 * dth * acc_a);
        ib[(size_t)b * nx * ny + p] = (float)(0.5 * dth * acc_b);
    }
}

void launch_fbp_pair(const Geom& g, const float* sino_a, const float* sino_b, int nsino, float* q,
                     float* img_a, float* img_b, hipStream_t st) {
    const size_t lds = 2 * (size_t)g.nd * sizeof(double);
    const size_t n = (size_t)nsino * g.nv * g.nd;
    hipLaunchKernelGGL(k_fbp_filter, dim3(g.nv, nsino), dim3(256), lds, st, sino_a, g.nv, g.nd,
                       g.pitch, g.offset, g.sid, g.sdd, q);
    hipLaunchKernelGGL(k_fbp_filter, dim3(g.nv, nsino), dim3(256), lds, st, sino_b, g.nv, g.nd,
                       g.pitch, g.offset, g.sid, g.sdd, q + n);
    const int npix = g.nx * g.ny;
    hipLaunchKernelGGL(k_fbp_bp2, dim3((npix + 255) / 256, nsino), dim3(256), 0, st, q, q + n, g.nx, g.ny,
                       g.nv, g.nd, g.dx, g.angle0, g.arc, g.pitch, g.offset, g.sid, g.sdd, img_a, img_b);
}

void launch_fbp(const Geom& g, const float* sino, int nsino, float* q, float* img,
                hipStream_t st) {
    const size_t lds = 2 * (size_t)g.nd * sizeof(double);
    hipLaunchKernelGGL(k_fbp_filter, dim3(g.nv, nsino), dim3(256), lds, st, sino, g.nv, g.nd,
                       g.pitch, g.offset, g.sid, g.sdd, q);
    const int npix = g.nx * g.ny;
    hipLaunchKernelGGL(k_fbp_bp, dim3((npix + 255) / 256, nsino), dim3(256), 0, st, q, g.nx, g.ny,
                       g.nv, g.nd, g.dx, g.angle0, g.arc, g.pitch, g.offset, g.sid, g.sdd, img);
}

}  // namespace dect
