// Periodic solve (c + beta*D^T D) x = rhs by 2-D FFT, the closed form of the
// g-subproblem in Section II-C (F(1) read as 1) and of the rho_e subproblem:
// X = F(rhs) / (c + beta*(|F dx|^2 + |F dy|^2)), |F dx|^2 = 4 sin^2(pi kx/nx).
//
// Three passes over a complex scratch image:
//   rows_fwd: build the right-hand side of one row (fused with the hard
//             threshold of eq. (9) and D^T), FFT along x;
//   cols:     FFT along y, spectral division, inverse FFT along y;
//   rows_inv: inverse FFT along x, real part / (nx*ny).
// Transforms are Stockham autosort (radix 4, 3, 2) in LDS; twiddles come from
// FP64 sincos rounded to FP32.
#include "dect_internal.h"
#include "device_util.h"

namespace dect {

struct FftPlan {
    int n;
    int nst;
    int rad[12];
};

static bool make_plan(int n, FftPlan* p) {
    if (n < 8 || n > 1024) return false;
    int m = n, a = 0, b = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++a;
    }
    while (m % 3 == 0) {
        m /= 3;
        ++b;
    }
    if (m != 1 || b > 1) return false;
    p->n = n;
    p->nst = 0;
    if (b) p->rad[p->nst++] = 3;
    while (a >= 2) {
        p->rad[p->nst++] = 4;
        a -= 2;
    }
    if (a) p->rad[p->nst++] = 2;
    return true;
}

bool fft_size_ok(int n) {
    FftPlan p;
    return make_plan(n, &p);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// tw[e] = exp(-2 pi i e / n); 2e/n is exact in FP32 for n <= 1024
__device__ void fill_twiddles(float2* tw, int n) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        float s, c;
        sincospif(-2.0f * (float)e / (float)n, &s, &c);
        tw[e] = make_float2(c, s);
    }
}

// nb interleaved transforms of length P.n: element e of transform t at e*nb + t.
// INV = false: forward (e^{-i}); true: inverse without 1/n.  Returns the buffer
// that holds the result.  Ends with a barrier.
template <bool INV>
__device__ float2* fft_lds(float2* a, float2* b, const float2* tw, const FftPlan& P, int nb) {
    int p = 1;
    const int n = P.n;
    for (int s = 0; s < P.nst; ++s) {
        const int r = P.rad[s];
        const int m = n / r;
        const int tstep = n / (p * r);
        for (int idx = threadIdx.x; idx < m * nb; idx += blockDim.x) {
            const int i = idx / nb, t = idx - (idx / nb) * nb;
            const int k = i % p;
            float2 x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q < r) x[q] = a[(size_t)(i + q * m) * nb + t];
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                if (q < r) {
                    float2 w = tw[(q * k * tstep) % n];
                    if (INV) w.y = -w.y;
                    x[q] = cmul(x[q], w);
                }
            }
            float2 y[4];
            if (r == 2) {
                y[0] = make_float2(x[0].x + x[1].x, x[0].y + x[1].y);
                y[1] = make_float2(x[0].x - x[1].x, x[0].y - x[1].y);
            } else if (r == 3) {
                const float h = 0.86602540378443865f;   // sqrt(3)/2
                const float2 t1 = make_float2(x[1].x + x[2].x, x[1].y + x[2].y);
                const float2 t2 = make_float2(x[1].x - x[2].x, x[1].y - x[2].y);
                y[0] = make_float2(x[0].x + t1.x, x[0].y + t1.y);
                const float2 m1 = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
                // forward: m2 = -i*h*t2; inverse: +i*h*t2
                const float2 m2 = INV ? make_float2(-h * t2.y, h * t2.x) : make_float2(h * t2.y, -h * t2.x);
                y[1] = make_float2(m1.x + m2.x, m1.y + m2.y);
                y[2] = make_float2(m1.x - m2.x, m1.y - m2.y);
            } else {
                const float2 aa = make_float2(x[0].x + x[2].x, x[0].y + x[2].y);
                const float2 bb = make_float2(x[0].x - x[2].x, x[0].y - x[2].y);
                const float2 cc = make_float2(x[1].x + x[3].x, x[1].y + x[3].y);
                const float2 dd = make_float2(x[1].x - x[3].x, x[1].y - x[3].y);
                // forward: y1 = bb - i dd, y3 = bb + i dd
                const float2 mid = INV ? make_float2(-dd.y, dd.x) : make_float2(dd.y, -dd.x);
                y[0] = make_float2(aa.x + cc.x, aa.y + cc.y);
                y[2] = make_float2(aa.x - cc.x, aa.y - cc.y);
                y[1] = make_float2(bb.x + mid.x, bb.y + mid.y);
                y[3] = make_float2(bb.x - mid.x, bb.y - mid.y);
            }
            const int jj = (i - k) * r + k;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q < r) b[(size_t)(jj + q * p) * nb + t] = y[q];
        }
        __syncthreads();
        float2* tmp = a;
        a = b;
        b = tmp;
        p *= r;
    }
    return a;
}

// Thresholded-away gradients S at (row ra, column k) of an image held as rows
// ra, rb (rb = the next row down): (dx, dy) where eq. (9) zeroes them, else
// (0, 0).  `kept` receives the complementary kept pair.  The decision is taken
// in FP32 with separately rounded squares.
__device__ __forceinline__ float2 ht_small(const float* ra, const float* rb, int k, int nx,
                                           float thr, float2* kept) {
    const int k1 = (k + 1 == nx) ? 0 : k + 1;
    const float dx = ra[k1] - ra[k];
    const float dy = rb[k] - ra[k];
    const bool keep = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)) > thr;
    if (kept) *kept = keep ? make_float2(dx, dy) : make_float2(0.f, 0.f);
    return keep ? make_float2(0.f, 0.f) : make_float2(dx, dy);
}

// r = b - H f of the image-domain f-subproblem at pixel q, both bases (FP64
// per pixel: the data and coupling residuals cancel to small values near
// convergence)
__device__ __forceinline__ float2 imgf_residual(const FftArgs& a, size_t q) {
    const float2 f = a.f[q];
    const double f1 = f.x, f2 = f.y;
    const double rL = (double)a.mu_lo[q] - (a.cL0 * f1 + a.cL1 * f2);
    const double rH = (double)a.mu_hi[q] - (a.cH0 * f1 + a.cH1 * f2);
    const double r = a.rho_in[q], t = a.t_in[q];
    const double c1 = r * (a.ta0 * t + a.tpsi0) - (a.m00 * f1 + a.m01 * f2);
    const double c2 = r * (a.ta1 * t + a.tpsi1) - (a.m10 * f1 + a.m11 * f2);
    const double v1 = a.eta_img * (a.cL0 * rL + a.cH0 * rH) + a.xi_img * (a.m00 * c1 + a.m10 * c2);
    const double v2 = a.eta_img * (a.cL1 * rL + a.cH1 * rH) + a.xi_img * (a.m01 * c1 + a.m11 * c2);
    return make_float2((float)v1, (float)v2);
}

__device__ __forceinline__ bool skip_slice(const FftArgs& a, int z) {
    return a.skip && a.skip[(size_t)z * a.skip_zstride];
}

// diagonal shift c of slice z (all threads; uses LDS and barriers)
__device__ float shift_of(const FftArgs& a, int z) {
    __shared__ double shs[4];
    if (!a.c_parts) return (float)a.c;
    const double s = block_sum_array<256>(a.c_parts + (size_t)z * a.c_zstride, a.c_n, 1, shs);
    __shared__ float bc;
    if (threadIdx.x == 0) bc = (float)fmax(a.c_scale * s, 1e-12);
    __syncthreads();
    const float r = bc;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_fft_rows_fwd(FftPlan P, int ny, FftArgs a,
                                                      float2* __restrict__ scratch) {
    extern __shared__ float2 sm2[];
    const int nx = P.n;
    float2* A = sm2;
    float2* B = sm2 + nx;
    float2* tw = sm2 + 2 * nx;
    float* rows = reinterpret_cast<float*>(sm2 + 3 * nx);   // 3 rows of the HT input
    const int i = blockIdx.x, z = blockIdx.y;
    slice_beta_thr(a, z);
    if (skip_slice(a, z)) return;
    const size_t npix = (size_t)nx * ny;
    if (a.src == FFT_SRC_IMGF) {
        // both bases: two interleaved transforms (A, B hold 2 nx values each),
        // three rows of each basis for the hard threshold
        float2* A2 = sm2;
        float2* B2 = sm2 + 2 * nx;
        float2* tw2 = sm2 + 4 * nx;
        float* rows2 = reinterpret_cast<float*>(sm2 + 5 * nx);
        fill_twiddles(tw2, nx);
        const int im = (i == 0) ? ny - 1 : i - 1, ip = (i + 1 == ny) ? 0 : i + 1;
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            const float2 fm = a.f[z * npix + (size_t)im * nx + k];
            const float2 f0 = a.f[z * npix + (size_t)i * nx + k];
            const float2 fp = a.f[z * npix + (size_t)ip * nx + k];
            rows2[k] = fm.x;
            rows2[nx + k] = f0.x;
            rows2[2 * nx + k] = fp.x;
            rows2[3 * nx + k] = fm.y;
            rows2[4 * nx + k] = f0.y;
            rows2[5 * nx + k] = fp.y;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            const int km = (k == 0) ? nx - 1 : k - 1;
            const float2 res = imgf_residual(a, z * npix + (size_t)i * nx + k);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float* rm = rows2 + 3 * c * nx;
                const float* r0 = rm + nx;
                const float* rp = rm + 2 * nx;
                const float2 sc = ht_small(r0, rp, k, nx, a.thr, nullptr);
                const float2 sl = ht_small(r0, rp, km, nx, a.thr, nullptr);
                const float2 su = ht_small(rm, r0, k, nx, a.thr, nullptr);
                const float dts = (sl.x - sc.x) + (su.y - sc.y);
                A2[2 * k + c] = make_float2((c == 0 ? res.x : res.y) - a.beta * dts, 0.f);
            }
        }
        __syncthreads();
        const float2* R2 = fft_lds<false>(A2, B2, tw2, P, 2);
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            scratch[(2 * (size_t)z) * npix + (size_t)i * nx + k] = R2[2 * k];
            scratch[(2 * (size_t)z + 1) * npix + (size_t)i * nx + k] = R2[2 * k + 1];
        }
        return;
    }
    fill_twiddles(tw, nx);
    if (a.src == FFT_SRC_PLAIN) {
        const float cz = a.scale_w2 ? shift_of(a, z) : 0.f;
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            const size_t q = z * npix + (size_t)i * nx + k;
            float v = a.in[q];
            if (a.scale_w2) v *= sqrtf((cz + 4.f * a.beta) / (a.scale_w2[q] + 4.f * a.beta));
            A[k] = make_float2(v, 0.f);
        }
    } else {
        const int im = (i == 0) ? ny - 1 : i - 1, ip = (i + 1 == ny) ? 0 : i + 1;
        const size_t bs = (size_t)a.bstride;
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            rows[k] = a.base[(z * npix + (size_t)im * nx + k) * bs];
            rows[nx + k] = a.base[(z * npix + (size_t)i * nx + k) * bs];
            rows[2 * nx + k] = a.base[(z * npix + (size_t)ip * nx + k) * bs];
        }
        __syncthreads();
        const float* rm = rows;
        const float* r0 = rows + nx;
        const float* rp = rows + 2 * nx;
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            const int km = (k == 0) ? nx - 1 : k - 1;
            float2 kept;
            const float2 sc = ht_small(r0, rp, k, nx, a.thr, &kept);   // at (i, k)
            const float2 sl = ht_small(r0, rp, km, nx, a.thr, nullptr); // at (i, k-1)
            const float2 su = ht_small(rm, r0, k, nx, a.thr, nullptr);  // at (i-1, k)
            const float dts = (sl.x - sc.x) + (su.y - sc.y);
            const float g = r0[k];
            float diff;
            if (a.src == FFT_SRC_RHO) {
                const float2 f = a.f[z * npix + (size_t)i * nx + k];
                const double M1 = a.m00 * (double)f.x + a.m01 * (double)f.y;
                const double M2 = a.m10 * (double)f.x + a.m11 * (double)f.y;
                diff = (float)((M1 * a.e1n - M2 * a.e2n) * a.inv_crho - (double)g);
            } else {
                diff = a.in[z * npix + (size_t)i * nx + k] - g;
                if (a.h_out) a.h_out[z * npix + (size_t)i * nx + k] = kept.x;
                if (a.v_out) a.v_out[z * npix + (size_t)i * nx + k] = kept.y;
            }
            A[k] = make_float2(diff - a.beta * dts, 0.f);
        }
    }
    __syncthreads();
    const float2* R = fft_lds<false>(A, B, tw, P, 1);
    for (int k = threadIdx.x; k < nx; k += blockDim.x) scratch[z * npix + (size_t)i * nx + k] = R[k];
}

__global__ __launch_bounds__(256) void k_fft_cols(FftPlan P, int nx, int cols, FftArgs a,
                                                  float2* __restrict__ scratch) {
    extern __shared__ float2 sm2[];
    __shared__ double sh[4];
    __shared__ float cz_sh;
    const int ny = P.n;
    const int ncomp = a.src == FFT_SRC_IMGF ? 2 : 1;
    float2* A = sm2;
    float2* B = sm2 + (size_t)ny * cols;
    float2* tw = sm2 + (size_t)2 * ny * cols * ncomp;
    float* lamy = reinterpret_cast<float*>(tw + ny);
    float* lamx = lamy + ny;
    // workgroups go round-robin to the 8 XCDs; give each XCD a contiguous run
    // of columns so that the row segments it reads share L2 lines
    const int nbx = gridDim.x;
    const int bx = (nbx & 7) == 0 ? (blockIdx.x & 7) * (nbx >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    const int c0 = bx * cols, z = blockIdx.y;
    slice_beta_thr(a, z);
    if (skip_slice(a, z)) return;
    const size_t npix = (size_t)nx * ny;
    {
        const float c = shift_of(a, z);
        if (threadIdx.x == 0) cz_sh = c;
    }
    fill_twiddles(tw, ny);
    for (int e = threadIdx.x; e < ny; e += blockDim.x) {
        const float s = sinpif((float)e / (float)ny);
        lamy[e] = 4.0f * s * s;
    }
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
        const float s = sinpif((float)(c0 + c) / (float)nx);
        lamx[c] = 4.0f * s * s;
    }
    if (a.src == FFT_SRC_IMGF) {
        // both bases of the same columns: transform t < cols is basis 0,
        // t >= cols basis 1; the 2x2 system of (13a) couples them per frequency
        const int nb = 2 * cols;
        float2* A2 = sm2;
        float2* B2 = sm2 + (size_t)ny * nb;
        for (int idx = threadIdx.x; idx < ny * nb; idx += blockDim.x) {
            const int e = idx / nb, r = idx - (idx / nb) * nb;
            const int comp = r >= cols, c = r - comp * cols;
            A2[idx] = (c0 + c < nx) ? scratch[(2 * (size_t)z + comp) * npix + (size_t)e * nx + c0 + c]
                                    : make_float2(0.f, 0.f);
        }
        __syncthreads();
        float2* R2 = fft_lds<false>(A2, B2, tw, P, nb);
        float2* S2 = (R2 == A2) ? B2 : A2;
        const float c1 = (float)a.c, c2 = (float)a.c_b, o = (float)a.c_o, d0 = (float)a.c_det;
        for (int idx = threadIdx.x; idx < ny * cols; idx += blockDim.x) {
            const int e = idx / cols, c = idx - (idx / cols) * cols;
            const float bl = a.beta * (lamx[c] + lamy[e]);
            // det = (c1 + bl)(c2 + bl) - o^2 = d0 + bl (c1 + c2 + bl), d0 formed in FP64
            const float inv = 1.0f / (d0 + bl * (c1 + c2 + bl));
            const float a11 = c1 + bl, a22 = c2 + bl;
            const float2 x1 = R2[(size_t)e * nb + c], x2 = R2[(size_t)e * nb + cols + c];
            R2[(size_t)e * nb + c] =
                make_float2((a22 * x1.x - o * x2.x) * inv, (a22 * x1.y - o * x2.y) * inv);
            R2[(size_t)e * nb + cols + c] =
                make_float2((a11 * x2.x - o * x1.x) * inv, (a11 * x2.y - o * x1.y) * inv);
        }
        __syncthreads();
        const float2* O2 = fft_lds<true>(R2, S2, tw, P, nb);
        for (int idx = threadIdx.x; idx < ny * nb; idx += blockDim.x) {
            const int e = idx / nb, r = idx - (idx / nb) * nb;
            const int comp = r >= cols, c = r - comp * cols;
            if (c0 + c < nx) scratch[(2 * (size_t)z + comp) * npix + (size_t)e * nx + c0 + c] = O2[idx];
        }
        return;
    }
    for (int idx = threadIdx.x; idx < ny * cols; idx += blockDim.x) {
        const int e = idx / cols, c = idx - (idx / cols) * cols;
        A[idx] = (c0 + c < nx) ? scratch[z * npix + (size_t)e * nx + c0 + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    float2* R = fft_lds<false>(A, B, tw, P, cols);
    float2* S = (R == A) ? B : A;
    const float cz = cz_sh;
    for (int idx = threadIdx.x; idx < ny * cols; idx += blockDim.x) {
        const int e = idx / cols, c = idx - (idx / cols) * cols;
        const float sc = 1.0f / (cz + a.beta * (lamx[c] + lamy[e]));
        R[idx] = make_float2(R[idx].x * sc, R[idx].y * sc);
    }
    __syncthreads();
    const float2* O = fft_lds<true>(R, S, tw, P, cols);
    for (int idx = threadIdx.x; idx < ny * cols; idx += blockDim.x) {
        const int e = idx / cols, c = idx - (idx / cols) * cols;
        if (c0 + c < nx) scratch[z * npix + (size_t)e * nx + c0 + c] = O[idx];
    }
}

__global__ __launch_bounds__(256) void k_fft_rows_inv(FftPlan P, int ny, FftArgs a,
                                                      const float2* __restrict__ scratch) {
    extern __shared__ float2 sm2[];
    __shared__ double sh[4];
    const int nx = P.n;
    float2* A = sm2;
    float2* B = sm2 + nx;
    float2* tw = sm2 + 2 * nx;
    const int i = blockIdx.x, z = blockIdx.y;
    slice_beta_thr(a, z);
    if (skip_slice(a, z)) return;
    const size_t npix = (size_t)nx * ny;
    if (a.src == FFT_SRC_IMGF) {
        float2* A2 = sm2;
        float2* B2 = sm2 + 2 * nx;
        float2* tw2 = sm2 + 4 * nx;
        fill_twiddles(tw2, nx);
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            A2[2 * k] = scratch[(2 * (size_t)z) * npix + (size_t)i * nx + k];
            A2[2 * k + 1] = scratch[(2 * (size_t)z + 1) * npix + (size_t)i * nx + k];
        }
        __syncthreads();
        const float2* R2 = fft_lds<true>(A2, B2, tw2, P, 2);
        const float sc2 = (float)(1.0 / ((double)nx * (double)ny));
        float2* out2 = reinterpret_cast<float2*>(a.out);
        for (int k = threadIdx.x; k < nx; k += blockDim.x) {
            const size_t q = z * npix + (size_t)i * nx + k;
            const float2 f = a.f[q];
            out2[q] = make_float2(f.x + R2[2 * k].x * sc2, f.y + R2[2 * k + 1].x * sc2);
        }
        return;
    }
    fill_twiddles(tw, nx);
    for (int k = threadIdx.x; k < nx; k += blockDim.x) A[k] = scratch[z * npix + (size_t)i * nx + k];
    __syncthreads();
    const float2* R = fft_lds<true>(A, B, tw, P, 1);
    const float sc = (float)(1.0 / ((double)nx * (double)ny));
    const bool corr = a.src != FFT_SRC_PLAIN;
    const float cz = a.scale_w2 ? shift_of(a, z) : 0.f;
    double dot = 0.0;
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
        const size_t q = z * npix + (size_t)i * nx + k;
        float d = R[k].x * sc;
        if (a.scale_w2) d *= sqrtf((cz + 4.f * a.beta) / (a.scale_w2[q] + 4.f * a.beta));
        const float v = corr ? a.base[q * a.bstride] + d : d;
        a.out[q * a.ostride] = v;
        if (a.dot_with) dot += (double)v * (double)a.dot_with[q];
    }
    if (a.dot_parts) {
        const double s = block_sum<256>(dot, sh);
        if (threadIdx.x == 0) a.dot_parts[(size_t)z * a.dot_zstride + i] = s;
    }
}

size_t fft_scratch_bytes(int ny, int nx, int batch) {
    return (size_t)batch * ny * nx * sizeof(float2);
}

static int cols_for(int ny, int nx, int batch, int ncomp) {
    // two ping-pong buffers of ny*cols*ncomp complex values within 64 KiB of
    // LDS, and at least 256 workgroups (one per CU) where the image allows
    int cols = 8;
    while (cols > 1 && (size_t)2 * ny * cols * ncomp * sizeof(float2) + ny * 16 > 64 * 1024) cols /= 2;
    while (cols > 2 && ((nx + cols - 1) / cols) * batch < 256) cols /= 2;
    return cols;
}

void launch_fft_solve(int ny, int nx, int batch, const FftArgs& a, float2* scratch,
                      hipStream_t st) {
    FftPlan px, py;
    make_plan(nx, &px);
    make_plan(ny, &py);
    // the joint f-subproblem carries both bases through every pass
    const int ncomp = a.src == FFT_SRC_IMGF ? 2 : 1;
    const size_t lds_row = ncomp == 2 ? (size_t)5 * nx * sizeof(float2) + (size_t)6 * nx * sizeof(float)
                                      : (size_t)3 * nx * sizeof(float2) + (size_t)3 * nx * sizeof(float);
    hipLaunchKernelGGL(k_fft_rows_fwd, dim3(ny, batch), dim3(256), lds_row, st, px, ny, a, scratch);
    const int cols = cols_for(ny, nx, batch, ncomp);
    const size_t lds_col = (size_t)2 * ny * cols * ncomp * sizeof(float2) + ny * sizeof(float2) +
                           (size_t)ny * sizeof(float) + (size_t)cols * sizeof(float);
    hipLaunchKernelGGL(k_fft_cols, dim3((nx + cols - 1) / cols, batch), dim3(256), lds_col, st, py, nx,
                       cols, a, scratch);
    const size_t lds_inv = (size_t)(ncomp == 2 ? 5 : 3) * nx * sizeof(float2);
    hipLaunchKernelGGL(k_fft_rows_inv, dim3(ny, batch), dim3(256), lds_inv, st, px, ny, a, scratch);
}

}  // namespace dect
