// Fan-beam system matrix A on gfx950: ray table, ray-driven forward projector
// and the matched voxel-driven back-projector.
//
// Both operators evaluate the same chord lengths from the same FP32 ray table:
// a ray advances along its major pixel axis (|slope| <= 1), so inside one
// major step it crosses at most one minor grid line; the step's chord L is
// split between minor pixels r0 and r0 +/- 1 in proportion w0 : 1 - w0, where
// w0 is the fraction of the step spent before the crossing.  This reproduces
// the exact intersection lengths of the ray with the half-open pixel squares
// (Siddon 1985) while giving every lane of a wavefront the same trip count.
// The minor coordinate is a 32.32 fixed-point integer that each step advances
// by the slope exactly, so crossings are placed to 2^-32 pixel however flat
// the ray; projector and back-projector derive identical weights from it.
#include <algorithm>
#include <climits>

#include "dect_internal.h"
#include "device_util.h"

namespace dect {

size_t ray_table_bytes(const Geom& g) {
    const size_t nr = (size_t)table_views(g) * g.nd;
    return nr * (sizeof(int4) + sizeof(float2) + sizeof(int2)) + (size_t)table_views(g) * sizeof(float4);
}

__device__ __forceinline__ long long fix_a0(int4 f) {
    return (long long)(((unsigned long long)(unsigned)f.y << 32) | (unsigned)f.x);
}
__device__ __forceinline__ long long fix_s(int4 f) {
    return (long long)(((unsigned long long)(unsigned)f.w << 32) | (unsigned)f.z);
}
// Fraction of the major step [y, y + s] spent in pixel floor(y): (1 - frac)/s
// when s >= 0, frac/|s| when s < 0, capped at 1.  lo = fractional bits of y;
// xmask = ~0 when s >= 0 (then lo ^ xmask = 2^32 - 1 - lo, which is 1 - frac
// to 2^-32), else 0; ainv32 = 2^-32 / |s| (table entry).
__device__ __forceinline__ float first_weight(unsigned lo, unsigned xmask, float ainv32) {
    return fminf((float)(lo ^ xmask) * ainv32, 1.0f);
}
// The same for a step [l, l + |s|] given by its lower end l (any direction):
// the fraction below the next boundary, (2^32 - lo) * ainv32 with the
// distance exact in fixed-point units, capped at 1 (s = 0: ainv32 = inf, 1).
__device__ __forceinline__ float lower_weight(unsigned lo, float ainv32) {
    return fminf(fmaf((float)(~lo), ainv32, ainv32), 1.0f);
}

// ---------------------------------------------------------------------------
// ray table (FP64 geometry, FP32 storage)
// ---------------------------------------------------------------------------
// xq > 0 (slices with the transpose symmetry, xq = nv / 4): the rays of views
// xq/2 < v < xq are the transposes of rays (xq - v, nd - 1 - j), the same
// fixed-point entries with the other major axis, so that the transpose is an
// exact symmetry of the projector
__global__ void k_build_ray_table(Geom g, int xq, int4* __restrict__ fix, float2* __restrict__ flt,
                                  int2* __restrict__ span, float4* __restrict__ view) {
    const int j0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int v0 = blockIdx.y;
    if (j0 == 0) {
        const double th0 = g.angle0 + (double)v0 * (g.arc / (double)g.nv);
        double sn0, cs0;
        sincos(th0, &sn0, &cs0);
        const double h = 0.5 * g.dx;
        view[v0] = make_float4((float)cs0, (float)sn0, (float)(h * (fabs(cs0) + fabs(sn0))), 0.f);
    }
    if (j0 >= g.nd) return;
    const bool tr = xq > 0 && 2 * v0 > xq;
    const int v = tr ? xq - v0 : v0, j = tr ? g.nd - 1 - j0 : j0;
    const double th = g.angle0 + (double)v * (g.arc / (double)g.nv);
    double sn, cs;
    sincos(th, &sn, &cs);
    const double u = ((double)j - 0.5 * (double)(g.nd - 1)) * g.pitch + g.offset;
    const double Sx = g.sid * cs, Sy = g.sid * sn;
    const double Qx = -(g.sdd - g.sid) * cs - u * sn;
    const double Qy = -(g.sdd - g.sid) * sn + u * cs;
    const double dxr = Qx - Sx, dyr = Qy - Sy;
    // source in pixel units from the image corner
    const double sx = (Sx + 0.5 * g.nx * g.dx) / g.dx;
    const double sy = (Sy + 0.5 * g.ny * g.dx) / g.dx;
    const bool xmaj = fabs(dxr) >= fabs(dyr);
    double slope;
    int nmaj, nmin;
    if (xmaj) {
        slope = dyr / dxr;
        nmaj = g.nx;
        nmin = g.ny;
    } else {
        slope = dxr / dyr;
        nmaj = g.ny;
        nmin = g.nx;
    }
    if (fabs(slope) < 0x1p-30) slope = 0.0;   // keeps sign(S) == sign(slope)
    const double a0 = xmaj ? sy - sx * slope : sx - sy * slope;
    const double L = g.dx * sqrt(1.0 + slope * slope);
    int klo, khi;
    if (slope == 0.0) {
        if (a0 >= 0.0 && a0 < (double)nmin) {
            klo = 0;
            khi = nmaj - 1;
        } else {
            klo = 1;
            khi = 0;
        }
    } else {
        double xa = (0.0 - a0) / slope, xb = ((double)nmin - a0) / slope;
        if (xa > xb) {
            const double t = xa;
            xa = xb;
            xb = t;
        }
        double lo = floor(xa) - 1.0, hi = ceil(xb);
        lo = fmax(lo, 0.0);
        hi = fmin(hi, (double)(nmaj - 1));
        if (lo > hi) {
            klo = 1;
            khi = 0;
        } else {
            klo = (int)lo;
            khi = (int)hi;
        }
    }
    const long long A0 = llrint(a0 * 4294967296.0);
    const long long S = llrint(slope * 4294967296.0);
    const size_t r = (size_t)v0 * g.nd + j0;
    fix[r] = make_int4((int)(unsigned)(A0 & 0xffffffffLL), (int)(A0 >> 32),
                       (int)(unsigned)(S & 0xffffffffLL), (int)(S >> 32));
    flt[r] = make_float2(slope == 0.0 ? __builtin_inff() : (float)(fabs(1.0 / slope) * 0x1p-32),
                         xmaj != tr ? (float)L : -(float)L);
    span[r] = make_int2(klo, khi);
}

SliceDesc make_slice_desc(const Geom& g, int ray0, int view0, long long sino0, double eta) {
    SliceDesc d;
    d.nv = g.nv;
    d.nd = g.nd;
    d.ray0 = ray0;
    d.view0 = view0;
    d.sino0 = sino0;
    d.sid = (float)g.sid;
    d.sdd = (float)g.sdd;
    d.u0 = (float)(-0.5 * (g.nd - 1) * g.pitch + g.offset);
    d.inv_pitch = (float)(1.0 / g.pitch);
    d.eta = eta;
    d.sym = sym8(g) ? 2 : (sym4(g) ? 1 : 0);
    return d;
}

__global__ void k_set_desc(SliceDesc* desc, int z, SliceDesc d) { desc[z] = d; }
__global__ void k_set_int(int* p, int value) { *p = value; }

void launch_set_desc(SliceDesc* desc, int z, const SliceDesc& d, hipStream_t st) {
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, st, desc, z, d);
}

void launch_set_int(int* p, int value, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, value);
}

void launch_build_ray_table(const Geom& g, RayTable t, hipStream_t st) {
    dim3 grid((g.nd + 255) / 256, table_views(g));
    hipLaunchKernelGGL(k_build_ray_table, grid, dim3(256), 0, st, g, sym8(g) ? g.nv / 4 : 0, t.fix,
                       t.flt, t.span, t.view);
}

// ---------------------------------------------------------------------------
// packing into the padded pair layouts
// ---------------------------------------------------------------------------
template <typename SRC>
__global__ __launch_bounds__(256) void k_pack(const SRC* __restrict__ src, int nsrc, int nx, int ny,
                                              PadLayout P, float2* __restrict__ pad) {
    __shared__ float2 tile[32][33];
    const int z = blockIdx.z;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const size_t npix = (size_t)nx * ny;
    float2* pn = pad + (size_t)z * P.pair;
    float2* pt = pn + P.offT;
    float2* pnr = pn + P.offNR;   // reversed layouts (P.rev: square image)
    float2* ptr = pn + P.offTR;
    const float2 zero = make_float2(0.f, 0.f);
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, k = bx + tx;
        float2 val = zero;
        if (i < ny && k < nx) {
            if constexpr (sizeof(SRC) == sizeof(float2)) {
                val = reinterpret_cast<const float2*>(src)[(size_t)z * npix + (size_t)i * nx + k];
            } else {
                const float* s = reinterpret_cast<const float*>(src);
                val.x = s[(size_t)(2 * z) * npix + (size_t)i * nx + k];
                if (2 * z + 1 < nsrc) val.y = s[(size_t)(2 * z + 1) * npix + (size_t)i * nx + k];
            }
            pn[(size_t)i * P.ldN + k + kPad] = val;
            if (P.rev) pnr[(size_t)i * P.ldN + (nx - 1 - k) + kPad] = val;
        }
        tile[r][tx] = val;
        if (i < ny && tx < kPad) {   // zero ends of row i
            if (blockIdx.x == 0) pn[(size_t)i * P.ldN + tx] = zero;
            if (blockIdx.x == gridDim.x - 1) pn[(size_t)i * P.ldN + kPad + nx + tx] = zero;
            if (P.rev && blockIdx.x == 0) pnr[(size_t)i * P.ldN + tx] = zero;
            if (P.rev && blockIdx.x == gridDim.x - 1) pnr[(size_t)i * P.ldN + kPad + nx + tx] = zero;
        }
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int k = bx + r, i = by + tx;
        if (k < nx && i < ny) {
            pt[(size_t)k * P.ldT + i + kPad] = tile[tx][r];
            if (P.rev) ptr[(size_t)k * P.ldT + (ny - 1 - i) + kPad] = tile[tx][r];
        }
        if (k < nx && tx < kPad) {   // zero ends of column k
            if (blockIdx.y == 0) pt[(size_t)k * P.ldT + tx] = zero;
            if (blockIdx.y == gridDim.y - 1) pt[(size_t)k * P.ldT + kPad + ny + tx] = zero;
            if (P.rev && blockIdx.y == 0) ptr[(size_t)k * P.ldT + tx] = zero;
            if (P.rev && blockIdx.y == gridDim.y - 1) ptr[(size_t)k * P.ldT + kPad + ny + tx] = zero;
        }
    }
}

// zero lines of a non-square image's layouts: padN rows ny.., padT columns nx..
__global__ void k_zero_lines(PadLayout P, int nx, int ny, float2* __restrict__ pad) {
    const size_t nN = (size_t)(P.lines - ny) * P.ldN, nT = (size_t)(P.lines - nx) * P.ldT;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    float2* b = pad + (size_t)blockIdx.y * P.pair;
    if (e < nN)
        b[(size_t)ny * P.ldN + e] = make_float2(0.f, 0.f);
    else if (e < nN + nT)
        b[P.offT + (size_t)nx * P.ldT + (e - nN)] = make_float2(0.f, 0.f);
}

static void launch_zero_lines(const Geom& g, const PadLayout& P, int npairs, float2* pad,
                              hipStream_t st) {
    if (g.nx == g.ny) return;
    const size_t n = (size_t)(P.lines - g.ny) * P.ldN + (size_t)(P.lines - g.nx) * P.ldT;
    hipLaunchKernelGGL(k_zero_lines, dim3((unsigned)((n + 255) / 256), npairs), dim3(256), 0, st, P,
                       g.nx, g.ny, pad);
}

void launch_pack_pairs(const Geom& g, const PadLayout& P, const float* img, int nimg, float2* pad,
                       hipStream_t st) {
    dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, (nimg + 1) / 2);
    hipLaunchKernelGGL(k_pack<float>, grid, dim3(256), 0, st, img, nimg, g.nx, g.ny, P, pad);
    launch_zero_lines(g, P, (nimg + 1) / 2, pad, st);
}

void launch_pack_f2(const Geom& g, const PadLayout& P, const float2* src, int npairs, float2* pad,
                    hipStream_t st) {
    dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, npairs);
    hipLaunchKernelGGL(k_pack<float2>, grid, dim3(256), 0, st, src, 2 * npairs, g.nx, g.ny, P, pad);
    launch_zero_lines(g, P, npairs, pad, st);
}

__global__ void k_pair_sinos(const float* __restrict__ s, int nsino, size_t nray,
                             float2* __restrict__ out) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y;
    if (r >= nray) return;
    float2 v;
    v.x = s[(size_t)(2 * z) * nray + r];
    v.y = (2 * z + 1 < nsino) ? s[(size_t)(2 * z + 1) * nray + r] : 0.f;
    out[(size_t)z * nray + r] = v;
}

void launch_pair_sinos(const Geom& g, const float* sino, int nsino, float2* out, hipStream_t st) {
    const size_t nray = (size_t)g.nv * g.nd;
    dim3 grid((unsigned)((nray + 255) / 256), (nsino + 1) / 2);
    hipLaunchKernelGGL(k_pair_sinos, grid, dim3(256), 0, st, sino, nsino, nray, out);
}

// ---------------------------------------------------------------------------
// forward projector: one lane per ray, kProjLanes adjacent bins of one view per block
// ---------------------------------------------------------------------------
// clamp to [lo, hi] (lo <= hi) in one VALU operation
__device__ __forceinline__ int clamp_med3(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// lanes (bins) per projector block
constexpr int kProjLanes = 128;

// line-search partials per slice: blocks of kProjLanes bins times views rounded up
// to a multiple of 4 (the four-ray form's grid), the same stride in both forms
int proj_nblocks(int nv, int nd) { return ((nd + kProjLanes - 1) / kProjLanes) * ((nv + 3) & ~3); }

// the two minor entries of one major step: float2 (f1, f2) per pixel, or one
// 32-bit word of two BF16 values per pixel
template <bool PB>
__device__ __forceinline__ void load_step(const char* zb, unsigned off, float2& A, float2& B) {
    if constexpr (PB) {
        A = bf16x2_unpack(*reinterpret_cast<const unsigned*>(zb + off));
        B = bf16x2_unpack(*reinterpret_cast<const unsigned*>(zb + off + 4));
    } else {
        A = *reinterpret_cast<const float2*>(zb + off);
        B = *reinterpret_cast<const float2*>(zb + off + 8);
    }
}

template <bool RB>
__device__ __forceinline__ void store_res(float2* res, long long i, float x, float y) {
    if constexpr (RB)
        reinterpret_cast<unsigned*>(res)[i] = bf16x2_pack(x, y);
    else
        res[i] = make_float2(x, y);
}

// PB: the pair blocks hold BF16 pairs; RB: the output sinogram pairs are BF16
// Both forward-projector forms compute every value exactly as written (no
// contraction of the epilogue's products into fused multiply-adds, which the
// compiler could otherwise choose differently in the two kernels), so that a
// symmetric slice's rays are the same bit for bit in either form.
template <int MODE, bool PB, bool RB>
__global__ __launch_bounds__(kProjLanes) void k_project(const void* __restrict__ pad, PadLayout P,
                                                 RayTable T, int nx, int ny, ProjArgs a) {
#pragma clang fp contract(off)
    constexpr unsigned ES = PB ? 4u : 8u;   // bytes per pixel entry
    constexpr int LS = PB ? 2 : 3;
    const int v = blockIdx.y, z = blockIdx.z;
    const SliceDesc D = T.desc[T.desc_stride * z];
    if (a.plain_only && D.sym) return;   // block-uniform: k_project4 takes this slice
    const int nd = D.nd;
    const int j = blockIdx.x * kProjLanes + threadIdx.x;
    const bool valid = j < nd && v < D.nv;   // the grid covers the batch's largest slice
    const size_t r = (size_t)v * nd + j;     // ray within the slice
    // quarter-turn symmetry: view v = vt + rot * nv/4 takes ray (vt, j) of the
    // table, applied to the image turned rot times
    int rot = 0, vt = v;
    if (D.sym) {
        const int q4 = D.nv >> 2;
        rot = min(v / q4, 3);
        vt = v - rot * q4;
    }
    const size_t rt = (size_t)D.ray0 + (size_t)vt * nd + j;   // its table entry
    const long long s0 = D.sino0 + (long long)z * T.sino_zstride;
    const int4 fx = valid ? T.fix[rt] : make_int4(0, 0, 0, 0);
    const float2 fl = valid ? T.flt[rt] : make_float2(__builtin_inff(), 1.f);
    const int2 sp = valid ? T.span[rt] : make_int2(1, 0);
    const bool xmaj = fl.y > 0.f;
    const float L = fabsf(fl.y);
    const float ainv32 = fl.x;
    const long long S = fix_s(fx);
    const bool up = S >= 0;
    const unsigned xmask = up ? ~0u : 0u;
    const int nmin = xmaj ? ny : nx;
    // Step k reads minor entries r' and r' + 1 of major line k, r' = r0 (s >= 0:
    // pixels r0, r0 + 1) or r0 - 1 (s < 0: pixels r0, r0 - 1), with r0 = floor(y)
    // clamped so that both entries stay inside the line's zero ends; a clamped
    // step reads zeros only.  Byte offsets are 32-bit, relative to the pair block.
    const int rlo = up ? -kPad : 1 - kPad, rhi = up ? nmin : nmin + 1;
    const float wa = up ? 0.f : 1.f, wb = up ? 1.f : -1.f;   // weight of entry r': wa + wb * w0
    // layout read at major step k: pixel (minor m, major k) of the turned image
    // is entry m of line k (or nmaj - 1 - k) of padT / padN or their reversed
    // copies (square images only when turned)
    bool useT = xmaj, rev_line = false, rev_entry = false;
    if (rot) {
        useT = xmaj != ((rot & 1) != 0);
        rev_line = xmaj ? rot >= 2 : (rot == 1 || rot == 2);
        rev_entry = xmaj ? (rot == 1 || rot == 2) : rot >= 2;
    }
    const unsigned lbase = (unsigned)(useT ? (rev_entry ? P.offTR : P.offT) : (rev_entry ? P.offNR : 0));
    const unsigned lstep_abs = ES * (unsigned)(useT ? P.ldT : P.ldN);
    const unsigned lstep = rev_line ? 0u - lstep_abs : lstep_abs;   // modulo 2^32
    const int nmaj = xmaj ? nx : ny;
    int klo = sp.x, khi = sp.y;
    if (klo > khi) {
        klo = INT_MAX;
        khi = INT_MIN;
    }
    const int ks = max(wave_min(klo), 0), ke = min(wave_max(khi), max(nx, ny) - 1);
    const int k0 = ks == INT_MAX ? 0 : ks;
    long long y = fix_a0(fx) + (long long)k0 * S;
    const int kl0 = rev_line ? nmaj - 1 - k0 : k0;   // physical line of step k0
    unsigned loff = ES * (lbase + (unsigned)(kPad + (up ? 0 : -1))) + (unsigned)kl0 * lstep_abs;
    const char* zb = reinterpret_cast<const char*>(pad) + (size_t)z * P.pair * ES;
    float s1 = 0.f, c1 = 0.f, s2 = 0.f, c2 = 0.f;
    const int nstep = ks <= ke ? ke - ks + 1 : 0;   // wave-uniform
    int k = 0;
    for (; k + 4 <= nstep; k += 4) {
        float2 A[4], B[4];
        float W[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r0 = clamp_med3((int)(y >> 32), rlo, rhi);
            load_step<PB>(zb, loff + ((unsigned)r0 << LS), A[u], B[u]);
            W[u] = fmaf(wb, first_weight((unsigned)y, xmask, ainv32), wa);
            y += S;
            loff += lstep;
        }
        // four steps summed pairwise, the group sum added with compensation
        float v1[4], v2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v1[u] = fmaf(W[u], A[u].x - B[u].x, B[u].x);
            v2[u] = fmaf(W[u], A[u].y - B[u].y, B[u].y);
        }
        kahan_add(s1, c1, (v1[0] + v1[1]) + (v1[2] + v1[3]));
        kahan_add(s2, c2, (v2[0] + v2[1]) + (v2[2] + v2[3]));
    }
    for (; k < nstep; ++k) {
        const int r0 = clamp_med3((int)(y >> 32), rlo, rhi);
        float2 A, B;
        load_step<PB>(zb, loff + ((unsigned)r0 << LS), A, B);
        const float W = fmaf(wb, first_weight((unsigned)y, xmask, ainv32), wa);
        kahan_add(s1, c1, fmaf(W, A.x - B.x, B.x));
        kahan_add(s2, c2, fmaf(W, A.y - B.y, B.y));
        y += S;
        loff += lstep;
    }
    const double Y1 = (double)L * ((double)s1 - (double)c1);
    const double Y2 = (double)L * ((double)s2 - (double)c2);
    const size_t nray = (size_t)D.nv * nd;
    if constexpr (MODE == PROJ_PLAIN) {
        if (valid) {
            a.out[(size_t)(2 * s0) + r] = (float)Y1;
            if (2 * z + 1 < a.nout) a.out[(size_t)(2 * s0) + nray + r] = (float)Y2;
        }
    } else if constexpr (MODE == PROJ_RESID) {
        if (valid) {
            const double rl = (double)a.c00 * Y1 + (double)a.c01 * Y2 - (double)a.p_lo[s0 - a.p_base + r];
            const double rh = (double)a.c10 * Y1 + (double)a.c11 * Y2 - (double)a.p_hi[s0 - a.p_base + r];
            store_res<RB>(a.res, s0 + r, (float)(D.eta * ((double)a.c00 * rl + (double)a.c10 * rh)),
                          (float)(D.eta * ((double)a.c01 * rl + (double)a.c11 * rh)));
        }
    } else {   // PROJ_LINESEARCH
        __shared__ double sh[kProjLanes / 64];
        double part = 0.0;
        if (valid) {
            const double yl = (double)a.c00 * Y1 + (double)a.c01 * Y2;
            const double yh = (double)a.c10 * Y1 + (double)a.c11 * Y2;
            store_res<RB>(a.res, s0 + r, (float)(D.eta * ((double)a.c00 * yl + (double)a.c10 * yh)),
                          (float)(D.eta * ((double)a.c01 * yl + (double)a.c11 * yh)));
            part = D.eta * (yl * yl + yh * yh);
        }
        // partials in the slice's own block order (the launch may cover a larger
        // slice of the batch), so a slice reduces exactly as it does alone
        const int nbx = (nd + kProjLanes - 1) / kProjLanes;
        if (v >= D.nv || (int)blockIdx.x >= nbx) return;
        const int bid = v * nbx + blockIdx.x;
        double* zp = a.partials + (size_t)z * a.part_stride;
        const double bs = block_sum<kProjLanes>(part, sh);
        if (threadIdx.x == 0) zp[bid] = bs;
    }
}

// Forward projector of quarter-turn symmetric slices: lane j of block vt
// steps ray (vt, j) of the table once and reads the four turned images at
// every step, producing rays (vt + t nv/4, j), t = 0..3.  The traversal, the
// clamp and the step weight are shared by the four rays; each ray's value is
// summed exactly as k_project sums it (same steps, same grouping), so the two
// kernels agree bit for bit.  Line-search partials go to the same per-view
// block slots.
template <int MODE, bool PB, bool RB>
__global__ __launch_bounds__(kProjLanes) void k_project4(const void* __restrict__ pad, PadLayout P,
                                                  RayTable T, int n, ProjArgs a) {
#pragma clang fp contract(off)
    constexpr unsigned ES = PB ? 4u : 8u;
    constexpr int LS = PB ? 2 : 3;
    const int vt = blockIdx.y, z = blockIdx.z;
    const SliceDesc D = T.desc[T.desc_stride * z];
    const int nd = D.nd, q4 = D.nv >> 2;
    if (!D.sym || vt >= q4) return;   // block-uniform
    const int j = blockIdx.x * kProjLanes + threadIdx.x;
    const bool valid = j < nd;
    const size_t rt = (size_t)D.ray0 + (size_t)vt * nd + j;
    const long long s0 = D.sino0 + (long long)z * T.sino_zstride;
    const int4 fx = valid ? T.fix[rt] : make_int4(0, 0, 0, 0);
    const float2 fl = valid ? T.flt[rt] : make_float2(__builtin_inff(), 1.f);
    const int2 sp = valid ? T.span[rt] : make_int2(1, 0);
    const bool xmaj = fl.y > 0.f;
    const float L = fabsf(fl.y);
    const float ainv32 = fl.x;
    const long long S = fix_s(fx);
    const bool up = S >= 0;
    const unsigned xmask = up ? ~0u : 0u;
    const int rlo = up ? -kPad : 1 - kPad, rhi = up ? n : n + 1;
    const float wa = up ? 0.f : 1.f, wb = up ? 1.f : -1.f;
    int klo = sp.x, khi = sp.y;
    if (klo > khi) {
        klo = INT_MAX;
        khi = INT_MIN;
    }
    const int ks = max(wave_min(klo), 0), ke = min(wave_max(khi), n - 1);
    const int k0 = ks == INT_MAX ? 0 : ks;
    const unsigned lstep_abs = ES * (unsigned)P.ldN;   // square image: ldN == ldT
    unsigned loff[4], lstep[4];
#pragma unroll
    for (int rot = 0; rot < 4; ++rot) {
        bool useT = xmaj, rev_line = false, rev_entry = false;
        if (rot) {
            useT = xmaj != ((rot & 1) != 0);
            rev_line = xmaj ? rot >= 2 : (rot == 1 || rot == 2);
            rev_entry = xmaj ? (rot == 1 || rot == 2) : rot >= 2;
        }
        const unsigned lbase =
            (unsigned)(useT ? (rev_entry ? P.offTR : P.offT) : (rev_entry ? P.offNR : 0));
        const int kl0 = rev_line ? n - 1 - k0 : k0;
        loff[rot] = ES * (lbase + (unsigned)(kPad + (up ? 0 : -1))) + (unsigned)kl0 * lstep_abs;
        lstep[rot] = rev_line ? 0u - lstep_abs : lstep_abs;
    }
    long long y = fix_a0(fx) + (long long)k0 * S;
    const char* zb = reinterpret_cast<const char*>(pad) + (size_t)z * P.pair * ES;
    float s1[4], c1[4], s2[4], c2[4];
#pragma unroll
    for (int rot = 0; rot < 4; ++rot) s1[rot] = c1[rot] = s2[rot] = c2[rot] = 0.f;
    const int nstep = ks <= ke ? ke - ks + 1 : 0;   // wave-uniform
    int k = 0;
    for (; k + 4 <= nstep; k += 4) {
        unsigned eo[4];
        float W[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            eo[u] = (unsigned)clamp_med3((int)(y >> 32), rlo, rhi) << LS;
            W[u] = fmaf(wb, first_weight((unsigned)y, xmask, ainv32), wa);
            y += S;
        }
#pragma unroll
        for (int rot = 0; rot < 4; ++rot) {
            float2 A[4], B[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) load_step<PB>(zb, loff[rot] + (unsigned)u * lstep[rot] + eo[u], A[u], B[u]);
            float v1[4], v2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v1[u] = fmaf(W[u], A[u].x - B[u].x, B[u].x);
                v2[u] = fmaf(W[u], A[u].y - B[u].y, B[u].y);
            }
            kahan_add(s1[rot], c1[rot], (v1[0] + v1[1]) + (v1[2] + v1[3]));
            kahan_add(s2[rot], c2[rot], (v2[0] + v2[1]) + (v2[2] + v2[3]));
            loff[rot] += 4u * lstep[rot];
        }
    }
    for (; k < nstep; ++k) {
        const unsigned eo = (unsigned)clamp_med3((int)(y >> 32), rlo, rhi) << LS;
        const float W = fmaf(wb, first_weight((unsigned)y, xmask, ainv32), wa);
#pragma unroll
        for (int rot = 0; rot < 4; ++rot) {
            float2 A, B;
            load_step<PB>(zb, loff[rot] + eo, A, B);
            kahan_add(s1[rot], c1[rot], fmaf(W, A.x - B.x, B.x));
            kahan_add(s2[rot], c2[rot], fmaf(W, A.y - B.y, B.y));
            loff[rot] += lstep[rot];
        }
        y += S;
    }
    const size_t nray = (size_t)D.nv * nd;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rot = 0; rot < 4; ++rot) {
        const double Y1 = (double)L * ((double)s1[rot] - (double)c1[rot]);
        const double Y2 = (double)L * ((double)s2[rot] - (double)c2[rot]);
        const size_t r = (size_t)(vt + rot * q4) * nd + j;   // ray of view vt + rot nv/4
        if (!valid) continue;
        if constexpr (MODE == PROJ_PLAIN) {
            a.out[(size_t)(2 * s0) + r] = (float)Y1;
            if (2 * z + 1 < a.nout) a.out[(size_t)(2 * s0) + nray + r] = (float)Y2;
        } else if constexpr (MODE == PROJ_RESID) {
            const double rl = (double)a.c00 * Y1 + (double)a.c01 * Y2 - (double)a.p_lo[s0 - a.p_base + r];
            const double rh = (double)a.c10 * Y1 + (double)a.c11 * Y2 - (double)a.p_hi[s0 - a.p_base + r];
            store_res<RB>(a.res, s0 + r, (float)(D.eta * ((double)a.c00 * rl + (double)a.c10 * rh)),
                          (float)(D.eta * ((double)a.c01 * rl + (double)a.c11 * rh)));
        } else {
            const double yl = (double)a.c00 * Y1 + (double)a.c01 * Y2;
            const double yh = (double)a.c10 * Y1 + (double)a.c11 * Y2;
            store_res<RB>(a.res, s0 + r, (float)(D.eta * ((double)a.c00 * yl + (double)a.c10 * yh)),
                          (float)(D.eta * ((double)a.c01 * yl + (double)a.c11 * yh)));
            part[rot] = D.eta * (yl * yl + yh * yh);
        }
    }
    if constexpr (MODE == PROJ_LINESEARCH) {
        __shared__ double sh[kProjLanes / 64];
        const int nbx = (nd + kProjLanes - 1) / kProjLanes;
        if ((int)blockIdx.x >= nbx) return;
        double* zp = a.partials + (size_t)z * a.part_stride;
#pragma unroll
        for (int rot = 0; rot < 4; ++rot) {
            const double bs = block_sum<kProjLanes>(part[rot], sh);
            if (threadIdx.x == 0) zp[(vt + rot * q4) * nbx + blockIdx.x] = bs;
        }
    }
}

// Exact line-search step of each slice, one block per slice: alpha = num / den
// from the gradient kernel's image partials (num, coupling, regulariser) and
// the projector's per-block data partials, each summed in its fixed slot
// order, so a slice's step does not depend on the batch or the launch form.
constexpr int kAlphaThreads = 1024;

__global__ __launch_bounds__(kAlphaThreads) void k_alpha(RayTable T, ProjArgs a) {
    __shared__ double sh[4 * (kAlphaThreads / 64)];
    const int z = blockIdx.x;
    const SliceDesc D = T.desc[T.desc_stride * z];
    const int nblk = ((D.nd + kProjLanes - 1) / kProjLanes) * D.nv;
    const double* zp = a.partials + (size_t)z * a.part_stride;
    const double* ip = a.img_partials + (size_t)z * a.img_nblocks * 3;
    // (data, num, coupling, regulariser), each thread over its own slots in
    // ascending order (unrolled so that the loads are issued together; the
    // additions keep their order)
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int i = threadIdx.x; i < nblk; i += kAlphaThreads) s[0] += zp[i];
#pragma unroll 2
    for (int i = threadIdx.x; i < a.img_nblocks; i += kAlphaThreads) {
        s[1] += ip[3 * i];
        s[2] += ip[3 * i + 1];
        s[3] += ip[3 * i + 2];
    }
    block_sum_n<kAlphaThreads, 4>(s, sh);
    if (threadIdx.x == 0) {
        const double wr = a.beta_z ? 2.0 * a.beta_z[z] : a.w_reg;
        const double den = a.w_data * s[0] + a.w_coup * s[2] + wr * s[3];
        a.alpha[z] = den > 0.0 ? s[1] / den : 0.0;
    }
}

static void launch_rays(const Geom& g, const PadLayout& P, const RayTable& t, const void* pad, int npairs,
                        int mode, ProjArgs a, hipStream_t st) {
    if (a.four_ray && P.rev) {
        dim3 grid4((t.nd_max + kProjLanes - 1) / kProjLanes, (t.nv_max + 3) / 4, npairs);
        if (mode == PROJ_PLAIN)
            hipLaunchKernelGGL((k_project4<PROJ_PLAIN, false, false>), grid4, dim3(kProjLanes), 0, st, pad, P, t,
                               g.nx, a);
        else if (mode == PROJ_RESID && a.res_bf16)
            hipLaunchKernelGGL((k_project4<PROJ_RESID, false, true>), grid4, dim3(kProjLanes), 0, st, pad, P, t,
                               g.nx, a);
        else if (mode == PROJ_RESID)
            hipLaunchKernelGGL((k_project4<PROJ_RESID, false, false>), grid4, dim3(kProjLanes), 0, st, pad, P, t,
                               g.nx, a);
        else if (a.pad_bf16)
            hipLaunchKernelGGL((k_project4<PROJ_LINESEARCH, true, true>), grid4, dim3(kProjLanes), 0, st, pad, P,
                               t, g.nx, a);
        else
            hipLaunchKernelGGL((k_project4<PROJ_LINESEARCH, false, false>), grid4, dim3(kProjLanes), 0, st, pad,
                               P, t, g.nx, a);
        if (!a.has_plain) return;
        a.plain_only = true;   // the other slices in the per-view form
    }
    dim3 grid((t.nd_max + kProjLanes - 1) / kProjLanes, t.nv_max, npairs);
    if (mode == PROJ_PLAIN)
        hipLaunchKernelGGL((k_project<PROJ_PLAIN, false, false>), grid, dim3(kProjLanes), 0, st, pad, P, t,
                           g.nx, g.ny, a);
    else if (mode == PROJ_RESID && a.res_bf16)
        hipLaunchKernelGGL((k_project<PROJ_RESID, false, true>), grid, dim3(kProjLanes), 0, st, pad, P, t,
                           g.nx, g.ny, a);
    else if (mode == PROJ_RESID)
        hipLaunchKernelGGL((k_project<PROJ_RESID, false, false>), grid, dim3(kProjLanes), 0, st, pad, P, t,
                           g.nx, g.ny, a);
    else if (a.pad_bf16)
        hipLaunchKernelGGL((k_project<PROJ_LINESEARCH, true, true>), grid, dim3(kProjLanes), 0, st, pad, P,
                           t, g.nx, g.ny, a);
    else
        hipLaunchKernelGGL((k_project<PROJ_LINESEARCH, false, false>), grid, dim3(kProjLanes), 0, st, pad,
                           P, t, g.nx, g.ny, a);
}

void launch_project(const Geom& g, const PadLayout& P, const RayTable& t, const void* pad, int npairs,
                    int mode, const ProjArgs& a_in, hipStream_t st) {
    ProjArgs a = a_in;
    a.part_stride = (size_t)proj_nblocks(t.nv_max, t.nd_max);
    a.plain_only = false;
    launch_rays(g, P, t, pad, npairs, mode, a, st);
    if (mode == PROJ_LINESEARCH)
        hipLaunchKernelGGL(k_alpha, dim3(npairs), dim3(kAlphaThreads), 0, st, t, a);
}

// ---------------------------------------------------------------------------
// back-projector: voxel-driven, exact transpose of the projector's weights.
// A block covers a 16 x 16 pixel tile with 8 wavefronts; each lane owns a
// 2 x 2 pixel quad (so one ray-table read serves four pixels) and wavefront
// w takes views w, w + 8, ...  Per view, the lanes' detector footprints
// (bounding box of the quad, projected from the source) give each lane its
// candidate bins; the union window is staged once per wavefront in LDS, so
// the candidate loop reads LDS only.  The 8 partial sums of every pixel are
// added in a fixed order at the end (deterministic, no atomics).
// ---------------------------------------------------------------------------
constexpr int kBpWaves = 8;
constexpr int kBpViewChunk = 256;

// SB: the sinogram pairs are BF16 (one 32-bit word per ray)
template <bool SB>
__global__ __launch_bounds__(kBpWaves * 64) void k_backproject(
    const void* __restrict__ sino, RayTable T, int nx, int ny, float dxmm,
    float2* __restrict__ out_pairs, float* __restrict__ out_split, int nout) {
    __shared__ float4 vs[kBpViewChunk];
    __shared__ int4 sfix[kBpWaves][64];
    __shared__ float4 sray[kBpWaves][64];      // (2^-32/|s|, +-L, L sino lo, L sino hi)
    __shared__ float red[kBpWaves][8][64];
    const int z = blockIdx.z;
    const SliceDesc D = T.desc[T.desc_stride * z];
    if (D.sym) return;   // quarter-turn symmetric slices: k_backproject_sym
    const int nv = D.nv, nd = D.nd;
    const float sid = D.sid, sdd = D.sdd, u0 = D.u0, inv_pitch = D.inv_pitch;
    const int4* __restrict__ fix = T.fix + D.ray0;
    const float2* __restrict__ flt = T.flt + D.ray0;
    const float4* __restrict__ view = T.view + D.view0;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // w: wave-uniform
    const int i0 = blockIdx.y * 16 + 2 * (lane >> 3), k0 = blockIdx.x * 16 + 2 * (lane & 7);
    // quad centre (between pixels k0, k0 + 1 and rows i0, i0 + 1)
    const float x = ((float)k0 + 0.5f - 0.5f * (float)(nx - 1)) * dxmm;
    const float y = ((float)i0 + 0.5f - 0.5f * (float)(ny - 1)) * dxmm;
    const long long sbase = D.sino0 + (long long)z * T.sino_zstride;
    const float2* sz = reinterpret_cast<const float2*>(sino) + sbase;
    const unsigned* szb = reinterpret_cast<const unsigned*>(sino) + sbase;
    // acc[di][dk]: pixel (i0 + di, k0 + dk), both channels
    float a00x = 0.f, a00y = 0.f, a01x = 0.f, a01y = 0.f;
    float a10x = 0.f, a10y = 0.f, a11x = 0.f, a11y = 0.f;
    for (int v0 = 0; v0 < nv; v0 += kBpViewChunk) {
        const int nvc = min(kBpViewChunk, nv - v0);
        __syncthreads();
        for (int q = threadIdx.x; q < nvc; q += kBpWaves * 64) vs[q] = view[v0 + q];
        __syncthreads();
        for (int vv = w; vv < nvc; vv += kBpWaves) {
            const float4 vc = vs[vv];
            const float e = 2.f * vc.z;   // half-extent of the quad along both view axes
            const float U = sid - (x * vc.x + y * vc.y);
            const float W = y * vc.x - x * vc.y;
            const float rm = __builtin_amdgcn_rcpf(U - e);
            const float rp = __builtin_amdgcn_rcpf(U + e);
            const float hi = W + e, lo = W - e;
            const float umax = sdd * hi * (hi >= 0.f ? rm : rp);
            const float umin = sdd * lo * (lo >= 0.f ? rp : rm);
            int jl = max((int)ceilf((umin - u0) * inv_pitch - 1e-3f), 0);
            int jh = min((int)floorf((umax - u0) * inv_pitch + 1e-3f), nd - 1);
            if (jl > jh) {
                jl = INT_MAX;
                jh = INT_MIN;
            }
            // (clamped to the detector: empty stays empty)
            const int Jlo = max(wave_min(jl), 0), Jhi = min(wave_max(jh), nd - 1);
            if (Jlo > Jhi) continue;   // wave-uniform
            const int v = v0 + vv;
            for (int base = Jlo; base <= Jhi; base += 64) {
                const int jj = base + lane;
                if (jj <= Jhi) {
                    const size_t r = (size_t)v * nd + jj;
                    const float2 fl = flt[r];
                    const float2 sv = SB ? bf16x2_unpack(szb[r]) : sz[r];
                    const float L = fabsf(fl.y);
                    sfix[w][lane] = fix[r];
                    sray[w][lane] = make_float4(fl.x, fl.y, L * sv.x, L * sv.y);
                }
                __builtin_amdgcn_wave_barrier();
                const int ja = max(jl, base), jb = min(jh, base + 63);
                for (int j = ja; j <= jb; ++j) {
                    const int4 fx = sfix[w][j - base];
                    const float4 fs = sray[w][j - base];
                    const bool xm = fs.y > 0.f;
                    const long long S = fix_s(fx);
                    const bool up = S >= 0;
                    const int maj0 = xm ? k0 : i0, mnr0 = xm ? i0 : k0;
                    const long long ya = fix_a0(fx) + (long long)(unsigned)maj0 * S;
                    const long long yb = ya + S;
                    const unsigned xmask = up ? ~0u : 0u;
                    const float wa = first_weight((unsigned)ya, xmask, fs.x);
                    const float wb = first_weight((unsigned)yb, xmask, fs.x);
                    // minor row r0 = floor(y) gets w0, its neighbour r0 +- 1 gets 1 - w0;
                    // e = r0 - mnr0, and row n of the quad is the neighbour when e == o_n
                    const int ea = (int)(ya >> 32) - mnr0, eb = (int)(yb >> 32) - mnr0;
                    const int o0 = up ? -1 : 1, o1 = up ? 0 : 2;
                    const float ca0 = ea == 0 ? wa : (ea == o0 ? 1.f - wa : 0.f);
                    const float ca1 = ea == 1 ? wa : (ea == o1 ? 1.f - wa : 0.f);
                    const float cb0 = eb == 0 ? wb : (eb == o0 ? 1.f - wb : 0.f);
                    const float cb1 = eb == 1 ? wb : (eb == o1 ? 1.f - wb : 0.f);
                    // (major, minor) offsets -> (row, column) offsets of the quad
                    const float c01 = xm ? cb0 : ca1, c10 = xm ? ca1 : cb0;
                    const float s1 = fs.z, s2 = fs.w;
                    a00x = fmaf(ca0, s1, a00x);
                    a00y = fmaf(ca0, s2, a00y);
                    a01x = fmaf(c01, s1, a01x);
                    a01y = fmaf(c01, s2, a01y);
                    a10x = fmaf(c10, s1, a10x);
                    a10y = fmaf(c10, s2, a10y);
                    a11x = fmaf(cb1, s1, a11x);
                    a11y = fmaf(cb1, s2, a11y);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    red[w][0][lane] = a00x;
    red[w][1][lane] = a00y;
    red[w][2][lane] = a01x;
    red[w][3][lane] = a01y;
    red[w][4][lane] = a10x;
    red[w][5][lane] = a10y;
    red[w][6][lane] = a11x;
    red[w][7][lane] = a11y;
    __syncthreads();
    if (threadIdx.x >= 256) return;
    const int ti = threadIdx.x >> 4, tk = threadIdx.x & 15;
    const int i = blockIdx.y * 16 + ti, k = blockIdx.x * 16 + tk;
    if (i >= ny || k >= nx) return;
    const int ql = (ti >> 1) * 8 + (tk >> 1);
    const int slot = ((ti & 1) * 2 + (tk & 1)) * 2;
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int q = 0; q < kBpWaves; ++q) {
        s1 += red[q][slot][ql];
        s2 += red[q][slot + 1][ql];
    }
    const size_t npix = (size_t)nx * ny;
    const size_t p = (size_t)i * nx + k;
    if (out_pairs) {
        out_pairs[(size_t)z * npix + p] = make_float2(s1, s2);
    } else {
        out_split[(size_t)(2 * z) * npix + p] = s1;
        if (2 * z + 1 < nout) out_split[(size_t)(2 * z + 1) * npix + p] = s2;
    }
}

// ---------------------------------------------------------------------------
// back-projector of quarter-turn symmetric slices.  The turn R(i, k) =
// (k, n - 1 - i) maps tile T0 of the image's first quadrant to T1 = R T0,
// T2 = R^2 T0 and T3 = R^3 T0, and ray (v + t nv/4, j) meets pixel R^t p with
// the weight that ray (v, j) of the table has on p.  A block owns the four
// tiles of one orbit with 16 wavefronts: wavefront w works on tile w & 3 and
// table views v = w >> 2 (mod 4).  Each lane owns a 2 x 2 quad of its tile,
// evaluates the weights of ray (v, j) on its quad once, exactly as the
// voxel-driven kernel does, and accumulates them times the residuals of
// views v + t nv/4, t = 0..3, for the quads R^t of its own.  The partial
// sums reach the tiles in LDS in a fixed order (turn, view class), so the
// result is deterministic.  Blocks loop over the orbits; for one slice the
// grid covers at most half the CUs, so that the short kernels of the
// concurrent PCG find CUs free of these long-lived workgroups.
// ---------------------------------------------------------------------------
constexpr int kBsWaves = 16;

template <bool SB>
__global__ __launch_bounds__(kBsWaves * 64) void k_backproject_sym(
    const void* __restrict__ sino, RayTable T, int n, float dxmm, float2* __restrict__ out_pairs,
    float* __restrict__ out_split, int nout, int norb_z) {
    __shared__ float4 vs[kBpViewChunk];
    __shared__ int4 sfix[kBsWaves][64];
    __shared__ float2 sfl[kBsWaves][64];        // (2^-32/|s|, +-L)
    __shared__ float4 ssn[kBsWaves][64][2];     // L times the residual pairs of the four turns
    // the four tiles' sums [tile][channel][row][column], in ssn's memory once
    // every view is done
    float(*acc_t)[2][16][17] = reinterpret_cast<float(*)[2][16][17]>(&ssn[0][0][0]);
    static_assert(sizeof(ssn) >= sizeof(float) * 4 * 2 * 16 * 17, "tile sums");
    const int nq = n / 32;   // orbits per axis (first-quadrant tiles)
    for (int orb = blockIdx.x; orb < nq * nq * norb_z; orb += gridDim.x) {
    const int z = orb / (nq * nq);
    const int obx = orb % nq, oby = (orb / nq) % nq;
    const SliceDesc D = T.desc[T.desc_stride * z];
    if (D.sym != 1) continue;   // block-uniform (sym == 2: k_backproject_sym8)
    const int nd = D.nd, q4 = D.nv >> 2;
    const float sid = D.sid, sdd = D.sdd, u0 = D.u0, inv_pitch = D.inv_pitch;
    const int4* __restrict__ fix = T.fix + D.ray0;
    const float2* __restrict__ flt = T.flt + D.ray0;
    const float4* __restrict__ view = T.view + D.view0;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // w: wave-uniform
    const int a = w & 3, cls = w >> 2;
    // tile origins (row, column) of T0..T3
    const int ty0 = oby * 16, tx0 = obx * 16;
    const int oy[4] = {ty0, tx0, n - 16 - ty0, n - 16 - tx0};
    const int ox[4] = {tx0, n - 16 - ty0, n - 16 - tx0, ty0};
    const int i0 = oy[a] + 2 * (lane >> 3), k0 = ox[a] + 2 * (lane & 7);
    const float x = ((float)k0 + 0.5f - 0.5f * (float)(n - 1)) * dxmm;
    const float y = ((float)i0 + 0.5f - 0.5f * (float)(n - 1)) * dxmm;
    const long long sbase = D.sino0 + (long long)z * T.sino_zstride;
    const float2* sz = reinterpret_cast<const float2*>(sino) + sbase;
    const unsigned* szb = reinterpret_cast<const unsigned*>(sino) + sbase;
    const size_t tstep = (size_t)q4 * nd;   // rays of one quarter of the views
    // acc[t][q]: turn t, q = 2 * (2 * di + dk) + channel for pixel (i0 + di, k0 + dk)
    float acc[4][8];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[t][q] = 0.f;
    for (int v0 = 0; v0 < q4; v0 += kBpViewChunk) {
        const int nvc = min(kBpViewChunk, q4 - v0);
        __syncthreads();
        for (int q = threadIdx.x; q < nvc; q += kBsWaves * 64) vs[q] = view[v0 + q];
        __syncthreads();
        for (int vv = cls; vv < nvc; vv += 4) {
            const float4 vc = vs[vv];
            const float e = 2.f * vc.z;
            const float U = sid - (x * vc.x + y * vc.y);
            const float W = y * vc.x - x * vc.y;
            const float rm = __builtin_amdgcn_rcpf(U - e);
            const float rp = __builtin_amdgcn_rcpf(U + e);
            const float hi = W + e, lo = W - e;
            const float umax = sdd * hi * (hi >= 0.f ? rm : rp);
            const float umin = sdd * lo * (lo >= 0.f ? rp : rm);
            int jl = max((int)ceilf((umin - u0) * inv_pitch - 1e-3f), 0);
            int jh = min((int)floorf((umax - u0) * inv_pitch + 1e-3f), nd - 1);
            if (jl > jh) {
                jl = INT_MAX;
                jh = INT_MIN;
            }
            // (clamped to the detector: empty stays empty)
            const int Jlo = max(wave_min(jl), 0), Jhi = min(wave_max(jh), nd - 1);
            if (Jlo > Jhi) continue;   // wave-uniform
            const int v = v0 + vv;
            for (int base = Jlo; base <= Jhi; base += 64) {
                const int jj = base + lane;
                if (jj <= Jhi) {
                    const size_t r = (size_t)v * nd + jj;
                    float2 s4[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        s4[t] = SB ? bf16x2_unpack(szb[r + t * tstep]) : sz[r + t * tstep];
                    const float2 fl = flt[r];
                    const float L = fabsf(fl.y);
                    sfix[w][lane] = fix[r];
                    sfl[w][lane] = fl;
                    ssn[w][lane][0] = make_float4(L * s4[0].x, L * s4[0].y, L * s4[1].x, L * s4[1].y);
                    ssn[w][lane][1] = make_float4(L * s4[2].x, L * s4[2].y, L * s4[3].x, L * s4[3].y);
                }
                __builtin_amdgcn_wave_barrier();
                const int ja = max(jl, base), jb = min(jh, base + 63);
                for (int j = ja; j <= jb; ++j) {
                    const int4 fx = sfix[w][j - base];
                    const float2 fs = sfl[w][j - base];
                    const bool xm = fs.y > 0.f;
                    const long long S = fix_s(fx);
                    const bool up = S >= 0;
                    const int maj0 = xm ? k0 : i0, mnr0 = xm ? i0 : k0;
                    const long long ya = fix_a0(fx) + (long long)(unsigned)maj0 * S;
                    const long long yb = ya + S;
                    const unsigned xmask = up ? ~0u : 0u;
                    const float wa = first_weight((unsigned)ya, xmask, fs.x);
                    const float wb = first_weight((unsigned)yb, xmask, fs.x);
                    const int ea = (int)(ya >> 32) - mnr0, eb = (int)(yb >> 32) - mnr0;
                    const int o0 = up ? -1 : 1, o1 = up ? 0 : 2;
                    const float ca0 = ea == 0 ? wa : (ea == o0 ? 1.f - wa : 0.f);
                    const float ca1 = ea == 1 ? wa : (ea == o1 ? 1.f - wa : 0.f);
                    const float cb0 = eb == 0 ? wb : (eb == o0 ? 1.f - wb : 0.f);
                    const float cb1 = eb == 1 ? wb : (eb == o1 ? 1.f - wb : 0.f);
                    const float c01 = xm ? cb0 : ca1, c10 = xm ? ca1 : cb0;
                    const float4 sA = ssn[w][j - base][0], sB = ssn[w][j - base][1];
                    const float sv[8] = {sA.x, sA.y, sA.z, sA.w, sB.x, sB.y, sB.z, sB.w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float s1 = sv[2 * t], s2 = sv[2 * t + 1];
                        acc[t][0] = fmaf(ca0, s1, acc[t][0]);
                        acc[t][1] = fmaf(ca0, s2, acc[t][1]);
                        acc[t][2] = fmaf(c01, s1, acc[t][2]);
                        acc[t][3] = fmaf(c01, s2, acc[t][3]);
                        acc[t][4] = fmaf(c10, s1, acc[t][4]);
                        acc[t][5] = fmaf(c10, s2, acc[t][5]);
                        acc[t][6] = fmaf(cb1, s1, acc[t][6]);
                        acc[t][7] = fmaf(cb1, s2, acc[t][7]);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    // the four tiles in LDS: turn t of tile a lands in tile (a + t) & 3; in each
    // round one view class adds one turn, its four wavefronts into four tiles
    __syncthreads();
    for (int q = threadIdx.x; q < 4 * 2 * 16 * 17; q += kBsWaves * 64) (&acc_t[0][0][0][0])[q] = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = (a + t) & 3;
        for (int c = 0; c < 4; ++c) {
            __syncthreads();
            if (cls != c) continue;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int gi0 = i0 + (d >> 1), gk0 = k0 + (d & 1);
                int gi = gi0, gk = gk0;   // R^t (gi0, gk0)
                if (t == 1) {
                    gi = gk0;
                    gk = n - 1 - gi0;
                } else if (t == 2) {
                    gi = n - 1 - gi0;
                    gk = n - 1 - gk0;
                } else if (t == 3) {
                    gi = n - 1 - gk0;
                    gk = gi0;
                }
                const int li = gi - oy[b], lk = gk - ox[b];
                acc_t[b][0][li][lk] += acc[t][2 * d];
                acc_t[b][1][li][lk] += acc[t][2 * d + 1];
            }
        }
    }
    __syncthreads();
    const size_t npix = (size_t)n * n;
    for (int q = threadIdx.x; q < 4 * 256; q += kBsWaves * 64) {
        const int b = q >> 8, li = (q >> 4) & 15, lk = q & 15;
        const size_t p = (size_t)(oy[b] + li) * n + (ox[b] + lk);
        const float s1 = acc_t[b][0][li][lk], s2 = acc_t[b][1][li][lk];
        if (out_pairs) {
            out_pairs[(size_t)z * npix + p] = make_float2(s1, s2);
        } else {
            out_split[(size_t)(2 * z) * npix + p] = s1;
            if (2 * z + 1 < nout) out_split[(size_t)(2 * z + 1) * npix + p] = s2;
        }
    }
    }   // orbits
}

// ---------------------------------------------------------------------------
// back-projector of slices with the transpose symmetry as well (sym == 2).
// T(i, k) = (k, i) maps ray (v, j) of the table to ray (nv/4 - v, nd - 1 - j),
// whose table entry is its exact transpose, and T R^s = R^-s T.  The tiles of
// the image's first quadrant fall into orbits of the group generated by R and
// T: a pair (P, P^T) of off-diagonal tiles and their turns (8 tiles), or one
// diagonal tile and its turns (4 tiles).  A lane evaluates the weights of
// table ray (v, j), v <= nv/8, on its quad q once and adds them, times the
// residuals of the rays R^t r and R^t T r, to the pixels R^t q and R^t T q
// (views v = 0 and v = nv/8 are their own transposes' turns and take the
// four turns only).  A work unit is one 8-tile orbit or two 4-tile orbits,
// so the units of a slice are of equal size: 16 wavefronts as 8 tiles x 2
// view classes, or 4 tiles x 4 classes.  The partial sums reach the tiles in
// LDS in a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int kB8Waves = 16;

__device__ __forceinline__ float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// work units of one slice: 8-tile orbits, then pairs of 4-tile orbits
__host__ __device__ inline int sym8_units(int n) {
    const int nq = n / 32;
    return nq * (nq - 1) / 2 + (nq + 1) / 2;
}

// Work item of the block's r-th round.  Workgroups go round-robin to the 8
// XCDs, each with its own L2, so the items are relabelled to give the blocks
// of one XCD a contiguous run of items (slot b + r G keeps its block and
// round, so every block does the same amount of work as without relabelling).
// Only for launches whose slices are all eight-fold symmetric: the units of
// other slices are skipped, and a run of them would leave its XCD idle.
__device__ __forceinline__ int sym8_xcd_item(int b, int r, int G, int N) {
    const int x = b & 7, R = N / G, rem = N - R * G;
    int off = 0;
    for (int y = 0; y < x; ++y) off += R * ((G + 7 - y) >> 3) + ((rem + 7 - y) >> 3);
    return off + r * ((G + 7 - x) >> 3) + (b >> 3);
}

// The orbits of work unit u of a slice, in an order where consecutive units
// are close in the image.  The first-quadrant tile pairs (a, b), a <= b, fall
// into 4 x 4 blocks (A, B), A <= B: first the diagonal blocks (A, A), each
// with its off-diagonal pairs row by row, then its diagonal tiles two at a
// time; then the off-diagonal blocks row by row, each with its 16 pairs row
// by row.  At 512^2 (16 x 16 tiles) that gives every XCD two diagonal blocks
// or one 64 x 64 pixel block, whose sinogram windows overlap.
__device__ __forceinline__ void sym8_unit_orbits(int u, int nq, int& norb, int pa[2], int pb[2]) {
    const int nb = (nq + 3) >> 2;
    int r = u;
    norb = 1;
    pa[1] = pb[1] = 0;
    for (int A = 0; A < nb; ++A) {
        const int ha = min(4, nq - 4 * A), nh = ha * (ha - 1) / 2;
        if (r < nh) {
            int a = 0;
            while (r >= ha - 1 - a) {
                r -= ha - 1 - a;
                ++a;
            }
            pa[0] = 4 * A + a;
            pb[0] = 4 * A + a + 1 + r;
            return;
        }
        r -= nh;
        if (r < (ha + 1) / 2) {
            const int d0 = 4 * A + 2 * r;
            norb = min(2, nq - d0);
            pa[0] = pb[0] = d0;
            pa[1] = pb[1] = d0 + 1;
            return;
        }
        r -= (ha + 1) / 2;
    }
    for (int A = 0; A < nb; ++A) {
        const int ha = min(4, nq - 4 * A);
        for (int B = A + 1; B < nb; ++B) {
            const int hb = min(4, nq - 4 * B);
            if (r < ha * hb) {
                pa[0] = 4 * A + r / hb;
                pb[0] = 4 * B + r % hb;
                return;
            }
            r -= ha * hb;
        }
    }
}

template <bool SB>
__global__ __launch_bounds__(kB8Waves * 64) void k_backproject_sym8(
    const void* __restrict__ sino, RayTable T, int n, float dxmm, float2* __restrict__ out_pairs,
    float* __restrict__ out_split, int nout, int npairs, bool by_xcd) {
    // staged rays, one struct so that the arrays read per ray in the
    // innermost loop sit at the lowest LDS addresses (constant offsets that
    // fit the ds_read offset field)
    struct Stage {
        int4 fix[kB8Waves][64];
        float2 fl[kB8Waves][64];        // (2^-32/|s|, +-L)
        float4 sn[kB8Waves][64][4];     // L times the residual pairs of R^t r, then of R^t T r
    };
    __shared__ Stage stg;
    __shared__ float4 vs[kBpViewChunk];
    auto& sfix = stg.fix;
    auto& sfl = stg.fl;
    auto& ssn = stg.sn;
    // the tiles' sums [tile][channel][row][column], in ssn's memory once every
    // view is done
    float(*acc_t)[2][16][17] = reinterpret_cast<float(*)[2][16][17]>(&ssn[0][0][0]);
    static_assert(sizeof(ssn) >= sizeof(float) * 8 * 2 * 16 * 17, "tile sums");
    const int nq = n / 32;
    const int nunit = sym8_units(n), nitem = nunit * npairs;
    // the wavefront index in a scalar register (wave-uniform; as a vector
    // register, values derived from it are spilled across the view loop)
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int slot = blockIdx.x, round = 0; slot < nitem; slot += gridDim.x, ++round) {
    const int unit = by_xcd ? sym8_xcd_item(blockIdx.x, round, gridDim.x, nitem) : slot;
    const int z = unit / nunit, u = unit - z * nunit;
    const SliceDesc D = T.desc[T.desc_stride * z];
    if (D.sym != 2) continue;   // block-uniform
    // the unit's orbits, by the first-quadrant tile row and column of P
    int norb, pa[2], pb[2];
    sym8_unit_orbits(u, nq, norb, pa, pb);
    const int nd = D.nd, q4 = D.nv >> 2, vmax = q4 >> 1;
    // slice constants in scalar registers (uniform; as vector registers they
    // would be spilled across the view loop)
    const float sid = uniform_f(D.sid), sdd = uniform_f(D.sdd), u0 = uniform_f(D.u0),
                inv_pitch = uniform_f(D.inv_pitch);
    const int4* __restrict__ fix = T.fix + D.ray0;
    const float2* __restrict__ flt = T.flt + D.ray0;
    const float4* __restrict__ view = T.view + D.view0;
    const long long sbase = D.sino0 + (long long)z * T.sino_zstride;
    const float2* sz = reinterpret_cast<const float2*>(sino) + sbase;
    const unsigned* szb = reinterpret_cast<const unsigned*>(sino) + sbase;
    const size_t tstep = (size_t)q4 * nd;   // rays of one quarter of the views
    for (int o = 0; o < norb; ++o) {
    const bool heavy = pa[o] != pb[o];   // block-uniform
    const int ntile = heavy ? 8 : 4, ncls = heavy ? 2 : 4;
    const int d = heavy ? (w & 7) : (w & 3), cls = heavy ? (w >> 3) : (w >> 2);
    // tile d = 4 f + s is R^s of P (f = 0) or of P^T (f = 1); R maps the tile
    // at (ty, tx) to the one at (tx, n - 16 - ty)
    int oy[8], ox[8];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int ty = 16 * (f ? pb[o] : pa[o]), tx = 16 * (f ? pa[o] : pb[o]);
        oy[4 * f + 0] = ty;
        ox[4 * f + 0] = tx;
        oy[4 * f + 1] = tx;
        ox[4 * f + 1] = n - 16 - ty;
        oy[4 * f + 2] = n - 16 - ty;
        ox[4 * f + 2] = n - 16 - tx;
        oy[4 * f + 3] = n - 16 - tx;
        ox[4 * f + 3] = ty;
    }
    const int di = 2 * (lane >> 3), dk = 2 * (lane & 7);   // the lane's quad in the tile
    const int ty = oy[d], tx = ox[d];
    const int i0 = ty + di, k0 = tx + dk;
    const float x = ((float)k0 + 0.5f - 0.5f * (float)(n - 1)) * dxmm;
    const float y = ((float)i0 + 0.5f - 0.5f * (float)(n - 1)) * dxmm;
    // acc[t][q]: ray R^t r at pixel R^t (i0 + di, k0 + dk), q = 2 (2 di + dk) + channel;
    // acx[t][q]: ray R^t T r at pixel R^t T (i0 + di, k0 + dk)
    float acc[4][8], acx[4][8];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[t][q] = acx[t][q] = 0.f;
    for (int v0 = 0; v0 <= vmax; v0 += kBpViewChunk) {
        const int nvc = min(kBpViewChunk, vmax + 1 - v0);
        __syncthreads();
        for (int q = threadIdx.x; q < nvc; q += kB8Waves * 64) vs[q] = view[v0 + q];
        __syncthreads();
        // the lane's bins whose rays can reach its quad in view vv of the
        // chunk (the circle through the quad's corners); empty: INT_MAX, INT_MIN
        auto window = [&](int vv, int& jl, int& jh) {
            const float4 vc = vs[vv];
            const float e = 2.f * vc.z;
            const float U = sid - (x * vc.x + y * vc.y);
            const float W = y * vc.x - x * vc.y;
            const float rm = __builtin_amdgcn_rcpf(U - e);
            const float rp = __builtin_amdgcn_rcpf(U + e);
            const float hi = W + e, lo = W - e;
            const float umax = sdd * hi * (hi >= 0.f ? rm : rp);
            const float umin = sdd * lo * (lo >= 0.f ? rp : rm);
            jl = max((int)ceilf((umin - u0) * inv_pitch - 1e-3f), 0);
            jh = min((int)floorf((umax - u0) * inv_pitch + 1e-3f), nd - 1);
            if (jl > jh) {
                jl = INT_MAX;
                jh = INT_MIN;
            }
        };
        // stage ray (v, jj) of the table in slot sl of this wavefront: its
        // fixed-point entry made tile-relative, its step data, and L times the
        // residual pairs of its four turns (and, for a pair view pr, of the
        // turns of its transpose, ray (q4 - v, nd - 1 - jj))
        auto stage = [&](int v, int jj, int sl, bool pr) {
            const size_t r = (size_t)v * nd + jj;
            const float2 fl = flt[r];
            const float L = fabsf(fl.y);
            float2 s4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) s4[t] = SB ? bf16x2_unpack(szb[r + t * tstep]) : sz[r + t * tstep];
            // the ray's minor coordinate on the tile's first major line,
            // relative to the tile's first minor line and moved to the lower
            // end of the ray's minor extent over that line's step (fixed
            // point, exact)
            const int4 f4 = fix[r];
            const long long Sr = fix_s(f4);
            const bool xr = fl.y > 0.f;
            const long long a = fix_a0(f4) + (long long)(xr ? tx : ty) * Sr -
                                ((long long)(xr ? ty : tx) << 32) + (Sr < 0 ? Sr : 0);
            sfix[w][sl] = make_int4((int)(unsigned)a, (int)(a >> 32), f4.z, f4.w);
            sfl[w][sl] = fl;
            ssn[w][sl][0] = make_float4(L * s4[0].x, L * s4[0].y, L * s4[1].x, L * s4[1].y);
            ssn[w][sl][1] = make_float4(L * s4[2].x, L * s4[2].y, L * s4[3].x, L * s4[3].y);
            if (pr) {
                const size_t rx = (size_t)(q4 - v) * nd + (nd - 1 - jj);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    s4[t] = SB ? bf16x2_unpack(szb[rx + t * tstep]) : sz[rx + t * tstep];
                ssn[w][sl][2] = make_float4(L * s4[0].x, L * s4[0].y, L * s4[1].x, L * s4[1].y);
                ssn[w][sl][3] = make_float4(L * s4[2].x, L * s4[2].y, L * s4[3].x, L * s4[3].y);
            }
        };
        // the lane's chords of bins ja..jb, staged from slot s0 for bin j0
        auto chords = [&](int ja, int jb, int s0, int j0, bool pr) {
            for (int j = ja; j <= jb; ++j) {
                const int4 fx = sfix[w][s0 + j - j0];
                const float2 fs = sfl[w][s0 + j - j0];
                const bool xm = fs.y > 0.f;
                // the quad's offset in the tile along the ray's major and minor axes
                const int dm = xm ? dk : di, dn = xm ? di : dk;
                // lower ends la, lb of the ray's minor extent over the
                // quad's two major steps: a + dm S (dm <= 14, so the high
                // word takes dm times S's high word, 0 or -1), then + S
                const unsigned long long t =
                    (((unsigned long long)(unsigned)fx.y << 32) | (unsigned)fx.x) +
                    (unsigned long long)(unsigned)dm * (unsigned)fx.z;
                const long long la =
                    (long long)((((unsigned long long)((unsigned)(t >> 32) + (unsigned)__mul24(dm, fx.w))) << 32) |
                                (unsigned)t);
                const long long lb = la + fix_s(fx);
                // row floor(l) takes the part of the step below the next
                // boundary, the row above it the rest
                const float wa = lower_weight((unsigned)la, fs.x);
                const float wb = lower_weight((unsigned)lb, fs.x);
                const int ea = (int)(la >> 32) - dn, eb = (int)(lb >> 32) - dn;
                const float ca0 = ea == 0 ? wa : (ea == -1 ? 1.f - wa : 0.f);
                const float ca1 = ea == 1 ? wa : (ea == 0 ? 1.f - wa : 0.f);
                const float cb0 = eb == 0 ? wb : (eb == -1 ? 1.f - wb : 0.f);
                const float cb1 = eb == 1 ? wb : (eb == 0 ? 1.f - wb : 0.f);
                const float c01 = xm ? cb0 : ca1, c10 = xm ? ca1 : cb0;
                const float4 sA = ssn[w][s0 + j - j0][0], sB = ssn[w][s0 + j - j0][1];
                const float sv[8] = {sA.x, sA.y, sA.z, sA.w, sB.x, sB.y, sB.z, sB.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float s1 = sv[2 * t], s2 = sv[2 * t + 1];
                    acc[t][0] = fmaf(ca0, s1, acc[t][0]);
                    acc[t][1] = fmaf(ca0, s2, acc[t][1]);
                    acc[t][2] = fmaf(c01, s1, acc[t][2]);
                    acc[t][3] = fmaf(c01, s2, acc[t][3]);
                    acc[t][4] = fmaf(c10, s1, acc[t][4]);
                    acc[t][5] = fmaf(c10, s2, acc[t][5]);
                    acc[t][6] = fmaf(cb1, s1, acc[t][6]);
                    acc[t][7] = fmaf(cb1, s2, acc[t][7]);
                }
                if (pr) {
                    const float4 sC = ssn[w][s0 + j - j0][2], sD = ssn[w][s0 + j - j0][3];
                    const float sx[8] = {sC.x, sC.y, sC.z, sC.w, sD.x, sD.y, sD.z, sD.w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float s1 = sx[2 * t], s2 = sx[2 * t + 1];
                        acx[t][0] = fmaf(ca0, s1, acx[t][0]);
                        acx[t][1] = fmaf(ca0, s2, acx[t][1]);
                        acx[t][2] = fmaf(c01, s1, acx[t][2]);
                        acx[t][3] = fmaf(c01, s2, acx[t][3]);
                        acx[t][4] = fmaf(c10, s1, acx[t][4]);
                        acx[t][5] = fmaf(c10, s2, acx[t][5]);
                        acx[t][6] = fmaf(cb1, s1, acx[t][6]);
                        acx[t][7] = fmaf(cb1, s2, acx[t][7]);
                    }
                }
            }
        };
        // views vv and vv + ncls of the class, in rounds of one staging each:
        // both views in one round (halves of the wavefront) when both windows
        // fit 32 bins, else view A's 64-bin rounds, then view B's.  Every
        // accumulator takes the views in the same order, bins ascending.
        for (int vv = cls; vv < nvc; vv += 2 * ncls) {
            const int vb = vv + ncls;
            const bool two = vb < nvc;   // wave-uniform
            const int vA = v0 + vv, vB = v0 + vb;
            const bool prA = vA > 0 && 2 * vA != q4, prB = vB > 0 && 2 * vB != q4;
            int jlA, jhA, jlB = INT_MAX, jhB = INT_MIN;
            window(vv, jlA, jhA);
            if (two) window(vb, jlB, jhB);
            // (clamped to the detector: empty stays empty)
            const int JloA = max(wave_min(jlA), 0), JhiA = min(wave_max(jhA), nd - 1);
            const int JloB = two ? max(wave_min(jlB), 0) : INT_MAX;
            const int JhiB = two ? min(wave_max(jhB), nd - 1) : INT_MIN;
            const bool emA = JloA > JhiA, emB = JloB > JhiB;   // wave-uniform
            const bool packed = (emA || JhiA - JloA < 32) && (emB || JhiB - JloB < 32);
            const int nA = emA ? 0 : (JhiA - JloA) / 64 + 1, nB = emB ? 0 : (JhiB - JloB) / 64 + 1;
            const int nround = packed ? 1 : nA + nB;
            for (int rd = 0; rd < nround; ++rd) {
                // bins baseA..hiA of view A in slots from 0, baseB..hiB of
                // view B in slots from sB (an empty part has hi = INT_MIN)
                int baseA = 0, hiA = INT_MIN, baseB = 0, hiB = INT_MIN, sB = 64;
                if (packed) {   // (an empty view keeps base 0: Jlo is INT_MAX there)
                    baseA = emA ? 0 : JloA;
                    hiA = emA ? INT_MIN : JhiA;
                    baseB = emB ? 0 : JloB;
                    hiB = emB ? INT_MIN : JhiB;
                    sB = 32;
                } else if (rd < nA) {
                    baseA = JloA + 64 * rd;
                    hiA = min(JhiA, baseA + 63);
                } else {
                    baseB = JloB + 64 * (rd - nA);
                    hiB = min(JhiB, baseB + 63);
                    sB = 0;
                }
                const bool hb = lane >= sB;   // this lane's slot holds view B
                const int jj = hb ? baseB + (lane - sB) : baseA + lane;   // no overflow: base <= nd - 1
                if (jj >= 0 && jj <= (hb ? hiB : hiA)) stage(hb ? vB : vA, jj, lane, hb ? prB : prA);
                __builtin_amdgcn_wave_barrier();
#pragma unroll 1
                for (int h = 0; h < 2; ++h)
                    chords(h ? max(jlB, baseB) : max(jlA, baseA), h ? min(jhB, hiB) : min(jhA, hiA),
                           h ? sB : 0, h ? baseB : baseA, h ? prB : prA);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    // the tiles in LDS: in each round (image g, turn t, view class c) the
    // wavefronts of class c add into distinct tiles; R^t maps tile 4 f + s to
    // 4 f + (s + t) mod 4, R^t T to 4 (1 - f) + (t - s) mod 4 (for a 4-tile
    // orbit P^T = P: tile (t - s) mod 4)
    __syncthreads();
    for (int q = threadIdx.x; q < ntile * 2 * 16 * 17; q += kB8Waves * 64) (&acc_t[0][0][0][0])[q] = 0.f;
    const int f = d >> 2, s = d & 3;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int b = g == 0 ? 4 * f + ((s + t) & 3) : (heavy ? 4 * (1 - f) : 0) + ((t - s) & 3);
            for (int c = 0; c < ncls; ++c) {
                __syncthreads();
                if (cls != c) continue;
#pragma unroll
                for (int dq = 0; dq < 4; ++dq) {
                    const int pi = i0 + (dq >> 1), pk = k0 + (dq & 1);
                    int gi = g ? pk : pi, gk = g ? pi : pk;   // T p for g = 1
#pragma unroll
                    for (int r = 0; r < 3; ++r) {   // R^t: R(i, k) = (k, n - 1 - i)
                        if (r < t) {
                            const int ni = gk;
                            gk = n - 1 - gi;
                            gi = ni;
                        }
                    }
                    const int li = gi - oy[b], lk = gk - ox[b];
                    acc_t[b][0][li][lk] += g ? acx[t][2 * dq] : acc[t][2 * dq];
                    acc_t[b][1][li][lk] += g ? acx[t][2 * dq + 1] : acc[t][2 * dq + 1];
                }
            }
        }
    }
    __syncthreads();
    const size_t npix = (size_t)n * n;
    for (int q = threadIdx.x; q < ntile * 256; q += kB8Waves * 64) {
        const int b = q >> 8, li = (q >> 4) & 15, lk = q & 15;
        const size_t p = (size_t)(oy[b] + li) * n + (ox[b] + lk);
        const float s1 = acc_t[b][0][li][lk], s2 = acc_t[b][1][li][lk];
        if (out_pairs) {
            out_pairs[(size_t)z * npix + p] = make_float2(s1, s2);
        } else {
            out_split[(size_t)(2 * z) * npix + p] = s1;
            if (2 * z + 1 < nout) out_split[(size_t)(2 * z + 1) * npix + p] = s2;
        }
    }
    __syncthreads();   // acc_t (in ssn) is reused by the next orbit
    }   // orbits of the unit
    }   // units
}

// Workgroups of the symmetric back-projector for `norb` orbits, spread so that
// every block takes the same number of orbits.  By default (pct = 0): up to
// one orbit per CU (a single slice), at most half the CUs, so that the
// latency-bound PCG kernels of the concurrent stream run on the other half;
// larger batches, where every stream's work is throughput-bound, take all
// CUs.  pct > 0 caps the workgroups at pct percent of the CUs instead.
static int sym_bp_grid(int norb, int pct) {
    static const int ncu = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 256;
        }
        return std::max(n, 2);
    }();
    const int cap = pct > 0 ? std::max(1, ncu * pct / 100) : (norb <= ncu ? ncu / 2 : ncu);
    const int rounds = (norb + cap - 1) / cap;
    return (norb + rounds - 1) / rounds;
}

void launch_backproject(const Geom& g, const RayTable& t, const void* sino, int npairs,
                        float2* out_pairs, float* out_split, int nout, hipStream_t st,
                        bool sino_bf16, int kinds, int bp_pct) {
    if (kinds & kSlicePlain) {
        dim3 grid((g.nx + 15) / 16, (g.ny + 15) / 16, npairs);
        if (sino_bf16)
            hipLaunchKernelGGL(k_backproject<true>, grid, dim3(kBpWaves * 64), 0, st, sino, t, g.nx,
                               g.ny, (float)g.dx, out_pairs, out_split, nout);
        else
            hipLaunchKernelGGL(k_backproject<false>, grid, dim3(kBpWaves * 64), 0, st, sino, t, g.nx,
                               g.ny, (float)g.dx, out_pairs, out_split, nout);
    }
    if ((kinds & kSliceQuarter) && grid_sym4(g)) {
        const int norb = (g.nx / 32) * (g.nx / 32) * npairs;   // tile orbits of all pairs
        dim3 grid(sym_bp_grid(norb, bp_pct));
        if (sino_bf16)
            hipLaunchKernelGGL(k_backproject_sym<true>, grid, dim3(kBsWaves * 64), 0, st, sino, t, g.nx,
                               (float)g.dx, out_pairs, out_split, nout, npairs);
        else
            hipLaunchKernelGGL(k_backproject_sym<false>, grid, dim3(kBsWaves * 64), 0, st, sino, t, g.nx,
                               (float)g.dx, out_pairs, out_split, nout, npairs);
    }
    if ((kinds & kSliceOcto) && grid_sym4(g)) {
        const int nunit = sym8_units(g.nx) * npairs;   // work units of all pairs
        dim3 grid(sym_bp_grid(nunit, bp_pct));
        const bool by_xcd = kinds == kSliceOcto;
        if (sino_bf16)
            hipLaunchKernelGGL(k_backproject_sym8<true>, grid, dim3(kB8Waves * 64), 0, st, sino, t, g.nx,
                               (float)g.dx, out_pairs, out_split, nout, npairs, by_xcd);
        else
            hipLaunchKernelGGL(k_backproject_sym8<false>, grid, dim3(kB8Waves * 64), 0, st, sino, t, g.nx,
                               (float)g.dx, out_pairs, out_split, nout, npairs, by_xcd);
    }
}

}  // namespace dect
