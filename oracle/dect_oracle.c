/*
 * FP64 CPU oracle: geometric operators of the sinogram-domain method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Nothing in the product path may link,
 * load or call it; it shares no code, headers or tables with the HIP library.
 *
 * Contents
 *   ora_project      system matrix A: for every ray (view v, bin j) the sum of
 *                    image values times the length of the ray inside each
 *                    pixel square.  Entries are computed with Siddon's exact
 *                    parametric method (R. L. Siddon, Med. Phys. 12, 1985):
 *                    all crossings of the ray with the grid lines are listed,
 *                    sorted, and each gap between consecutive crossings is one
 *                    pixel chord.  The pixel of a gap is found by comparing
 *                    its mid parameter with the crossing parameters of the
 *                    grid lines (not with rounded coordinates), so a ray that
 *                    runs within rounding of a grid line is classified exactly
 *                    as the per-pixel clipper classifies it.
 *   ora_backproject  exact transpose A^T, by scattering each ray's chords.
 *   ora_ray_chords   the nonzeros of one row of A (for tests).
 *   ora_clip_chord   brute-force chord of one ray and one pixel by clipping the
 *                    line against the pixel square (Liang-Barsky); an
 *                    independent check of the Siddon entries.
 *   ora_fbp          flat-detector fan-beam filtered back-projection
 *                    (Kak & Slaney, "Principles of Computerized Tomographic
 *                    Imaging", ch. 3, equally spaced collinear detectors), the
 *                    stand-in for the scanner-reconstructed input images that
 *                    the paper's Algorithm 1 requires.
 *
 * Geometry (mm, radians), shared by all functions:
 *   pixel (row i, column k) is the half-open square
 *     [x0 + k*dx, x0 + (k+1)*dx) x [y0 + i*dx, y0 + (i+1)*dx),
 *     x0 = -nx*dx/2, y0 = -ny*dx/2;
 *   view v: theta = angle0 + v*arc/nv, source S = sid*(cos, sin) (exact at
 *   multiples of 90 degrees);
 *   detector centre -(sdd - sid)*(cos, sin), axis e = (-sin, cos);
 *   bin j centre: u_j = (j - (nd-1)/2)*pitch + offset along e;
 *   ray (v, j) = line from S to the bin centre.
 * Images are [ny][nx] row-major, sinograms [nv][nd] row-major.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny;
    double dx;
    int nv;
    double angle0, arc;
    int nd;
    double pitch, offset, sid, sdd;
} OraGeom;

/* cos and sin of view angle th; at an exact multiple of 90 degrees (to 1e-12
 * rad) the exact values, so that such a view's rays are exactly parallel to
 * the grid and a ray on a grid line is decided by the half-open rule above,
 * not by the rounding of cos(pi/2) etc. */
static void view_cos_sin(double th, double *c, double *s) {
    const double q = th / (0.5 * M_PI);
    const double qr = floor(q + 0.5);
    if (fabs(q - qr) * (0.5 * M_PI) < 1e-12) {
        const long k = ((long)qr % 4 + 4) % 4;
        *c = k == 0 ? 1.0 : (k == 2 ? -1.0 : 0.0);
        *s = k == 1 ? 1.0 : (k == 3 ? -1.0 : 0.0);
        return;
    }
    *c = cos(th);
    *s = sin(th);
}

static void ray_of(const OraGeom *g, int v, int j, double S[2], double Q[2]) {
    double th = g->angle0 + (double)v * (g->arc / (double)g->nv);
    double c, s;
    view_cos_sin(th, &c, &s);
    double u = ((double)j - 0.5 * (double)(g->nd - 1)) * g->pitch + g->offset;
    S[0] = g->sid * c;
    S[1] = g->sid * s;
    Q[0] = -(g->sdd - g->sid) * c + u * (-s);
    Q[1] = -(g->sdd - g->sid) * s + u * c;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Grid line q of axis a (x: a = 0, y: a = 1); every function uses this
 * expression so that equal lines give bit-equal crossing parameters. */
static double grid_line(const OraGeom *g, int a, int q) {
    int n = a == 0 ? g->nx : g->ny;
    return -0.5 * n * g->dx + q * g->dx;
}

/* Index c in [0, n) of the slab [line c, line c+1) that contains the ray at
 * parameter tm, decided from crossing parameters t_q = (line q - S)/d, which
 * increase with q when d > 0 and decrease when d < 0.  Half-open slabs. */
static int slab_of(const double *tl, int n, double d, double tm) {
    int lo = 0, hi = n;                    /* answer in [lo, hi) or n = outside */
    if (d > 0) {                           /* largest c with tl[c] <= tm */
        if (tm < tl[0] || !(tm < tl[n])) return -1;
        while (hi - lo > 1) { int mid = (lo + hi) / 2; if (tl[mid] <= tm) lo = mid; else hi = mid; }
    } else {                               /* c with tl[c+1] < tm <= tl[c] */
        if (tm > tl[0] || !(tm > tl[n])) return -1;
        while (hi - lo > 1) { int mid = (lo + hi) / 2; if (tl[mid] >= tm) lo = mid; else hi = mid; }
    }
    return lo;
}

/* Siddon: fill pix[] (i*nx + k) and len[] (mm) for ray (v, j); return count.
 * work must hold 3*(nx + ny + 4) doubles; pix/len nx + ny + 3 entries. */
static int siddon_ray(const OraGeom *g, int v, int j, double *work, int *pix, double *len) {
    double S[2], Q[2];
    ray_of(g, v, j, S, Q);
    double d[2] = {Q[0] - S[0], Q[1] - S[1]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1]);
    int n[2] = {g->nx, g->ny};
    int cap = g->nx + g->ny + 4;
    double *tbuf = work, *tl[2] = {work + cap, work + 2 * cap};
    double tmin = 0.0, tmax = 1.0;
    int fixed[2] = {-1, -1};
    for (int a = 0; a < 2; ++a) {
        if (d[a] == 0.0) {                 /* parallel to the lines of this axis */
            for (int q = 0; q < n[a]; ++q)
                if (S[a] >= grid_line(g, a, q) && S[a] < grid_line(g, a, q + 1)) fixed[a] = q;
            if (fixed[a] < 0) return 0;
            continue;
        }
        for (int q = 0; q <= n[a]; ++q) tl[a][q] = (grid_line(g, a, q) - S[a]) / d[a];
        double t0 = tl[a][0], t1 = tl[a][n[a]];
        if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    if (!(tmax > tmin)) return 0;
    int m = 0;
    tbuf[m++] = tmin;
    for (int a = 0; a < 2; ++a) {
        if (d[a] == 0.0) continue;
        for (int q = 0; q <= n[a]; ++q)
            if (tl[a][q] > tmin && tl[a][q] < tmax) tbuf[m++] = tl[a][q];
    }
    tbuf[m++] = tmax;
    qsort(tbuf, (size_t)m, sizeof(double), cmp_double);
    int cnt = 0;
    for (int q = 0; q + 1 < m; ++q) {
        double ta = tbuf[q], tb = tbuf[q + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        int c[2];
        for (int a = 0; a < 2; ++a)
            c[a] = d[a] == 0.0 ? fixed[a] : slab_of(tl[a], n[a], d[a], tm);
        if (c[0] < 0 || c[1] < 0) continue;
        pix[cnt] = c[1] * g->nx + c[0];
        len[cnt] = (tb - ta) * dn;
        ++cnt;
    }
    return cnt;
}

int ora_ray_chords(const OraGeom *g, int v, int j, int *pix, double *len) {
    double *work = (double *)malloc(sizeof(double) * 3 * (size_t)(g->nx + g->ny + 4));
    int c = siddon_ray(g, v, j, work, pix, len);
    free(work);
    return c;
}

void ora_project(const OraGeom *g, const double *img, double *sino, int batch, int nthreads) {
    size_t npix = (size_t)g->nx * g->ny, nray = (size_t)g->nv * g->nd;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int cap = g->nx + g->ny + 4;
        double *tbuf = (double *)malloc(sizeof(double) * 3 * cap);
        int *pix = (int *)malloc(sizeof(int) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 16)
        for (long r = 0; r < (long)nray; ++r) {
            int v = (int)(r / g->nd), j = (int)(r % g->nd);
            int c = siddon_ray(g, v, j, tbuf, pix, len);
            for (int b = 0; b < batch; ++b) {
                const double *im = img + (size_t)b * npix;
                double acc = 0.0;
                for (int q = 0; q < c; ++q) acc += len[q] * im[pix[q]];
                sino[(size_t)b * nray + r] = acc;
            }
        }
        free(tbuf); free(pix); free(len);
    }
}

void ora_backproject(const OraGeom *g, const double *sino, double *img, int batch, int nthreads) {
    size_t npix = (size_t)g->nx * g->ny, nray = (size_t)g->nv * g->nd;
    memset(img, 0, sizeof(double) * npix * batch);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nt * npix * batch, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + (size_t)tid * npix * batch;
        int cap = g->nx + g->ny + 4;
        double *tbuf = (double *)malloc(sizeof(double) * 3 * cap);
        int *pix = (int *)malloc(sizeof(int) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(static)
        for (long r = 0; r < (long)nray; ++r) {
            int v = (int)(r / g->nd), j = (int)(r % g->nd);
            int c = siddon_ray(g, v, j, tbuf, pix, len);
            for (int b = 0; b < batch; ++b) {
                double y = sino[(size_t)b * nray + r];
                double *im = mine + (size_t)b * npix;
                for (int q = 0; q < c; ++q) im[pix[q]] += len[q] * y;
            }
        }
        free(tbuf); free(pix); free(len);
    }
    for (int t = 0; t < nt; ++t) {
        const double *src = part + (size_t)t * npix * batch;
        for (size_t p = 0; p < npix * batch; ++p) img[p] += src[p];
    }
    free(part);
}

/* Brute force: clip ray (v, j) against the half-open square of pixel (i, k). */
double ora_clip_chord(const OraGeom *g, int v, int j, int i, int k) {
    double S[2], Q[2];
    ray_of(g, v, j, S, Q);
    double d[2] = {Q[0] - S[0], Q[1] - S[1]};
    int c[2] = {k, i};
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 2; ++a) {
        double lo = grid_line(g, a, c[a]), hi = grid_line(g, a, c[a] + 1);
        if (d[a] == 0.0) {
            if (S[a] < lo || S[a] >= hi) return 0.0;
            continue;
        }
        double ta = (lo - S[a]) / d[a], tb = (hi - S[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t1 > t0)) return 0.0;
    return (t1 - t0) * sqrt(d[0] * d[0] + d[1] * d[1]);
}

/* Fan-beam FBP of one batch of sinograms; see the header comment. */
void ora_fbp(const OraGeom *g, const double *sino, double *img, int batch, int nthreads) {
    int nd = g->nd, nv = g->nv;
    size_t npix = (size_t)g->nx * g->ny, nray = (size_t)nv * nd;
    double mag = g->sid / g->sdd;
    double dp = g->pitch * mag;                 /* virtual-detector pitch */
    double *q = (double *)malloc(sizeof(double) * nray * batch);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    /* 1) cosine weighting and ramp filtering, row by row */
#pragma omp parallel
    {
        double *pw = (double *)malloc(sizeof(double) * nd);
#pragma omp for schedule(static)
        for (long r = 0; r < (long)nv * batch; ++r) {
            int b = (int)(r / nv), v = (int)(r % nv);
            const double *p = sino + (size_t)b * nray + (size_t)v * nd;
            for (int j = 0; j < nd; ++j) {
                double up = (((double)j - 0.5 * (nd - 1)) * g->pitch + g->offset) * mag;
                pw[j] = p[j] * g->sid / sqrt(g->sid * g->sid + up * up);
            }
            double *out = q + (size_t)b * nray + (size_t)v * nd;
            for (int j = 0; j < nd; ++j) {
                double acc = 0.0;
                for (int l = 0; l < nd; ++l) {
                    int n = j - l;
                    double h;
                    if (n == 0) h = 1.0 / (4.0 * dp * dp);
                    else if (n % 2 == 0) h = 0.0;
                    else h = -1.0 / (M_PI * M_PI * (double)n * (double)n * dp * dp);
                    acc += h * pw[l];
                }
                out[j] = dp * acc;
            }
        }
        free(pw);
    }
    /* 2) distance-weighted back-projection with linear interpolation */
    double dth = g->arc / nv;
    double u0 = (-0.5 * (nd - 1) * g->pitch + g->offset) * mag;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)npix; ++p) {
        int i = (int)(p / g->nx), k = (int)(p % g->nx);
        double x = ((double)k - 0.5 * (g->nx - 1)) * g->dx;
        double y = ((double)i - 0.5 * (g->ny - 1)) * g->dx;
        for (int b = 0; b < batch; ++b) {
            const double *qb = q + (size_t)b * nray;
            double acc = 0.0;
            for (int v = 0; v < nv; ++v) {
                double th = g->angle0 + (double)v * dth;
                double c = cos(th), s = sin(th);
                double U = g->sid - (x * c + y * s);
                double w = -x * s + y * c;
                double up = g->sid * w / U;
                double f = (up - u0) / dp;
                double j0 = floor(f);
                double t = f - j0;
                int a = (int)j0;
                double va = (a >= 0 && a < nd) ? qb[(size_t)v * nd + a] : 0.0;
                double vb = (a + 1 >= 0 && a + 1 < nd) ? qb[(size_t)v * nd + a + 1] : 0.0;
                acc += (g->sid * g->sid) / (U * U) * ((1.0 - t) * va + t * vb);
            }
            img[(size_t)b * npix + p] = 0.5 * dth * acc;
        }
    }
    free(q);
}
