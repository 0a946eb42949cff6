/*
 * FP64 CPU oracle for direct algebraic CT reconstruction by QR.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library: the two are written separately so that one can check the other.
 *
 * What it computes (paper: Sec. 2, Eqs. (system), (qr), (solve)):
 *   A X = B with A the M x N weights matrix of the scanner (a_ij = contribution
 *   of ray i to pixel j), A = Q R, and X = R^{-1} (Q^T B), where Q is kept as
 *   Householder reflectors and R^{-1} is never formed (Sec. 2).
 *
 * Everything is plain, unblocked, double precision.  The only parallelism is
 * an OpenMP split of independent columns in the rank-1 reflector update and of
 * independent right-hand sides; every output element sees the same sequence
 * of floating-point operations as the serial loop.
 *
 * Readings where the paper is silent (geometry, projector, sign convention)
 * are fixed below and listed in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_pix, n_angles, n_det;
    int32_t projector;              /* 0: Siddon, 1: Joseph */
    double grid_width, sid, sdd, det_length, angle0;
} orc_geometry;

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. 3.1 "Simulated scanner parameters", Table 1: 360-degree    */
/* circular fan-beam scan).  Reading: flat equispaced detector centred on    */
/* the line through the isocentre, one ray per bin from the source point to  */
/* the bin centre, view k at angle angle0 + 2 pi k / n_angles, counter-      */
/* clockwise; row index i = k * n_det + d (angles x detectors).              */
/* ------------------------------------------------------------------------ */
void orc_ray_endpoints(const orc_geometry* g, double* rays /* m x 4 row-major */)
{
    const double pitch = g->det_length / (double)g->n_det;
    for (int k = 0; k < g->n_angles; ++k) {
        const double th = g->angle0 + 2.0 * M_PI * (double)k / (double)g->n_angles;
        const double c = cos(th), s = sin(th);
        const double sx = g->sid * c, sy = g->sid * s;            /* source */
        const double dcx = (g->sid - g->sdd) * c;                 /* detector centre */
        const double dcy = (g->sid - g->sdd) * s;
        for (int d = 0; d < g->n_det; ++d) {
            const double u = ((double)d - 0.5 * (double)(g->n_det - 1)) * pitch;
            double* r = rays + 4 * ((int64_t)k * g->n_det + d);
            r[0] = sx;
            r[1] = sy;
            r[2] = dcx - u * s;                                    /* axis (-sin, cos) */
            r[3] = dcy + u * c;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Siddon (1985) exact intersection lengths of one ray with an N x N grid of */
/* width W centred at the origin.  Pixel (ix, iy) covers                     */
/* [-W/2 + ix W/N, -W/2 + (ix+1) W/N] x [same in y]; column j = iy N + ix.   */
/* Steps: clip the parametric ray p(a) = p0 + a (p1 - p0), a in [0, 1], to   */
/* the square; gather every grid-line crossing a inside the clipped range;   */
/* sort; each consecutive pair is one segment whose pixel is the one holding */
/* the segment midpoint and whose length is (a_{t+1} - a_t) |p1 - p0|.       */
/* Segments shorter than 1e-14 W are dropped.                                */
/* Returns the number of (pixel, length) pairs written (at most 2N + 2).     */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

int64_t orc_siddon_ray(double x0, double y0, double x1, double y1, int32_t N,
                       double W, int32_t* pix, double* len, double* work /* >= 2N+4 */)
{
    const double dx = x1 - x0, dy = y1 - y0;
    const double lo = -0.5 * W, hi = 0.5 * W, h = W / (double)N;
    double amin = 0.0, amax = 1.0;
    /* slab clip in x */
    if (dx != 0.0) {
        double a0 = (lo - x0) / dx, a1 = (hi - x0) / dx;
        if (a0 > a1) { double t = a0; a0 = a1; a1 = t; }
        if (a0 > amin) amin = a0;
        if (a1 < amax) amax = a1;
    } else if (x0 < lo || x0 > hi) {
        return 0;
    }
    /* slab clip in y */
    if (dy != 0.0) {
        double a0 = (lo - y0) / dy, a1 = (hi - y0) / dy;
        if (a0 > a1) { double t = a0; a0 = a1; a1 = t; }
        if (a0 > amin) amin = a0;
        if (a1 < amax) amax = a1;
    } else if (y0 < lo || y0 > hi) {
        return 0;
    }
    if (!(amax > amin)) return 0;

    int64_t na = 0;
    work[na++] = amin;
    work[na++] = amax;
    for (int i = 0; i <= N; ++i) {
        const double plane = lo + (double)i * h;
        if (dx != 0.0) {
            const double a = (plane - x0) / dx;
            if (a > amin && a < amax) work[na++] = a;
        }
        if (dy != 0.0) {
            const double a = (plane - y0) / dy;
            if (a > amin && a < amax) work[na++] = a;
        }
    }
    qsort(work, (size_t)na, sizeof(double), cmp_double);

    const double dist = sqrt(dx * dx + dy * dy);
    int64_t cnt = 0;
    for (int64_t t = 0; t + 1 < na; ++t) {
        const double seg = (work[t + 1] - work[t]) * dist;
        if (seg < 1e-14 * W) continue;
        const double am = 0.5 * (work[t] + work[t + 1]);
        const double xm = x0 + am * dx, ym = y0 + am * dy;
        int ix = (int)floor((xm - lo) / h);
        int iy = (int)floor((ym - lo) / h);
        if (ix < 0) ix = 0;
        if (ix > N - 1) ix = N - 1;
        if (iy < 0) iy = 0;
        if (iy > N - 1) iy = N - 1;
        pix[cnt] = iy * N + ix;
        len[cnt] = seg;
        ++cnt;
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Joseph (1982) interpolating projector, the one the paper builds A with    */
/* (Sec. 3.1).  The ray is sampled once per pixel-centre line across its     */
/* dominant axis (x when |dx| >= |dy|): at the centre line of pixel column   */
/* ix it sits at height y; the image there is the linear interpolation of    */
/* the two pixels of that column whose centres bracket y (zero outside the   */
/* grid), and each sample stands for the ray length over one pixel width     */
/* along the dominant axis, h |p1 - p0| / |dx|.  So pixel (ix, iy) gets      */
/* (1 - f) h |p1-p0|/|dx| and pixel (ix, iy+1) gets f h |p1-p0|/|dx|, with   */
/* iy = floor(fy), f = fy - iy, fy = (y - lo)/h - 1/2.  Samples outside the  */
/* segment [p0, p1] are skipped; zero weights are not emitted.               */
/* Returns the number of (pixel, weight) pairs written (at most 2N).         */
/* ------------------------------------------------------------------------ */
int64_t orc_joseph_ray(double x0, double y0, double x1, double y1, int32_t N, double W,
                       int32_t* pix, double* wt)
{
    const double dx = x1 - x0, dy = y1 - y0;
    const double lo = -0.5 * W, h = W / (double)N;
    const int xmajor = fabs(dx) >= fabs(dy);
    const double dmaj = xmajor ? dx : dy, dmin = xmajor ? dy : dx;
    const double pmaj = xmajor ? x0 : y0, pmin = xmajor ? y0 : x0;
    if (dmaj == 0.0) return 0;
    const double scale = h * sqrt(dx * dx + dy * dy) / fabs(dmaj);
    int64_t cnt = 0;
    for (int32_t k = 0; k < N; ++k) {
        const double c = lo + ((double)k + 0.5) * h;       /* centre line of pixel column / row k */
        const double a = (c - pmaj) / dmaj;
        if (a < 0.0 || a > 1.0) continue;
        const double q = pmin + a * dmin;                  /* position across the dominant axis */
        const double fq = (q - lo) / h - 0.5;
        const double fl = floor(fq);
        const double f = fq - fl;
        const int64_t i0 = (int64_t)fl;
        for (int e = 0; e < 2; ++e) {
            const int64_t i = i0 + e;
            const double w = (e == 0 ? 1.0 - f : f) * scale;
            if (i < 0 || i >= N || !(w > 0.0)) continue;
            pix[cnt] = xmajor ? (int32_t)(i * N + k) : (int32_t)((int64_t)k * N + i);
            wt[cnt] = w;
            ++cnt;
        }
    }
    return cnt;
}

/* One ray of the geometry's projector: (pixel, weight) pairs, count returned */
static int64_t orc_ray(const orc_geometry* g, const double* p, int32_t* pix, double* len, double* work)
{
    if (g->projector == 1) return orc_joseph_ray(p[0], p[1], p[2], p[3], g->n_pix, g->grid_width, pix, len);
    return orc_siddon_ray(p[0], p[1], p[2], p[3], g->n_pix, g->grid_width, pix, len, work);
}

/* Joseph rows for an explicit list of rays (r x 4), dense row-major r x N^2. */
void orc_joseph_rows(const double* rays, int64_t r, int32_t N, double W, double* rows)
{
    const int64_t n = (int64_t)N * N;
    int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * N + 8));
    double* wt = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
    for (int64_t i = 0; i < r; ++i) {
        double* row = rows + i * n;
        memset(row, 0, sizeof(double) * (size_t)n);
        const double* p = rays + 4 * i;
        const int64_t c = orc_joseph_ray(p[0], p[1], p[2], p[3], N, W, pix, wt);
        for (int64_t t = 0; t < c; ++t) row[pix[t]] += wt[t];
    }
    free(pix); free(wt);
}

/* Rows of A for an explicit list of rays (r x 4), dense row-major r x N^2. */
void orc_siddon_rows(const double* rays, int64_t r, int32_t N, double W, double* rows)
{
    const int64_t n = (int64_t)N * N;
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
        int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * N + 8));
        double* len = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < r; ++i) {
            double* row = rows + i * n;
            memset(row, 0, sizeof(double) * (size_t)n);
            const double* p = rays + 4 * i;
            const int64_t c = orc_siddon_ray(p[0], p[1], p[2], p[3], N, W, pix, len, work);
            for (int64_t t = 0; t < c; ++t) row[pix[t]] += len[t];
        }
        free(work); free(pix); free(len);
    }
}

/* Dense column-major A (m x n, leading dimension lda >= m) for a geometry. */
void orc_system_dense(const orc_geometry* g, double* A, int64_t lda)
{
    const int32_t N = g->n_pix;
    const int64_t m = (int64_t)g->n_angles * g->n_det, n = (int64_t)N * N;
    double* rays = (double*)malloc(sizeof(double) * 4 * (size_t)m);
    orc_ray_endpoints(g, rays);
    for (int64_t j = 0; j < n; ++j) memset(A + j * lda, 0, sizeof(double) * (size_t)lda);
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
        int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * N + 8));
        double* len = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            const double* p = rays + 4 * i;
            const int64_t c = orc_ray(g, p, pix, len, work);
            for (int64_t t = 0; t < c; ++t) A[i + (int64_t)pix[t] * lda] += len[t];
        }
        free(work); free(pix); free(len);
    }
    free(rays);
}

/* CSR copy of A (rows in ray order, columns ascending within a row).
 * Returns nnz, or -1 if it would exceed cap (row_ptr is then incomplete). */
int64_t orc_system_csr(const orc_geometry* g, int64_t* row_ptr, int32_t* col, double* val, int64_t cap)
{
    const int32_t N = g->n_pix;
    const int64_t m = (int64_t)g->n_angles * g->n_det;
    double* rays = (double*)malloc(sizeof(double) * 4 * (size_t)m);
    orc_ray_endpoints(g, rays);
    double* work = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
    int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * N + 8));
    double* len = (double*)malloc(sizeof(double) * (size_t)(2 * N + 8));
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        const double* p = rays + 4 * i;
        int64_t c = orc_ray(g, p, pix, len, work);
        /* insertion sort by column so that each row lists ascending pixels */
        for (int64_t a = 1; a < c; ++a) {
            int32_t kp = pix[a]; double kl = len[a]; int64_t b = a - 1;
            while (b >= 0 && pix[b] > kp) { pix[b + 1] = pix[b]; len[b + 1] = len[b]; --b; }
            pix[b + 1] = kp; len[b + 1] = kl;
        }
        if (nnz + c > cap) { free(rays); free(work); free(pix); free(len); return -1; }
        for (int64_t t = 0; t < c; ++t) { col[nnz] = pix[t]; val[nnz] = len[t]; ++nnz; }
        row_ptr[i + 1] = nnz;
    }
    free(rays); free(work); free(pix); free(len);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Householder QR, unblocked (Eq. (qr); the LAPACK geqrf factorization the   */
/* in-memory method calls, Sec. 2.1).  For column j:                         */
/*   x = A[j:m, j], sigma = ||x||_2,                                         */
/*   beta = -sign(x0) sigma (sign(0) = +1), tau = (beta - x0) / beta,        */
/*   v = [1; x[1:] / (x0 - beta)],  R_jj = beta,                             */
/*   A[j:m, j+1:n] -= tau v (v^T A[j:m, j+1:n]).                             */
/* The v below the diagonal overwrite A; R is in the upper triangle.         */
/* sigma == 0 gives tau = 0 (H = I) and the returned info is the first such  */
/* column + 1 (rank deficiency); 0 means every column had a nonzero norm.    */
/* ------------------------------------------------------------------------ */
int64_t orc_householder_qr(int64_t m, int64_t n, double* A, int64_t lda, double* tau)
{
    int64_t info = 0;
    const int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) {
        double* x = A + j + j * lda;
        const int64_t len = m - j;
        /* two-pass scaled 2-norm */
        double scale = 0.0;
        for (int64_t i = 0; i < len; ++i) { double a = fabs(x[i]); if (a > scale) scale = a; }
        double ssq = 0.0;
        if (scale > 0.0)
            for (int64_t i = 0; i < len; ++i) { double t = x[i] / scale; ssq += t * t; }
        const double sigma = scale * sqrt(ssq);
        if (sigma == 0.0) {
            tau[j] = 0.0;
            if (info == 0) info = j + 1;
            continue;
        }
        const double x0 = x[0];
        const double beta = (x0 >= 0.0) ? -sigma : sigma;
        const double t = (beta - x0) / beta;
        const double inv = 1.0 / (x0 - beta);
        for (int64_t i = 1; i < len; ++i) x[i] *= inv;
        x[0] = beta;
        tau[j] = t;
        /* apply H_j = I - t v v^T to the trailing columns */
#pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < n; ++k) {
            double* c = A + j + k * lda;
            double w = c[0];
            for (int64_t i = 1; i < len; ++i) w += x[i] * c[i];
            w *= t;
            c[0] -= w;
            for (int64_t i = 1; i < len; ++i) c[i] -= w * x[i];
        }
    }
    return info;
}

/* C = Q^T B (Eq. (solve), first half; ormqr in Sec. 2.1): for j = 0..k-1,
 * B[j:m, :] -= tau_j v_j (v_j^T B[j:m, :]).  B is m x nrhs, column-major. */
void orc_apply_qt(int64_t m, int64_t k, const double* V, int64_t ldv, const double* tau,
                  double* B, int64_t nrhs, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double* b = B + r * ldb;
        for (int64_t j = 0; j < k; ++j) {
            const double* v = V + j + j * ldv;
            double w = b[j];
            for (int64_t i = 1; i < m - j; ++i) w += v[i] * b[j + i];
            w *= tau[j];
            b[j] -= w;
            for (int64_t i = 1; i < m - j; ++i) b[j + i] -= w * v[i];
        }
    }
}

/* Y = Q Y: the same reflectors applied in reverse order, j = k-1..0. */
void orc_apply_q(int64_t m, int64_t k, const double* V, int64_t ldv, const double* tau,
                 double* B, int64_t nrhs, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double* b = B + r * ldb;
        for (int64_t j = k - 1; j >= 0; --j) {
            const double* v = V + j + j * ldv;
            double w = b[j];
            for (int64_t i = 1; i < m - j; ++i) w += v[i] * b[j + i];
            w *= tau[j];
            b[j] -= w;
            for (int64_t i = 1; i < m - j; ++i) b[j + i] -= w * v[i];
        }
    }
}

/* X = R^{-1} C by back-substitution (Eq. (solve), second half; trsm):
 * x_j = (c_j - sum_{k>j} R_jk x_k) / R_jj for j = n-1..0, in place on C.
 * Returns the first j+1 with R_jj == 0, or 0. */
int64_t orc_back_substitute(int64_t n, const double* R, int64_t ldr, double* C, int64_t nrhs, int64_t ldc)
{
    for (int64_t j = 0; j < n; ++j)
        if (R[j + j * ldr] == 0.0) return j + 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double* c = C + r * ldc;
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = c[j];
            for (int64_t k = j + 1; k < n; ++k) s -= R[j + k * ldr] * c[k];
            c[j] = s / R[j + j * ldr];
        }
    }
    return 0;
}

/* Z = R^{-T} G by forward substitution on R^T (lower triangular):
 * z_j = (g_j - sum_{k<j} R_kj z_k) / R_jj for j = 0..n-1, in place. */
int64_t orc_forward_substitute_rt(int64_t n, const double* R, int64_t ldr, double* G, int64_t nrhs, int64_t ldg)
{
    for (int64_t j = 0; j < n; ++j)
        if (R[j + j * ldr] == 0.0) return j + 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double* g = G + r * ldg;
        for (int64_t j = 0; j < n; ++j) {
            double s = g[j];
            for (int64_t k = 0; k < j; ++k) s -= R[k + j * ldr] * g[k];
            g[j] = s / R[j + j * ldr];
        }
    }
    return 0;
}

/* y = A x (CSR, FP64), the forward projection used for residuals. */
void orc_csr_matvec(int64_t m, const int64_t* row_ptr, const int32_t* col, const double* val,
                    const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s += val[p] * x[col[p]];
        y[i] = s;
    }
}
