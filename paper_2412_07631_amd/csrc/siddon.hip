// Assembly of the fan-beam system matrix A (Eq. (system): a_ij is the length
// of ray i inside pixel j) by Siddon's ray-driven walk (Siddon 1985), or, as a
// second mode, by Joseph's interpolating projector (Joseph 1982), the one the
// paper builds A with (Sec. 3.1).
//
// One lane per ray; the 64 lanes of a wavefront take 64 consecutive detector
// bins of one view, so their writes land on 64 consecutive rows of the
// column-major A and coalesce whenever neighbouring rays cross the same pixel
// column at the same step.  Each ray's crossings with the x- and y-grid lines
// are produced in increasing order by merging the two monotone sequences (no
// sort); each crossing parameter is evaluated from its plane index directly,
// never accumulated, so rounding does not drift along the ray.
#include "ct_internal.h"
#include <math.h>
#include <algorithm>

namespace ctqr {


// Ray i = k * n_det + d: source on the circle of radius sid at angle
// angle0 + 2 pi k / n_angles, flat detector at distance sdd from the source,
// centred on the line through the isocentre, bin centres equispaced.
__device__ inline void ray_points(const GeomDev& g, int64_t i, double& x0, double& y0, double& x1, double& y1)
{
    const int k = (int)(i / g.n_det);
    const int d = (int)(i - (int64_t)k * g.n_det);
    const double th = g.angle0 + 2.0 * M_PI * (double)k / (double)g.n_angles;
    double s, c;
    sincos(th, &s, &c);
    const double pitch = g.det_length / (double)g.n_det;
    const double u = ((double)d - 0.5 * (double)(g.n_det - 1)) * pitch;
    x0 = g.sid * c;
    y0 = g.sid * s;
    x1 = (g.sid - g.sdd) * c - u * s;
    y1 = (g.sid - g.sdd) * s + u * c;
}

// Walks one ray and calls emit(pixel, length) for every segment >= 1e-14 W.
// The pixel of a segment is the one containing its midpoint.
template <typename Emit>
__device__ inline void siddon_walk(double x0, double y0, double x1, double y1, int N, double W, Emit emit)
{
#pragma clang fp contract(off)
    const double dx = x1 - x0, dy = y1 - y0;
    const double lo = -0.5 * W, hi = 0.5 * W, h = W / (double)N;
    double amin = 0.0, amax = 1.0;
    if (dx != 0.0) {
        double a0 = (lo - x0) / dx, a1 = (hi - x0) / dx;
        if (a0 > a1) { const double t = a0; a0 = a1; a1 = t; }
        amin = fmax(amin, a0);
        amax = fmin(amax, a1);
    } else if (x0 < lo || x0 > hi) {
        return;
    }
    if (dy != 0.0) {
        double a0 = (lo - y0) / dy, a1 = (hi - y0) / dy;
        if (a0 > a1) { const double t = a0; a0 = a1; a1 = t; }
        amin = fmax(amin, a0);
        amax = fmin(amax, a1);
    } else if (y0 < lo || y0 > hi) {
        return;
    }
    if (!(amax > amin)) return;

    const double dist = sqrt(dx * dx + dy * dy);
    const double tiny = 1e-14 * W;
    // first candidate plane on each axis, then skip planes at or before amin
    const int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1;
    int ix = 0, iy = 0;
    if (dx != 0.0) {
        const double p = (x0 + amin * dx - lo) / h;
        ix = dx > 0.0 ? (int)floor(p) : (int)ceil(p);
        ix = ix < 0 ? 0 : (ix > N ? N : ix);
        while (ix >= 0 && ix <= N && (lo + (double)ix * h - x0) / dx <= amin) ix += sx;
    }
    if (dy != 0.0) {
        const double p = (y0 + amin * dy - lo) / h;
        iy = dy > 0.0 ? (int)floor(p) : (int)ceil(p);
        iy = iy < 0 ? 0 : (iy > N ? N : iy);
        while (iy >= 0 && iy <= N && (lo + (double)iy * h - y0) / dy <= amin) iy += sy;
    }
    double acur = amin;
    for (int guard = 0; guard < 2 * N + 4; ++guard) {
        const double ax = (dx != 0.0 && ix >= 0 && ix <= N) ? (lo + (double)ix * h - x0) / dx : INFINITY;
        const double ay = (dy != 0.0 && iy >= 0 && iy <= N) ? (lo + (double)iy * h - y0) / dy : INFINITY;
        double anext = fmin(ax, ay);
        const bool last = !(anext < amax);
        if (last) anext = amax;
        const double seg = (anext - acur) * dist;
        if (seg >= tiny) {
            const double am = 0.5 * (acur + anext);
            int px = (int)floor((x0 + am * dx - lo) / h);
            int py = (int)floor((y0 + am * dy - lo) / h);
            px = px < 0 ? 0 : (px > N - 1 ? N - 1 : px);
            py = py < 0 ? 0 : (py > N - 1 ? N - 1 : py);
            emit(py * N + px, seg);
        }
        if (last) break;
        if (ax == anext) ix += sx;
        if (ay == anext) iy += sy;
        acur = anext;
    }
}

// Joseph's projector: the ray is sampled once per pixel-centre line across
// its dominant axis (x when |dx| >= |dy|); there the image is linearly
// interpolated between the two pixels of that column (row) whose centres
// bracket the ray, zero outside the grid, and the sample stands for one pixel
// width along the dominant axis, h |p1 - p0| / |d_dominant|.  Calls
// emit(pixel, weight) for every positive weight (at most 2N).
template <typename Emit>
__device__ inline void joseph_walk(double x0, double y0, double x1, double y1, int N, double W, Emit emit)
{
#pragma clang fp contract(off)
    const double dx = x1 - x0, dy = y1 - y0;
    const double lo = -0.5 * W, h = W / (double)N;
    const bool xmajor = fabs(dx) >= fabs(dy);
    const double dmaj = xmajor ? dx : dy, dmin = xmajor ? dy : dx;
    const double pmaj = xmajor ? x0 : y0, pmin = xmajor ? y0 : x0;
    if (dmaj == 0.0) return;
    const double scale = h * sqrt(dx * dx + dy * dy) / fabs(dmaj);
    for (int k = 0; k < N; ++k) {
        const double c = lo + ((double)k + 0.5) * h;
        const double a = (c - pmaj) / dmaj;
        if (a < 0.0 || a > 1.0) continue;
        const double q = pmin + a * dmin;
        const double fq = (q - lo) / h - 0.5;
        const double fl = floor(fq);
        const double f = fq - fl;
        const int i0 = (int)fl;
        const double w0 = (1.0 - f) * scale, w1 = f * scale;
        if (i0 >= 0 && i0 < N && w0 > 0.0) emit(xmajor ? i0 * N + k : k * N + i0, w0);
        if (i0 + 1 >= 0 && i0 + 1 < N && w1 > 0.0) emit(xmajor ? (i0 + 1) * N + k : k * N + i0 + 1, w1);
    }
}

// The geometry's projector.
template <typename Emit>
__device__ inline void ray_walk(const GeomDev& g, double x0, double y0, double x1, double y1, Emit emit)
{
    if (g.proj == 1) joseph_walk(x0, y0, x1, y1, g.n_pix, g.W, emit);
    else siddon_walk(x0, y0, x1, y1, g.n_pix, g.W, emit);
}

template <typename T>
__global__ void __launch_bounds__(256) fill_zero_kernel(T* A, int64_t lda, int64_t m, int64_t n)
{
    // column-major m x n block with leading dimension lda; zero rows [0, m)
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        T* col = A + j * lda;
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x) col[i] = (T)0;
    }
}

template <typename T>
__global__ void __launch_bounds__(64) siddon_dense_kernel(GeomDev g, T* A, int64_t lda)
{
    const int64_t m = (int64_t)g.n_angles * g.n_det;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double x0, y0, x1, y1;
    ray_points(g, i, x0, y0, x1, y1);
    T* row = A + i;
    ray_walk(g, x0, y0, x1, y1, [&](int j, double len) { row[(int64_t)j * lda] = (T)len; });
}

__global__ void __launch_bounds__(64) siddon_count_kernel(GeomDev g, int64_t* counts)
{
    const int64_t m = (int64_t)g.n_angles * g.n_det;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double x0, y0, x1, y1;
    ray_points(g, i, x0, y0, x1, y1);
    int64_t c = 0;
    ray_walk(g, x0, y0, x1, y1, [&](int, double) { ++c; });
    counts[i + 1] = c;
}

// Exclusive prefix sum in place over row_ptr[0..m] where row_ptr[i+1] holds
// the count of row i on entry; one workgroup of 1024 lanes, chunked.
__global__ void __launch_bounds__(1024) csr_scan_kernel(int64_t* row_ptr, int64_t m)
{
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) { row_ptr[0] = 0; carry = 0; }
    __syncthreads();
    for (int64_t base = 0; base < m; base += 1024 * 8) {
        // each lane sums 8 consecutive counts
        int64_t loc[8];
        int64_t s = 0;
        for (int q = 0; q < 8; ++q) {
            const int64_t idx = base + (int64_t)t * 8 + q;
            loc[q] = idx < m ? row_ptr[idx + 1] : 0;
            s += loc[q];
        }
        part[t] = s;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t v = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        int64_t run = carry + (t > 0 ? part[t - 1] : 0);
        for (int q = 0; q < 8; ++q) {
            const int64_t idx = base + (int64_t)t * 8 + q;
            run += loc[q];
            if (idx < m) row_ptr[idx + 1] = run;
        }
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) siddon_csr_kernel(GeomDev g, const int64_t* row_ptr, int32_t* col,
                                                        double* val, int64_t cap)
{
    const int64_t m = (int64_t)g.n_angles * g.n_det;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (row_ptr[m] > cap) return;   // too small: nothing is written
    double x0, y0, x1, y1;
    ray_points(g, i, x0, y0, x1, y1);
    int64_t p = row_ptr[i];
    ray_walk(g, x0, y0, x1, y1, [&](int j, double len) {
        col[p] = j;
        val[p] = len;
        ++p;
    });
}

// Rows for an explicit list of rays (r x 4 end points), dense row-major.
__global__ void __launch_bounds__(64) siddon_rows_kernel(const double* rays, int64_t r, int32_t N, double W,
                                                         double* rows)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const double* p = rays + 4 * i;
    double* row = rows + i * (int64_t)N * N;
    siddon_walk(p[0], p[1], p[2], p[3], N, W, [&](int j, double len) { row[j] = len; });
}

// ---------------------------------------------------------------- launchers
hipError_t launch_siddon_dense(const GeomDev& g, int dtype, void* A, int64_t lda, hipStream_t s)
{
    const int64_t m = (int64_t)g.n_angles * g.n_det, n = (int64_t)g.n_pix * g.n_pix;
    const int blocks = (int)(n < 65536 ? n : 65536);
    const int rb = (int)((m + 63) / 64);
    if (dtype == 0) {
        fill_zero_kernel<double><<<blocks, 256, 0, s>>>((double*)A, lda, m, n);
        siddon_dense_kernel<double><<<rb, 64, 0, s>>>(g, (double*)A, lda);
    } else {
        fill_zero_kernel<float><<<blocks, 256, 0, s>>>((float*)A, lda, m, n);
        siddon_dense_kernel<float><<<rb, 64, 0, s>>>(g, (float*)A, lda);
    }
    return hipGetLastError();
}

hipError_t launch_siddon_csr(const GeomDev& g, int64_t* row_ptr, int32_t* col, double* val, int64_t cap,
                             hipStream_t s)
{
    const int64_t m = (int64_t)g.n_angles * g.n_det;
    const int rb = (int)((m + 63) / 64);
    siddon_count_kernel<<<rb, 64, 0, s>>>(g, row_ptr);
    csr_scan_kernel<<<1, 1024, 0, s>>>(row_ptr, m);
    if (col != nullptr && val != nullptr) siddon_csr_kernel<<<rb, 64, 0, s>>>(g, row_ptr, col, val, cap);
    return hipGetLastError();
}

hipError_t launch_csr_scan(int64_t* ptr, int64_t m, hipStream_t s)
{
    csr_scan_kernel<<<1, 1024, 0, s>>>(ptr, m);
    return hipGetLastError();
}

hipError_t launch_siddon_rows(const double* rays, int64_t r, int32_t N, double W, double* rows, hipStream_t s)
{
    const int64_t n = (int64_t)N * N;
    const int blocks = (int)(r < 65536 ? r : 65536);
    fill_zero_kernel<double><<<blocks, 256, 0, s>>>(rows, n, n, r);
    siddon_rows_kernel<<<(int)((r + 63) / 64), 64, 0, s>>>(rays, r, N, W, rows);
    return hipGetLastError();
}

}  // namespace ctqr

namespace ctqr {

// ----------------------------------------------------------------------------
// CSC copy (the rows of A^T) from the CSR copy, for the FP64 products A^T r.
// Entries of a column are sorted by row, so the copy -- and every product
// computed from it -- is independent of the scheduling of the fill.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) csc_count_kernel(const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col, int64_t m,
                                                        int64_t* col_ptr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
        atomicAdd((unsigned long long*)&col_ptr[(int64_t)col[p] + 1], 1ull);
}

__global__ void __launch_bounds__(256) csc_fill_kernel(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, int64_t m,
                                                       const int64_t* __restrict__ col_ptr, int32_t* fill,
                                                       int32_t* row, double* cval)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const int32_t c = col[p];
        const int64_t q = col_ptr[c] + atomicAdd(&fill[c], 1);
        row[q] = (int32_t)i;
        cval[q] = val[p];
    }
}

__global__ void __launch_bounds__(256) csc_sort_kernel(const int64_t* __restrict__ col_ptr, int64_t n, int32_t* row,
                                                       double* cval)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int64_t s = col_ptr[j], e = col_ptr[j + 1];
    for (int64_t a = s + 1; a < e; ++a) {
        const int32_t kr = row[a];
        const double kv = cval[a];
        int64_t b = a - 1;
        while (b >= s && row[b] > kr) {
            row[b + 1] = row[b];
            cval[b + 1] = cval[b];
            --b;
        }
        row[b + 1] = kr;
        cval[b + 1] = kv;
    }
}

__global__ void __launch_bounds__(256) zero_i64_kernel(int64_t* p, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) p[e] = 0;
}

__global__ void __launch_bounds__(256) zero_i32_kernel(int32_t* p, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) p[e] = 0;
}

hipError_t launch_csc(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, int64_t n,
                      int64_t* col_ptr, int32_t* row, double* cval, int32_t* work, hipStream_t s)
{
    const unsigned gz = (unsigned)std::min<int64_t>((n + 256) / 256, 4096);
    zero_i64_kernel<<<gz, 256, 0, s>>>(col_ptr, n + 1);
    zero_i32_kernel<<<gz, 256, 0, s>>>(work, n);
    const unsigned gm = (unsigned)((m + 255) / 256);
    csc_count_kernel<<<gm, 256, 0, s>>>(row_ptr, col, m, col_ptr);
    csr_scan_kernel<<<1, 1024, 0, s>>>(col_ptr, n);
    csc_fill_kernel<<<gm, 256, 0, s>>>(row_ptr, col, val, m, col_ptr, work, row, cval);
    csc_sort_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(col_ptr, n, row, cval);
    return hipGetLastError();
}

}  // namespace ctqr
