// Triangular diagonal-block solves, the FP64 residual, and small elementwise
// kernels of the solve path (Eq. (solve): X = R^{-1} C with R kept triangular
// and never inverted; the blocked back-substitution of Sec. 2.2 alternates
// these diagonal solves with GEMM updates of the rows above).
#include "ct_internal.h"

#include <algorithm>

namespace ctqr {

constexpr int kTrsmBlock = 128;

// X_b = R_bb^{-1} C_b (UPPER) or Z_b = R_bb^{-T} C_b (!UPPER) in place, for a
// bo x bo diagonal block (bo <= 128) and nrhs columns.  R_bb sits in LDS as
// FP64 (leading dimension bo + 1 against bank conflicts); one wavefront per
// right-hand side, two rows per lane, one substitution step per row.
template <typename TS, bool UPPER>
__global__ void __launch_bounds__(256) trsm_diag_kernel(const TS* __restrict__ R, int64_t ldr, int bo,
                                                        TS* __restrict__ B, int64_t ldb, int nrhs,
                                                        const int32_t* desc)
{
    extern __shared__ double Rs[];
    if (desc) {
        B += (int64_t)desc_offset(desc) * ldb;
        nrhs = desc_count(desc, nrhs);
    }
    if (blockIdx.x * 4 >= nrhs) return;
    const int ld = bo + 1;
    for (int e = threadIdx.x; e < bo * bo; e += 256) {
        const int q = e / bo, p = e - q * bo;
        Rs[p + q * ld] = p <= q ? (double)R[p + (int64_t)q * ldr] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j = blockIdx.x * 4 + wv; j < nrhs; j += gridDim.x * 4) {
        TS* col = B + (int64_t)j * ldb;
        double x0 = lane < bo ? (double)col[lane] : 0.0;
        double x1 = lane + 64 < bo ? (double)col[lane + 64] : 0.0;
        if (UPPER) {
            for (int jj = bo - 1; jj >= 0; --jj) {
                const int owner = jj & 63;
                const double cj = __shfl(jj < 64 ? x0 : x1, owner, 64);
                const double z = cj / Rs[jj + jj * ld];
                if (lane == owner) {
                    if (jj < 64) x0 = z; else x1 = z;
                }
                if (lane < jj) x0 -= Rs[lane + jj * ld] * z;
                if (lane + 64 < jj) x1 -= Rs[lane + 64 + jj * ld] * z;
            }
        } else {
            for (int jj = 0; jj < bo; ++jj) {
                const int owner = jj & 63;
                const double cj = __shfl(jj < 64 ? x0 : x1, owner, 64);
                const double z = cj / Rs[jj + jj * ld];
                if (lane == owner) {
                    if (jj < 64) x0 = z; else x1 = z;
                }
                if (lane > jj && lane < bo) x0 -= Rs[jj + lane * ld] * z;
                if (lane + 64 > jj && lane + 64 < bo) x1 -= Rs[jj + (lane + 64) * ld] * z;
            }
        }
        if (lane < bo) col[lane] = (TS)x0;
        if (lane + 64 < bo) col[lane + 64] = (TS)x1;
    }
}

// Solve-side copies of R, built once per factorization, for 256-row blocks.
// Step 1: the inverse of every 128-row diagonal block, one workgroup each.
// The block (upper triangle) and its inverse are kept packed in LDS as FP64
// (column-major triangle: entry (i, j), i <= j, at j (j + 1) / 2 + i); thread j
// computes column j of the inverse by back-substitution against the unit
// vector e_j, independently of the other columns.  Written in FP64 to the
// diagonal of its 256-row block in Ri64 (block k at k * 256^2, ld 256).
__global__ void __launch_bounds__(128) rinv128_kernel(const void* __restrict__ Av, int f64, int64_t lda, int64_t n,
                                                      double* __restrict__ Ri64)
{
    extern __shared__ double tri[];
    constexpr int B = 128;
    constexpr int NP = B * (B + 1) / 2;
    double* Rp = tri;
    double* Xp = tri + NP;
    const int64_t k0 = (int64_t)blockIdx.x * B;
    const int bo = (int)((n - k0) < B ? (n - k0) : B);
    const int t = threadIdx.x;
    for (int j = 0; j < bo; ++j)
        for (int i = t; i <= j; i += B) {
            const int64_t e = (k0 + i) + (k0 + j) * lda;
            Rp[j * (j + 1) / 2 + i] = f64 ? ((const double*)Av)[e] : (double)((const float*)Av)[e];
        }
    __syncthreads();
    if (t < bo) {
        const int j = t;
        const int cj = j * (j + 1) / 2;
        Xp[cj + j] = 1.0 / Rp[cj + j];
        for (int i = j - 1; i >= 0; --i) {
            double s0 = 0.0, s1 = 0.0;
            int l = i + 1;
            for (; l + 1 <= j; l += 2) {
                s0 += Rp[l * (l + 1) / 2 + i] * Xp[cj + l];
                s1 += Rp[(l + 1) * (l + 2) / 2 + i] * Xp[cj + l + 1];
            }
            if (l <= j) s0 += Rp[l * (l + 1) / 2 + i] * Xp[cj + l];
            Xp[cj + i] = -(s0 + s1) / Rp[i * (i + 1) / 2 + i];
        }
    }
    __syncthreads();
    double* out = Ri64 + (size_t)(blockIdx.x >> 1) * 256 * 256 + (size_t)(blockIdx.x & 1) * B * 257;
    for (int e = t; e < B * B; e += B) {
        const int i = e % B, j = e / B;
        out[i + (size_t)j * 256] = (i <= j && j < bo) ? Xp[j * (j + 1) / 2 + i] : 0.0;
    }
}

// Step 2: the coupling block of each 256-row block's inverse,
//   [A B; 0 D]^{-1} = [A^{-1}  -A^{-1} B D^{-1}; 0  D^{-1}],
// STEP 0: M = B D^{-1} (128 x n2, ld 128), STEP 1: X12 = -A^{-1} M; block
// k = blockIdx.y, one output per thread.
template <int STEP>
__global__ void __launch_bounds__(256) rinv_join_kernel(const void* __restrict__ Av, int f64, int64_t lda, int64_t n,
                                                        double* __restrict__ Ri64, double* __restrict__ M)
{
    const int64_t k0 = (int64_t)blockIdx.y * 256;
    const int bo = (int)((n - k0) < 256 ? (n - k0) : 256);
    const int n2 = bo - 128;
    if (n2 <= 0) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 128 * n2) return;
    const int r = e % 128, q = e / 128;
    double* X = Ri64 + (size_t)blockIdx.y * 256 * 256;
    double* Mk = M + (size_t)blockIdx.y * 128 * 128;
    double s0 = 0.0, s1 = 0.0;
    if (STEP == 0) {
        const double* Dinv = X + 128 + (size_t)128 * 256;
        for (int l = 0; l <= q; ++l) {
            const int64_t ei = (k0 + r) + (k0 + 128 + l) * lda;
            const double b = f64 ? ((const double*)Av)[ei] : (double)((const float*)Av)[ei];
            if (l & 1) s1 += b * Dinv[l + (size_t)q * 256];
            else s0 += b * Dinv[l + (size_t)q * 256];
        }
        Mk[r + q * 128] = s0 + s1;
    } else {
        const double* mq = Mk + (size_t)q * 128;
        int l = r;
        for (; l + 1 < 128; l += 2) {
            s0 += X[r + (size_t)l * 256] * mq[l];
            s1 += X[r + (size_t)(l + 1) * 256] * mq[l + 1];
        }
        if (l < 128) s0 += X[r + (size_t)l * 256] * mq[l];
        X[r + (size_t)(128 + q) * 256] = -(s0 + s1);
    }
}

// Step 3: the inverses in the storage type, row-major (RiR, for X_b =
// R_bb^{-1} C_b) and column-major (RiC, for Z_b = R_bb^{-T} C_b), 256 x 256
// per block with zeros outside the triangle.
template <typename TS>
__global__ void __launch_bounds__(256) rinv_store_kernel(const double* __restrict__ Ri64, int64_t n,
                                                         TS* __restrict__ RiR, TS* __restrict__ RiC)
{
    const int64_t k0 = (int64_t)blockIdx.y * 256;
    const int bo = (int)((n - k0) < 256 ? (n - k0) : 256);
    const double* X = Ri64 + (size_t)blockIdx.y * 256 * 256;
    TS* R = RiR + (size_t)blockIdx.y * 256 * 256;
    TS* C = RiC + (size_t)blockIdx.y * 256 * 256;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < 256 * 256; e += gridDim.x * 256) {
        const int i = e / 256, j = e % 256;     // row-major walk: (i, j) at i * 256 + j
        R[e] = (i <= j && j < bo) ? (TS)X[i + (size_t)j * 256] : (TS)0;
        const int jc = e / 256, ic = e % 256;   // column-major walk: (ic, jc) at jc * 256 + ic
        C[e] = (ic <= jc && jc < bo) ? (TS)X[ic + (size_t)jc * 256] : (TS)0;
    }
}

// Row-major copies of R above its diagonal, for the products of the blocked
// back-substitution, in two levels of blocks: outer blocks of ob columns
// (a multiple of 256) and, inside each, 256-column blocks.
//   outer block B (columns K0 = ob B .. K0 + ob): rows 0..K0 of those
//     columns, Rt4_B[p * ob + c] = R[p][K0 + c] (zero past column n), at
//     element ob^2 B (B - 1) / 2;
//   inner block i >= 1 of B (columns K0 + 256 i .. + 256): rows K0 .. K0 + 256 i,
//     Rin_{B,i}[(p - K0) * 256 + c] = R[p][K0 + 256 i + c], at element
//     ob^2 nbo (nbo - 1) / 2 + B 256^2 q (q - 1) / 2 + 256^2 i (i - 1) / 2
//     (nbo outer blocks, q = ob / 256).
// With ob = 256 this is the one-level layout: every 256-column block's rows
// above its diagonal block.  Tiles of 16 rows x 256 columns pass through LDS
// so that both the column-major reads and the row-major writes are coalesced.
// Grid: x row tiles, y outer blocks, z < q the outer block's 256-column
// chunks, z >= q its inner blocks i = z - q + 1.
size_t rt_elems(int64_t n, int ob)
{
    const int64_t nbo = (n + ob - 1) / ob, q = ob / 256;
    return (size_t)ob * ob * (size_t)(nbo * (nbo - 1) / 2) + (size_t)nbo * 256 * 256 * (size_t)(q * (q - 1) / 2);
}

template <typename TS>
__global__ void __launch_bounds__(256) rt_kernel(const TS* __restrict__ A, int64_t lda, int64_t n, int ob,
                                                 TS* __restrict__ Rt)
{
    constexpr int B = 256, TR = 16;
    __shared__ TS tile[B][TR + 1];
    const int64_t ob_ = ob, q = ob / 256, nbo = (n + ob - 1) / ob;
    const int64_t Bk = blockIdx.y, K0 = Bk * ob_;
    const int z = blockIdx.z;
    int64_t c0, p0, p1;          // source columns c0 .. c0 + 256, rows p0 .. p1
    TS* out;
    int64_t ldo;
    if (z < q) {
        c0 = K0 + (int64_t)z * B;
        p0 = (int64_t)blockIdx.x * TR;
        p1 = K0;
        out = Rt + (size_t)ob_ * ob_ * (size_t)(Bk * (Bk - 1) / 2) + (size_t)z * B;
        ldo = ob_;
    } else {
        const int64_t i = z - q + 1;
        c0 = K0 + i * B;
        p0 = K0 + (int64_t)blockIdx.x * TR;
        p1 = K0 + i * B;
        out = Rt + (size_t)ob_ * ob_ * (size_t)(nbo * (nbo - 1) / 2) + (size_t)Bk * B * B * (size_t)(q * (q - 1) / 2) +
              (size_t)B * B * (size_t)(i * (i - 1) / 2) - (size_t)K0 * B;
        ldo = B;
    }
    if (p0 >= p1 || c0 >= n) return;          // (columns past n are never read)
    const int64_t cols = n - c0;
    const int t = threadIdx.x;
    for (int e = t; e < B * TR; e += 256) {
        const int c = e / TR, r = e % TR;        // r fastest: along a column of R
        const int64_t p = p0 + r;
        tile[c][r] = (c < cols && p < p1) ? A[p + (c0 + c) * lda] : (TS)0;
    }
    __syncthreads();
    for (int e = t; e < B * TR; e += 256) {
        const int r = e / B, c = e % B;          // c fastest: along a row of the copy
        const int64_t p = p0 + r;
        if (p < p1) out[p * ldo + c] = tile[c][r];
    }
}

// dst[:, q] = src[:, q] for rows [0, rows) and the batch's columns; the
// batch descriptor (if any) offsets the source columns.
template <typename TS>
__global__ void __launch_bounds__(256) copy_block_kernel(const TS* __restrict__ src, int64_t lds,
                                                         TS* __restrict__ dst, int64_t ldd, int rows, int cols,
                                                         const int32_t* desc)
{
    cols = desc_count(desc, cols);
    src += (int64_t)desc_offset(desc) * lds;
    for (int q = blockIdx.y; q < cols; q += gridDim.y)
        for (int r = blockIdx.x * 256 + threadIdx.x; r < rows; r += gridDim.x * 256)
            dst[r + (int64_t)q * ldd] = src[r + (int64_t)q * lds];
}

// R = B - A X in FP64 from the CSR copy of A; one lane per row, eight
// right-hand sides per lane so each CSR entry is read once per eight columns.
__global__ void __launch_bounds__(256) residual_kernel(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, int64_t m,
                                                       const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ B, int64_t ldb, double* R,
                                                       int64_t ldr, int nrhs)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * 8;
    if (i >= m) return;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    const int nq = nrhs - j0 < 8 ? nrhs - j0 : 8;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const double v = val[p];
        const int64_t c = col[p];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < nq) acc[q] += v * X[c + (int64_t)(j0 + q) * ldx];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < nq) R[i + (int64_t)(j0 + q) * ldr] = B[i + (int64_t)(j0 + q) * ldb] - acc[q];
}

// S = A^T R in FP64 from the CSC copy of A (entries of a column sorted by
// row); one lane per column, eight right-hand sides per lane.
__global__ void __launch_bounds__(256) residual_t_kernel(const int64_t* __restrict__ col_ptr,
                                                         const int32_t* __restrict__ row,
                                                         const double* __restrict__ cval, int64_t n,
                                                         const double* __restrict__ R, int64_t ldr, double* S,
                                                         int64_t lds, int nrhs)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c0 = blockIdx.y * 8;
    if (j >= n) return;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    const int nq = nrhs - c0 < 8 ? nrhs - c0 : 8;
    for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
        const double v = cval[p];
        const int64_t i = row[p];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < nq) acc[q] += v * R[i + (int64_t)(c0 + q) * ldr];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < nq) S[j + (int64_t)(c0 + q) * lds] = acc[q];
}

// ---------------------------------------------------------------------------
// Slice-contiguous ("transposed") layouts for the refinement: a vector block
// Zt of r rows and nrhs slices stores element (i, j) at Zt[i * ld + j], so one
// wavefront reads the 64 slices of a row with one coalesced load.
// Rt = Bt - A Xt (CSR) and St = A^T Rt (CSC), one wavefront per matrix row
// (column); CSR/CSC entries are wave-uniform scalar loads.  Rows are dealt
// to the 8 XCDs in contiguous ranges so neighbouring rays, which cross
// nearly the same pixels, share an L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_row(int64_t b, int64_t rows)
{
    if (rows % 8 != 0) return b;
    return (b % 8) * (rows / 8) + b / 8;
}

__global__ void __launch_bounds__(64) spmv_rows_t_kernel(const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const double* __restrict__ val, int64_t rows,
                                                         const double* __restrict__ Xt, const double* __restrict__ Bt,
                                                         double* __restrict__ Rt, int64_t ld, int nrhs)
{
    const int64_t i = xcd_row(blockIdx.x, rows);
    const int lane = threadIdx.x;
    const int64_t p0 = ptr[i], p1 = ptr[i + 1];
    for (int j0 = 0; j0 < nrhs; j0 += 512) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int64_t p = p0; p < p1; ++p) {
            const double v = val[p];
            const double* xr = Xt + (int64_t)idx[p] * ld + j0 + lane;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (j0 + lane + 64 * q < nrhs) acc[q] += v * xr[64 * q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + lane + 64 * q;
            if (j < nrhs) Rt[i * ld + j] = (Bt ? Bt[i * ld + j] : 0.0) - acc[q];
        }
    }
}

// St[j][q] = sum_{p in column j} cval[p] Rt[row[p]][q]  (sign +)
__global__ void __launch_bounds__(64) spmv_cols_t_kernel(const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const double* __restrict__ val, int64_t cols,
                                                         const double* __restrict__ Rt, double* __restrict__ St,
                                                         int64_t ld, int nrhs)
{
    const int64_t jc = xcd_row(blockIdx.x, cols);
    const int lane = threadIdx.x;
    const int64_t p0 = ptr[jc], p1 = ptr[jc + 1];
    for (int j0 = 0; j0 < nrhs; j0 += 512) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int64_t p = p0; p < p1; ++p) {
            const double v = val[p];
            const double* rr = Rt + (int64_t)idx[p] * ld + j0 + lane;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (j0 + lane + 64 * q < nrhs) acc[q] += v * rr[64 * q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + lane + 64 * q;
            if (j < nrhs) St[jc * ld + j] = acc[q];
        }
    }
}

// out[j] = ||Zt[:, j]||_2 over `rows` rows of a slice-contiguous block
constexpr int kNormChunks = 256;

// Column norms of a slice-contiguous block, in two deterministic passes:
// workgroup (x, ch) sums the squares of rows ch, ch + kNormChunks, ... for 64
// slices into part[ch][j]; the second pass adds the chunks in order.
__global__ void __launch_bounds__(256) colnorm_t_kernel(const double* __restrict__ Zt, int64_t ld, int64_t rows,
                                                        int nrhs, double* __restrict__ part)
{
    __shared__ double red[4][64];
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int sub = threadIdx.x >> 6;
    double s = 0.0;
    if (j < nrhs)
        for (int64_t i = blockIdx.y + (int64_t)kNormChunks * sub; i < rows; i += 4 * kNormChunks) {
            const double v = Zt[i * ld + j];
            s += v * v;
        }
    red[sub][threadIdx.x & 63] = s;
    __syncthreads();
    if (sub == 0 && j < nrhs)
        part[(size_t)blockIdx.y * nrhs + j] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

__global__ void __launch_bounds__(256) colnorm_sum_kernel(const double* __restrict__ part, int nrhs,
                                                          double* __restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nrhs) return;
    double s = 0.0;
    for (int ch = 0; ch < kNormChunks; ++ch) s += part[(size_t)ch * nrhs + j];
    out[j] = sqrt(s);
}

// Transpose with conversion between a column-major block (rows x cols, ld ldc)
// and a slice-contiguous block (element (i, j) at Zt[i * ldt + j]).
//   TO_T: column-major -> slice-contiguous, else the reverse.  ACC adds.
template <typename TI, typename TO, bool TO_T, bool ACC>
__global__ void __launch_bounds__(256) transpose_kernel(const TI* __restrict__ in, TO* __restrict__ out, int64_t rows,
                                                        int cols, int64_t ldc, int64_t ldt)
{
    __shared__ double tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int t = threadIdx.x;
    if (TO_T) {
        for (int e = t; e < 64 * 64; e += 256) {
            const int jj = e / 64, ii = e % 64;
            const int64_t i = i0 + ii;
            const int j = j0 + jj;
            tile[jj][ii] = (i < rows && j < cols) ? (double)in[i + (int64_t)j * ldc] : 0.0;
        }
        __syncthreads();
        for (int e = t; e < 64 * 64; e += 256) {
            const int ii = e / 64, jj = e % 64;
            const int64_t i = i0 + ii;
            const int j = j0 + jj;
            if (i < rows && j < cols) {
                TO* d = out + i * ldt + j;
                *d = ACC ? (TO)((double)*d + tile[jj][ii]) : (TO)tile[jj][ii];
            }
        }
    } else {
        for (int e = t; e < 64 * 64; e += 256) {
            const int ii = e / 64, jj = e % 64;
            const int64_t i = i0 + ii;
            const int j = j0 + jj;
            tile[jj][ii] = (i < rows && j < cols) ? (double)in[i * ldt + j] : 0.0;
        }
        __syncthreads();
        for (int e = t; e < 64 * 64; e += 256) {
            const int jj = e / 64, ii = e % 64;
            const int64_t i = i0 + ii;
            const int j = j0 + jj;
            if (i < rows && j < cols) {
                TO* d = out + i + (int64_t)j * ldc;
                *d = ACC ? (TO)((double)*d + tile[jj][ii]) : (TO)tile[jj][ii];
            }
        }
    }
}

// Y (rows x cols, ldy) = (TO) X (ldx)
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) convert_kernel(const TI* __restrict__ X, int64_t ldx, TO* __restrict__ Y,
                                                      int64_t ldy, int64_t rows, int cols)
{
    for (int j = blockIdx.y; j < cols; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
            Y[i + (int64_t)j * ldy] = (TO)X[i + (int64_t)j * ldx];
}

// X (FP64) += D
template <typename TD>
__global__ void __launch_bounds__(256) accumulate_kernel(double* __restrict__ X, int64_t ldx,
                                                         const TD* __restrict__ D, int64_t ldd, int64_t rows,
                                                         int cols)
{
    for (int j = blockIdx.y; j < cols; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
            X[i + (int64_t)j * ldx] += (double)D[i + (int64_t)j * ldd];
}

template <typename T>
__global__ void __launch_bounds__(256) zero_rows_kernel(T* __restrict__ Y, int64_t ldy, int64_t r0, int64_t r1,
                                                        int cols)
{
    for (int j = blockIdx.y; j < cols; j += gridDim.y)
        for (int64_t i = r0 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < r1; i += (int64_t)gridDim.x * 256)
            Y[i + (int64_t)j * ldy] = (T)0;
}

// Relative size of a refinement correction per slice, for the stop rule:
// ratio[j] = ||D[:, j]||_2 / ||X[:, j]||_2 (FP64 sums in a fixed-order tree,
// one workgroup per slice), and the largest over the slices into *maxw as
// the bit pattern of a non-negative double (ordered like the values).
template <typename TD>
__global__ void __launch_bounds__(256) corr_ratio_kernel(const TD* __restrict__ D, int64_t ldd,
                                                         const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                         double* __restrict__ ratio,
                                                         unsigned long long* __restrict__ maxw)
{
    __shared__ double rd[256], rx[256];
    const int j = blockIdx.x;
    double sd = 0.0, sx = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        const double d = (double)D[i + (int64_t)j * ldd], x = X[i + (int64_t)j * ldx];
        sd += d * d;
        sx += x * x;
    }
    rd[threadIdx.x] = sd;
    rx[threadIdx.x] = sx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rd[threadIdx.x] += rd[threadIdx.x + w];
            rx[threadIdx.x] += rx[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nd = sqrt(rd[0]), nx = sqrt(rx[0]);
        const double r = nx > 0.0 ? nd / nx : (nd > 0.0 ? __builtin_huge_val() : 0.0);
        ratio[j] = r;
        atomicMax(maxw, (unsigned long long)__double_as_longlong(r));
    }
}

__global__ void zero_word_kernel(unsigned long long* w) { *w = 0ull; }

// out[j] = ||X[:, j]||_2 in FP64 (fixed-order tree, one workgroup per column)
__global__ void __launch_bounds__(256) colnorm_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                      double* out)
{
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        const double v = X[i + (int64_t)j * ldx];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sqrt(red[0]);
}

// Sums of squares of the columns of a column-major block (fixed-order tree,
// one workgroup per column): out[j] = sum_i C[i + j ldc]^2, in FP64.
template <typename T>
__global__ void __launch_bounds__(256) colsq_kernel(const T* __restrict__ C, int64_t ldc, int64_t rows,
                                                    double* __restrict__ out)
{
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        const double v = (double)C[i + (int64_t)j * ldc];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

// Per-slice coefficient of the conjugate-gradient updates: num / den^2 when den
// is a norm (the step length gamma / ||A p||^2), num / den otherwise (the
// ratio of successive gammas); zero where the denominator vanishes (a slice
// whose residual is already zero keeps its image).
__device__ inline double cg_coef(const double* num, const double* den, int j, bool den_is_norm)
{
    const double d = den_is_norm ? den[j] * den[j] : den[j];
    return d > 0.0 ? num[j] / d : 0.0;
}

// Slice-contiguous blocks (element (i, j) at i * ld + j), one coefficient c_j
// per slice:  mode 0: y += c_j x,  mode 1: y = x + c_j y.
__global__ void __launch_bounds__(256) cg_update_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                        int64_t rows, int nrhs, int64_t ld,
                                                        const double* __restrict__ num,
                                                        const double* __restrict__ den, int mode)
{
    const int64_t total = rows * ld;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int j = (int)(e % ld);
        if (j >= nrhs) continue;
        const double c = cg_coef(num, den, j, mode == 0);
        y[e] = mode == 0 ? y[e] + c * x[e] : x[e] + c * y[e];
    }
}

// Stop rule of the conjugate-gradient refinement: the step of slice j is
// c_j p_j with c_j = gamma_j / ||A p_j||^2; its size relative to the updated
// image, max over slices into *maxw (the bits of a non-negative double).
__global__ void __launch_bounds__(256) cg_ratio_kernel(const double* __restrict__ gam,
                                                       const double* __restrict__ qn,
                                                       const double* __restrict__ pn,
                                                       const double* __restrict__ xn, int nrhs,
                                                       unsigned long long* __restrict__ maxw)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nrhs) return;
    const double step = fabs(cg_coef(gam, qn, j, true)) * pn[j];
    const double r = xn[j] > 0.0 ? step / xn[j] : (step > 0.0 ? __builtin_huge_val() : 0.0);
    atomicMax(maxw, (unsigned long long)__double_as_longlong(r));
}

// ------------------------------------------------------------------ launchers
static inline dim3 grid2(int64_t rows, int cols)
{
    int64_t gx = (rows + 255) / 256;
    if (gx > 1024) gx = 1024;
    int gy = cols < 65535 ? cols : 65535;
    return dim3((unsigned)(gx > 0 ? gx : 1), (unsigned)(gy > 0 ? gy : 1));
}

template <typename TS, bool UPPER>
hipError_t launch_trsm_diag(const TS* R, int64_t ldr, int bo, TS* B, int64_t ldb, int nrhs, hipStream_t s,
                            const int32_t* desc)
{
    const size_t sh = (size_t)bo * (bo + 1) * sizeof(double);
    int blocks = (nrhs + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL((trsm_diag_kernel<TS, UPPER>), dim3(blocks), dim3(256), sh, s, R, ldr, bo, B, ldb, nrhs, desc);
    return hipGetLastError();
}

// Inverses of the 256-row diagonal blocks of R (RiR row-major, RiC
// column-major, 256^2 elements per block); Ri64 (n_blocks x 256^2 FP64) and M
// (n_blocks x 128^2 FP64) are scratch.
template <typename TS>
hipError_t launch_rinv(const TS* A, int64_t lda, int64_t n, TS* RiR, TS* RiC, double* Ri64, double* M, hipStream_t s)
{
    const unsigned b128 = (unsigned)((n + 127) / 128), b256 = (unsigned)((n + 255) / 256);
    const size_t sh = (size_t)128 * 129 * sizeof(double);   // two packed triangles
    const int f64 = sizeof(TS) == 8;
    hipLaunchKernelGGL(rinv128_kernel, dim3(b128), dim3(128), sh, s, (const void*)A, f64, lda, n, Ri64);
    const dim3 gj(128 * 128 / 256, b256);
    hipLaunchKernelGGL((rinv_join_kernel<0>), gj, dim3(256), 0, s, (const void*)A, f64, lda, n, Ri64, M);
    hipLaunchKernelGGL((rinv_join_kernel<1>), gj, dim3(256), 0, s, (const void*)A, f64, lda, n, Ri64, M);
    hipLaunchKernelGGL(rinv_store_kernel<TS>, dim3(64, b256), dim3(256), 0, s, (const double*)Ri64, n, RiR, RiC);
    return hipGetLastError();
}

// C (column-major, ld ld, rows x cols) = the identity on its leading w x w
// block, zero elsewhere
template <typename TS>
__global__ void __launch_bounds__(256) eye_kernel(TS* __restrict__ C, int64_t ld, int64_t rows, int cols, int w)
{
    for (int j = blockIdx.y; j < cols; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
            C[i + (int64_t)j * ld] = (i == j && i < w) ? (TS)1 : (TS)0;
}

template <typename TS>
hipError_t launch_eye(TS* C, int64_t ld, int64_t rows, int cols, int w, hipStream_t s)
{
    const dim3 grid((unsigned)((rows + 255) / 256), (unsigned)(cols < 65535 ? cols : 65535));
    hipLaunchKernelGGL(eye_kernel<TS>, grid, dim3(256), 0, s, C, ld, rows, cols, w);
    return hipGetLastError();
}
template hipError_t launch_eye<float>(float*, int64_t, int64_t, int, int, hipStream_t);

template <typename TS>
hipError_t launch_rt(const TS* A, int64_t lda, int64_t n, int ob, TS* Rt, hipStream_t s)
{
    const int64_t nbo = (n + ob - 1) / ob, q = ob / 256;
    if (nbo < 2 && q < 2) return hipSuccess;
    const int64_t rows = std::max<int64_t>((nbo - 1) * ob, ob);    // the most rows any part copies
    hipLaunchKernelGGL(rt_kernel<TS>, dim3((unsigned)((rows + 15) / 16), (unsigned)nbo, (unsigned)(2 * q - 1)),
                       dim3(256), 0, s, A, lda, n, ob, Rt);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_copy_block(const TS* src, int64_t lds, TS* dst, int64_t ldd, int rows, int cols, hipStream_t s,
                             const int32_t* desc)
{
    unsigned gx = (unsigned)((rows + 255) / 256);
    const unsigned gy = (unsigned)(cols < 65535 ? (cols > 0 ? cols : 1) : 65535);
    hipLaunchKernelGGL(copy_block_kernel<TS>, dim3(gx, gy), dim3(256), 0, s, src, lds, dst, ldd, rows, cols, desc);
    return hipGetLastError();
}

// One diagonal step of a blocked triangular solve with a stored inverse
// block, B[0:bo, q] <- Ri B[0:bo, q] (Ri: bo x bo of a 256 x 256 row-major
// array), in BF16x3 on the bfloat16 MFMA: each FP32 operand is split into
// bfloat16 halves and the product formed as hi*hi + hi*lo + lo*hi with FP32
// accumulation.  Workgroup w takes slices 16w .. 16w + 15, stages them in LDS
// (split), then writes its results in place: no other workgroup reads them.
// Wave v computes rows 64v .. 64v + 63.  FULL: bo = 256 (no guards).
template <bool FULL>
__global__ void __launch_bounds__(256) diag_x3_kernel(const float* __restrict__ Ri, float* __restrict__ B, int64_t ldb,
                                                      int bo, int nrhs)
{
    constexpr int LDK = 256 + 8;                  // 528-byte rows: conflict-free 16-byte lane reads
    __shared__ __attribute__((aligned(16))) __bf16 Bh[16 * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[16 * LDK];
    const int t = threadIdx.x;
    const int q0 = blockIdx.x * 16;
    const int lane = t & 63, wv = t >> 6;
    const int c = lane & 15, g = lane >> 4;
    // this lane's 8 consecutive K values of row 64 wv + 16 i + c at K offset kk
    auto load_a = [&](int kk, float (&a)[4][8]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = 64 * wv + 16 * i + c;
            const int k = kk + 8 * g;
            if (FULL || (p < bo && k + 8 <= bo)) {
                const f4_t u = *(const f4_t*)(Ri + (int64_t)p * 256 + k);
                const f4_t w = *(const f4_t*)(Ri + (int64_t)p * 256 + k + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    a[i][e] = u[e];
                    a[i][4 + e] = w[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) a[i][e] = (p < bo && k + e < bo) ? Ri[(int64_t)p * 256 + k + e] : 0.f;
            }
        }
    };
    float an[4][8];
    load_a(0, an);
    float bv[16];
#pragma unroll
    for (int qs = 0; qs < 16; ++qs) {
        const int q = q0 + qs;
        bv[qs] = (q < nrhs && (FULL || t < bo)) ? B[(int64_t)q * ldb + t] : 0.f;
    }
#pragma unroll
    for (int qs = 0; qs < 16; ++qs) {
        const __bf16 h = (__bf16)bv[qs];
        Bh[qs * LDK + t] = h;
        Bl[qs * LDK + t] = (__bf16)(bv[qs] - (float)h);
    }
    __syncthreads();
    f4_t acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < bo; kk += 32) {
        float a[4][8];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 8; ++e) a[i][e] = an[i][e];
        if (kk + 32 < bo) load_a(kk + 32, an);     // next K step's operands in flight
        const bf8_t bh = *(const bf8_t*)&Bh[c * LDK + kk + 8 * g];
        const bf8_t bl = *(const bf8_t*)&Bl[c * LDK + kk + 8 * g];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf8_t ah, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                ah[e] = (__bf16)a[i][e];
                al[e] = (__bf16)(a[i][e] - (float)ah[e]);
            }
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i], 0, 0, 0);
        }
    }
    const int q = q0 + c;
    if (q >= nrhs) return;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 64 * wv + 16 * i + 4 * g + r;
            if (p < bo) B[(int64_t)q * ldb + p] = acc[i][r];
        }
}

hipError_t launch_diag_x3(const float* Ri, float* B, int64_t ldb, int bo, int nrhs, hipStream_t s)
{
    if (nrhs <= 0 || bo <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrhs + 15) / 16));
    if (bo == 256) hipLaunchKernelGGL(diag_x3_kernel<true>, grid, dim3(256), 0, s, Ri, B, ldb, bo, nrhs);
    else hipLaunchKernelGGL(diag_x3_kernel<false>, grid, dim3(256), 0, s, Ri, B, ldb, bo, nrhs);
    return hipGetLastError();
}

// The same diagonal step in FP32 on the FP32 MFMA (16 x 16 x 4), for FP32
// factors and graph-captured solves: B[0:bo, q] <- Ri B[0:bo, q] in place,
// one launch instead of a copy and a split product.  Workgroup w (512
// threads) takes slices 16w .. 16w + 15 (of the batch record's columns when
// desc is given: offset desc[0], count desc[1], at most nrhs) and stages them
// in LDS; wave v forms rows 32v .. 32v + 31 as two 16 x 16 tiles.  Lane (c, g)
// supplies row c's K values 16s + 4g .. 16s + 4g + 3 of each 16-wide slab s as
// one 16-byte load (the A operands of four MFMAs), all of them issued before
// the first product (the inverse block is read cold, once per step), and reads
// column c's matching four values from LDS.
template <bool FULL>
__global__ void __launch_bounds__(512) diag_f32_kernel(const float* __restrict__ Ri, float* __restrict__ B, int64_t ldb,
                                                       int bo, int nrhs, const int32_t* desc)
{
    constexpr int LDK = 256 + 4;
    __shared__ __attribute__((aligned(16))) float Bs[16 * LDK];
    int cnt = nrhs;
    if (desc) {
        B += (int64_t)desc[0] * ldb;
        if (desc[1] < cnt) cnt = desc[1];
    }
    const int q0 = blockIdx.x * 16;
    if (q0 >= cnt) return;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int c = lane & 15, g = lane >> 4;
    f4_t a[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int p = 32 * wv + 16 * i + c;
#pragma unroll
        for (int sl = 0; sl < 16; ++sl) {
            const int k = 16 * sl + 4 * g;
            if (FULL || (p < bo && k + 4 <= bo)) {
                a[i][sl] = *(const f4_t*)(Ri + (int64_t)p * 256 + k);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) a[i][sl][e] = (p < bo && k + e < bo) ? Ri[(int64_t)p * 256 + k + e] : 0.f;
            }
        }
    }
    {
        const int row = t & 255, qh = (t >> 8) * 8;
#pragma unroll
        for (int qs = 0; qs < 8; ++qs) {
            const int q = q0 + qh + qs;
            Bs[(qh + qs) * LDK + row] = (q < cnt && (FULL || row < bo)) ? B[(int64_t)q * ldb + row] : 0.f;
        }
    }
    __syncthreads();
    f4_t acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sl = 0; sl < 16; ++sl) {
        const f4_t bq = *(const f4_t*)&Bs[c * LDK + 16 * sl + 4 * g];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][sl][e], bq[e], acc[i], 0, 0, 0);
    }
    const int q = q0 + c;
    if (q >= cnt) return;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 32 * wv + 16 * i + 4 * g + r;
            if (p < bo) B[(int64_t)q * ldb + p] = acc[i][r];
        }
}

hipError_t launch_diag_f32(const float* Ri, float* B, int64_t ldb, int bo, int nrhs, const int32_t* desc,
                           hipStream_t s)
{
    if (nrhs <= 0 || bo <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrhs + 15) / 16));
    if (bo == 256) hipLaunchKernelGGL(diag_f32_kernel<true>, grid, dim3(512), 0, s, Ri, B, ldb, bo, nrhs, desc);
    else hipLaunchKernelGGL(diag_f32_kernel<false>, grid, dim3(512), 0, s, Ri, B, ldb, bo, nrhs, desc);
    return hipGetLastError();
}

hipError_t rinv_set_max_lds(size_t bytes)
{
    return hipFuncSetAttribute((const void*)rinv128_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template hipError_t launch_rinv<double>(const double*, int64_t, int64_t, double*, double*, double*, double*,
                                        hipStream_t);
template hipError_t launch_rinv<float>(const float*, int64_t, int64_t, float*, float*, double*, double*, hipStream_t);
template hipError_t launch_rt<double>(const double*, int64_t, int64_t, int, double*, hipStream_t);
template hipError_t launch_rt<float>(const float*, int64_t, int64_t, int, float*, hipStream_t);
template hipError_t launch_copy_block<double>(const double*, int64_t, double*, int64_t, int, int, hipStream_t,
                                              const int32_t*);
template hipError_t launch_copy_block<float>(const float*, int64_t, float*, int64_t, int, int, hipStream_t,
                                             const int32_t*);

// First node of a graph-captured solve: check the caller's descriptor
// [cur, nbatch, off_0, cnt_0, off_1, cnt_1, ...] at the current batch and
// write the batch record rec = (offset, count) that the solve kernels read.
// An entry outside 0 <= off, 0 <= cnt <= max_cols, off + cnt <= b_cols, or a
// launch past the last batch, gives count 0 (the launch solves nothing) and
// sets bit 2 of the error word.
__global__ void begin_batch_kernel(const int32_t* desc, int32_t* rec, int max_cols, int64_t b_cols, int32_t* err)
{
    const int cur = desc[0], nb = desc[1];
    int off = 0, cnt = 0;
    bool ok = cur >= 0 && cur < nb;
    if (ok) {
        off = desc[2 + 2 * cur];
        cnt = desc[3 + 2 * cur];
        ok = off >= 0 && cnt >= 0 && cnt <= max_cols && (int64_t)off + cnt <= b_cols;
    }
    rec[0] = ok ? off : 0;
    rec[1] = ok ? cnt : 0;
    if (!ok) __hip_atomic_fetch_or(err, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last node: advance the batch cursor, never past the batch count.
__global__ void end_batch_kernel(int32_t* desc)
{
    if (desc[0] >= 0 && desc[0] < desc[1]) desc[0] += 1;
}

hipError_t launch_begin_batch(const int32_t* desc, int32_t* rec, int max_cols, int64_t b_cols, int32_t* err,
                              hipStream_t s)
{
    hipLaunchKernelGGL(begin_batch_kernel, dim3(1), dim3(1), 0, s, desc, rec, max_cols, b_cols, err);
    return hipGetLastError();
}

hipError_t launch_end_batch(int32_t* desc, hipStream_t s)
{
    hipLaunchKernelGGL(end_batch_kernel, dim3(1), dim3(1), 0, s, desc);
    return hipGetLastError();
}

hipError_t trsm_set_max_lds(size_t bytes)
{
    hipError_t e;
    e = hipFuncSetAttribute((const void*)trsm_diag_kernel<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)trsm_diag_kernel<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)trsm_diag_kernel<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)trsm_diag_kernel<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_residual(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int nrhs, hipStream_t s)
{
    dim3 grid((unsigned)((m + 255) / 256), (unsigned)((nrhs + 7) / 8));
    hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, s, row_ptr, col, val, m, X, ldx, B, ldb, R, ldr, nrhs);
    return hipGetLastError();
}

hipError_t launch_residual_t(const int64_t* col_ptr, const int32_t* row, const double* cval, int64_t n,
                             const double* R, int64_t ldr, double* S, int64_t lds, int nrhs, hipStream_t s)
{
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((nrhs + 7) / 8));
    hipLaunchKernelGGL(residual_t_kernel, grid, dim3(256), 0, s, col_ptr, row, cval, n, R, ldr, S, lds, nrhs);
    return hipGetLastError();
}

hipError_t launch_spmv_rows_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows,
                              const double* Xt, const double* Bt, double* Rt, int64_t ld, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(spmv_rows_t_kernel, dim3((unsigned)rows), dim3(64), 0, s, ptr, idx, val, rows, Xt, Bt, Rt, ld,
                       nrhs);
    return hipGetLastError();
}

hipError_t launch_spmv_cols_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t cols,
                              const double* Rt, double* St, int64_t ld, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(spmv_cols_t_kernel, dim3((unsigned)cols), dim3(64), 0, s, ptr, idx, val, cols, Rt, St, ld, nrhs);
    return hipGetLastError();
}

hipError_t launch_colnorm_t(const double* Zt, int64_t ld, int64_t rows, int nrhs, double* out, double* part,
                            hipStream_t s)
{
    hipLaunchKernelGGL(colnorm_t_kernel, dim3((unsigned)((nrhs + 63) / 64), kNormChunks), dim3(256), 0, s, Zt, ld, rows,
                       nrhs, part);
    hipLaunchKernelGGL(colnorm_sum_kernel, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, s, part, nrhs, out);
    return hipGetLastError();
}

template <typename TI, typename TO, bool TO_T, bool ACC>
hipError_t launch_transpose(const TI* in, TO* out, int64_t rows, int cols, int64_t ldc, int64_t ldt, hipStream_t s)
{
    dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
    hipLaunchKernelGGL((transpose_kernel<TI, TO, TO_T, ACC>), grid, dim3(256), 0, s, in, out, rows, cols, ldc, ldt);
    return hipGetLastError();
}
template hipError_t launch_transpose<double, double, true, false>(const double*, double*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<float, double, true, false>(const float*, double*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<float, double, true, true>(const float*, double*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<double, double, true, true>(const double*, double*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<double, float, false, false>(const double*, float*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<double, double, false, false>(const double*, double*, int64_t, int, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<float, float, true, false>(const float*, float*, int64_t, int, int64_t, int64_t, hipStream_t);

template <typename TI, typename TO>
hipError_t launch_convert(const TI* X, int64_t ldx, TO* Y, int64_t ldy, int64_t rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL((convert_kernel<TI, TO>), grid2(rows, cols), dim3(256), 0, s, X, ldx, Y, ldy, rows, cols);
    return hipGetLastError();
}

template <typename TD>
hipError_t launch_corr_ratio(const TD* D, int64_t ldd, const double* X, int64_t ldx, int64_t rows, int cols,
                             double* ratio, unsigned long long* maxw, hipStream_t s)
{
    hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, maxw);
    hipLaunchKernelGGL((corr_ratio_kernel<TD>), dim3(cols), dim3(256), 0, s, D, ldd, X, ldx, rows, ratio, maxw);
    return hipGetLastError();
}
template hipError_t launch_corr_ratio<float>(const float*, int64_t, const double*, int64_t, int64_t, int, double*,
                                             unsigned long long*, hipStream_t);
template hipError_t launch_corr_ratio<double>(const double*, int64_t, const double*, int64_t, int64_t, int, double*,
                                              unsigned long long*, hipStream_t);

template <typename TD>
hipError_t launch_accumulate(double* X, int64_t ldx, const TD* D, int64_t ldd, int64_t rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL((accumulate_kernel<TD>), grid2(rows, cols), dim3(256), 0, s, X, ldx, D, ldd, rows, cols);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero_rows(T* Y, int64_t ldy, int64_t r0, int64_t r1, int cols, hipStream_t s)
{
    if (r1 <= r0) return hipSuccess;
    hipLaunchKernelGGL((zero_rows_kernel<T>), grid2(r1 - r0, cols), dim3(256), 0, s, Y, ldy, r0, r1, cols);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colsq(const T* C, int64_t ldc, int64_t rows, int cols, double* out, hipStream_t s)
{
    hipLaunchKernelGGL((colsq_kernel<T>), dim3(cols), dim3(256), 0, s, C, ldc, rows, out);
    return hipGetLastError();
}
template hipError_t launch_colsq<float>(const float*, int64_t, int64_t, int, double*, hipStream_t);
template hipError_t launch_colsq<double>(const double*, int64_t, int64_t, int, double*, hipStream_t);

hipError_t launch_cg_update(const double* x, double* y, int64_t rows, int nrhs, int64_t ld, const double* num,
                            const double* den, int mode, hipStream_t s)
{
    int64_t g = (rows * ld + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(cg_update_kernel, dim3((unsigned)(g > 0 ? g : 1)), dim3(256), 0, s, x, y, rows, nrhs, ld, num,
                       den, mode);
    return hipGetLastError();
}

hipError_t launch_cg_ratio(const double* gam, const double* qn, const double* pn, const double* xn, int nrhs,
                           unsigned long long* maxw, hipStream_t s)
{
    hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, maxw);
    hipLaunchKernelGGL(cg_ratio_kernel, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, s, gam, qn, pn, xn, nrhs,
                       maxw);
    return hipGetLastError();
}

hipError_t launch_colnorm(const double* X, int64_t ldx, int64_t rows, int cols, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(colnorm_kernel, dim3(cols), dim3(256), 0, s, X, ldx, rows, out);
    return hipGetLastError();
}

template hipError_t launch_trsm_diag<double, true>(const double*, int64_t, int, double*, int64_t, int, hipStream_t,
                                                   const int32_t*);
template hipError_t launch_trsm_diag<double, false>(const double*, int64_t, int, double*, int64_t, int, hipStream_t,
                                                    const int32_t*);
template hipError_t launch_trsm_diag<float, true>(const float*, int64_t, int, float*, int64_t, int, hipStream_t,
                                                  const int32_t*);
template hipError_t launch_trsm_diag<float, false>(const float*, int64_t, int, float*, int64_t, int, hipStream_t,
                                                   const int32_t*);
template hipError_t launch_convert<double, float>(const double*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<float, float>(const float*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_accumulate<float>(double*, int64_t, const float*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_accumulate<double>(double*, int64_t, const double*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_zero_rows<float>(float*, int64_t, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_zero_rows<double>(double*, int64_t, int64_t, int64_t, int, hipStream_t);

}  // namespace ctqr
