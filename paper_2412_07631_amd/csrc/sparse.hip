// Grouped copies of the FP64 sparse matrix for the refinement's products
// with many slices (r = b - A x with the rays as rows, A^T r with the pixels
// as rows).  Consecutive rows are taken `group` at a time -- adjacent rays of
// one view cross nearly the same pixels, adjacent pixels of an image row are
// crossed by nearly the same rays -- and each group keeps the sorted union of
// its rows' column indices once, with a dense group-wide block of weights
// (zero where a row does not touch that column).  A product then reads each
// slice-contiguous row of the dense operand once per group instead of once
// per stored entry.
#include "ct_internal.h"

#include <stdint.h>

namespace ctqr {

hipError_t launch_csr_scan(int64_t* ptr, int64_t m, hipStream_t s);

constexpr int kGroupCap = 8192;    // stored entries of one group held in LDS while it is built

// bitonic sort of n (a power of two) 64-bit keys, with optional payloads, in
// LDS by the whole workgroup
__device__ void lds_bitonic(uint64_t* key, double* val, int n)
{
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = key[i], b = key[l];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[l] = a;
                        if (val) {
                            const double t = val[i];
                            val[i] = val[l];
                            val[l] = t;
                        }
                    }
                }
            }
            __syncthreads();
        }
}

__device__ __forceinline__ int pow2_at_least(int e)
{
    int n = 1;
    while (n < e) n <<= 1;
    return n;
}

// Pass 1: the number of distinct columns of each group into cnt[g + 1].
__global__ void __launch_bounds__(256) group_count_kernel(const int64_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ idx, int64_t rows, int group,
                                                          int64_t* __restrict__ cnt, int32_t* __restrict__ err)
{
    extern __shared__ __attribute__((aligned(16))) char glds[];
    uint64_t* key = (uint64_t*)glds;
    __shared__ int red[256];
    const int64_t g = blockIdx.x, r0 = g * group;
    const int64_t r1 = r0 + group < rows ? r0 + group : rows;
    const int64_t p0 = ptr[r0];
    const int e = (int)(ptr[r1] - p0);
    if (e > kGroupCap) {
        if (threadIdx.x == 0) {
            cnt[g + 1] = 0;
            atomicOr(err, 1);
        }
        return;
    }
    const int n2 = pow2_at_least(e > 0 ? e : 1);
    for (int i = threadIdx.x; i < n2; i += 256) key[i] = i < e ? (uint64_t)(uint32_t)idx[p0 + i] : ~0ull;
    __syncthreads();
    lds_bitonic(key, nullptr, n2);
    int u = 0;
    for (int i = threadIdx.x; i < e; i += 256) u += (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
    red[threadIdx.x] = u;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[g + 1] = red[0];
}

// Pass 2: each group's sorted distinct columns into gidx[gptr[g] ..] and its
// entries into the dense weights gval[(gptr[g] + position) * group + row].
__global__ void __launch_bounds__(256) group_fill_kernel(const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const double* __restrict__ val, int64_t rows, int group,
                                                         const int64_t* __restrict__ gptr, int32_t* __restrict__ gidx,
                                                         double* __restrict__ gval)
{
    extern __shared__ __attribute__((aligned(16))) char glds[];
    uint64_t* key = (uint64_t*)glds;
    double* pv = (double*)(glds + (size_t)kGroupCap * 8);
    __shared__ int part[257];
    const int64_t g = blockIdx.x, r0 = g * group;
    const int64_t r1 = r0 + group < rows ? r0 + group : rows;
    const int64_t p0 = ptr[r0];
    const int e = (int)(ptr[r1] - p0);
    if (e > kGroupCap || e == 0) return;
    const int n2 = pow2_at_least(e);
    const int shift = 32 - __builtin_clz((unsigned)group);        // bits for the row within the group
    for (int i = threadIdx.x; i < n2; i += 256) {
        if (i < e) {
            const int64_t p = p0 + i;
            int r = 0;
            while (r0 + r + 1 < r1 && ptr[r0 + r + 1] <= p) ++r;
            key[i] = ((uint64_t)(uint32_t)idx[p] << shift) | (uint64_t)r;
            pv[i] = val[p];
        } else {
            key[i] = ~0ull;
            pv[i] = 0.0;
        }
    }
    __syncthreads();
    lds_bitonic(key, pv, n2);
    // distinct-column positions: each thread counts the column starts in its
    // contiguous chunk, the chunk counts are scanned, then positions assigned
    const int chunk = (e + 255) / 256;
    const int b0 = threadIdx.x * chunk, b1 = b0 + chunk < e ? b0 + chunk : e;
    int c = 0;
    for (int i = b0; i < b1; ++i) c += (i == 0 || (key[i] >> shift) != (key[i - 1] >> shift)) ? 1 : 0;
    part[threadIdx.x + 1] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[0] = 0;
        for (int t = 1; t <= 256; ++t) part[t] += part[t - 1];
    }
    __syncthreads();
    int pos = part[threadIdx.x] - 1;
    const int64_t base = gptr[g];
    for (int i = b0; i < b1; ++i) {
        const uint64_t k = key[i];
        if (i == 0 || (k >> shift) != (key[i - 1] >> shift)) {
            ++pos;
            gidx[base + pos] = (int32_t)(k >> shift);
        }
        // a repeated (column, row) pair, if any, is summed by the first of its run
        if (i > 0 && k == key[i - 1]) continue;
        double v = pv[i];
        for (int j = i + 1; j < e && key[j] == k; ++j) v += pv[j];
        gval[(base + pos) * group + (int64_t)(k & ((1u << shift) - 1))] = v;
    }
}

__global__ void __launch_bounds__(256) fill_f64_kernel(double* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0;
}

hipError_t group_set_lds()
{
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)group_fill_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kGroupCap * 16);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)group_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kGroupCap * 8);
    if (e == hipSuccess) done = true;
    return e;
}

__global__ void zero_i32_kernel(int32_t* w) { *w = 0; }

hipError_t launch_group_count(const int64_t* ptr, const int32_t* idx, int64_t rows, int group, int64_t* gptr,
                              int32_t* err, hipStream_t s)
{
    hipError_t e = group_set_lds();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, err);
    const int64_t ng = (rows + group - 1) / group;
    hipLaunchKernelGGL(group_count_kernel, dim3((unsigned)ng), dim3(256), kGroupCap * 8, s, ptr, idx, rows, group,
                       gptr, err);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_csr_scan(gptr, ng, s);
}

hipError_t launch_group_fill(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, int group,
                             const int64_t* gptr, int32_t* gidx, double* gval, int64_t count, hipStream_t s)
{
    hipError_t e = group_set_lds();
    if (e != hipSuccess) return e;
    const int64_t ng = (rows + group - 1) / group;
    const int64_t nv = count * group;
    int64_t fb = (nv + 255) / 256;
    if (fb > 8192) fb = 8192;
    if (fb < 1) fb = 1;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)fb), dim3(256), 0, s, gval, nv);
    hipLaunchKernelGGL(group_fill_kernel, dim3((unsigned)ng), dim3(256), kGroupCap * 16, s, ptr, idx, val, rows, group,
                       gptr, gidx, gval);
    return hipGetLastError();
}

// ----------------------------------------------------------- the products
// out[(r0 + r) * ld + j] = (sub ? (B ? B[..] : 0) - acc : acc) for the rows of
// group g, acc = sum over the group's columns c of w[c][r] Z[c * ld + j];
// slice-contiguous operands (element (i, j) at i * ld + j), one workgroup per
// group, 256 slices per pass of its threads.
template <int G>
__global__ void __launch_bounds__(256) group_spmm_kernel(const int64_t* __restrict__ gptr,
                                                         const int32_t* __restrict__ gidx,
                                                         const double* __restrict__ gval, int64_t rows,
                                                         const double* __restrict__ Z, const double* __restrict__ B,
                                                         double* __restrict__ out, int64_t ld, int nrhs, int sub)
{
    const int64_t ng = (rows + G - 1) / G;
    int64_t g = blockIdx.x;
    if (ng % 8 == 0) g = (g % 8) * (ng / 8) + g / 8;      // consecutive groups on one XCD
    const int64_t r0 = g * G;
    const int64_t u0 = gptr[g], u1 = gptr[g + 1];
    for (int j0 = 0; j0 < nrhs; j0 += 512) {
        const int ja = j0 + threadIdx.x, jb = ja + 256;
        const bool va = ja < nrhs, vb = jb < nrhs;
        double acc[2][G];
#pragma unroll
        for (int r = 0; r < G; ++r) acc[0][r] = acc[1][r] = 0.0;
#pragma unroll 4
        for (int64_t u = u0; u < u1; ++u) {
            const double* zr = Z + (int64_t)gidx[u] * ld;
            const double za = va ? zr[ja] : 0.0, zb = vb ? zr[jb] : 0.0;
            const double* w = gval + u * G;
#pragma unroll
            for (int r = 0; r < G; ++r) {
                acc[0][r] += w[r] * za;
                acc[1][r] += w[r] * zb;
            }
        }
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const int64_t i = r0 + r;
            if (i >= rows) break;
            if (va) out[i * ld + ja] = sub ? (B ? B[i * ld + ja] : 0.0) - acc[0][r] : acc[0][r];
            if (vb) out[i * ld + jb] = sub ? (B ? B[i * ld + jb] : 0.0) - acc[1][r] : acc[1][r];
        }
    }
}

hipError_t launch_group_spmm(const int64_t* gptr, const int32_t* gidx, const double* gval, int group, int64_t rows,
                             const double* Z, const double* B, double* out, int64_t ld, int nrhs, bool sub,
                             hipStream_t s)
{
    const int64_t ng = (rows + group - 1) / group;
    const dim3 grid((unsigned)ng), block(256);
    switch (group) {
        case 8: hipLaunchKernelGGL(group_spmm_kernel<8>, grid, block, 0, s, gptr, gidx, gval, rows, Z, B, out, ld, nrhs, sub ? 1 : 0); break;
        case 4: hipLaunchKernelGGL(group_spmm_kernel<4>, grid, block, 0, s, gptr, gidx, gval, rows, Z, B, out, ld, nrhs, sub ? 1 : 0); break;
        case 2: hipLaunchKernelGGL(group_spmm_kernel<2>, grid, block, 0, s, gptr, gidx, gval, rows, Z, B, out, ld, nrhs, sub ? 1 : 0); break;
        case 1: hipLaunchKernelGGL(group_spmm_kernel<1>, grid, block, 0, s, gptr, gidx, gval, rows, Z, B, out, ld, nrhs, sub ? 1 : 0); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ctqr
