// Persistent fused solve: X = R^{-1} Q^T B (Eq. (solve)) for a batch of
// right-hand sides in one launch of one workgroup per CU (cooperative, so the
// launch is refused rather than under-scheduled).
//
// The batch is taken in chunks of KC columns.  Per chunk:
//   Q^T B, outer block by outer block (Q = I - V T V^T per block, compact WY):
//     A   W partials: each workgroup sums V[rows, cols]^T B[rows] over its
//         rows (V from the row-major reflector copy, B staged in LDS)
//     B1  W = sum of the partials (fixed order, FP64)
//     B2  W' = T^T W (T upper triangular, FP64)
//     C   B[rows] -= V[rows, :] W', the rows split over the workgroups
//     with a grid-wide barrier after each phase;
//   R^{-1}: back-substitution over 256-row blocks whose x blocks are
//     published to the other workgroups through flags as the chain of
//     dependent blocks reaches them.
// Two forms.  Chunks of at most 8 columns of an FP32-storage factor (the
// latency path): one contiguous row range per workgroup in phases A and C,
// phase C as MFMA products, and a back-substitution on Rh =
// blockdiag(R_qq^{-1}) R with each block split over four workgroups
// (narrow_*).  Wider chunks and FP64 factors: row groups x 128-column groups
// in phase A, FMA products, and a back-substitution that multiplies each
// block by its stored inverse on the chain, one workgroup per block
// (fused_phase_*, fused_update, fused_solve_block).  The cross-workgroup
// waits are bounded in time like the factorization's (bit 3 of the error
// word on a time-out).
#include "ct_internal.h"

namespace ctqr {

constexpr int kFusedMaxOwn = 2;     // 256-row blocks per workgroup in the back-substitution
constexpr int kFusedErr = 8;

__host__ __device__ inline size_t fused_up256(size_t x) { return (x + 255) / 256 * 256; }

// Scratch layout (bytes): barrier words, per-block flags, W (KC x nbo FP64),
// W' (nbo x KC), the published x blocks (nbq 256 x KC), the W partials
// (nrg x KC x nbo).
struct FusedLayout {
    size_t flags, W, Wt, Xp, P, total;
};
__host__ __device__ inline FusedLayout fused_layout(int nbo, int64_t nbq, int nrg, int KC, size_t es)
{
    FusedLayout L;
    L.flags = 256;
    L.W = L.flags + fused_up256((size_t)nbq * 16);   // four flags a block (one a quarter)
    L.Wt = L.W + fused_up256((size_t)KC * nbo * 8);
    L.Xp = L.Wt + fused_up256((size_t)nbo * KC * es);
    L.P = L.Xp + fused_up256((size_t)nbq * 256 * KC * es);
    L.total = L.P + (size_t)nrg * KC * nbo * es;
    return L;
}

__device__ inline size_t fused_vt_off(const FusedArgs& a, int64_t b)
{
    return (size_t)(b * a.m - (int64_t)a.nbo * (b * (b - 1) / 2)) * (size_t)((a.nbo + 15) / 16 * 16);
}

__device__ inline void fused_err(int32_t* err)
{
    __hip_atomic_fetch_or(err, kFusedErr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded spin of thread 0 until *p != v (want_ne) or *p == v.
__device__ inline bool fused_wait(uint32_t* p, uint32_t v, bool want_ne, int32_t* err, uint64_t ticks)
{
    uint64_t t0 = 0;
    uint32_t spins = 0;
    for (;;) {
        const uint32_t x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (want_ne ? x != v : x == v) return true;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spins == 16) {
                t0 = now;
            } else if (now - t0 >= ticks) {
                fused_err(err);
                return false;
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kFusedErr | 1)) return false;
        }
    }
}

// Bounded spin of thread 0 until the four words p[0..3] all equal v: the four
// loads of a round are issued together (one memory round trip a poll, not
// four).
__device__ inline bool fused_wait4(uint32_t* p, uint32_t v, int32_t* err, uint64_t ticks)
{
    uint64_t t0 = 0;
    uint32_t spins = 0;
    for (;;) {
        const uint32_t x0 = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t x1 = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t x2 = __hip_atomic_load(p + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t x3 = __hip_atomic_load(p + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (x0 == v && x1 == v && x2 == v && x3 == v) return true;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spins == 16) {
                t0 = now;
            } else if (now - t0 >= ticks) {
                fused_err(err);
                return false;
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kFusedErr | 1)) return false;
        }
    }
}

// Grid-wide barrier: the last workgroup to arrive resets the count and
// advances the generation; the others wait for the generation to change.
// Self-resetting, so one reset before the launch is all it needs.  Only
// thread 0 fences at agent scope: the workgroup barrier before it waits for
// every wavefront's stores to reach L2 (and orders them before thread 0's
// release, which writes L2 back), and its acquire (an L2 and L1 invalidate)
// comes before the barrier after it.  One writeback and one invalidate per
// workgroup instead of one per wavefront: 6 us a barrier instead of 20 on
// 256 workgroups.
__device__ inline bool fused_sync(uint32_t* bar, uint32_t& gen, int G, int32_t* err, uint64_t ticks, int* flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* count = bar;
        uint32_t* gw = bar + 32;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool ok = true;
        if (old == (uint32_t)G - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(gw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = fused_wait(gw, gen, true, err, ticks);
        }
        gen += 1;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = ok ? 1 : 0;
    }
    __syncthreads();
    return *flag != 0;
}

// Barrier for LDS hand-over only: waits for this wave's LDS operations, not
// for its global loads (a workgroup fence would also wait for the next tile's
// loads, issued into registers before the barrier to overlap the multiply).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);    // lgkmcnt(0); vmcnt and expcnt at their maximum
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <typename TS> struct Vec4;
template <> struct Vec4<float> { typedef float4 t; };
template <> struct Vec4<double> { typedef double4 t; };

template <typename TS>
__device__ inline typename Vec4<TS>::t ld4(const TS* p) { return *(const typename Vec4<TS>::t*)p; }

// ---------------------------------------------------------------- Q^T phases
// A: W partials of block b over row group rg, column group cg.  Rows go in
// sub-chunks of RS: the next sub-chunk's V row segments and B values are
// loaded into registers while the current one is multiplied.
template <typename TS, int KC>
__device__ __forceinline__ void fused_phase_a(const FusedArgs& a, char* lds, const TS* Bc, int kc, int64_t b, int bo, int64_t mk,
                              int nrg, int ncg, TS* P)
{
    typedef typename Vec4<TS>::t V4;
    const int g = blockIdx.x, t = threadIdx.x;
    if (g >= ncg * nrg) return;
    const int cg = g % ncg, rg = g / ncg;
    const int cq = t & 31, rl = t >> 5;
    const int64_t k0 = b * a.nbo;
    const int64_t rch = (mk + nrg - 1) / nrg;
    const int64_t rb = rg * rch, re = rb + rch < mk ? rb + rch : mk;
    const int ldv = (bo + 15) / 16 * 16;
    const TS* Vb = (const TS*)a.Vt + fused_vt_off(a, b);
    const int c = cg * 128 + 4 * cq;
    const bool cvalid = c < ldv;
    constexpr int BL = KC + 64 / (int)sizeof(TS);   // rows of 192 or 256 bytes: aligned vector reads
    constexpr int RS = 32;                           // rows per sub-chunk (RS / 8 per thread)
    constexpr int NU = RS / 8;
    constexpr int NB = RS * KC / 256;                // B values staged per thread and sub-chunk
    TS* Bs = (TS*)lds;                               // RS x BL
    TS acc[KC][4];
#pragma unroll
    for (int j = 0; j < KC; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] = (TS)0;
    V4 vn[NU];
    TS bn[NB];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int64_t r = r0 + rl + 8 * u;
            vn[u] = (r < re && cvalid) ? ld4<TS>(Vb + r * ldv + c) : V4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = t + 256 * u, rr = e % RS, j = e / RS;
            const int64_t r = r0 + rr;
            bn[u] = (r < re && j < kc) ? Bc[k0 + r + (int64_t)j * a.ldb] : (TS)0;
        }
    };
    if (rb < re) fetch(rb);
    for (int64_t r0 = rb; r0 < re; r0 += RS) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = t + 256 * u;
            Bs[(e % RS) * BL + e / RS] = bn[u];
        }
        V4 v[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) v[u] = vn[u];
        lds_barrier();
        if (r0 + RS < re) fetch(r0 + RS);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const TS* br = Bs + (rl + 8 * u) * BL;
#pragma unroll
            for (int j = 0; j < KC; j += 4) {
                const V4 bb = ld4<TS>(br + j);
                const TS bj[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    acc[j + w][0] += v[u].x * bj[w];
                    acc[j + w][1] += v[u].y * bj[w];
                    acc[j + w][2] += v[u].z * bj[w];
                    acc[j + w][3] += v[u].w * bj[w];
                }
            }
        }
        lds_barrier();
    }
    __syncthreads();
    // sum the 8 row lanes in LDS: red[rl][j][128]
    TS* red = (TS*)lds;
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        V4 w = {acc[j][0], acc[j][1], acc[j][2], acc[j][3]};
        *(V4*)(red + ((size_t)(rl * KC + j) * 128 + 4 * cq)) = w;
    }
    __syncthreads();
    for (int e = t; e < KC * 128; e += 256) {
        const int j = e >> 7, cc = e & 127;
        TS s = (TS)0;
#pragma unroll
        for (int l = 0; l < 8; ++l) s += red[(size_t)(l * KC + j) * 128 + cc];
        const int col = cg * 128 + cc;
        if (col < bo) P[((size_t)rg * KC + j) * a.nbo + col] = s;
    }
    __syncthreads();
}

// B1: W[c][j] = sum over row groups (fixed order), FP64
template <typename TS, int KC>
__device__ __forceinline__ void fused_phase_b1(const FusedArgs& a, int bo, int nrg, const TS* P, double* W)
{
    const int64_t total = (int64_t)KC * bo;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int j = (int)(e / bo), c = (int)(e % bo);
        double s = 0.0;
        for (int rg = 0; rg < nrg; ++rg) s += (double)P[((size_t)rg * KC + j) * a.nbo + c];
        W[(size_t)c * KC + j] = s;
    }
}

// B2: W'[c][j] = sum_{l <= c} T[l, c] W[l][j]; workgroup g takes columns
// c = g, g + G, ...; its threads split the sum over l in 256 / KC slices
// (coalesced rows of W), reduced in LDS in a fixed order.
template <typename TS, int KC>
__device__ __forceinline__ void fused_phase_b2(const FusedArgs& a, char* lds, int64_t b, int bo, const double* W, TS* Wt)
{
    constexpr int NS = 256 / KC;
    const int t = threadIdx.x, j = t % KC, sl = t / KC;
    const double* Tb = a.T + (size_t)b * a.nbo * a.nbo;
    double* red = (double*)lds;                      // NS x KC
    for (int c = blockIdx.x; c < bo; c += gridDim.x) {
        const double* tc = Tb + (size_t)c * a.nbo;
        const int len = (c + 1 + NS - 1) / NS;
        const int l0 = sl * len, l1 = l0 + len < c + 1 ? l0 + len : c + 1;
        double s = 0.0;
#pragma unroll 8
        for (int l = l0; l < l1; ++l) s += tc[l] * W[(size_t)l * KC + j];
        red[sl * KC + j] = s;
        __syncthreads();
        if (t < KC) {
            double r = 0.0;
            for (int q = 0; q < NS; ++q) r += red[q * KC + t];
            Wt[(size_t)c * KC + t] = (TS)r;
        }
        __syncthreads();
    }
}

// C: B[k0 + r] -= V[r, :] W' for the rows of this workgroup.  W' (bo x KC)
// goes to LDS once; thread t takes rows rb + t, rb + t + 256, ... and walks
// the row along the columns of V read in place (column-major: the 64 lanes
// of a wavefront read 64 consecutive rows of one column, one coalesced load),
// the triangle above V's unit diagonal masked; each column's W' row is one
// broadcast LDS read per 4 slices.
template <typename TS, int KC>
__device__ __forceinline__ void fused_phase_c(const FusedArgs& a, char* lds, TS* Bc, int kc, int64_t b, int bo,
                                              int64_t mk, const TS* Wt)
{
    typedef typename Vec4<TS>::t V4;
    const int g = blockIdx.x, t = threadIdx.x, G = gridDim.x;
    const int64_t k0 = b * a.nbo;
    const int64_t rpw = (mk + G - 1) / G;
    const int64_t rb = g * rpw, re = rb + rpw < mk ? rb + rpw : mk;
    if (rb >= re) return;
    TS* Ws = (TS*)lds;                 // bo x KC
    for (int e = 4 * t; e < bo * KC; e += 1024) *(V4*)(Ws + e) = ld4<TS>(Wt + e);
    __syncthreads();
    const TS* V0 = (const TS*)a.A + k0 + k0 * a.lda;     // V[r][c] = V0[r + c lda] below the diagonal
    constexpr int U = 8;
    for (int64_t r = rb + t; r - t < re; r += 256) {
        const bool live = r < re;
        const TS* vr = V0 + (live ? r : rb);
        TS acc[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) acc[j] = (TS)0;
        // columns c < min(r, bo) are stored, c == r is the unit diagonal;
        // the next group of U columns is loaded while this one is multiplied
        const int cs = r < bo ? (int)r : bo;
        const int cfull = cs / U * U;
        TS vc[U], vn[U];
        if (cfull > 0)
#pragma unroll
            for (int u = 0; u < U; ++u) vc[u] = vr[(int64_t)u * a.lda];
        int c = 0;
        for (; c < cfull; c += U) {
            const bool more = c + U < cfull;
            if (more)
#pragma unroll
                for (int u = 0; u < U; ++u) vn[u] = vr[(int64_t)(c + U + u) * a.lda];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const TS* wc = Ws + (c + u) * KC;
#pragma unroll
                for (int j = 0; j < KC; j += 4) {
                    const V4 w = ld4<TS>(wc + j);
                    acc[j] += vc[u] * w.x;
                    acc[j + 1] += vc[u] * w.y;
                    acc[j + 2] += vc[u] * w.z;
                    acc[j + 3] += vc[u] * w.w;
                }
            }
            if (more)
#pragma unroll
                for (int u = 0; u < U; ++u) vc[u] = vn[u];
        }
        for (; c < cs; ++c) {
            const TS v = vr[(int64_t)c * a.lda];
            const TS* wc = Ws + c * KC;
#pragma unroll
            for (int j = 0; j < KC; ++j) acc[j] += v * wc[j];
        }
        if (r < bo) {
            const TS* wc = Ws + r * KC;
#pragma unroll
            for (int j = 0; j < KC; ++j) acc[j] += wc[j];
        }
        if (live)
#pragma unroll
            for (int j = 0; j < KC; ++j)
                if (j < kc) {
                    TS* p = Bc + k0 + r + (int64_t)j * a.ldb;
                    *p = *p - acc[j];
                }
    }
    __syncthreads();
}

// ------------------------------------------------- Q^T phases, narrow FP32 chunks
// Chunks of at most kNarrow columns of an FP32 factor.  The rows of a block
// are split in nrw contiguous ranges, one per workgroup, and thread t owns
// columns 4t .. 4t+3 of the row-major reflector copy: one wavefront load reads
// 1 KB of a row, the workgroup reads whole rows, and every workgroup streams
// one contiguous stretch of the block.  Phase C walks its range backwards, so
// that the rows phase A read last (the likeliest still cached) come first;
// its products are MFMAs.  LDS: the range's B rows (row-major, 8 floats a
// row) at 0, the FP64 W of phase B2 and the reduction buffers at kNarrowWs.
constexpr int kNarrow = 8;
constexpr int kNarrowCh = 1024;                       // B rows staged at a time
constexpr int kNarrowGr = 8;                          // rows per group of phase A's loads (two groups in flight)
constexpr int kNarrowStage = kNarrowCh + 4 * kNarrowGr; // staged rows: phase A reads up to two groups past the chunk
constexpr size_t kNarrowWs = 34816;
static_assert(kNarrowWs >= (size_t)kNarrowStage * kNarrow * 4, "B rows overlap the FP64 W");
static_assert(kNarrowWs + (1024 + 4) * kNarrow * 8 <= 131072, "narrow phases exceed the LDS of the wide ones");

__device__ __forceinline__ void narrow_range(int64_t mk, int nrw, int g, int64_t& rb, int64_t& re)
{
    const int64_t rpw = (mk + nrw - 1) / nrw;
    rb = (int64_t)g * rpw;
    if (rb > mk) rb = mk;
    re = rb + rpw < mk ? rb + rpw : mk;
}

// Reduce-scatter over the 64 lanes of a wavefront: N values a lane (N a power
// of two, 2..64) are summed over the lanes, value i ending in lane i (64 / N)
// .. lane (i + 1)(64 / N) - 1; halving steps with lane offsets 32, 16, ...,
// then a butterfly over the offsets left, so that every such lane holds the
// whole sum.  Fixed order: the result does not depend on timing.
template <typename T, int N, int n>
__device__ __forceinline__ void wave_rs_step(T (&v)[N], int lane)
{
    if constexpr (n > 1) {
        constexpr int o = 32 * n / N, h = n / 2;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int k = 0; k < h; ++k) {
            const T send = up ? v[k] : v[k + h];
            const T keep = up ? v[k + h] : v[k];
            v[k] = keep + __shfl_xor(send, o);
        }
        wave_rs_step<T, N, h>(v, lane);
    }
}

template <typename T, int o>
__device__ __forceinline__ T wave_bfly(T x)
{
    if constexpr (o >= 1) return wave_bfly<T, o / 2>(x + __shfl_xor(x, o));
    else return x;
}

template <typename T, int N>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[N], int lane)
{
    static_assert(N >= 2 && N <= 64 && (N & (N - 1)) == 0, "N: a power of two up to 64");
    wave_rs_step<T, N, N>(v, lane);
    return wave_bfly<T, 32 / N>(v[0]);
}

// Stage B[k0 + r, j] for rows c0 .. c0 + kNarrowStage - 1 (zero past c1 and
// for j >= kc) into Bs, row-major; all loads issued before the first store.
__device__ __forceinline__ void narrow_stage_b(const FusedArgs& a, float* Bs, const float* Bc, int kc, int64_t k0,
                                               int64_t c0, int64_t c1)
{
    constexpr int NI = (kNarrowStage + 255) / 256;
    float bv[NI][kNarrow];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int64_t r = c0 + threadIdx.x + 256 * k;
#pragma unroll
        for (int j = 0; j < kNarrow; ++j) bv[k][j] = (r < c1 && j < kc) ? Bc[k0 + r + (int64_t)j * a.ldb] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < kNarrowStage) {
            *(float4*)(Bs + 8 * i) = float4{bv[k][0], bv[k][1], bv[k][2], bv[k][3]};
            *(float4*)(Bs + 8 * i + 4) = float4{bv[k][4], bv[k][5], bv[k][6], bv[k][7]};
        }
    }
}

// A: P[c / 4][g][j][c % 4] = sum over the rows r of range g of V[r, c] B[k0 + r, j]
// (thread t writes the 128 contiguous bytes of its column quad; phase B1 then
// reads one contiguous stretch per quad).
__device__ __forceinline__ void narrow_phase_a(const FusedArgs& a, char* lds, const float* Bc, int kc, int64_t b,
                                               int bo, int64_t mk, float* P)
{
    const int g = blockIdx.x, t = threadIdx.x;
    if (g >= a.nrw) return;
    int64_t rb, re;
    narrow_range(mk, a.nrw, g, rb, re);
    const int64_t k0 = b * a.nbo;
    const int ldv = (bo + 15) / 16 * 16;
    const float* Vb = (const float*)a.Vt + fused_vt_off(a, b) + 4 * t;
    const bool cv = 4 * t < ldv;
    float* Bs = (float*)lds;
    float acc[kNarrow][4];
#pragma unroll
    for (int j = 0; j < kNarrow; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] = 0.f;
    constexpr int GR = kNarrowGr;
    for (int64_t c0 = rb; c0 < re; c0 += kNarrowCh) {
        const int64_t c1 = c0 + kNarrowCh < re ? c0 + kNarrowCh : re;
        float4 va[GR], vb[GR];
        auto ld = [&](float4 (&v)[GR], int64_t r0) {
#pragma unroll
            for (int u = 0; u < GR; ++u) {
                const int64_t r = r0 + u;
                v[u] = (r < c1 && cv) ? *(const float4*)(Vb + r * ldv) : float4{0.f, 0.f, 0.f, 0.f};
            }
        };
        auto mac = [&](const float4 (&v)[GR], int64_t r0) {
            const float* br = Bs + 8 * (r0 - c0);
#pragma unroll
            for (int u = 0; u < GR; ++u) {
                const float4 b0 = *(const float4*)(br + 8 * u), b1 = *(const float4*)(br + 8 * u + 4);
                const float bj[kNarrow] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                for (int j = 0; j < kNarrow; ++j) {
                    acc[j][0] += v[u].x * bj[j];
                    acc[j][1] += v[u].y * bj[j];
                    acc[j][2] += v[u].z * bj[j];
                    acc[j][3] += v[u].w * bj[j];
                }
            }
        };
        lds_barrier();                      // the previous chunk's reads of Bs are done
        narrow_stage_b(a, Bs, Bc, kc, k0, c0, c1);
        ld(va, c0);
        ld(vb, c0 + GR);
        lds_barrier();
        for (int64_t r0 = c0; r0 < c1; r0 += 2 * GR) {
            mac(va, r0);
            ld(va, r0 + 2 * GR);
            mac(vb, r0 + GR);
            ld(vb, r0 + 3 * GR);
        }
    }
    if (4 * t < a.nbo)
#pragma unroll
        for (int j = 0; j < kNarrow; ++j)
            *(float4*)(P + (((size_t)t * a.nrw + g) * kNarrow + j) * 4) = float4{acc[j][0], acc[j][1], acc[j][2], acc[j][3]};
}

// B1: W[c][j] = sum of the nrw partials (fixed order, FP64); workgroup g
// takes the column quads g, g + G, ..., thread p loads partial p (128
// contiguous bytes: the workgroup reads its quad's partials in one stretch).
__device__ __forceinline__ void narrow_phase_b1(const FusedArgs& a, char* lds, int bo, const float* P, double* W)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double* red = (double*)(lds + kNarrowWs);          // 4 waves x 32
    const int nq = (bo + 3) / 4;
    for (int cq = blockIdx.x; cq < nq; cq += gridDim.x) {
        double v[4 * kNarrow];
#pragma unroll
        for (int e = 0; e < 4 * kNarrow; ++e) v[e] = 0.0;
        for (int p = t; p < a.nrw; p += 256) {
            float4 x[kNarrow];
#pragma unroll
            for (int j = 0; j < kNarrow; ++j) x[j] = *(const float4*)(P + (((size_t)cq * a.nrw + p) * kNarrow + j) * 4);
#pragma unroll
            for (int j = 0; j < kNarrow; ++j) {
                v[4 * j] += (double)x[j].x;
                v[4 * j + 1] += (double)x[j].y;
                v[4 * j + 2] += (double)x[j].z;
                v[4 * j + 3] += (double)x[j].w;
            }
        }
        const double s = wave_reduce_scatter<double, 4 * kNarrow>(v, lane);
        if ((lane & 1) == 0) red[wv * 32 + (lane >> 1)] = s;
        __syncthreads();
        if (t < 32) {
            const int c = 4 * cq + (t & 3), j = t >> 2;
            if (c < bo) W[(size_t)c * kNarrow + j] = ((red[t] + red[32 + t]) + red[64 + t]) + red[96 + t];
        }
        __syncthreads();
    }
}

// B2: W'[c][j] = sum_{l <= c} T[l, c] W[l][j]; W in LDS, workgroup g takes
// columns g, g + G, ..., four at a time with all their loads of T issued
// together (thread t: rows t, t + 256, t + 512, t + 768).
__device__ __forceinline__ void narrow_phase_b2(const FusedArgs& a, char* lds, int64_t b, int bo, const double* W,
                                                float* Wt)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, G = gridDim.x;
    if ((int)blockIdx.x >= bo) return;
    double* Ws = (double*)(lds + kNarrowWs);            // bo x 8
    double* red = Ws + 1024 * kNarrow;                  // 4 waves x 8
    for (int e = t; e < bo * kNarrow / 2; e += 256) ((double2*)Ws)[e] = ((const double2*)W)[e];
    __syncthreads();
    const double* Tb = a.T + (size_t)b * a.nbo * a.nbo;
    for (int c0 = blockIdx.x; c0 < bo; c0 += 4 * G) {
        double tv[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c0 + k * G;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int l = t + 256 * i;
                tv[k][i] = (c < bo && l <= c) ? Tb[(size_t)c * a.nbo + l] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c0 + k * G;
            if (c >= bo) break;
            double sj[kNarrow];
#pragma unroll
            for (int j = 0; j < kNarrow; ++j) sj[j] = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int l = t + 256 * i;
                if (l <= c) {
                    const double2* w = (const double2*)(Ws + (size_t)l * kNarrow);
#pragma unroll
                    for (int j = 0; j < kNarrow / 2; ++j) {
                        const double2 x = w[j];
                        sj[2 * j] += tv[k][i] * x.x;
                        sj[2 * j + 1] += tv[k][i] * x.y;
                    }
                }
            }
            const double s = wave_reduce_scatter<double, kNarrow>(sj, lane);
            if ((lane & 7) == 0) red[wv * kNarrow + (lane >> 3)] = s;
            __syncthreads();
            if (t < kNarrow)
                Wt[(size_t)c * kNarrow + t] = (float)(((red[t] + red[kNarrow + t]) + red[2 * kNarrow + t]) + red[3 * kNarrow + t]);
            __syncthreads();
        }
    }
}

// C: B[k0 + r, j] -= sum_c V[r, c] W'[c][j] over the rows of range g, last row
// group first, as MFMA products (16 x 16 x 4, FP32): wavefront w takes columns
// 256w .. 256w + 255 of 16 rows at a time, lane (c, g4) = (lane % 16, lane / 16)
// loading row c's columns 256w + 16k + 4g4 .. +3 (k < 16) as one 16-byte
// vector whose four values are the A operands of four MFMAs; the B operands
// (W' of the same columns, rhs c, zero for c >= 8) stay in registers.  The
// four wavefronts' 16 x 16 tiles are added through LDS (double-buffered, one
// barrier a group).  The B values come from the LDS copy phase A staged when
// the range is one chunk.
constexpr int kNarrowCr = 16;                 // rows per MFMA group

__device__ __forceinline__ void narrow_phase_c(const FusedArgs& a, char* lds, float* Bc, int kc, int64_t b, int bo,
                                               int64_t mk, const float* Wt)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int c16 = lane & 15, g4 = lane >> 4;
    if (g >= a.nrw) return;
    int64_t rb, re;
    narrow_range(mk, a.nrw, g, rb, re);
    if (rb >= re) return;
    const int64_t k0 = b * a.nbo;
    const int ldv = (bo + 15) / 16 * 16;
    const int cb = 256 * w + 4 * g4;              // this lane's first column; slab k adds 16k
    const float* Vb = (const float*)a.Vt + fused_vt_off(a, b) + cb;
    float wf[16][4];
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = cb + 16 * k + q;
            wf[k][q] = (c16 < kNarrow && col < bo) ? Wt[(size_t)col * kNarrow + c16] : 0.f;
        }
    float* Bs = (float*)lds;
    float* red = (float*)(lds + kNarrowWs);       // 2 x 4 wavefronts x 16 x 16
    constexpr int GR = kNarrowCr;
    const int64_t nch = (re - rb + kNarrowCh - 1) / kNarrowCh;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        const int64_t c0 = rb + ch * kNarrowCh;
        const int64_t c1 = c0 + kNarrowCh < re ? c0 + kNarrowCh : re;
        const int ng = (int)((c1 - c0 + GR - 1) / GR);
        // group i: rows c1 - GR (i + 1) .. c1 - GR i - 1, those below c0 masked
        float4 va[16], vb[16];
        auto ld = [&](float4 (&v)[16], int i) {
            const int64_t r = c1 - (int64_t)GR * (i + 1) + c16;
            const bool rv = i < ng && r >= c0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int col = cb + 16 * k;
                float4 x = (rv && col < ldv) ? *(const float4*)(Vb + r * ldv + 16 * k) : float4{0.f, 0.f, 0.f, 0.f};
                if (col + 4 > bo) {           // past the last column (the padding of a narrow last block)
                    x.x = col < bo ? x.x : 0.f;
                    x.y = col + 1 < bo ? x.y : 0.f;
                    x.z = col + 2 < bo ? x.z : 0.f;
                    x.w = 0.f;
                }
                v[k] = x;
            }
        };
        auto grp = [&](const float4 (&v)[16], int i) {
            f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[k].x, wf[k][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[k].y, wf[k][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[k].z, wf[k][2], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[k].w, wf[k][3], acc, 0, 0, 0);
            }
            // lane (c16, g4) holds rows 4 g4 .. 4 g4 + 3 of column c16
            float* rd = red + (i & 1) * 1024;
#pragma unroll
            for (int q = 0; q < 4; ++q) rd[w * 256 + (4 * g4 + q) * 16 + c16] = acc[q];
            lds_barrier();
            if (t < GR * kNarrow) {
                const int u = t >> 3, j = t & 7;
                const float sum = ((rd[u * 16 + j] + rd[256 + u * 16 + j]) + rd[512 + u * 16 + j]) + rd[768 + u * 16 + j];
                const int64_t r = c1 - (int64_t)GR * (i + 1) + u;
                if (r >= c0 && j < kc) Bc[k0 + r + (int64_t)j * a.ldb] = Bs[8 * (r - c0) + j] - sum;
            }
        };
        if (nch > 1) {
            lds_barrier();
            narrow_stage_b(a, Bs, Bc, kc, k0, c0, c1);
        }
        ld(va, 0);
        ld(vb, 1);
        lds_barrier();
        for (int i = 0; i < ng; i += 2) {
            grp(va, i);
            ld(va, i + 2);
            if (i + 1 < ng) {
                grp(vb, i + 1);
                ld(vb, i + 3);
            }
        }
    }
}

// ------------------------------------------------------------ back-substitution
// Columns of R (or of a stored inverse) are taken RW at a time, all RW loads
// of a thread issued together; the critical path (the owner of the next
// block) loads its first round of both before it waits for the flag.
template <typename TS, int KC> struct Rw { static constexpr int v = KC <= 8 ? 64 : 32; };

template <typename TS, int RW>
__device__ __forceinline__ void load_cols(const TS* base, int64_t stride, int c0, int bo, TS (&r)[RW])
{
#pragma unroll
    for (int u = 0; u < RW; ++u) r[u] = c0 + u < bo ? base[(int64_t)(c0 + u) * stride] : (TS)0;
}

// acc (+)= sum over the round's columns of r[u] * src[c0 + u][:]  (SUB: -=)
template <typename TS, int KC, int RW, bool SUB>
__device__ __forceinline__ void round_fma(TS (&acc)[KC], const TS (&r)[RW], const TS* src, int c0)
{
    typedef typename Vec4<TS>::t V4;
#pragma unroll
    for (int u = 0; u < RW; ++u) {
        const TS* xc = src + (c0 + u) * KC;
#pragma unroll
        for (int j = 0; j < KC; j += 4) {
            const V4 w = ld4<TS>(xc + j);
            if (SUB) {
                acc[j] -= r[u] * w.x;
                acc[j + 1] -= r[u] * w.y;
                acc[j + 2] -= r[u] * w.z;
                acc[j + 3] -= r[u] * w.w;
            } else {
                acc[j] += r[u] * w.x;
                acc[j + 1] += r[u] * w.y;
                acc[j + 2] += r[u] * w.z;
                acc[j + 3] += r[u] * w.w;
            }
        }
    }
}

// x_q = R_qq^{-1} y_q (stored inverse), into xs, the published copy and B.
// r holds the inverse's first round of columns (row threadIdx.x).
template <typename TS, int KC>
__device__ __forceinline__ void fused_solve_block(const FusedArgs& a, TS* ys, TS* xs, const TS (&y)[KC], int64_t q,
                                                  TS* Bc, int kc, TS* Xp, uint32_t* flags, uint32_t stamp,
                                                  TS (&r)[Rw<TS, KC>::v])
{
    typedef typename Vec4<TS>::t V4;
    constexpr int RW = Rw<TS, KC>::v;
    const int t = threadIdx.x;
    const int bo = (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256);
#pragma unroll
    for (int j = 0; j < KC; j += 4) {
        V4 w = {y[j], y[j + 1], y[j + 2], y[j + 3]};
        *(V4*)(ys + t * KC + j) = w;
    }
    __syncthreads();
    const TS* Ri = (const TS*)a.RiC + (size_t)q * 256 * 256 + t;
    TS acc[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) acc[j] = (TS)0;
    for (int c0 = 0; c0 < bo; c0 += RW) {
        if (c0 > 0) load_cols<TS, RW>(Ri, 256, c0, bo, r);
        round_fma<TS, KC, RW, false>(acc, r, ys, c0);
    }
    TS* xp = Xp + ((size_t)q * 256 + t) * KC;
#pragma unroll
    for (int j = 0; j < KC; j += 4) {
        V4 w = {acc[j], acc[j + 1], acc[j + 2], acc[j + 3]};
        *(V4*)(xs + t * KC + j) = w;
        *(V4*)(xp + j) = w;
    }
    if (t < bo)
#pragma unroll
        for (int j = 0; j < KC; ++j)
            if (j < kc) Bc[256 * q + t + (int64_t)j * a.ldb] = acc[j];
    // the workgroup barrier waits for every wavefront's stores; thread 0's
    // release writes them back before the flag (as in fused_sync)
    __syncthreads();
    if (t == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(flags + q, stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// y -= R[rows of block q, columns of block b] x_b  (R read in place); r holds
// the first round of columns (row 256 q + threadIdx.x)
template <typename TS, int KC>
__device__ __forceinline__ void fused_update(const FusedArgs& a, TS (&y)[KC], int64_t q, int64_t b, const TS* xs,
                                             TS (&r)[Rw<TS, KC>::v])
{
    constexpr int RW = Rw<TS, KC>::v;
    const int bo = (int)(a.n - 256 * b < 256 ? a.n - 256 * b : 256);
    const TS* Rc = (const TS*)a.A + (256 * q + threadIdx.x) + 256 * b * a.lda;
    for (int c0 = 0; c0 < bo; c0 += RW) {
        if (c0 > 0) load_cols<TS, RW>(Rc, a.lda, c0, bo, r);
        round_fma<TS, KC, RW, true>(y, r, xs, c0);
    }
}

template <typename TS, int KC>
__device__ __forceinline__ const TS* r_block(const FusedArgs& a, int64_t q, int64_t b)
{
    return (const TS*)a.A + (256 * q + threadIdx.x) + 256 * b * a.lda;
}

// ------------------------------------ back-substitution, narrow FP32 chunks
// With Rh = blockdiag(R_qq^{-1}) R (right of the diagonal blocks),
//   x_q = R_qq^{-1} c_q - sum_{b > q} Rh[q, b] x_b,
// so the chain of dependent blocks has no inverse product on it.  Each
// 256-row block is split in four quarters of 64 rows; quarter Q = 4q + s
// belongs to workgroup Q mod G (its k-th: Q = g + k G), and wavefront w holds
// the partial sums over columns 64w .. 64w + 63 of every product, lane i row
// i of the quarter.  Step bb, once the four quarters of x_bb are published:
// the owner of a quarter of block bb - 1 applies x_bb with the slice it loaded
// before waiting, adds its four wavefronts' sums and publishes those 64 rows
// of x_{bb-1} (flag per quarter); then every workgroup applies x_bb to its
// other quarters, the highest block first (the next on the chain).  The
// quarters' partial sums live in LDS, each thread's in its own slots, so that
// a quarter is addressed by its index at run time (no unrolled copy of the
// update per quarter).
constexpr int kNarrowMaxQ = 8;     // quarters a workgroup (blocks <= 2 G)

// Columns 64w .. 64w + 63 of block b in rows 64 s + lane of block q of Rh
// (zero past the last column).
__device__ __forceinline__ void narrow_slice(const FusedArgs& a, int64_t q, int s, int64_t b, float (&S)[64])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int bo = (int)(a.n - 256 * b < 256 ? a.n - 256 * b : 256);
    const float* base = (const float*)a.Rh + fused_rh_off(q, a.n) + (size_t)(256 * (b - q - 1) + 64 * w) * 256 + 64 * s + lane;
#pragma unroll
    for (int u = 0; u < 64; ++u) S[u] = 64 * w + u < bo ? base[(size_t)u * 256] : 0.f;
}

// p (+|-)= sum_u S[u] x[64 w + u][:]; x in LDS, 8 floats a row (a broadcast read)
template <bool SUB>
__device__ __forceinline__ void narrow_fma(float (&p)[kNarrow], const float (&S)[64], const float* xs)
{
    const float* xr = xs + 64 * (threadIdx.x >> 6) * kNarrow;
#pragma unroll
    for (int u = 0; u < 64; ++u) {
        const float4 x0 = *(const float4*)(xr + u * 8), x1 = *(const float4*)(xr + u * 8 + 4);
        const float xv[kNarrow] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int j = 0; j < kNarrow; ++j) {
            if (SUB)
                p[j] -= S[u] * xv[j];
            else
                p[j] += S[u] * xv[j];
        }
    }
}

// Sum the four wavefronts' partials of quarter (q, s), store its rows of x
// (zero past the last row) in the published copy and in B, then the flag.
__device__ __forceinline__ void narrow_publish(const FusedArgs& a, float* red, const float (&p)[kNarrow], int64_t q, int s,
                                               float* Bc, int kc, float* Xp, uint32_t* flags, uint32_t stamp)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    float* r = red + (w * 64 + lane) * kNarrow;
    *(float4*)r = float4{p[0], p[1], p[2], p[3]};
    *(float4*)(r + 4) = float4{p[4], p[5], p[6], p[7]};
    __syncthreads();
    const int i = t >> 2, jj = (t & 3) * 2;
    const int bo = (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256);
    const bool valid = 64 * s + i < bo;
    float x0 = 0.f, x1 = 0.f;
    if (valid) {
        x0 = ((red[i * 8 + jj] + red[(64 + i) * 8 + jj]) + red[(128 + i) * 8 + jj]) + red[(192 + i) * 8 + jj];
        x1 = ((red[i * 8 + jj + 1] + red[(64 + i) * 8 + jj + 1]) + red[(128 + i) * 8 + jj + 1]) + red[(192 + i) * 8 + jj + 1];
    }
    const int64_t row = 256 * q + 64 * s + i;
    *(float2*)(Xp + (size_t)row * kNarrow + jj) = float2{x0, x1};
    if (valid) {
        if (jj < kc) Bc[row + (int64_t)jj * a.ldb] = x0;
        if (jj + 1 < kc) Bc[row + (int64_t)(jj + 1) * a.ldb] = x1;
    }
    __syncthreads();
    if (t == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(flags + 4 * q + s, stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void narrow_pload(const float* pl, int k, float (&v)[kNarrow])
{
    const float4* q = (const float4*)(pl + ((size_t)k * 256 + threadIdx.x) * kNarrow);
    const float4 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ void narrow_pstore(float* pl, int k, const float (&v)[kNarrow])
{
    float4* q = (float4*)(pl + ((size_t)k * 256 + threadIdx.x) * kNarrow);
    q[0] = float4{v[0], v[1], v[2], v[3]};
    q[1] = float4{v[4], v[5], v[6], v[7]};
}

// x_b (in LDS) applied to this workgroup's quarters below block lim, the
// highest first: quarters 0 .. kq - 1 of the workgroup (blocks rise with k).
__device__ __forceinline__ void narrow_bulk(const FusedArgs& a, float* pl, const float* xsrc, int64_t b, int64_t lim)
{
    const int G = gridDim.x, g = blockIdx.x;
    const int64_t nbq = (a.n + 255) / 256;
    int kq = 0;
    for (int k = 0; k < kNarrowMaxQ; ++k) {
        const int64_t Qd = g + (int64_t)G * k;
        if (Qd < 4 * nbq && (Qd >> 2) < lim) kq = k + 1;
    }
    for (int k = kq - 1; k >= 0; --k) {
        const int64_t Qd = g + (int64_t)G * k;
        float S[64], v[kNarrow];
        narrow_slice(a, Qd >> 2, (int)(Qd & 3), b, S);
        narrow_pload(pl, k, v);
        narrow_fma<true>(v, S, xsrc);
        narrow_pstore(pl, k, v);
    }
}

__device__ __forceinline__ bool narrow_backsub(const FusedArgs& a, char* lds, int* sflag, float* Bc, int kc,
                                               uint32_t* flags, float* Xp, uint32_t stamp)
{
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x, w = t >> 6;
    const int64_t nbq = (a.n + 255) / 256;
    float* xs = (float*)lds;                      // 256 x 8: x_bb
    float* red = xs + 256 * kNarrow;              // 4 wavefronts x 64 rows x 8
    float* pl = red + 4 * 64 * kNarrow;           // the quarters' partial sums, each thread its own (k, t) slots
    // p = wavefront w's part of R_qq^{-1} c_q for every quarter owned
    for (int k = 0; k < kNarrowMaxQ; ++k) {
        const int64_t Qd = g + (int64_t)G * k;
        if (Qd >= 4 * nbq) break;
        const int64_t q = Qd >> 2;
        const int s = (int)(Qd & 3);
        const int bo = (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256);
        float S[64], v[kNarrow];
        const float* Ri = (const float*)a.RiC + (size_t)q * 65536 + (size_t)(64 * w) * 256 + 64 * s + (t & 63);
#pragma unroll
        for (int u = 0; u < 64; ++u) S[u] = 64 * w + u < bo ? Ri[(size_t)u * 256] : 0.f;
        __syncthreads();                          // earlier readers of xs are done
        {
            float bv[kNarrow];
#pragma unroll
            for (int j = 0; j < kNarrow; ++j) bv[j] = (t < bo && j < kc) ? Bc[256 * q + t + (int64_t)j * a.ldb] : 0.f;
            *(float4*)(xs + t * 8) = float4{bv[0], bv[1], bv[2], bv[3]};
            *(float4*)(xs + t * 8 + 4) = float4{bv[4], bv[5], bv[6], bv[7]};
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kNarrow; ++j) v[j] = 0.f;
        narrow_fma<false>(v, S, xs);
        narrow_pstore(pl, k, v);
    }
    const int64_t last = nbq - 1;
    for (int k = 0; k < kNarrowMaxQ; ++k) {
        const int64_t Qd = g + (int64_t)G * k;
        if (Qd < 4 * nbq && (Qd >> 2) == last) {
            float v[kNarrow];
            narrow_pload(pl, k, v);
            narrow_publish(a, red, v, last, (int)(Qd & 3), Bc, kc, Xp, flags, stamp);
        }
    }
    for (int64_t bb = last; bb >= 1; --bb) {
        const int64_t an = bb - 1;
        int kan = -1, san = 0;
        for (int s = 0; s < 4; ++s)
            if ((4 * an + s) % G == g) {
                kan = (int)((4 * an + s) / G);
                san = s;
            }
        float S[64];
        if (kan >= 0) narrow_slice(a, an, san, bb, S);     // the critical path's slice, before the wait
        if (t == 0) {
            const bool ok = fused_wait4(flags + 4 * bb, stamp, a.err, a.wait_ticks);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *sflag = ok ? 1 : 0;
        }
        __syncthreads();
        if (!*sflag) return false;
        {
            const float4* src = (const float4*)(Xp + (size_t)bb * 256 * kNarrow);
            ((float4*)xs)[t] = src[t];
            ((float4*)xs)[t + 256] = src[t + 256];
        }
        __syncthreads();
        if (kan >= 0) {
            float v[kNarrow];
            narrow_pload(pl, kan, v);
            narrow_fma<true>(v, S, xs);
            narrow_publish(a, red, v, an, san, Bc, kc, Xp, flags, stamp);
        }
        narrow_bulk(a, pl, xs, bb, an);
    }
    return true;
}

// One chunk of at most KC columns: Q^T then R^{-1}.  False: a wait gave up.
template <typename TS, int KC>
__device__ __forceinline__ bool fused_chunk(const FusedArgs& a, char* lds, int* sflag, uint32_t* bar, uint32_t& gen, TS* Bc, int kc,
                            uint32_t stamp, const FusedLayout& L)
{
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x;
    const int64_t nbq = (a.n + 255) / 256;
    uint32_t* flags = (uint32_t*)(a.scratch + L.flags);
    double* W = (double*)(a.scratch + L.W);
    TS* Wt = (TS*)(a.scratch + L.Wt);
    TS* Xp = (TS*)(a.scratch + L.Xp);
    TS* P = (TS*)(a.scratch + L.P);
    // ---- Q^T B
    for (int64_t b = 0; b < a.nblocks; ++b) {
        const int64_t k0 = b * a.nbo;
        const int bo = (int)(a.n - k0 < a.nbo ? a.n - k0 : a.nbo);
        const int64_t mk = a.m - k0;
        const int ncg = (bo + 127) / 128;
        int nrg = G / ncg;
        if (nrg > a.nrg_cap) nrg = a.nrg_cap;
        const int64_t rmax = (mk + 63) / 64;
        if (nrg > rmax) nrg = (int)rmax;
        if (nrg < 1) nrg = 1;
        if constexpr (sizeof(TS) == 4 && KC == kNarrow) {
            narrow_phase_a(a, lds, Bc, kc, b, bo, mk, P);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
            narrow_phase_b1(a, lds, bo, P, W);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
            narrow_phase_b2(a, lds, b, bo, W, Wt);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
            narrow_phase_c(a, lds, Bc, kc, b, bo, mk, Wt);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
            continue;
        }
        fused_phase_a<TS, KC>(a, lds, Bc, kc, b, bo, mk, nrg, ncg, P);
        if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
        fused_phase_b1<TS, KC>(a, bo, nrg, P, W);
        if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
        fused_phase_b2<TS, KC>(a, lds, b, bo, W, Wt);
        if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
        fused_phase_c<TS, KC>(a, lds, Bc, kc, b, bo, mk, Wt);
        if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, sflag)) return false;
    }
    // ---- R^{-1}
    if constexpr (sizeof(TS) == 4 && KC == kNarrow)
        if (a.Rh) return narrow_backsub(a, lds, sflag, Bc, kc, flags, Xp, stamp);
    constexpr int RW = Rw<TS, KC>::v;
    TS* ys = (TS*)lds;                  // then two x buffers of 256 x KC
    TS y[kFusedMaxOwn][KC];
#pragma unroll
    for (int s = 0; s < kFusedMaxOwn; ++s) {
        const int64_t q = g + (int64_t)s * G;
        const int bo = q < nbq ? (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256) : 0;
#pragma unroll
        for (int j = 0; j < KC; ++j) y[s][j] = (t < bo && j < kc) ? Bc[256 * q + t + (int64_t)j * a.ldb] : (TS)0;
    }
    int cur = 0;
    bool have = false;
    const int64_t last = nbq - 1;
    TS ru[RW], ri[RW];
    if (last % G == g) {
        const int s = (int)(last / G);
        const int bo = (int)(a.n - 256 * last);
        load_cols<TS, RW>((const TS*)a.RiC + (size_t)last * 256 * 256 + t, 256, 0, bo, ri);
#pragma unroll
        for (int ss = 0; ss < kFusedMaxOwn; ++ss)
            if (ss == s)
                fused_solve_block<TS, KC>(a, ys, ys + (1 + cur) * 256 * KC, y[ss], last, Bc, kc, Xp, flags, stamp,
                                          ri);
        have = true;
    }
    for (int64_t bb = last; bb >= 1; --bb) {
        const int64_t an = bb - 1;
        const bool mine = an % G == g;
        const int bob = (int)(a.n - 256 * bb < 256 ? a.n - 256 * bb : 256);
        if (mine) {
            // the critical path: first rounds of R[an, bb] and of R_an,an^{-1}
            load_cols<TS, RW>(r_block<TS, KC>(a, an, bb), a.lda, 0, bob, ru);
            load_cols<TS, RW>((const TS*)a.RiC + (size_t)an * 256 * 256 + t, 256, 0, 256, ri);
        }
        if (!have) {
            // x_b published by its owner
            if (t == 0) {
                const bool ok = fused_wait(flags + bb, stamp, false, a.err, a.wait_ticks);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                *sflag = ok ? 1 : 0;
            }
            __syncthreads();
            if (!*sflag) return false;
            const TS* src = Xp + (size_t)bb * 256 * KC;
            TS* dst = ys + (1 + cur) * 256 * KC;
            for (int e = 4 * t; e < 256 * KC; e += 1024) *(typename Vec4<TS>::t*)(dst + e) = ld4<TS>(src + e);
        }
        __syncthreads();
        const TS* xs = ys + (1 + cur) * 256 * KC;
        have = false;
        if (mine) {
            const int s = (int)(an / G);
#pragma unroll
            for (int ss = 0; ss < kFusedMaxOwn; ++ss)
                if (ss == s) {
                    fused_update<TS, KC>(a, y[ss], an, bb, xs, ru);
                    fused_solve_block<TS, KC>(a, ys, ys + (2 - cur) * 256 * KC, y[ss], an, Bc, kc, Xp, flags, stamp,
                                              ri);
                }
            have = true;
        }
#pragma unroll
        for (int ss = 0; ss < kFusedMaxOwn; ++ss) {
            const int64_t q = g + (int64_t)ss * G;
            if (q < an) {
                load_cols<TS, RW>(r_block<TS, KC>(a, q, bb), a.lda, 0, bob, ru);
                fused_update<TS, KC>(a, y[ss], q, bb, xs, ru);
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    return true;
}

// Chunks of up to KCB columns; a batch of at most KCS columns (a small
// batch) runs the narrow variant, whose products do a quarter of the work.
template <typename TS, int KCB, int KCS>
__global__ void __launch_bounds__(256, 1) fused_solve_kernel(FusedArgs a)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ int sflag;
    const int t = threadIdx.x;
    const int off = a.rec ? a.rec[0] : 0;
    const int cnt = a.rec ? (a.rec[1] < a.nrhs ? a.rec[1] : a.nrhs) : a.nrhs;
    if (cnt <= 0) return;
    const int64_t nbq = (a.n + 255) / 256;
    const FusedLayout L = fused_layout(a.nbo, nbq, a.nrg_cap, KCB, sizeof(TS));
    uint32_t* bar = (uint32_t*)a.scratch;
    uint32_t gen = 0;
    if (t == 0) gen = __hip_atomic_load(bar + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    TS* B = (TS*)a.B + (int64_t)off * a.ldb;
    if (cnt <= KCS) {
        fused_chunk<TS, KCS>(a, lds, &sflag, bar, gen, B, cnt, 1u, L);
        return;
    }
    uint32_t stamp = 0;
    for (int j0 = 0; j0 < cnt; j0 += KCB) {
        const int kc = cnt - j0 < KCB ? cnt - j0 : KCB;
        if (!fused_chunk<TS, KCB>(a, lds, &sflag, bar, gen, B + (int64_t)j0 * a.ldb, kc, ++stamp, L)) return;
    }
}

__global__ void fused_reset_kernel(uint32_t* bar, uint32_t* flags, int64_t nbq)
{
    const int t = threadIdx.x;
    if (t == 0) bar[0] = 0u;
    for (int64_t q = t; q < 4 * nbq; q += 256) flags[q] = 0u;
}

template <typename TS>
static constexpr int fused_kc() { return sizeof(TS) == 4 ? 32 : 16; }
constexpr int kFusedSmall = kNarrow;

template <typename TS>
static size_t fused_lds_bytes()
{
    constexpr int KC = fused_kc<TS>();
    const size_t a = (size_t)8 * KC * 128 * sizeof(TS);                 // phase A reduction (aliases B staging)
    const size_t c = (size_t)1024 * KC * sizeof(TS);                      // phase C: W' of a block
    const size_t s = (size_t)3 * 256 * KC * sizeof(TS);                  // back-substitution
    size_t m = a > c ? a : c;
    return m > s ? m : s;
}

// Row groups of the W partials (chunks of kc columns) that fit `bytes` of
// scratch after the fixed part of the layout, at most cap; 0: none fits.
int fused_row_groups(int nbo, int64_t n, size_t es, size_t bytes, int kc, int cap)
{
    const int KC = es == 4 ? 32 : 16;
    const int64_t nbq = (n + 255) / 256;
    const FusedLayout L0 = fused_layout(nbo, nbq, 0, KC, es);
    if (bytes <= L0.total) return 0;
    const size_t per = (size_t)kc * nbo * es;
    const size_t r = (bytes - L0.total) / per;
    return r > (size_t)cap ? cap : (int)r;
}

template <typename TS>
hipError_t launch_fused_solve(const FusedArgs& a, int G, bool cooperative, hipStream_t s)
{
    constexpr int KC = fused_kc<TS>();
    static bool attr = false;
    const size_t lds = fused_lds_bytes<TS>();
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fused_solve_kernel<TS, KC, kFusedSmall>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int64_t nbq = (a.n + 255) / 256;
    const FusedLayout L = fused_layout(a.nbo, nbq, a.nrg_cap, KC, sizeof(TS));
    hipLaunchKernelGGL(fused_reset_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)a.scratch,
                       (uint32_t*)(a.scratch + L.flags), nbq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    FusedArgs args = a;
    void* kargs[] = {&args};
    if (cooperative)
        return hipLaunchCooperativeKernel((const void*)fused_solve_kernel<TS, KC, kFusedSmall>, dim3(G), dim3(256),
                                          kargs, lds, s);
    hipLaunchKernelGGL((fused_solve_kernel<TS, KC, kFusedSmall>), dim3(G), dim3(256), lds, s, args);
    return hipGetLastError();
}
template hipError_t launch_fused_solve<float>(const FusedArgs&, int, bool, hipStream_t);
template hipError_t launch_fused_solve<double>(const FusedArgs&, int, bool, hipStream_t);

size_t fused_scratch_bytes(int nbo, int64_t n, size_t es, int nrg)
{
    const int KC = es == 4 ? 32 : 16;
    return fused_layout(nbo, (n + 255) / 256, nrg, KC, es).total;
}

}  // namespace ctqr
