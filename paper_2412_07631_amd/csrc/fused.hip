// Persistent fused solve: X = R^{-1} Q^T B (Eq. (solve)) for a batch of
// right-hand sides in one launch of one workgroup per CU (cooperative, so the
// launch is refused rather than under-scheduled).
//
// The batch is taken in chunks of KC columns.  Per chunk:
//   Q^T B, outer block by outer block (Q = I - V T V^T per block, compact WY):
//     A   W partials: the rows of the block split in row groups, its columns in
//         groups of 128; each workgroup sums V[rows, cols]^T B[rows] over its
//         rows (V from the row-major reflector copy, B staged in LDS)
//     B1  W = sum of the partials (fixed order, FP64)
//     B2  W' = T^T W (T upper triangular, FP64)
//     C   B[rows] -= V[rows, :] W', the rows split over all workgroups
//     with a grid-wide barrier after each phase;
//   R^{-1}: back-substitution over 256-row blocks, block q owned by workgroup
//     q mod G; the owner of block q, once every later block's x has been
//     applied to its rows, multiplies by the stored inverse of R_qq and
//     publishes x_q with a flag; every workgroup takes the published x_b in
//     order b = last .. 1 and subtracts R[q, b] x_b from the rows it owns,
//     first the block right below in the chain, which it then solves at once.
// All arithmetic is FMA in the storage type (W and T W in FP64).  The
// cross-workgroup waits are bounded in time like the factorization's (bit 3
// of the error word on a time-out).
#include "ct_internal.h"

namespace ctqr {

constexpr int kFusedMaxOwn = 2;     // 256-row blocks per workgroup in the back-substitution
constexpr int kFusedErr = 8;

struct FusedArgs {
    const void* A;        // V\R in place, column-major
    int64_t lda;
    const void* Vt;       // row-major reflector blocks: block b at vt_off(b), ld round16(width)
    const double* T;      // T of block b at b nbo^2, column-major, upper triangular
    const void* RiC;      // inverses of the 256 x 256 diagonal blocks of R, column-major, block q at q 256^2
    int64_t m, n;
    int nbo, nblocks;
    void* B;
    int64_t ldb;
    int nrhs;             // columns (eager), or the largest batch (graph)
    const int32_t* rec;   // batch record (offset, count) of a graph-captured solve, or null
    char* scratch;
    int nrg_cap;          // row groups of the W partials at most
    int32_t* err;
    uint64_t wait_ticks;
};

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
    L.W = L.flags + fused_up256((size_t)nbq * 4);
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

// Grid-wide barrier: the last workgroup to arrive resets the count and
// advances the generation; the others wait for the generation to change.
// Self-resetting, so one reset before the launch is all it needs.
__device__ inline bool fused_sync(uint32_t* bar, uint32_t& gen, int G, int32_t* err, uint64_t ticks, int* flag)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
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
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
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
            if (t == 0) *sflag = fused_wait(flags + bb, stamp, false, a.err, a.wait_ticks) ? 1 : 0;
            __syncthreads();
            if (!*sflag) return false;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
    for (int64_t q = t; q < nbq; q += 256) flags[q] = 0u;
}

template <typename TS>
static constexpr int fused_kc() { return sizeof(TS) == 4 ? 32 : 16; }
constexpr int kFusedSmall = 8;

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

// Scratch bytes with nrg row groups; the largest nrg that fits `bytes`.
int fused_row_groups(int nbo, int64_t n, size_t es, size_t bytes)
{
    const int KC = es == 4 ? 32 : 16;
    const int64_t nbq = (n + 255) / 256;
    const FusedLayout L0 = fused_layout(nbo, nbq, 0, KC, es);
    if (bytes <= L0.total) return 0;
    const size_t per = (size_t)KC * nbo * es;
    const size_t r = (bytes - L0.total) / per;
    return r > 32 ? 32 : (int)r;
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
