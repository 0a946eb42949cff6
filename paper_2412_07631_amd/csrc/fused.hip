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

constexpr int kFusedMaxOwn = 4;     // 256-row blocks per workgroup in the back-substitution
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

template <typename TS> struct Vec4;
template <> struct Vec4<float> { typedef float4 t; };
template <> struct Vec4<double> { typedef double4 t; };

template <typename TS>
__device__ inline typename Vec4<TS>::t ld4(const TS* p) { return *(const typename Vec4<TS>::t*)p; }

// ---------------------------------------------------------------- Q^T phases
// A: W partials of block b over row group rg, column group cg.
template <typename TS, int KC>
__device__ void fused_phase_a(const FusedArgs& a, char* lds, const TS* Bc, int kc, int64_t b, int bo, int64_t mk,
                              int nrg, int ncg, TS* P)
{
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
    constexpr int BL = KC + 64 / (int)sizeof(TS);   // rows of 192 bytes: aligned vector reads
    TS* Bs = (TS*)lds;                        // 64 x BL
    TS acc[KC][4];
#pragma unroll
    for (int j = 0; j < KC; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] = (TS)0;
    for (int64_t r0 = rb; r0 < re; r0 += 64) {
        for (int e = t; e < 64 * KC; e += 256) {
            const int rr = e & 63, j = e >> 6;
            const int64_t r = r0 + rr;
            Bs[rr * BL + j] = (r < re && j < kc) ? Bc[k0 + r + (int64_t)j * a.ldb] : (TS)0;
        }
        __syncthreads();
        const int nr = re - r0 < 64 ? (int)(re - r0) : 64;
        for (int rr = rl; rr < nr; rr += 8) {
            typename Vec4<TS>::t v = {0, 0, 0, 0};
            if (cvalid) v = ld4<TS>(Vb + (r0 + rr) * ldv + c);
            const TS* br = Bs + rr * BL;
#pragma unroll
            for (int j = 0; j < KC; j += 4) {
                const typename Vec4<TS>::t bb = ld4<TS>(br + j);
                const TS bj[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[j + u][0] += v.x * bj[u];
                    acc[j + u][1] += v.y * bj[u];
                    acc[j + u][2] += v.z * bj[u];
                    acc[j + u][3] += v.w * bj[u];
                }
            }
        }
        __syncthreads();
    }
    // sum the 8 row lanes in LDS: red[rl][j][128]
    TS* red = (TS*)lds;
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        typename Vec4<TS>::t w = {acc[j][0], acc[j][1], acc[j][2], acc[j][3]};
        *(typename Vec4<TS>::t*)(red + ((size_t)(rl * KC + j) * 128 + 4 * cq)) = w;
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

// B1: W[j][c] = sum over row groups (fixed order), FP64
template <typename TS, int KC>
__device__ void fused_phase_b1(const FusedArgs& a, int bo, int nrg, const TS* P, double* W)
{
    const int64_t total = (int64_t)KC * bo;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int j = (int)(e / bo), c = (int)(e % bo);
        double s = 0.0;
        for (int rg = 0; rg < nrg; ++rg) s += (double)P[((size_t)rg * KC + j) * a.nbo + c];
        W[(size_t)j * a.nbo + c] = s;
    }
}

// B2: W'[c][j] = sum_{l <= c} T[l, c] W[j][l]
template <typename TS, int KC>
__device__ void fused_phase_b2(const FusedArgs& a, int64_t b, int bo, const double* W, TS* Wt)
{
    const double* Tb = a.T + (size_t)b * a.nbo * a.nbo;
    const int64_t total = (int64_t)KC * bo;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int c = (int)(e / KC), j = (int)(e % KC);
        const double* tc = Tb + (size_t)c * a.nbo;
        const double* wr = W + (size_t)j * a.nbo;
        double s = 0.0;
        for (int l = 0; l <= c; ++l) s += tc[l] * wr[l];
        Wt[(size_t)c * KC + j] = (TS)s;
    }
}

// C: B[k0 + r] -= V[r, :] W' for the rows of this workgroup
template <typename TS, int KC>
__device__ void fused_phase_c(const FusedArgs& a, char* lds, TS* Bc, int kc, int64_t b, int bo, int64_t mk,
                              const TS* Wt)
{
    const int g = blockIdx.x, t = threadIdx.x, G = gridDim.x;
    const int64_t k0 = b * a.nbo;
    const int64_t rpw = (mk + G - 1) / G;
    const int64_t rb = g * rpw, re = rb + rpw < mk ? rb + rpw : mk;
    const int ldv = (bo + 15) / 16 * 16;
    const TS* Vb = (const TS*)a.Vt + fused_vt_off(a, b);
    constexpr int KQ = KC / 4;
    TS* Vs = (TS*)lds;                 // 64 x 65
    TS* Ws = Vs + 64 * 65;             // 64 x KC
    const int rr = t & 63, jg = t >> 6;
    for (int64_t r0 = rb; r0 < re; r0 += 64) {
        TS acc[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) acc[q] = (TS)0;
        for (int c0 = 0; c0 < bo; c0 += 64) {
            for (int e = t; e < 64 * 64; e += 256) {
                const int r2 = e >> 6, cc = e & 63;
                const int64_t r = r0 + r2;
                Vs[r2 * 65 + cc] = (r < re && c0 + cc < ldv) ? Vb[r * ldv + c0 + cc] : (TS)0;
            }
            for (int e = t; e < 64 * KC; e += 256) {
                const int cc = e / KC, j = e % KC;
                Ws[e] = (c0 + cc < bo) ? Wt[(size_t)(c0 + cc) * KC + j] : (TS)0;
            }
            __syncthreads();
            const TS* vr = Vs + rr * 65;
            const TS* wc = Ws + jg * KQ;
#pragma unroll 8
            for (int cc = 0; cc < 64; ++cc) {
                const TS v = vr[cc];
#pragma unroll
                for (int q = 0; q < KQ; q += 4) {
                    const typename Vec4<TS>::t w = ld4<TS>(wc + cc * KC + q);
                    acc[q] += v * w.x;
                    acc[q + 1] += v * w.y;
                    acc[q + 2] += v * w.z;
                    acc[q + 3] += v * w.w;
                }
            }
            __syncthreads();
        }
        const int64_t r = r0 + rr;
        if (r < re) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const int j = jg * KQ + q;
                if (j < kc) {
                    TS* p = Bc + k0 + r + (int64_t)j * a.ldb;
                    *p = *p - acc[q];
                }
            }
        }
    }
}

// ------------------------------------------------------------ back-substitution
// x_q = R_qq^{-1} y_q (stored inverse), into xs, the published copy and B
template <typename TS, int KC>
__device__ void fused_solve_block(const FusedArgs& a, TS* ys, TS* xs, const TS (&y)[KC], int64_t q, TS* Bc, int kc,
                                  TS* Xp, uint32_t* flags, uint32_t stamp)
{
    const int t = threadIdx.x;
    const int bo = (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256);
#pragma unroll
    for (int j = 0; j < KC; j += 4) {
        typename Vec4<TS>::t w = {y[j], y[j + 1], y[j + 2], y[j + 3]};
        *(typename Vec4<TS>::t*)(ys + t * KC + j) = w;
    }
    __syncthreads();
    const TS* Ri = (const TS*)a.RiC + (size_t)q * 256 * 256;
    TS acc[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) acc[j] = (TS)0;
#pragma unroll 4
    for (int c = 0; c < bo; ++c) {
        const TS r = Ri[(size_t)c * 256 + t];
        const TS* yc = ys + c * KC;
#pragma unroll
        for (int j = 0; j < KC; j += 4) {
            const typename Vec4<TS>::t w = ld4<TS>(yc + j);
            acc[j] += r * w.x;
            acc[j + 1] += r * w.y;
            acc[j + 2] += r * w.z;
            acc[j + 3] += r * w.w;
        }
    }
    TS* xp = Xp + ((size_t)q * 256 + t) * KC;
#pragma unroll
    for (int j = 0; j < KC; j += 4) {
        typename Vec4<TS>::t w = {acc[j], acc[j + 1], acc[j + 2], acc[j + 3]};
        *(typename Vec4<TS>::t*)(xs + t * KC + j) = w;
        *(typename Vec4<TS>::t*)(xp + j) = w;
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

// y -= R[rows of block q, columns of block b] x_b  (R read in place)
template <typename TS, int KC>
__device__ void fused_update(const FusedArgs& a, TS (&y)[KC], int64_t q, int64_t b, const TS* xs)
{
    const int t = threadIdx.x;
    const int bo = (int)(a.n - 256 * b < 256 ? a.n - 256 * b : 256);
    const TS* Rc = (const TS*)a.A + (256 * q + t) + 256 * b * a.lda;
#pragma unroll 4
    for (int c = 0; c < bo; ++c) {
        const TS r = Rc[(int64_t)c * a.lda];
        const TS* xc = xs + c * KC;
#pragma unroll
        for (int j = 0; j < KC; j += 4) {
            const typename Vec4<TS>::t w = ld4<TS>(xc + j);
            y[j] -= r * w.x;
            y[j + 1] -= r * w.y;
            y[j + 2] -= r * w.z;
            y[j + 3] -= r * w.w;
        }
    }
}

template <typename TS, int KC>
__global__ void __launch_bounds__(256, 1) fused_solve_kernel(FusedArgs a)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ int sflag;
    const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x;
    const int off = a.rec ? a.rec[0] : 0;
    const int cnt = a.rec ? (a.rec[1] < a.nrhs ? a.rec[1] : a.nrhs) : a.nrhs;
    if (cnt <= 0) return;
    const int64_t nbq = (a.n + 255) / 256;
    const FusedLayout L = fused_layout(a.nbo, nbq, a.nrg_cap, KC, sizeof(TS));
    uint32_t* bar = (uint32_t*)a.scratch;
    uint32_t* flags = (uint32_t*)(a.scratch + L.flags);
    double* W = (double*)(a.scratch + L.W);
    TS* Wt = (TS*)(a.scratch + L.Wt);
    TS* Xp = (TS*)(a.scratch + L.Xp);
    TS* P = (TS*)(a.scratch + L.P);
    uint32_t gen = 0;
    if (t == 0) gen = __hip_atomic_load(bar + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    TS* B = (TS*)a.B + (int64_t)off * a.ldb;
    uint32_t stamp = 0;
    for (int j0 = 0; j0 < cnt; j0 += KC) {
        const int kc = cnt - j0 < KC ? cnt - j0 : KC;
        TS* Bc = B + (int64_t)j0 * a.ldb;
        ++stamp;
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
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, &sflag)) return;
            fused_phase_b1<TS, KC>(a, bo, nrg, P, W);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, &sflag)) return;
            fused_phase_b2<TS, KC>(a, b, bo, W, Wt);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, &sflag)) return;
            fused_phase_c<TS, KC>(a, lds, Bc, kc, b, bo, mk, Wt);
            if (!fused_sync(bar, gen, G, a.err, a.wait_ticks, &sflag)) return;
        }
        // ---- R^{-1}
        TS* ys = (TS*)lds;
        TS* xsb[2] = {ys + 256 * KC, ys + 2 * 256 * KC};
        TS y[kFusedMaxOwn][KC];
#pragma unroll
        for (int s = 0; s < kFusedMaxOwn; ++s) {
            const int64_t q = g + (int64_t)s * G;
            const int bo = q < nbq ? (int)(a.n - 256 * q < 256 ? a.n - 256 * q : 256) : 0;
#pragma unroll
            for (int j = 0; j < KC; ++j)
                y[s][j] = (t < bo && j < kc) ? Bc[256 * q + t + (int64_t)j * a.ldb] : (TS)0;
        }
        int cur = 0;
        bool have = false;
        const int64_t last = nbq - 1;
        if (last % G == g) {
            const int s = (int)(last / G);
#pragma unroll
            for (int ss = 0; ss < kFusedMaxOwn; ++ss)
                if (ss == s) fused_solve_block<TS, KC>(a, ys, xsb[cur], y[ss], last, Bc, kc, Xp, flags, stamp);
            have = true;
        }
        for (int64_t bb = last; bb >= 1; --bb) {
            if (!have) {
                // x_b published by its owner
                if (t == 0) sflag = fused_wait(flags + bb, stamp, false, a.err, a.wait_ticks) ? 1 : 0;
                __syncthreads();
                if (!sflag) return;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const TS* src = Xp + (size_t)bb * 256 * KC;
                TS* dst = xsb[cur];
                for (int e = 4 * t; e < 256 * KC; e += 1024)
                    *(typename Vec4<TS>::t*)(dst + e) = ld4<TS>(src + e);
            }
            __syncthreads();
            const TS* xs = xsb[cur];
            const int64_t an = bb - 1;
            have = false;
            if (an % G == g) {
                const int s = (int)(an / G);
#pragma unroll
                for (int ss = 0; ss < kFusedMaxOwn; ++ss)
                    if (ss == s) {
                        fused_update<TS, KC>(a, y[ss], an, bb, xs);
                        fused_solve_block<TS, KC>(a, ys, xsb[cur ^ 1], y[ss], an, Bc, kc, Xp, flags, stamp);
                    }
                have = true;
            }
#pragma unroll
            for (int ss = 0; ss < kFusedMaxOwn; ++ss) {
                const int64_t q = g + (int64_t)ss * G;
                if (q < an) fused_update<TS, KC>(a, y[ss], q, bb, xs);
            }
            __syncthreads();
            cur ^= 1;
        }
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

template <typename TS>
static size_t fused_lds_bytes()
{
    constexpr int KC = fused_kc<TS>();
    const size_t a = (size_t)8 * KC * 128 * sizeof(TS);                 // phase A reduction (aliases B staging)
    const size_t c = (size_t)(64 * 65 + 64 * KC) * sizeof(TS);            // phase C tiles
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
        hipError_t e = hipFuncSetAttribute((const void*)fused_solve_kernel<TS, KC>,
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
        return hipLaunchCooperativeKernel((const void*)fused_solve_kernel<TS, KC>, dim3(G), dim3(256), kargs, lds, s);
    hipLaunchKernelGGL((fused_solve_kernel<TS, KC>), dim3(G), dim3(256), lds, s, args);
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
