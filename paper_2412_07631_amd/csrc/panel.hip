// Householder panel factorization (Eq. (qr), the geqrf step of Sec. 2.1) of
// an mk x nbp column panel, nbp <= 32, as ONE cooperative launch.
//
// The panel is spread over P workgroups by rows; each holds its rows in LDS
// as FP64 for the whole panel.  Column j needs, after all earlier reflectors,
//   s_c = sum_{i>j} a_ij a_ic  (all c)   and the pivot row a_jc,
// from which every workgroup derives, redundantly and identically,
//   sigma = sqrt(a_jj^2 + s_j), beta = -sign(a_jj) sigma, tau = (beta-a_jj)/beta,
//   v_i = a_ij / (a_jj - beta) (i > j), w_c = tau (a_jc + s_c / (a_jj - beta)),
// and applies H_j = I - tau v v^T to its own rows: a_ic -= w_c v_i.  So one
// cross-workgroup reduction (of the Gram row s and the pivot row) per column
// is the only synchronisation; norms, tau and the reflector scaling are FP64
// whatever the storage type.  Partials are summed in a fixed order by the
// last workgroup to arrive, which publishes the sums, so the result is
// bitwise reproducible.
//
// The same reduction also yields the inner products of the new reflector
// with the earlier ones: for c < j, v_c is final and
//   v_c^T v_j = a_jc + s_c / (a_jj - beta),
// so workgroup 0 grows the compact-WY factor T (Schreiber & Van Loan 1989)
// one column per step in LDS, T_jj = tau_j, T[0:j, j] = -tau_j T[0:j,0:j] (V^T v_j)[0:j],
// with no extra pass over the panel: H_0 ... H_{nbp-1} = I - V T V^T.
//
// Two-reduction path (panel_cqr_kernel, tried first when the panel fits): the
// same V, T, R and tau in exact arithmetic from two Gram reductions instead of
// one per column.  CholeskyQR2 gives the thin factor Q with orthonormal
// columns: G = A^T A, R1 = chol(G), Q1 = A R1^-1, R2 = chol(Q1^T Q1),
// Q = Q1 R2^-1, A = Q (R2 R1).  The Householder form follows from the LU
// factorization without pivoting Q_top - S = L1 U of the top nbp x nbp block,
// with the sign S_j = -sign of the eliminated diagonal entry (so every pivot
// has modulus >= 1): V = [L1; Q_bottom U^-1], T = -U S L1^-T, R = S R2 R1
// (Ballard, Demmel, Grigori, Jacquelin, Knight, Nguyen, "Reconstructing
// Householder vectors from tall-skinny QR", 2015).  The sign choice is the
// no-cancellation choice of the column-wise path, so both give the LAPACK
// convention.  Each workgroup sums a slice of the Gram partials of all
// workgroups and publishes it; the top block travels with the first
// reduction, so the small factorizations (two Cholesky, one LU) run
// redundantly and identically in every workgroup.  A Cholesky pivot below a
// relative threshold (rank deficiency, or a panel too ill-conditioned for
// CholeskyQR2 in FP64) sends every workgroup, uniformly, to the column-wise
// path on the original panel.
#include "ct_internal.h"

#include <stdlib.h>
#include <string.h>
#include <math.h>

namespace ctqr {

constexpr int kPanelMax = 32;

template <typename TS>
struct PanelArgs {
    TS* A;              // top-left of the panel, column-major
    int64_t lda;
    int64_t mk;         // rows of the panel (m - k0)
    int nbp;            // columns of the panel, <= 32
    int rw;             // rows held by one workgroup
    int P;              // workgroups
    double* tau;        // tau[0..nbp)
    double* T;          // nbp x nbp compact-WY factor, column-major
    int64_t ldt;
    double* part;       // [2][P][64] per-column partials (double buffered), then [2][64] results
    uint64_t* counter;  // arrival counter (monotone)
    uint64_t base;      // its value before this launch
    uint64_t col_base;  // columns factored by earlier launches (parity of the result slots)
    int64_t* info;      // first zero-norm column + 1 (0: none so far)
    int64_t col0;       // global index of the panel's first column
    int32_t* err;
    uint64_t wait_ticks; // time limit of one wait (100 MHz ticks)
    double* cq;         // two-reduction path scratch (kCqWords)
    uint64_t cq_par;    // parity of this launch among the two-reduction launches
};

// Result slots follow the double-buffered partial rows (2 x 256 x 64) in the
// part buffer; an empty slot entry holds this NaN bit pattern.
constexpr size_t kPartRes = (size_t)2 * 256 * 64;
constexpr uint64_t kEmpty = 0x7FF4C0FFEE5107D5ull;

// LDS words besides the panel: red 256, vec 64, wv 32, sc 8, Tl 32*33, gl 32
constexpr int kPanelAux = 256 + 64 + 32 + 8 + kPanelMax * (kPanelMax + 1) + kPanelMax;

// Two-reduction path: a reduction carries the packed upper triangle of a
// 32 x 32 Gram matrix (kNV values); the first also carries the panel's top
// 32 x 32 block (published by workgroup 0, not summed).  The scratch buffer
// holds the partials of both reductions for both launch parities, then the
// result slots of both parities; every word reads as kEmpty until written.
constexpr int kNV = 32 * 33 / 2;
constexpr int kNA = kNV + 32 * 32;
constexpr int kCqSlotLen = kNA + kNV;
constexpr size_t kCqPartLen = (size_t)256 * kNV;
constexpr size_t kCqSlot = 4 * kCqPartLen;
constexpr size_t kCqWords = kCqSlot + 2 * (size_t)kCqSlotLen;
// LDS words of that path besides the 32-column panel and kPanelAux:
// K1..K4 (32 x 32 each), S, 1/diag, Gram phase partials (36 blocks x 7 x 16)
constexpr int kGramPh = 7;
constexpr int kCqAux = 4 * 1024 + 32 + 32 + 36 * kGramPh * 16;
constexpr double kCholTol1 = 1e-13;   // pivot / diagonal of A^T A
constexpr double kCholTol2 = 0.25;    // pivot of Q1^T Q1 (close to 1)

struct PanelLds {
    double *pan, *red, *vec, *wv, *sc, *Tl, *gl;
};

__device__ __forceinline__ PanelLds panel_lds(double* lds, int rw, int ncols)
{
    PanelLds L;
    L.pan = lds;                               // pan[c * rw + r]
    L.red = lds + (size_t)ncols * rw;          // 256
    L.vec = L.red + 256;                       // 64: s_c then the pivot row
    L.wv = L.vec + 64;                         // 32
    L.sc = L.wv + 32;                          // 8 scalars
    L.Tl = L.sc + 8;                           // 32 x 33 (workgroup 0)
    L.gl = L.Tl + kPanelMax * (kPanelMax + 1); // 32
    return L;
}

__device__ __forceinline__ void set_err(int32_t* err)
{
    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait for a published word (anything but the kEmpty pattern).  The
// clock and the error word are read only every 16 polls, so a normal
// (microsecond) wait costs neither.  False: the wait gave up (time limit, or
// an earlier wait of the factorization did).
__device__ __forceinline__ bool wait_word(uint64_t* p, uint64_t& bits, int32_t* err, uint64_t wait_ticks)
{
    uint64_t t0 = 0;
    uint32_t spins = 0;
    while ((bits = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kEmpty) {
        if (wait_ticks == 0) {
            set_err(err);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spins == 16) {
                t0 = now;
            } else if (now - t0 >= wait_ticks) {
                set_err(err);
                return false;
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) return false;
        }
    }
    return true;
}

// The same for the arrival counter: wait until it reaches `target`.
__device__ __forceinline__ bool wait_count(uint64_t* counter, uint64_t target, int32_t* err, uint64_t wait_ticks)
{
    uint64_t t0 = 0;
    uint32_t spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (wait_ticks == 0) {
            set_err(err);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spins == 16) {
                t0 = now;
            } else if (now - t0 >= wait_ticks) {
                set_err(err);
                return false;
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) return false;
        }
    }
    return true;
}

// Column-wise Householder steps on the panel in LDS: one cross-workgroup
// reduction per column, arrivals counted from `target` on.  False: a wait
// gave up (every workgroup then leaves).
template <typename TS>
__device__ bool column_steps(const PanelArgs<TS>& a, const PanelLds& L, int w, int t, int rows, int64_t r0,
                             uint64_t target)
{
    const int nbp = a.nbp, rw = a.rw;
    double* pan = L.pan;
    double* red = L.red;
    double* vec = L.vec;
    double* wv = L.wv;
    double* sc = L.sc;
    double* Tl = L.Tl;
    double* gl = L.gl;
    if (w == 0)
        for (int e = t; e < kPanelMax * (kPanelMax + 1); e += 256) Tl[e] = 0.0;
    __syncthreads();
    for (int j = 0; j < nbp; ++j) {
        // (1) this workgroup's partial Gram row (all columns) and pivot row
        {
            const int c = t & 31, g = t >> 5;
            double s = 0.0;
            if (c < nbp) {
                int rs = (int)((int64_t)j + 1 - r0);
                if (rs < 0) rs = 0;
                const double* pj = pan + j * rw;
                const double* pc = pan + c * rw;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int r = rs + g;
                for (; r + 24 < rows; r += 32) {
                    s0 += pj[r] * pc[r];
                    s1 += pj[r + 8] * pc[r + 8];
                    s2 += pj[r + 16] * pc[r + 16];
                    s3 += pj[r + 24] * pc[r + 24];
                }
                for (; r < rows; r += 8) s0 += pj[r] * pc[r];
                s = (s0 + s1) + (s2 + s3);
            }
            red[g * 32 + c] = s;
        }
        __syncthreads();
        if (t < 64) {
            double v = 0.0;
            if (t < 32) {
                for (int g = 0; g < 8; ++g) v += red[g * 32 + t];
            } else {
                const int c = t - 32;
                const int64_t lr = (int64_t)j - r0;
                if (lr >= 0 && lr < rows && c < nbp) v = pan[c * rw + (int)lr];
            }
            a.part[((size_t)(j & 1) * a.P + w) * 64 + t] = v;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        // (2) arrival; the last workgroup to arrive sums the partials in a
        // fixed order and publishes the 64 sums in a result slot; the others
        // poll that slot.  Two slots alternate by global column parity; a slot
        // reads as empty (kEmpty bit pattern) until published, and the
        // publisher empties the other slot, for the next column, first.
        if (t == 0) {
            const uint64_t old =
                __hip_atomic_fetch_add(a.counter, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sc[4] = (old + 1 == target + (uint64_t)a.P) ? 1.0 : 0.0;
        }
        target += (uint64_t)a.P;
        __syncthreads();
        const bool last = sc[4] != 0.0;
        const uint64_t gpar = (a.col_base + (uint64_t)j) & 1;
        uint64_t* slot = (uint64_t*)(a.part + kPartRes) + gpar * 64;
        uint64_t* other = (uint64_t*)(a.part + kPartRes) + (gpar ^ 1) * 64;
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int v = t & 63, g = t >> 6;
            const double* base = a.part + (size_t)(j & 1) * a.P * 64 + v;
            // every load of this lane is issued before any is consumed: one
            // round trip for up to 136 workgroups (136 rows per WG-column of
            // 4 lanes x 34), a second one for the rest (P <= 256)
            double s = 0.0;
            {
                double x[34];
#pragma unroll
                for (int u = 0; u < 34; ++u) {
                    const int q = g + 4 * u;
                    x[u] = q < a.P ? base[(size_t)q * 64] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 34; ++u) s += x[u];
            }
            if (a.P > 136) {
                double x[30];
#pragma unroll
                for (int u = 0; u < 30; ++u) {
                    const int q = g + 4 * (u + 34);
                    x[u] = q < a.P ? base[(size_t)q * 64] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 30; ++u) s += x[u];
            }
            red[g * 64 + v] = s;
            __syncthreads();
            if (t < 64) {
                const double r = ((red[t] + red[64 + t]) + red[128 + t]) + red[192 + t];
                vec[t] = r;
                __hip_atomic_store(other + t, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(slot + t, __builtin_bit_cast(uint64_t, r), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            if (t < 64) {
                uint64_t bits = 0;
                if (!wait_word(slot + t, bits, a.err, a.wait_ticks)) sc[5] = 1.0;
                // what the publisher wrote before the slot (the emptied
                // other slot) is visible from here on
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                vec[t] = __builtin_bit_cast(double, bits);
            }
            __syncthreads();
            if (sc[5] != 0.0) return false;      // uniform: the whole workgroup leaves
        }
        __syncthreads();
        // (3) the reflector, computed alike by the 32 lanes that then form
        // w_c = tau (v_j^T a_c) for their column c (same inputs, same values)
        if (t < 32) {
            const double alpha = vec[32 + j], ssum = vec[j];
            const double sigma = sqrt(alpha * alpha + ssum);
            double beta, tau, scl;
            if (sigma == 0.0) {
                beta = alpha;
                tau = 0.0;
                scl = 0.0;
            } else {
                beta = alpha >= 0.0 ? -sigma : sigma;
                tau = (beta - alpha) / beta;
                scl = 1.0 / (alpha - beta);
            }
            if (t == 0) {
                sc[0] = scl;
                sc[1] = beta;
                sc[2] = tau;
                sc[3] = sigma == 0.0 ? 1.0 : 0.0;
                if (w == 0) {
                    a.tau[j] = tau;
                    if (sigma == 0.0 && *a.info == 0) *a.info = a.col0 + j + 1;
                }
            }
            const int c = t;
            const double h = vec[32 + c] + scl * vec[c];
            wv[c] = (c > j && c < nbp) ? tau * h : 0.0;
            if (w == 0) gl[c] = (c < j && sigma != 0.0) ? h : 0.0;   // v_c^T v_j
        }
        __syncthreads();
        if (w == 0 && t < 32) {
            // T[c][j] = -tau_j sum_{l=c}^{j-1} T[c][l] g_l ;  T[j][j] = tau_j
            const int c = t;
            if (c < j) {
                double acc = 0.0;
                for (int l = c; l < j; ++l) acc += Tl[l * 33 + c] * gl[l];
                Tl[j * 33 + c] = -sc[2] * acc;
            } else if (c == j) {
                Tl[j * 33 + j] = sc[2];
            }
        }
        // (4) apply H_j to this workgroup's rows: first v (column j scaled,
        // pivot set to beta), then the rank-1 update with one column per
        // thread and eight row phases, so the inner loop has no branches
        if (sc[3] == 0.0) {
            const double scl = sc[0], beta = sc[1];
            for (int r = t; r < rows; r += 256) {
                const int64_t gr = r0 + r;
                if (gr > j) pan[j * rw + r] *= scl;
                else if (gr == j) pan[j * rw + r] = beta;
            }
            __syncthreads();
            const int c = t & 31, g = t >> 5;
            if (c > j && c < nbp) {
                const double wc = wv[c];
                const double* vj = pan + j * rw;
                double* pc = pan + c * rw;
                int rs = (int)((int64_t)j - r0);
                if (rs < 0) rs = 0;
                // the pivot row (gr == j) takes v = 1
                if (rs < rows && r0 + rs == j && (rs & 7) == g) {
                    pc[rs] -= wc;
                    rs += 8;
                }
                int r = rs + ((g - rs) & 7);
                if (r < rows && r0 + r == j) r += 8;
                for (; r + 24 < rows; r += 32) {
                    const double v0 = vj[r], v1 = vj[r + 8], v2 = vj[r + 16], v3 = vj[r + 24];
                    const double x0 = pc[r], x1 = pc[r + 8], x2 = pc[r + 16], x3 = pc[r + 24];
                    pc[r] = x0 - wc * v0;
                    pc[r + 8] = x1 - wc * v1;
                    pc[r + 16] = x2 - wc * v2;
                    pc[r + 24] = x3 - wc * v3;
                }
                for (; r < rows; r += 8) pc[r] -= wc * vj[r];
            }
        }
        __syncthreads();
    }
    return true;
}

// Rows of the panel into LDS as FP64 (columns from nbp to ncols as zeros);
// every load of a row is issued before any is stored.
template <typename TS>
__device__ __forceinline__ void load_panel(const PanelArgs<TS>& a, double* pan, int ncols, int t, int rows, int64_t r0)
{
    for (int r = t; r < rows; r += 256) {
        const TS* src = a.A + (r0 + r);
        // unconditional loads (columns past nbp reread the last one), so the
        // compiler issues all 32 before waiting
        TS v[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) v[c] = src[(int64_t)(c < a.nbp ? c : a.nbp - 1) * a.lda];
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < ncols) pan[c * a.rw + r] = c < a.nbp ? (double)v[c] : 0.0;
    }
}

// V\R back to the matrix; workgroup 0 also writes T (zero below the diagonal).
template <typename TS>
__device__ __forceinline__ void store_panel(const PanelArgs<TS>& a, const PanelLds& L, int w, int t, int rows,
                                            int64_t r0)
{
    const int nbp = a.nbp;
    for (int c = 0; c < nbp; ++c)
        for (int r = t; r < rows; r += 256) a.A[(r0 + r) + (int64_t)c * a.lda] = (TS)L.pan[c * a.rw + r];
    if (w == 0)
        for (int e = t; e < nbp * nbp; e += 256) {
            const int q = e / nbp, p = e - q * nbp;
            a.T[p + (int64_t)q * a.ldt] = p <= q ? L.Tl[q * 33 + p] : 0.0;
        }
}

template <typename TS>
__global__ void __launch_bounds__(256) panel_qr_kernel(PanelArgs<TS> a)
{
    extern __shared__ double lds[];
    const int t = threadIdx.x, w = blockIdx.x;
    const PanelLds L = panel_lds(lds, a.rw, a.nbp);
    const int64_t r0 = (int64_t)w * a.rw;
    const int rows = (int)((a.mk - r0) < (int64_t)a.rw ? (a.mk - r0) : (int64_t)a.rw);

    // a wait of an earlier launch gave up: the factorization is already failed
    if (t == 0) L.sc[5] = (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) ? 1.0 : 0.0;
    __syncthreads();
    if (L.sc[5] != 0.0) return;
    load_panel(a, L.pan, a.nbp, t, rows, r0);
    __syncthreads();
    if (!column_steps(a, L, w, t, rows, r0, a.base)) return;
    store_panel(a, L, w, t, rows, r0);
}

// ------------------------------------------------- two-reduction panel path
// Packed upper triangle: entry (i, c), i <= c < 32, at c (c + 1) / 2 + i.
__device__ __forceinline__ void unpack_ut(int e, int& i, int& c)
{
    int cc = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    if ((cc + 1) * (cc + 2) / 2 <= e) ++cc;
    if (cc * (cc + 1) / 2 > e) --cc;
    c = cc;
    i = e - cc * (cc + 1) / 2;
}

// This workgroup's Gram partial of the 32 panel columns (rows in LDS) as the
// packed upper triangle, in pv[0..kNV).  Threads own 4 x 4 blocks of the
// upper block triangle (36 blocks) over kGramPh row phases; the phases are
// then summed per entry.  Ends with a barrier.
__device__ void gram_partial(const double* pan, int rw, int rows, double* red2, double* pv, int t)
{
    if (t < 36 * kGramPh) {
        const int blk = t % 36, ph = t / 36;
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
        const int bi = blk - bj * (bj + 1) / 2;
        const double* pa = pan + (4 * bi) * rw;
        const double* pc = pan + (4 * bj) * rw;
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
        for (int r = ph; r < rows; r += kGramPh) {
            double xa[4], xc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xa[u] = pa[u * rw + r];
                xc[u] = pc[u * rw + r];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += xa[u] * xc[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) red2[(ph * 36 + blk) * 16 + u * 4 + v] = acc[u][v];
    }
    __syncthreads();
    for (int e = t; e < kNV; e += 256) {
        int i, c;
        unpack_ut(e, i, c);
        const int bi = i >> 2, bj = c >> 2;
        const int blk = bj * (bj + 1) / 2 + bi;
        const int uv = (i & 3) * 4 + (c & 3);
        double s = 0.0;
        for (int ph = 0; ph < kGramPh; ++ph) s += red2[(ph * 36 + blk) * 16 + uv];
        pv[e] = s;
    }
    __syncthreads();
}

// Wave-uniform bounded poll: loads the NW words p[i] (i < n, compile-time
// bound NW) until none holds kEmpty in any lane of the wave; their bits go
// to v.  False: the wait gave up (time limit, or an earlier wait did).
template <int NW>
__device__ __forceinline__ bool poll_words(uint64_t* const (&p)[NW], int n, uint64_t (&v)[NW], int32_t* err,
                                           uint64_t wait_ticks)
{
    uint64_t t0 = 0;
    uint32_t spins = 0;
    for (;;) {
        bool all = true;
#pragma unroll
        for (int i = 0; i < NW; ++i)
            if (i < n) {
                v[i] = __hip_atomic_load(p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                all = all && v[i] != kEmpty;
            }
        if (__all(all)) return true;
        if (wait_ticks == 0) {
            set_err(err);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 15) == 0) {
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spins == 16) {
                t0 = now;
            } else if (now - t0 >= wait_ticks) {
                set_err(err);
                return false;
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) return false;
        }
    }
}

// One reduction of the two-reduction path.  Each workgroup writes its packed
// partial (pv, LDS) to its row of `part`, one polled word per entry; wave 0
// sums the workgroup's slice of entries (e = w + P k) over every partial in a
// fixed order and publishes the sums in `slot`; then the nread slot entries
// come back into LDS (packed entries to the upper triangle of K, row-major
// ld 32; entries from kNV on to Kt).  No counter, no fence: every word is
// its own flag.  False: a wait gave up.
template <typename TS>
__device__ bool cq_reduce(const PanelArgs<TS>& a, const double* pv, double* part, uint64_t* slot, int nread,
                          double* K, double* Kt, double* sc, int w, int t)
{
    const int P = a.P;
    uint64_t* pw = (uint64_t*)part;
    for (int e = t; e < kNV; e += 256)
        __hip_atomic_store(pw + (size_t)w * kNV + e, __builtin_bit_cast(uint64_t, pv[e]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (t < 64) {
        // lanes in groups of gsz, one slice entry per group and round; lane
        // `mem` of a group adds the partials q = mem + gsz i
        const int ns = (kNV - 1 - w) / P + 1;
        int p2 = 1;
        while (p2 < ns) p2 <<= 1;
        const int gsz = p2 >= 64 ? 1 : 64 / p2;
        const int ng = 64 / gsz, grp = t / gsz, mem = t % gsz;
        const int nq = mem < P ? (P - mem + gsz - 1) / gsz : 0;    // <= 24 (gsz >= P / 24 here)
        for (int k0 = 0; k0 < ns; k0 += ng) {
            const int k = k0 + grp;
            const int e = w + P * (k < ns ? k : 0);
            constexpr int NW = 24;
            uint64_t* ptr[NW];
            uint64_t bits[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) ptr[i] = pw + (size_t)(mem + gsz * i) * kNV + e;
            if (!poll_words<NW>(ptr, k < ns ? nq : 0, bits, a.err, a.wait_ticks)) {
                sc[5] = 1.0;
                break;
            }
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NW; ++i)
                if (i < nq && k < ns) s += __builtin_bit_cast(double, bits[i]);
            for (int o = 1; o < gsz; o <<= 1) s += __shfl_xor(s, o);
            if (k < ns && mem == 0)
                __hip_atomic_store(slot + e, __builtin_bit_cast(uint64_t, s), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    {
        constexpr int NW = (kNA + 255) / 256;
        uint64_t* ptr[NW];
        uint64_t bits[NW];
        int n = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int e = t + 256 * i;
            ptr[i] = slot + (e < nread ? e : 0);
            if (e < nread) n = i + 1;
        }
        if (!poll_words<NW>(ptr, n, bits, a.err, a.wait_ticks)) {
            sc[5] = 1.0;
        } else {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int e = t + 256 * i;
                if (e < nread) {
                    const double v = __builtin_bit_cast(double, bits[i]);
                    if (e < kNV) {
                        int r, c;
                        unpack_ut(e, r, c);
                        K[r * 32 + c] = v;
                    } else {
                        Kt[e - kNV] = v;
                    }
                }
            }
        }
    }
    __syncthreads();
    return sc[5] == 0.0;
}

// Value of v in lane `lane` (uniform lane index), for every lane.
__device__ __forceinline__ double bcast(double v, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Cholesky factor of the symmetric matrix in K (upper triangle, row-major
// ld 32, n x n leading block, zero elsewhere), by wave 0 in registers: lane i
// holds row i (lanes 32..63 repeat 0..31), right-looking, the pivot row
// broadcast from its lane, no barrier inside.  On success K's upper triangle
// holds R (R^T R = K) and dv[j] = 1/R_jj (0 past n).  Pivots must exceed tol
// times the original diagonal; the test reads broadcast values, so the
// outcome is the same in every lane and, through flag, every thread.
__device__ bool chol32(double* K, double* dv, double* flag, int n, double tol, int t)
{
    if (t < 64) {
        const int i = t & 31;
        double a[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) a[c] = c >= i ? K[i * 32 + c] : K[c * 32 + i];
        const double g0 = K[i * 33];
        bool ok = true;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if (j < n && ok) {
                const double d = bcast(a[j], j);
                if (!(d > tol * bcast(g0, j)) || !(d < 1.0e300)) {
                    ok = false;
                } else {
                    const double f = i > j ? a[j] / d : 0.0;
#pragma unroll
                    for (int c = j + 1; c < 32; ++c) a[c] -= f * bcast(a[c], j);
                }
            }
        }
        if (t < 32) {
            if (ok && i < n) {
                // this row's pivot (register chosen without a dynamic index)
                double ai = 0.0;
#pragma unroll
                for (int c = 0; c < 32; ++c) ai = c == i ? a[c] : ai;
                const double rd = sqrt(ai);
                const double ir = 1.0 / rd;
#pragma unroll
                for (int c = 0; c < 32; ++c)
                    if (c > i) K[i * 32 + c] = c < n ? a[c] * ir : 0.0;
                K[i * 33] = rd;
                dv[i] = ir;
            } else if (i >= n) {
                dv[i] = 0.0;
            }
            if (t == 0) flag[0] = ok ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    return flag[0] != 0.0;
}

// LU without pivoting of Q - S on the leading n x n block of K (column-major
// ld 32), S_j = -sign of the eliminated diagonal entry, by wave 0 in
// registers (lane i holds row i).  Leaves the unit lower factor's
// multipliers below the diagonal, U on and above it (U_jj = q_jj - S_j),
// S in Sv; diagonal entries past n are set to 1.
__device__ void lu32(double* K, double* Sv, int n, int t)
{
    if (t < 64) {
        const int i = t & 31;
        double a[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) a[c] = K[i + 32 * c];
        double si = 0.0;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if (j < n) {
                const double q = bcast(a[j], j);
                const double sj = q >= 0.0 ? -1.0 : 1.0;
                if (i == j) si = sj;
                const double l = (i > j && i < n) ? a[j] / (q - sj) : 0.0;
                if (i > j && i < n) a[j] = l;
#pragma unroll
                for (int c = j + 1; c < 32; ++c) a[c] -= l * bcast(a[c], j);
            }
        }
        if (t < 32) {
#pragma unroll
            for (int c = 0; c < 32; ++c) K[i + 32 * c] = c == i ? (i < n ? a[c] - si : 1.0) : a[c];
            Sv[i] = si;
        }
    }
    __syncthreads();
}

// x (one row of 32, registers) <- x M^-1, M upper triangular (row-major
// ld 32, 16-byte aligned; dv = 1/diag, zero beyond the leading block; UNIT:
// unit diagonal, dv unused).  Right-looking, so a step's updates are
// independent; each row of M comes in as 16-byte loads issued one step
// ahead, so a step waits on LDS once, not once per product.
template <bool UNIT>
__device__ __forceinline__ void row_times_inv(double (&x)[32], const double* M, const double* dv)
{
    const double2* M2 = (const double2*)M;
    double2 m[16];
    double d = UNIT ? 1.0 : dv[0];
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k] = M2[k];
#pragma unroll
    for (int l = 0; l < 32; ++l) {
        double2 mn[16];
        double dn = 1.0;
        if (l + 1 < 32) {
#pragma unroll
            for (int k = (l + 2) / 2; k < 16; ++k) mn[k] = M2[(l + 1) * 16 + k];
            if (!UNIT) dn = dv[l + 1];
        }
        if (!UNIT) x[l] *= d;
#pragma unroll
        for (int c = l + 1; c < 32; ++c) x[c] -= x[l] * ((c & 1) ? m[c >> 1].y : m[c >> 1].x);
        if (l + 1 < 32) {
#pragma unroll
            for (int k = (l + 2) / 2; k < 16; ++k) m[k] = mn[k];
            d = dn;
        }
    }
}

// Rows u, u + nt, ... (< n) of X (column-major, ld) times M^-1, in place.
__device__ __forceinline__ void rows_times_inv(double* X, int ld, int n, const double* M, const double* dv, int u,
                                               int nt)
{
    for (int r = u; r < n; r += nt) {
        double x[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) x[c] = X[c * ld + r];
        row_times_inv<false>(x, M, dv);
#pragma unroll
        for (int c = 0; c < 32; ++c) X[c * ld + r] = x[c];
    }
}

template <typename TS>
__global__ void __launch_bounds__(256) panel_cqr_kernel(PanelArgs<TS> a)
{
    extern __shared__ double lds[];
    const int t = threadIdx.x, w = blockIdx.x;
    const int nbp = a.nbp, rw = a.rw, P = a.P;
    const PanelLds L = panel_lds(lds, rw, 32);
    double* K1 = L.gl + kPanelMax;   // G, then R1 (row-major upper)
    double* K2 = K1 + 1024;          // Q1^T Q1, then R2 (row-major upper)
    double* K3 = K2 + 1024;          // top 32 x 32 block of A, of Q1, of Q, then L1 \ U (column-major)
    double* K4 = K3 + 1024;          // this workgroup's Gram partials, then U R2 (row-major upper)
    double* Sv = K4 + 1024;          // S
    double* dv = Sv + 32;            // 1 / diagonal of the current triangular factor
    double* red2 = dv + 32;          // Gram phase partials
    double* sc = L.sc;
    double* pan = L.pan;
    const int64_t r0 = (int64_t)w * rw;
    const int rows = (int)((a.mk - r0) < (int64_t)rw ? (a.mk - r0) : (int64_t)rw);
    const uint64_t par = a.cq_par;
    double* partA = a.cq + (par * 2 + 0) * kCqPartLen;
    double* partB = a.cq + (par * 2 + 1) * kCqPartLen;
    uint64_t* slotA = (uint64_t*)(a.cq + kCqSlot) + par * kCqSlotLen;
    uint64_t* slotB = slotA + kNA;

    if (t == 0) sc[5] = (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) ? 1.0 : 0.0;
    __syncthreads();
    if (sc[5] != 0.0) return;
    // Nothing in this launch reads the other parity's words: empty this
    // workgroup's partial rows and its share of the result slots there, for
    // the next two-reduction launch.  The column-wise path expects the slot
    // of parity col_base + nbp empty at its next launch.
    {
        uint64_t* q0 = (uint64_t*)(a.cq + ((par ^ 1) * 2 + 0) * kCqPartLen) + (size_t)w * kNV;
        uint64_t* q1 = (uint64_t*)(a.cq + ((par ^ 1) * 2 + 1) * kCqPartLen) + (size_t)w * kNV;
        for (int e = t; e < kNV; e += 256) {
            __hip_atomic_store(q0 + e, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(q1 + e, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        uint64_t* o = (uint64_t*)(a.cq + kCqSlot) + (par ^ 1) * kCqSlotLen;
        for (int e = w * 256 + t; e < kCqSlotLen; e += P * 256)
            __hip_atomic_store(o + e, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == 0 && t < 64) {
            uint64_t* cs = (uint64_t*)(a.part + kPartRes) + ((a.col_base + (uint64_t)nbp) & 1) * 64;
            __hip_atomic_store(cs + t, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    load_panel(a, pan, 32, t, rows, r0);
    for (int e = t; e < 4 * 1024; e += 256) K1[e] = 0.0;
    __syncthreads();
    // the panel's top 32 x 32 block, from workgroup 0 (whose rows they are)
    if (w == 0)
        for (int e = t; e < 1024; e += 256) {
            const int r = e & 31, c = e >> 5;
            const double v = r < rows ? pan[c * rw + r] : 0.0;
            __hip_atomic_store(slotA + kNV + e, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }

    bool done = false;
    do {
        // (A) G = A^T A and the top block
        gram_partial(pan, rw, rows, red2, K4, t);
        if (!cq_reduce(a, K4, partA, slotA, kNA, K1, K3, sc, w, t)) return;
        if (!chol32(K1, dv, sc + 6, nbp, kCholTol1, t)) break;
        // Q1 = A R1^-1 on this workgroup's rows and on the top block
        // (the top block's 32 rows go to threads idle in the panel rows'
        // last batch, when there are enough)
        {
            const int tail = rows & 255;
            const int t3 = rows < 256 ? rows : (tail == 0 ? 256 : tail);
            rows_times_inv(pan, rw, rows, K1, dv, t, 256);
            if (t3 + 32 <= 256) {
                if (t >= t3 && t < t3 + 32) rows_times_inv(K3, 32, 32, K1, dv, t - t3, 32);
            } else {
                __syncthreads();
                if (t < 32) rows_times_inv(K3, 32, 32, K1, dv, t, 32);
            }
        }
        __syncthreads();
        // (B) Q1^T Q1
        gram_partial(pan, rw, rows, red2, K4, t);
        if (!cq_reduce(a, K4, partB, slotB, kNV, K2, nullptr, sc, w, t)) return;
        if (!chol32(K2, dv, sc + 6, nbp, kCholTol2, t)) break;
        // top block of Q = Q1 R2^-1
        if (t < 32) rows_times_inv(K3, 32, 32, K2, dv, t, 32);
        __syncthreads();
        // LU of Q_top - S (leading nbp x nbp)
        lu32(K3, Sv, nbp, t);
        // K4 = U R2 (upper triangular, row-major), dv = its inverse diagonal
        for (int e = t; e < kNV; e += 256) {
            int i, c;
            unpack_ut(e, i, c);
            double s = 0.0;
            if (c < nbp)
                for (int l = i; l <= c; ++l) s += K3[i + 32 * l] * K2[l * 32 + c];
            K4[i * 32 + c] = s;
        }
        __syncthreads();
        if (t < 32) dv[t] = t < nbp ? 1.0 / K4[t * 33] : 0.0;
        __syncthreads();
        // V = Q1 (U R2)^-1 on rows nbp.. of the panel
        {
            const int lo = r0 >= nbp ? 0 : (int)(nbp - r0 < rows ? nbp - r0 : rows);
            rows_times_inv(pan + lo, rw, rows - lo, K4, dv, t, 256);
        }
        __syncthreads();
        if (w == 0) {
            // top rows: V below the diagonal, R = S R2 R1 on and above it
            for (int e = t; e < nbp * nbp; e += 256) {
                const int i = e % nbp, c = e / nbp;
                double v;
                if (i > c) {
                    v = K3[i + 32 * c];
                } else {
                    double s = 0.0;
                    for (int l = i; l <= c; ++l) s += K2[i * 32 + l] * K1[l * 32 + c];
                    v = Sv[i] * s;
                }
                pan[c * rw + i] = v;
            }
            // T = -U S L1^-T: row i of T solves T_i L1^T = -(U S)_i, and
            // L1^T read row-major is K3 (column-major L1) itself
            if (t < nbp) {
                const int i = t;
                double x[32];
#pragma unroll
                for (int c = 0; c < 32; ++c) x[c] = (c >= i && c < nbp) ? -K3[i + 32 * c] * Sv[c] : 0.0;
                row_times_inv<true>(x, K3, nullptr);
                double ti = 0.0;   // x[i], chosen without a dynamic index (which would put x in scratch)
#pragma unroll
                for (int c = 0; c < 32; ++c) {
                    L.Tl[c * 33 + i] = x[c];
                    ti = c == i ? x[c] : ti;
                }
                a.tau[i] = ti;
            }
        }
        __syncthreads();
        done = true;
    } while (false);

    if (done) {
        store_panel(a, L, w, t, rows, r0);
        // the arrivals the column-wise path would have made: the counter
        // advances by P nbp whichever path a launch takes
        if (t == 0) __hip_atomic_fetch_add(a.counter, (uint64_t)nbp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // Cholesky breakdown (every workgroup alike): the column-wise path from
    // the original panel
    load_panel(a, pan, nbp, t, rows, r0);
    __syncthreads();
    if (!column_steps(a, L, w, t, rows, r0, a.base)) return;
    store_panel(a, L, w, t, rows, r0);
}

// --------------------------------------------------------------- launcher
static uint64_t g_wait_ticks = kWaitTicks;
void panel_set_wait_limit(int64_t ticks) { g_wait_ticks = ticks < 0 ? kWaitTicks : (uint64_t)ticks; }
uint64_t panel_wait_limit() { return g_wait_ticks; }

// LDS: the panel plus the reduction scratch and the T factor.
size_t panel_lds_bytes(int nbp, int rw) { return ((size_t)nbp * rw + kPanelAux) * sizeof(double); }
int panel_aux_words() { return kPanelAux; }
size_t panel_scratch_words() { return kCqWords; }

// Two-reduction path: 32 panel columns, the column-wise scratch and its own.
static size_t cqr_lds_bytes(int rw) { return ((size_t)32 * rw + kPanelAux + kCqAux) * sizeof(double); }
static size_t g_lds_max = 64 * 1024;
static bool g_cqr = true;
static int g_cus = 256;
void panel_set_cholesky(bool on) { g_cqr = on; }
void panel_set_cus(int cus) { g_cus = cus < 1 ? 1 : (cus > 256 ? 256 : cus); }

// The slice sums of the two-reduction path hold at most 24 partials per lane
// (the same arithmetic as the kernel's lane grouping).
static bool cq_lanes_ok(int P)
{
    for (int w = 0; w < P; ++w) {
        const int ns = (kNV - 1 - w) / P + 1;
        int p2 = 1;
        while (p2 < ns) p2 <<= 1;
        const int gsz = p2 >= 64 ? 1 : 64 / p2;
        if ((P + gsz - 1) / gsz > 24) return false;
    }
    return true;
}

template <typename TS>
hipError_t launch_panel(TS* A, int64_t lda, int64_t mk, int nbp, int rw, double* tau, double* T, int64_t ldt,
                        double* part, double* gpart, uint64_t* counter, uint64_t* base, uint64_t* col_base,
                        uint64_t* cq_count, int64_t* info, int64_t col0, int32_t* err, hipStream_t s)
{
    PanelArgs<TS> a;
    a.A = A; a.lda = lda; a.mk = mk; a.nbp = nbp;
    a.tau = tau; a.T = T; a.ldt = ldt; a.part = part;
    a.counter = counter; a.base = *base; a.info = info; a.col0 = col0; a.err = err;
    a.col_base = *col_base;
    a.wait_ticks = g_wait_ticks;
    a.cq = gpart;
    a.cq_par = *cq_count & 1;
    // the two-reduction path spreads the rows over one workgroup per compute
    // unit (at most 256; odd row counts keep the column-major LDS panel free
    // of bank conflicts); workgroup 0 must hold the top nbp rows
    int64_t rq = (mk + g_cus - 1) / g_cus;
    if (rq < 33) rq = 33;
    if ((rq & 1) == 0) ++rq;
    // (at most 448 rows: the row-pair solves then need at most 224 threads
    // for the panel rows plus 16 for the top block)
    const bool cq = g_cqr && nbp <= 32 && rq <= 448 && cqr_lds_bytes((int)rq) <= g_lds_max &&
                    cq_lanes_ok((int)((mk + rq - 1) / rq));
    // Every workgroup of a panel waits for the others' published sums, so all
    // of them must be resident at once.  A cooperative launch guarantees that
    // or refuses the grid (hipErrorCooperativeLaunchTooLarge) instead of
    // scheduling part of it, which would leave the waits to time out.
    void* kargs[] = {&a};
    hipError_t e = hipErrorCooperativeLaunchTooLarge;
    if (cq) {
        a.rw = (int)rq;
        a.P = (int)((mk + rq - 1) / rq);
        e = hipLaunchCooperativeKernel((const void*)panel_cqr_kernel<TS>, dim3(a.P), dim3(256), kargs,
                                       (unsigned)cqr_lds_bytes(a.rw), s);
        if (e == hipSuccess) *cq_count += 1;
        else if (e == hipErrorCooperativeLaunchTooLarge) (void)hipGetLastError();
        else return e;
    }
    if (e != hipSuccess) {
        // the column-wise form (one reduction per column, smaller LDS panel)
        a.rw = rw;
        a.P = (int)((mk + rw - 1) / rw);
        e = hipLaunchCooperativeKernel((const void*)panel_qr_kernel<TS>, dim3(a.P), dim3(256), kargs,
                                       (unsigned)panel_lds_bytes(nbp, rw), s);
        if (e != hipSuccess) return e;
    }
    *base += (uint64_t)a.P * (uint64_t)nbp;
    *col_base += (uint64_t)nbp;
    return hipSuccess;
}


hipError_t panel_set_max_lds(size_t bytes)
{
    const void* k[4] = {(const void*)panel_qr_kernel<double>, (const void*)panel_qr_kernel<float>,
                        (const void*)panel_cqr_kernel<double>, (const void*)panel_cqr_kernel<float>};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    g_lds_max = bytes;
    return hipSuccess;
}

// Workgroups of a panel kernel (at `shmem` bytes of LDS) that one compute
// unit holds at once: the smallest over both forms and storage types.
hipError_t panel_max_active(int* per_cu, size_t shmem)
{
    // both panel forms, both storage types: the smallest residency of the
    // kernels a factorization may launch with this LDS size
    const void* k[4] = {(const void*)panel_qr_kernel<float>, (const void*)panel_qr_kernel<double>,
                        (const void*)panel_cqr_kernel<float>, (const void*)panel_cqr_kernel<double>};
    int lo = 1 << 30;
    for (const void* f : k) {
        int a = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f, 256, shmem);
        if (e != hipSuccess) return e;
        if (a < lo) lo = a;
    }
    *per_cu = lo;
    return hipSuccess;
}

template hipError_t launch_panel<double>(double*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                         double*, uint64_t*, uint64_t*, uint64_t*, uint64_t*, int64_t*, int64_t,
                                         int32_t*, hipStream_t);
template hipError_t launch_panel<float>(float*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                        double*, uint64_t*, uint64_t*, uint64_t*, uint64_t*, int64_t*, int64_t,
                                        int32_t*, hipStream_t);

// Empty every polled word (before the first panel of a factorization): the
// column-wise path's two result slots, and all of the two-reduction path's
// scratch.
__global__ void __launch_bounds__(256) panel_reset_kernel(double* part, double* gpart)
{
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e < 128) ((uint64_t*)(part + kPartRes))[e] = kEmpty;
    for (size_t i = e; i < kCqWords; i += (size_t)gridDim.x * 256) ((uint64_t*)gpart)[i] = kEmpty;
}

hipError_t panel_reset(double* part, double* gpart, hipStream_t s)
{
    hipLaunchKernelGGL(panel_reset_kernel, dim3(256), dim3(256), 0, s, part, gpart);
    return hipGetLastError();
}

}  // namespace ctqr
