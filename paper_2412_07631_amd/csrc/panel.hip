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
};

// Result slots follow the double-buffered partial rows (2 x 256 x 64) in the
// part buffer; an empty slot entry holds this NaN bit pattern.
constexpr size_t kPartRes = (size_t)2 * 256 * 64;
constexpr uint64_t kEmpty = 0x7FF4C0FFEE5107D5ull;

// LDS words besides the panel: red 256, vec 64, wv 32, sc 8, Tl 32*33, gl 32
constexpr int kPanelAux = 256 + 64 + 32 + 8 + kPanelMax * (kPanelMax + 1) + kPanelMax;

template <typename TS>
__global__ void __launch_bounds__(256) panel_qr_kernel(PanelArgs<TS> a)
{
    extern __shared__ double lds[];
    const int t = threadIdx.x, w = blockIdx.x;
    const int nbp = a.nbp, rw = a.rw;
    double* pan = lds;                        // pan[c * rw + r]
    double* red = lds + (size_t)nbp * rw;     // 256
    double* vec = red + 256;                  // 64: s_c then the pivot row
    double* wv = vec + 64;                    // 32
    double* sc = wv + 32;                     // 8 scalars
    double* Tl = sc + 8;                      // 32 x 33 (workgroup 0)
    double* gl = Tl + kPanelMax * (kPanelMax + 1);  // 32
    const int64_t r0 = (int64_t)w * rw;
    const int rows = (int)((a.mk - r0) < (int64_t)rw ? (a.mk - r0) : (int64_t)rw);

    // a wait of an earlier launch gave up: the factorization is already failed
    if (t == 0) sc[5] = (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) ? 1.0 : 0.0;
    __syncthreads();
    if (sc[5] != 0.0) return;
    for (int c = 0; c < nbp; ++c)
        for (int r = t; r < rows; r += 256) pan[c * rw + r] = (double)a.A[(r0 + r) + (int64_t)c * a.lda];
    if (w == 0)
        for (int e = t; e < kPanelMax * (kPanelMax + 1); e += 256) Tl[e] = 0.0;
    __syncthreads();

    uint64_t target = a.base;
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
                // poll this lane's entry; the clock and the error word are read
                // only every 16 polls, so a normal (microsecond) wait costs neither
                uint64_t t0 = 0, bits;
                uint32_t spins = 0;
                while ((bits = __hip_atomic_load(slot + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kEmpty) {
                    if (a.wait_ticks == 0) {
                        __hip_atomic_fetch_or(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        sc[5] = 1.0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    if ((++spins & 15) == 0) {
                        const uint64_t now = __builtin_amdgcn_s_memrealtime();
                        if (spins == 16) {
                            t0 = now;
                        } else if (now - t0 >= a.wait_ticks) {
                            __hip_atomic_fetch_or(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            sc[5] = 1.0;
                            break;
                        }
                        if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) {
                            sc[5] = 1.0;
                            break;
                        }
                    }
                }
                // what the publisher wrote before the slot (the emptied
                // other slot) is visible from here on
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                vec[t] = __builtin_bit_cast(double, bits);
            }
            __syncthreads();
            if (sc[5] != 0.0) return;      // uniform: the whole workgroup leaves
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

    for (int c = 0; c < nbp; ++c)
        for (int r = t; r < rows; r += 256) a.A[(r0 + r) + (int64_t)c * a.lda] = (TS)pan[c * rw + r];
    if (w == 0)
        for (int e = t; e < nbp * nbp; e += 256) {
            const int q = e / nbp, p = e - q * nbp;
            a.T[p + (int64_t)q * a.ldt] = p <= q ? Tl[q * 33 + p] : 0.0;
        }
}

// --------------------------------------------------------------- launcher
static uint64_t g_wait_ticks = kWaitTicks;
void panel_set_wait_limit(int64_t ticks) { g_wait_ticks = ticks < 0 ? kWaitTicks : (uint64_t)ticks; }

// LDS: the panel plus the reduction scratch and the T factor.
size_t panel_lds_bytes(int nbp, int rw) { return ((size_t)nbp * rw + kPanelAux) * sizeof(double); }
int panel_aux_words() { return kPanelAux; }

template <typename TS>
hipError_t launch_panel(TS* A, int64_t lda, int64_t mk, int nbp, int rw, double* tau, double* T, int64_t ldt,
                        double* part, double* gpart, uint64_t* counter, uint64_t* base, uint64_t* col_base,
                        int64_t* info, int64_t col0, int32_t* err, hipStream_t s)
{
    PanelArgs<TS> a;
    a.A = A; a.lda = lda; a.mk = mk; a.nbp = nbp; a.rw = rw;
    a.P = (int)((mk + rw - 1) / rw);
    a.tau = tau; a.T = T; a.ldt = ldt; a.part = part;
    (void)gpart;
    a.counter = counter; a.base = *base; a.info = info; a.col0 = col0; a.err = err;
    a.col_base = *col_base;
    a.wait_ticks = g_wait_ticks;
    const size_t shmem = panel_lds_bytes(nbp, rw);
    hipLaunchKernelGGL(panel_qr_kernel<TS>, dim3(a.P), dim3(256), shmem, s, a);
    *base += (uint64_t)a.P * (uint64_t)nbp;
    *col_base += (uint64_t)nbp;
    return hipGetLastError();
}


hipError_t panel_set_max_lds(size_t bytes)
{
    const void* k[2] = {(const void*)panel_qr_kernel<double>, (const void*)panel_qr_kernel<float>};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t panel_max_active(int* per_cu, size_t shmem)
{
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)panel_qr_kernel<float>, 256, shmem);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)panel_qr_kernel<double>, 256, shmem);
    *per_cu = a < b ? a : b;
    return e;
}

template hipError_t launch_panel<double>(double*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                         double*, uint64_t*, uint64_t*, uint64_t*, int64_t*, int64_t, int32_t*,
                                         hipStream_t);
template hipError_t launch_panel<float>(float*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                        double*, uint64_t*, uint64_t*, uint64_t*, int64_t*, int64_t, int32_t*,
                                        hipStream_t);

// Empty both result slots (before the first panel of a factorization).
__global__ void panel_reset_kernel(double* part)
{
    uint64_t* s = (uint64_t*)(part + kPartRes);
    s[threadIdx.x] = kEmpty;
}

hipError_t panel_reset(double* part, hipStream_t s)
{
    hipLaunchKernelGGL(panel_reset_kernel, dim3(1), dim3(128), 0, s, part);
    return hipGetLastError();
}

}  // namespace ctqr
