// Householder panel factorization (Eq. (qr), the geqrf step of Sec. 2.1) of
// an mk x nbp column panel, nbp <= 32, as ONE cooperative launch.
//
// The panel is spread over P workgroups by rows; each holds its rows in LDS
// as FP64 for the whole panel.  Column j needs, after all earlier reflectors,
//   s_c = sum_{i>j} a_ij a_ic  (c >= j)   and the pivot row a_jc,
// from which every workgroup derives, redundantly and identically,
//   sigma = sqrt(a_jj^2 + s_j), beta = -sign(a_jj) sigma, tau = (beta-a_jj)/beta,
//   v_i = a_ij / (a_jj - beta) (i > j), w_c = tau (a_jc + s_c / (a_jj - beta)),
// and applies H_j = I - tau v v^T to its own rows: a_ic -= w_c v_i.  So one
// cross-workgroup reduction (of the Gram row s and the pivot row) per column
// is the only synchronisation; norms, tau and the reflector scaling are FP64
// whatever the storage type.  Partials are summed in a fixed order, so the
// result is bitwise reproducible.
//
// After the last column each workgroup writes its rows back (rounded to the
// storage type) and its share of the Gram matrix V^T V of the stored
// reflectors; workgroup 0 then forms the compact-WY factor T in LDS
// (Schreiber & Van Loan 1989): T_jj = tau_j, T[0:j, j] = -tau_j T[0:j,0:j] (V^T v_j)[0:j],
// so that H_0 H_1 ... H_{nbp-1} = I - V T V^T.
#include "ct_internal.h"
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
    double* part;       // [2][P][64] per-column partials (double buffered)
    double* gpart;      // [P][32*32] Gram partials
    uint64_t* counter;  // barrier arrival counter (monotone)
    uint64_t base;      // arrivals before this launch
    int64_t* info;      // first zero-norm column + 1 (0: none so far)
    int64_t col0;       // global index of the panel's first column
    int32_t* err;
};

__device__ __forceinline__ void grid_arrive_wait(uint64_t* counter, uint64_t target, int32_t* err)
{
    // caller: thread 0 only, after its release fence
    __hip_atomic_fetch_add(counter, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit) {
            atomicOr(err, 1);
            break;
        }
    }
}

template <typename TS>
__global__ void __launch_bounds__(256) panel_qr_kernel(PanelArgs<TS> a)
{
    extern __shared__ double lds[];
    const int t = threadIdx.x, w = blockIdx.x;
    const int nbp = a.nbp, rw = a.rw;
    double* pan = lds;                  // pan[c * rw + r]
    double* red = lds + (size_t)nbp * rw;  // 256
    double* vec = red + 256;            // 64: s_c then pivot row
    double* wv = vec + 64;              // 32
    double* sc = wv + 32;               // 4 scalars
    const int64_t r0 = (int64_t)w * rw;
    const int rows = (int)((a.mk - r0) < (int64_t)rw ? (a.mk - r0) : (int64_t)rw);

    for (int c = 0; c < nbp; ++c)
        for (int r = t; r < rows; r += 256) pan[c * rw + r] = (double)a.A[(r0 + r) + (int64_t)c * a.lda];
    __syncthreads();

    uint64_t target = a.base;
    for (int j = 0; j < nbp; ++j) {
        // (1) this workgroup's partial Gram row and pivot row
        {
            const int c = t & 31, g = t >> 5;
            double s = 0.0;
            if (c >= j && c < nbp) {
                int rs = (int)((int64_t)j + 1 - r0);
                if (rs < 0) rs = 0;
                const double* pj = pan + j * rw;
                const double* pc = pan + c * rw;
                for (int r = rs + g; r < rows; r += 8) s += pj[r] * pc[r];
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
        target += (uint64_t)a.P;
        if (t == 0) grid_arrive_wait(a.counter, target, a.err);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // (2) sum the P partials in a fixed order
        {
            const int v = t & 63, g = t >> 6;
            const int c = v & 31;
            double s = 0.0;
            if (c >= j && c < nbp) {
                // eight independent chains so the loads are all in flight together
                const double* base = a.part + (size_t)(j & 1) * a.P * 64 + v;
                double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
                int q = g;
                for (; q + 28 < a.P; q += 32) {
                    s0 += base[(size_t)q * 64];
                    s1 += base[(size_t)(q + 4) * 64];
                    s2 += base[(size_t)(q + 8) * 64];
                    s3 += base[(size_t)(q + 12) * 64];
                    s4 += base[(size_t)(q + 16) * 64];
                    s5 += base[(size_t)(q + 20) * 64];
                    s6 += base[(size_t)(q + 24) * 64];
                    s7 += base[(size_t)(q + 28) * 64];
                }
                for (; q < a.P; q += 4) s0 += base[(size_t)q * 64];
                s = ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
            }
            red[g * 64 + v] = s;
        }
        __syncthreads();
        if (t < 64) vec[t] = ((red[t] + red[64 + t]) + red[128 + t]) + red[192 + t];
        __syncthreads();
        // (3) the reflector
        if (t == 0) {
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
            sc[0] = scl;
            sc[1] = beta;
            sc[2] = tau;
            sc[3] = sigma == 0.0 ? 1.0 : 0.0;
            if (w == 0) {
                a.tau[j] = tau;
                if (sigma == 0.0 && *a.info == 0) *a.info = a.col0 + j + 1;
            }
        }
        __syncthreads();
        if (t < 32) {
            const int c = t;
            wv[c] = (c > j && c < nbp) ? sc[2] * (vec[32 + c] + sc[0] * vec[c]) : 0.0;
        }
        __syncthreads();
        // (4) apply H_j to this workgroup's rows
        if (sc[3] == 0.0) {
            const double scl = sc[0], beta = sc[1];
            for (int r = t; r < rows; r += 256) {
                const int64_t gr = r0 + r;
                if (gr < j) continue;
                if (gr == j) {
                    pan[j * rw + r] = beta;
                    for (int c = j + 1; c < nbp; ++c) pan[c * rw + r] -= wv[c];
                } else {
                    const double v = pan[j * rw + r] * scl;
                    pan[j * rw + r] = v;
                    for (int c = j + 1; c < nbp; ++c) pan[c * rw + r] -= wv[c] * v;
                }
            }
        }
        __syncthreads();
    }

    // write back, rounding to the storage type; keep the rounded values for the Gram
    for (int c = 0; c < nbp; ++c)
        for (int r = t; r < rows; r += 256) {
            const TS v = (TS)pan[c * rw + r];
            a.A[(r0 + r) + (int64_t)c * a.lda] = v;
            pan[c * rw + r] = (double)v;
        }
    __syncthreads();

    // partial Gram of the unit-lower reflector block: G[p][q] = v_p^T v_q, p < q
    {
        const int p = t & 31, qg = t >> 5;
        for (int q = qg; q < kPanelMax; q += 8) {
            double s = 0.0;
            if (p < q && q < nbp) {
                for (int r = 0; r < rows; ++r) {
                    const int64_t gr = r0 + r;
                    if (gr < p) continue;   // v_p is zero above row p
                    const double vp = gr == p ? 1.0 : pan[p * rw + r];
                    const double vq = gr < q ? 0.0 : (gr == q ? 1.0 : pan[q * rw + r]);
                    s += vp * vq;
                }
            }
            a.gpart[(size_t)w * (kPanelMax * kPanelMax) + q * kPanelMax + p] = s;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    target += (uint64_t)a.P;
    if (t == 0) grid_arrive_wait(a.counter, target, a.err);
    __syncthreads();
    if (w != 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    double* G = lds;                        // 32 x 32, G[q * 32 + p]
    double* T = lds + kPanelMax * kPanelMax;  // 32 x 32, T[q * 32 + p]
    for (int e = t; e < kPanelMax * kPanelMax; e += 256) {
        const double* gp = a.gpart + e;
        const size_t st = kPanelMax * kPanelMax;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int q = 0;
        for (; q + 3 < a.P; q += 4) {
            s0 += gp[(size_t)q * st];
            s1 += gp[(size_t)(q + 1) * st];
            s2 += gp[(size_t)(q + 2) * st];
            s3 += gp[(size_t)(q + 3) * st];
        }
        for (; q < a.P; ++q) s0 += gp[(size_t)q * st];
        G[e] = (s0 + s1) + (s2 + s3);
        T[e] = 0.0;
    }
    __syncthreads();
    for (int q = 0; q < nbp; ++q) {
        // T[p][q] = -tau_q sum_{l=p}^{q-1} T[p][l] G[l][q]
        const double tq = a.tau[q];
        if (t < q) {
            double s = 0.0;
            for (int l = t; l < q; ++l) s += T[l * kPanelMax + t] * G[q * kPanelMax + l];
            T[q * kPanelMax + t] = -tq * s;
        } else if (t == q) {
            T[q * kPanelMax + q] = tq;
        }
        __syncthreads();
    }
    for (int e = t; e < nbp * nbp; e += 256) {
        const int q = e / nbp, p = e - q * nbp;
        a.T[p + (int64_t)q * a.ldt] = p <= q ? T[q * kPanelMax + p] : 0.0;
    }
}

// --------------------------------------------------------------- launcher
// LDS: the panel plus the reduction scratch, and at least room for the two
// 32 x 32 FP64 matrices (G, T) of the final phase.
size_t panel_lds_bytes(int nbp, int rw)
{
    size_t words = (size_t)nbp * rw + 256 + 64 + 32 + 4;
    if (words < 2 * kPanelMax * kPanelMax) words = 2 * kPanelMax * kPanelMax;
    return words * sizeof(double);
}

template <typename TS>
hipError_t launch_panel(TS* A, int64_t lda, int64_t mk, int nbp, int rw, double* tau, double* T, int64_t ldt,
                        double* part, double* gpart, uint64_t* counter, uint64_t* base, int64_t* info,
                        int64_t col0, int32_t* err, hipStream_t s)
{
    PanelArgs<TS> a;
    a.A = A; a.lda = lda; a.mk = mk; a.nbp = nbp; a.rw = rw;
    a.P = (int)((mk + rw - 1) / rw);
    a.tau = tau; a.T = T; a.ldt = ldt; a.part = part; a.gpart = gpart;
    a.counter = counter; a.base = *base; a.info = info; a.col0 = col0; a.err = err;
    const size_t shmem = panel_lds_bytes(nbp, rw);
    hipLaunchKernelGGL(panel_qr_kernel<TS>, dim3(a.P), dim3(256), shmem, s, a);
    *base += (uint64_t)a.P * (uint64_t)(nbp + 1);
    return hipGetLastError();
}


hipError_t panel_set_max_lds(size_t bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)panel_qr_kernel<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)panel_qr_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t panel_max_active(int* per_cu, size_t shmem)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)panel_qr_kernel<float>, 256, shmem);
}

template hipError_t launch_panel<double>(double*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                         double*, uint64_t*, uint64_t*, int64_t*, int64_t, int32_t*, hipStream_t);
template hipError_t launch_panel<float>(float*, int64_t, int64_t, int, int, double*, double*, int64_t, double*,
                                        double*, uint64_t*, uint64_t*, int64_t*, int64_t, int32_t*, hipStream_t);

}  // namespace ctqr
