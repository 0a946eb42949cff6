// Block-reflector application C <- (I - V op(T) V^T) C on the MFMA units:
//   W_z = V^T C      over row slice z  (gemm_tn: both operands K-contiguous)
//   W'  = op(T) sum_z W_z             (tw_kernel, fixed-order split-K sum)
//   C  -= V W'                         (gemm_nn_sub)
// This is the trailing-matrix update of the blocked Householder QR (Eq. (qr))
// and, applied to a block of sinograms, the Q^T B of Eq. (solve).  The same
// two GEMM kernels also serve the triangular solves (R blocks instead of V)
// and the Gram matrices V^T V that build the compact-WY factors.
//
// Each wavefront owns a (16*MB) x (16*NB) output tile built from 16x16 MFMA
// blocks; the workgroup is WM x WN wavefronts.  Fragments are read straight
// from global memory (the caches supply the reuse between the wavefronts of
// a workgroup): along K each lane owns KS consecutive elements, so every
// fragment load is one contiguous vector load.
#include "ct_internal.h"

namespace ctqr {

template <int MODE> struct ModeTraits;
template <> struct ModeTraits<M_F64> { typedef double E; typedef d4_t Acc; static constexpr int KS = 4; };
template <> struct ModeTraits<M_F32> { typedef float E; typedef f4_t Acc; static constexpr int KS = 4; };
template <> struct ModeTraits<M_BF16> { typedef float E; typedef f4_t Acc; static constexpr int KS = 16; };
template <> struct ModeTraits<M_F16> { typedef float E; typedef f4_t Acc; static constexpr int KS = 16; };
template <> struct ModeTraits<M_BF16X3> { typedef float E; typedef f4_t Acc; static constexpr int KS = 16; };

// KS consecutive elements p[0..KS) converted to E; only the first `valid` are read.
template <typename E, typename T, int KS>
__device__ __forceinline__ void load_run(const T* __restrict__ p, int valid, E (&out)[KS])
{
    if (valid >= KS) {
        if constexpr (sizeof(T) * KS % 16 == 0) {
            constexpr int NV = sizeof(T) * KS / 16;
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            u4 raw[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) raw[v] = ((const u4*)p)[v];
            const T* e = (const T*)raw;
#pragma unroll
            for (int s = 0; s < KS; ++s) out[s] = (E)e[s];
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s) out[s] = (E)p[s];
        }
    } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) out[s] = s < valid ? (E)p[s] : (E)0;
    }
}

template <int MODE>
__device__ __forceinline__ void mfma_step(typename ModeTraits<MODE>::Acc& acc,
                                          const typename ModeTraits<MODE>::E (&a)[ModeTraits<MODE>::KS],
                                          const typename ModeTraits<MODE>::E (&b)[ModeTraits<MODE>::KS])
{
    if constexpr (MODE == M_F64) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
    } else if constexpr (MODE == M_F32) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
    } else if constexpr (MODE == M_BF16) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf8_t x, y;
#pragma unroll
            for (int e = 0; e < 8; ++e) { x[e] = (__bf16)a[8 * h + e]; y[e] = (__bf16)b[8 * h + e]; }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc, 0, 0, 0);
        }
    } else if constexpr (MODE == M_F16) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            h8_t x, y;
#pragma unroll
            for (int e = 0; e < 8; ++e) { x[e] = (_Float16)a[8 * h + e]; y[e] = (_Float16)b[8 * h + e]; }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc, 0, 0, 0);
        }
    } else {  // M_BF16X3
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf8_t xh, xl, yh, yl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float av = a[8 * h + e], bv = b[8 * h + e];
                xh[e] = (__bf16)av;
                xl[e] = (__bf16)(av - (float)xh[e]);
                yh[e] = (__bf16)bv;
                yl[e] = (__bf16)(bv - (float)yh[e]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// gemm_tn: W[z][i + j*ldw] = sum_{k in slice z} opA(k, i) opB(k, j)
//   opA(k, i) = A[k + i*lda], opB(k, j) = B[k + j*ldb]; with MASKA (MASKB) the
//   operand is read as a unit-lower-trapezoidal reflector block: 0 for k < i,
//   1 for k == i.  i < M, j < N, k < K.
// ---------------------------------------------------------------------------
struct TnArgs {
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    void* W;
    int64_t ldw, wstride;
    int M, N;
    int64_t K, kslice;
};

template <int MODE, typename TA, typename TB, typename TW, bool MASKA, bool MASKB, int MB, int NB, int WM, int WN>
__global__ void __launch_bounds__(256) gemm_tn_kernel(TnArgs args)
{
    typedef ModeTraits<MODE> Tr;
    typedef typename Tr::E E;
    typedef typename Tr::Acc Acc;
    constexpr int KS = Tr::KS, KC = 4 * KS;
    const TA* __restrict__ A = (const TA*)args.A;
    const TB* __restrict__ B = (const TB*)args.B;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int wm = wv / WN, wn = wv % WN;
    const int i0 = (blockIdx.y * WM + wm) * 16 * MB;
    const int j0 = (blockIdx.x * WN + wn) * 16 * NB;
    const int64_t kbeg = (int64_t)blockIdx.z * args.kslice;
    int64_t kend = kbeg + args.kslice;
    if (kend > args.K) kend = args.K;

    Acc acc[MB][NB];
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) acc[bi][bj] = Acc{0, 0, 0, 0};

    if (i0 < args.M && j0 < args.N) {
        for (int64_t k = kbeg; k < kend; k += KC) {
            const int64_t kl = k + KS * g;            // first k of this lane
            const int valid = (int)(kend - kl < KS ? (kend - kl > 0 ? kend - kl : 0) : KS);
            E a[MB][KS], b[NB][KS];
#pragma unroll
            for (int bi = 0; bi < MB; ++bi) {
                const int i = i0 + 16 * bi + c;
                if (i < args.M) load_run<E, TA, KS>(A + kl + (int64_t)i * args.lda, valid, a[bi]);
                else
#pragma unroll
                    for (int s = 0; s < KS; ++s) a[bi][s] = (E)0;
                if (MASKA && k < i0 + 16 * MB) {
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const int64_t kk = kl + s;
                        if (kk < i) a[bi][s] = (E)0;
                        else if (kk == i) a[bi][s] = (E)1;
                    }
                }
            }
#pragma unroll
            for (int bj = 0; bj < NB; ++bj) {
                const int j = j0 + 16 * bj + c;
                if (j < args.N) load_run<E, TB, KS>(B + kl + (int64_t)j * args.ldb, valid, b[bj]);
                else
#pragma unroll
                    for (int s = 0; s < KS; ++s) b[bj][s] = (E)0;
                if (MASKB && k < j0 + 16 * NB) {
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const int64_t kk = kl + s;
                        if (kk < j) b[bj][s] = (E)0;
                        else if (kk == j) b[bj][s] = (E)1;
                    }
                }
            }
#pragma unroll
            for (int bi = 0; bi < MB; ++bi)
#pragma unroll
                for (int bj = 0; bj < NB; ++bj) mfma_step<MODE>(acc[bi][bj], a[bi], b[bj]);
        }
    }
    TW* W = (TW*)args.W + (int64_t)blockIdx.z * args.wstride;
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) {
            const int j = j0 + 16 * bj + c;
            if (j >= args.N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 16 * bi + d_row(MODE, g, q);
                if (i < args.M) W[i + (int64_t)j * args.ldw] = (TW)acc[bi][bj][q];
            }
        }
}

// ---------------------------------------------------------------------------
// gemm_nn_sub: C[r + j*ldc] -= sum_k opA(r, k) Bw(k, j)
//   opA(r, k) = A[r + k*lda] (MASKA: 0 for r < k, 1 for r == k)
//   Bw(k, j)  = Bhi[k + j*ldb]
//   r < M, j < N, k < K.
// ---------------------------------------------------------------------------
struct NnArgs {
    const void* A;
    int64_t lda;
    const void* Bhi;
    const void* Blo;
    int64_t ldb;
    void* C;
    int64_t ldc;
    int64_t M;
    int N, K;
    const int32_t* desc;   // batch descriptor: columns of Bhi and C start at its offset
};

template <int MODE, typename TA, typename TB, typename TC, bool MASKA, int MB, int NB, int WM, int WN>
__global__ void __launch_bounds__(256) gemm_nn_sub_kernel(NnArgs args)
{
    typedef ModeTraits<MODE> Tr;
    typedef typename Tr::E E;
    typedef typename Tr::Acc Acc;
    constexpr int KS = Tr::KS, KC = 4 * KS;
    const TA* __restrict__ A = (const TA*)args.A;
    const int doff = desc_offset(args.desc);
    const int Ne = desc_count(args.desc, args.N);
    const TB* __restrict__ Bh = (const TB*)args.Bhi + (int64_t)doff * args.ldb;
    TC* __restrict__ C = (TC*)args.C + (int64_t)doff * args.ldc;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int wm = wv / WN, wn = wv % WN;
    const int64_t r0 = ((int64_t)blockIdx.x * WM + wm) * 16 * MB;
    const int j0 = (blockIdx.y * WN + wn) * 16 * NB;
    if (r0 >= args.M || j0 >= Ne) return;

    Acc acc[MB][NB];
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) acc[bi][bj] = Acc{0, 0, 0, 0};

    for (int k = 0; k < args.K; k += KC) {
        const int kl = k + KS * g;
        const int valid = args.K - kl < KS ? (args.K - kl > 0 ? args.K - kl : 0) : KS;
        E a[MB][KS], b[NB][KS];
#pragma unroll
        for (int bi = 0; bi < MB; ++bi) {
            const int64_t r = r0 + 16 * bi + c;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                E v = (E)0;
                if (r < args.M && s < valid) v = (E)A[r + (int64_t)(kl + s) * args.lda];
                if (MASKA) {
                    if (r < kl + s) v = (E)0;
                    else if (r == kl + s) v = (E)1;
                }
                a[bi][s] = v;
            }
        }
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) {
            const int j = j0 + 16 * bj + c;
            if (j < Ne) {
                load_run<E, TB, KS>(Bh + kl + (int64_t)j * args.ldb, valid, b[bj]);
            } else {
#pragma unroll
                for (int s = 0; s < KS; ++s) b[bj][s] = (E)0;
            }
        }
#pragma unroll
        for (int bi = 0; bi < MB; ++bi)
#pragma unroll
            for (int bj = 0; bj < NB; ++bj) mfma_step<MODE>(acc[bi][bj], a[bi], b[bj]);
    }
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) {
            const int j = j0 + 16 * bj + c;
            if (j >= Ne) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + 16 * bi + d_row(MODE, g, q);
                if (r < args.M) {
                    TC* p = C + r + (int64_t)j * args.ldc;
                    *p = (TC)((E)*p - (E)acc[bi][bj][q]);
                }
            }
        }
}

// ---------------------------------------------------------------------------
// tw_kernel: combine the split-K partials of W (nbv x N, ld nbv, nz slices)
//   OP 0: out = T^T W      OP 1: out = T W      (T upper triangular, FP64)
//   OP 2: out = W (FP64 sum only)
//   OP 3: out(i, j) -= W(i, j) into a storage-typed matrix (ld ldo)
// Output element type TO (the element type of the consuming GEMM).
// One workgroup per 16 columns; the summed tile sits in LDS as FP64.
// ---------------------------------------------------------------------------
template <typename TWp, typename TO, int OP, bool SPLIT>
__global__ void __launch_bounds__(256) tw_kernel(const TWp* __restrict__ Wp, int64_t wstride, int nz, int nbv, int N,
                                                 const double* __restrict__ T, int64_t ldt, TO* out, TO* out_lo,
                                                 int64_t ldo, const int32_t* desc)
{
    extern __shared__ double sw[];   // nbv x 16
    N = desc_count(desc, N);
    const int j0 = blockIdx.x * 16;
    if (j0 >= N) return;
    const int t = threadIdx.x;
    const int ncol = N - j0 < 16 ? N - j0 : 16;
    for (int e = t; e < nbv * 16; e += 256) {
        const int jj = e / nbv, i = e - jj * nbv;
        double s = 0.0;
        if (jj < ncol)
            for (int z = 0; z < nz; ++z) s += (double)Wp[(int64_t)z * wstride + i + (int64_t)(j0 + jj) * nbv];
        sw[jj * nbv + i] = s;
    }
    __syncthreads();
    for (int e = t; e < nbv * 16; e += 256) {
        const int jj = e / nbv, i = e - jj * nbv;
        if (jj >= ncol) continue;
        double y;
        if (OP == 0) {
            y = 0.0;
            const double* tc = T + (int64_t)i * ldt;           // column i of T, rows 0..i
            for (int l = 0; l <= i; ++l) y += tc[l] * sw[jj * nbv + l];
        } else if (OP == 1) {
            y = 0.0;
            for (int l = i; l < nbv; ++l) y += T[i + (int64_t)l * ldt] * sw[jj * nbv + l];
        } else {
            y = sw[jj * nbv + i];
        }
        TO* p = out + i + (int64_t)(j0 + jj) * ldo;
        if (OP == 3) {
            *p = (TO)((double)*p - y);
        } else if (SPLIT) {
            const TO h = (TO)(float)y;
            *p = h;
            out_lo[i + (int64_t)(j0 + jj) * ldo] = (TO)((float)y - (float)h);
        } else {
            *p = (TO)y;
        }
    }
}

// ---------------------------------------------------------------------------
// Compact-WY factor of an outer reflector block from the factors of its
// panels.  For consecutive groups of reflectors V = [V1 V2] with factors T1,
// T2 (H1 H2 = I - V T V^T):
//   T = [ T1   -T1 (V1^T V2) T2 ]
//       [ 0     T2              ]
// The panels leave their factors on T's diagonal (width s); one level joins
// adjacent groups [a, a + s) and [a + s, c), pair i = blockIdx.y, a = 2 s i,
// using the block's Gram matrix G = V^T V for V1^T V2.
// STEP 0: M_i = G12 T2 (T2 upper triangular); STEP 1: T12 = -T1 M_i.
// One output per thread.
// ---------------------------------------------------------------------------
template <int STEP>
__global__ void __launch_bounds__(256) t_join_kernel(const double* __restrict__ G, int64_t ldg, double* T,
                                                     int64_t ldt, double* M, int sz, int bo)
{
    const int a = 2 * sz * blockIdx.y, b = a + sz;
    const int c = a + 2 * sz < bo ? a + 2 * sz : bo;
    const int n1 = sz, n2 = c - b;
    if (n2 <= 0) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n1 * n2) return;
    const int r = e % n1, q = e / n1;
    double* Mi = M + (size_t)blockIdx.y * sz * sz;          // n1 x n2, ld n1
    double s0 = 0.0, s1 = 0.0;
    if (STEP == 0) {
        // M[r][q] = sum_{l <= q} G[a + r][b + l] T[b + l][b + q]
        const double* g = G + (a + r) + (int64_t)b * ldg;
        const double* t2 = T + b + (int64_t)(b + q) * ldt;
        int l = 0;
        for (; l + 1 <= q; l += 2) {
            s0 += g[(int64_t)l * ldg] * t2[l];
            s1 += g[(int64_t)(l + 1) * ldg] * t2[l + 1];
        }
        if (l <= q) s0 += g[(int64_t)l * ldg] * t2[l];
        Mi[r + q * n1] = s0 + s1;
    } else {
        // T[a + r][b + q] = -sum_{l >= r} T[a + r][a + l] M[l][q]
        const double* t1 = T + (a + r) + (int64_t)a * ldt;
        const double* mq = Mi + (size_t)q * n1;
        int l = r;
        for (; l + 1 < n1; l += 2) {
            s0 += t1[(int64_t)l * ldt] * mq[l];
            s1 += t1[(int64_t)(l + 1) * ldt] * mq[l + 1];
        }
        if (l < n1) s0 += t1[(int64_t)l * ldt] * mq[l];
        T[(a + r) + (int64_t)(b + q) * ldt] = -(s0 + s1);
    }
}

// T[p][q] = 0 for p > q (n x n)
__global__ void __launch_bounds__(256) tril_zero_kernel(double* T, int64_t ldt, int n)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n * n) return;
    const int p = e % n, q = e / n;
    if (p > q) T[p + (int64_t)q * ldt] = 0.0;
}

hipError_t launch_t_join(const double* G, int64_t ldg, double* T, int64_t ldt, double* M, int nb_panel, int bo,
                         hipStream_t s)
{
    hipLaunchKernelGGL(tril_zero_kernel, dim3((unsigned)((bo * bo + 255) / 256)), dim3(256), 0, s, T, ldt, bo);
    for (int sz = nb_panel; sz < bo; sz *= 2) {
        const dim3 grid((unsigned)((sz * sz + 255) / 256), (unsigned)((bo + 2 * sz - 1) / (2 * sz)));
        hipLaunchKernelGGL((t_join_kernel<0>), grid, dim3(256), 0, s, G, ldg, T, ldt, M, sz, bo);
        hipLaunchKernelGGL((t_join_kernel<1>), grid, dim3(256), 0, s, G, ldg, T, ldt, M, sz, bo);
    }
    return hipGetLastError();
}

// S[e] = sum_z W[z][e] over `count` contiguous elements (fixed order in z);
// with a descriptor, count = per_col * (batch column count).
template <typename TWp, typename TS>
__global__ void __launch_bounds__(256) sum_slices_kernel(const TWp* __restrict__ Wp, int64_t wstride, int nz,
                                                         int64_t count, TS* __restrict__ S, const int32_t* desc,
                                                         int per_col)
{
    if (desc) count = (int64_t)per_col * desc_count(desc, (int)(count / per_col));
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int z = 0; z < nz; ++z) s += (double)Wp[(int64_t)z * wstride + e];
        S[e] = (TS)s;
    }
}

// The same sum for a small output (a few slices' worth of columns): 64
// elements a workgroup, its four wavefronts summing every fourth slice, the
// four partial sums added in a fixed order (four times the workgroups, a
// quarter of the dependent loads a thread).
template <typename TWp, typename TS>
__global__ void __launch_bounds__(256) sum_slices4_kernel(const TWp* __restrict__ Wp, int64_t wstride, int nz,
                                                          int64_t count, TS* __restrict__ S, const int32_t* desc,
                                                          int per_col)
{
    __shared__ double red[4][64];
    if (desc) count = (int64_t)per_col * desc_count(desc, (int)(count / per_col));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (e < count) {
#pragma unroll 8
        for (int z = wv; z < nz; z += 4) s += (double)Wp[(int64_t)z * wstride + e];
    }
    red[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && e < count) S[e] = (TS)(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

// ------------------------------------------------------------------ launchers
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <int MODE, typename TA, typename TB, typename TW, bool MA, bool MB_>
static hipError_t tn_dispatch(const TnArgs& a, int nz, hipStream_t s)
{
    if (a.M <= 32) {
        dim3 grid(cdiv(a.N, 16 * 4 * 4), cdiv(a.M, 32), nz);
        hipLaunchKernelGGL((gemm_tn_kernel<MODE, TA, TB, TW, MA, MB_, 2, 4, 1, 4>), grid, dim3(256), 0, s, a);
    } else {
        dim3 grid(cdiv(a.N, 16 * 4 * 2), cdiv(a.M, 16 * 4 * 2), nz);
        hipLaunchKernelGGL((gemm_tn_kernel<MODE, TA, TB, TW, MA, MB_, 4, 4, 2, 2>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// Split-K plan: enough workgroups to fill the chip, slices a multiple of kc.
static inline void plan_split(int64_t K, int tiles, int kc, int* nz, int64_t* kslice)
{
    int z = 1;
    const int target = 1024;
    while (tiles * z * 2 <= target && K / (z * 2) >= 4 * kc && z < 256) z *= 2;
    int64_t ks = (K + z - 1) / z;
    ks = (ks + kc - 1) / kc * kc;
    *nz = (int)((K + ks - 1) / ks);
    *kslice = ks;
}

int tn_tiles(int M, int N) { return M <= 32 ? cdiv(N, 256) * cdiv(M, 32) : cdiv(N, 128) * cdiv(M, 128); }

// W partials of opA^T opB; returns the number of slices in *nz_out.
template <int MODE, typename TA, typename TB, typename TW, bool MA, bool MB_>
hipError_t launch_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, TW* W, int M, int N, int64_t K,
                     int64_t wcap, int* nz_out, hipStream_t s)
{
    TnArgs a;
    a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.W = W; a.ldw = M; a.wstride = (int64_t)M * N;
    a.M = M; a.N = N; a.K = K;
    int nz;
    int64_t ks;
    plan_split(K, tn_tiles(M, N), 4 * ModeTraits<MODE>::KS, &nz, &ks);
    while (nz > 1 && (int64_t)nz * M * N > wcap) {
        ks *= 2;
        nz = (int)((K + ks - 1) / ks);
    }
    a.kslice = ks;
    *nz_out = nz;
    return tn_dispatch<MODE, TA, TB, TW, MA, MB_>(a, nz, s);
}

template <int MODE, typename TA, typename TB, typename TC, bool MA>
hipError_t launch_nn_sub(const TA* A, int64_t lda, const TB* Bhi, const TB* Blo, int64_t ldb, TC* C, int64_t ldc,
                         int64_t M, int N, int K, hipStream_t s, const int32_t* desc)
{
    NnArgs a;
    a.A = A; a.lda = lda; a.Bhi = Bhi; a.Blo = Blo; a.ldb = ldb; a.C = C; a.ldc = ldc; a.M = M; a.N = N; a.K = K;
    a.desc = desc;
    if (N <= 64) {
        dim3 grid(cdiv(M, 16 * 4 * 4), cdiv(N, 64), 1);
        hipLaunchKernelGGL((gemm_nn_sub_kernel<MODE, TA, TB, TC, MA, 4, 4, 4, 1>), grid, dim3(256), 0, s, a);
    } else {
        dim3 grid(cdiv(M, 16 * 4 * 2), cdiv(N, 16 * 4 * 2), 1);
        hipLaunchKernelGGL((gemm_nn_sub_kernel<MODE, TA, TB, TC, MA, 4, 4, 2, 2>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <typename TWp, typename TO, int OP, bool SPLIT>
hipError_t launch_tw(const TWp* Wp, int nz, int nbv, int N, const double* T, int64_t ldt, TO* out, TO* out_lo,
                     int64_t ldo, hipStream_t s, const int32_t* desc)
{
    const size_t sh = (size_t)nbv * 16 * sizeof(double);
    hipLaunchKernelGGL((tw_kernel<TWp, TO, OP, SPLIT>), dim3(cdiv(N, 16)), dim3(256), sh, s, Wp, (int64_t)nbv * N,
                       nz, nbv, N, T, ldt, out, out_lo, ldo, desc);
    return hipGetLastError();
}

template <typename TWp, typename TS>
hipError_t launch_sum_slices(const TWp* Wp, int64_t wstride, int nz, int64_t count, TS* S, hipStream_t s,
                             const int32_t* desc, int per_col)
{
    if (count <= 65536 && nz >= 8) {
        // few outputs, many slices: split the slices over the wavefronts
        hipLaunchKernelGGL((sum_slices4_kernel<TWp, TS>), dim3((unsigned)((count + 63) / 64)), dim3(256), 0, s, Wp,
                           wstride, nz, count, S, desc, per_col > 0 ? per_col : 1);
        return hipGetLastError();
    }
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((sum_slices_kernel<TWp, TS>), dim3((unsigned)blocks), dim3(256), 0, s, Wp, wstride, nz, count,
                       S, desc, per_col > 0 ? per_col : 1);
    return hipGetLastError();
}
template hipError_t launch_sum_slices<float, float>(const float*, int64_t, int, int64_t, float*, hipStream_t,
                                                    const int32_t*, int);
template hipError_t launch_sum_slices<double, double>(const double*, int64_t, int, int64_t, double*, hipStream_t,
                                                      const int32_t*, int);
template hipError_t launch_sum_slices<float, double>(const float*, int64_t, int, int64_t, double*, hipStream_t,
                                                     const int32_t*, int);

// ---------------------------------------------------------- instantiations
#define CT_TN(MODE, TA, TB, TW, MA, MB)                                                                       \
    template hipError_t launch_tn<MODE, TA, TB, TW, MA, MB>(const TA*, int64_t, const TB*, int64_t, TW*, int, \
                                                            int, int64_t, int64_t, int*, hipStream_t);
CT_TN(M_F64, double, double, double, true, false)
CT_TN(M_F64, double, double, double, true, true)
CT_TN(M_F64, double, double, double, false, false)
CT_TN(M_F64, float, float, double, true, true)
CT_TN(M_F32, float, float, float, true, false)
CT_TN(M_F32, float, float, float, false, false)
CT_TN(M_BF16, float, float, float, true, false)
CT_TN(M_F16, float, float, float, true, false)
CT_TN(M_BF16X3, float, float, float, true, false)

#define CT_NN(MODE, TA, TB, TC, MA)                                                                            \
    template hipError_t launch_nn_sub<MODE, TA, TB, TC, MA>(const TA*, int64_t, const TB*, const TB*, int64_t, \
                                                           TC*, int64_t, int64_t, int, int, hipStream_t,       \
                                                           const int32_t*);
CT_NN(M_F64, double, double, double, true)
CT_NN(M_F64, double, double, double, false)
CT_NN(M_F32, float, float, float, true)
CT_NN(M_F32, float, float, float, false)
CT_NN(M_BF16, float, float, float, true)
CT_NN(M_F16, float, float, float, true)
CT_NN(M_BF16X3, float, float, float, true)

#define CT_TW(TWp, TO, OP, SPLIT)                                                                          \
    template hipError_t launch_tw<TWp, TO, OP, SPLIT>(const TWp*, int, int, int, const double*, int64_t, TO*, \
                                                      TO*, int64_t, hipStream_t, const int32_t*);
CT_TW(double, double, 0, false)
CT_TW(double, double, 1, false)
CT_TW(double, double, 2, false)
CT_TW(double, double, 3, false)
CT_TW(float, float, 0, false)
CT_TW(float, float, 1, false)
CT_TW(float, float, 3, false)

}  // namespace ctqr
