// LDS-tiled MFMA kernel for the block-reflector update of the trailing matrix
// (the hot loop of the blocked Householder QR, Eq. (qr)) and of the Q^T B of
// Eq. (solve).  Both products of C <- C - V (op(T) (V^T C)) are written as
//     out[p][q] (+)= sum_k X[p][k] Y[q][k]            ("NT" form)
// with BOTH operands K-contiguous:
//   W  = V^T C :  X = Vm (masked reflector block, column-major: row i of X is
//                 column i of Vm), Y = C (column-major: row j of Y is column j)
//   C -= V W'  :  X = Vt (the same block transposed, row-major mk x nb),
//                 Y = W' (column-major nb x nc)
// so every global load is a 16-byte vector along K, tiles go to LDS without
// transposition, and the MFMA fragments are single ds_read_b128 (FP32) or two
// ds_read_b128 (FP64) per lane.
//
// Workgroup tile BP x BQ = 128 x 128, K step BK, 4 wavefronts in 2 x 2, each
// 64 x 64 (4 x 4 blocks of 16x16 MFMA).  Global->register prefetch of the next
// K step overlaps the MFMAs of the current one (two LDS buffers).  The tile
// order is remapped so the 8 XCDs of MI355X each walk a contiguous range of
// tiles and share their L2.
#include "ct_internal.h"

namespace ctqr {

template <typename T> struct LdsTraits;
template <> struct LdsTraits<double> { static constexpr int BK = 16, PAD = 2, KS = 4; typedef d4_t Acc; };
template <> struct LdsTraits<float> { static constexpr int BK = 32, PAD = 4, KS = 4; typedef f4_t Acc; };

constexpr int kBP = 128, kBQ = 128;

struct NtArgs {
    const void* X;   // BP rows of K-contiguous data, leading dimension ldx
    int64_t ldx;
    const void* Y;
    int64_t ldy;
    void* out;       // column-major P x Q (ld ldo) per split slice
    int64_t ldo, ostride;
    int64_t P;
    int Q;
    int64_t K, kslice;
    int tiles_p, tiles_q;
    int sub;         // 0: out = acc (split slice z at out + z*ostride), 1: out -= acc
    // optional batch record of a graph-captured solve (desc[0] = column
    // offset, desc[1] = column count of the current batch): Q is clipped to
    // the count, and Y (desc_y) or out (desc_out) start at the offset
    const int32_t* desc;
    int desc_y, desc_out;
    // X is a reflector block read in place (column p of the block from its
    // diagonal down): entries above the diagonal read as 0, the diagonal as 1
    int maskx;
    // split operands of the BF16x3 kernel: X / Y hold the bfloat16 high parts
    // and Xlo / Ylo the low parts, same leading dimension
    const void* Xlo;
    const void* Ylo;
    // non-subtracting form only: store element (p, q) at q + p ldo (the
    // transpose; a slice then spans P ldo elements)
    int tout;
    // only tiles that reach the diagonal or above it (a Gram matrix whose
    // lower triangle nobody reads); the others stay unwritten
    int upper;
};

__device__ __forceinline__ void apply_desc(const NtArgs& a, int& Q, const char*& Y, size_t ysz, char*& out, size_t osz)
{
    if (a.desc) {
        const int off = a.desc[0], cnt = a.desc[1];
        if (cnt < Q) Q = cnt;
        if (a.desc_y) Y += (size_t)off * a.ldy * ysz;
        if (a.desc_out) out += (size_t)off * a.ldo * osz;
    }
}

template <typename T>
__device__ __forceinline__ void mfma_nt(typename LdsTraits<T>::Acc& acc, const T (&a)[4], const T (&b)[4])
{
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
    }
}

// one 16-byte vector of T
template <typename T> struct V16;
template <> struct V16<float> { typedef f4_t t; static constexpr int N = 4; };
template <> struct V16<double> { typedef double t __attribute__((ext_vector_type(2))); static constexpr int N = 2; };

// SUB = false: partial products out[z] = X Y^T over K slice z (W = V^T C);
// SUB = true: out -= X Y^T (the rank-nb update C -= V W').
template <typename T, bool SUB, int BQ = kBQ>
__global__ void __launch_bounds__(256, 2) gemm_nt_kernel(NtArgs a)
{
    typedef LdsTraits<T> L;
    constexpr int BK = L::BK, LDK = BK + L::PAD;
    constexpr int VN = V16<T>::N;                  // elements per 16-byte vector
    constexpr int VPR = BK / VN;                   // vectors per tile row
    constexpr int ROWS_PER_PASS = 256 / VPR;       // tile rows loaded per pass of 256 threads
    constexpr int PASSES = kBP / ROWS_PER_PASS;
    constexpr int YPASSES = (BQ + ROWS_PER_PASS - 1) / ROWS_PER_PASS;
    // waves: 2 x 2 of 64 x 64 for the 128-wide tile, else 4 x 1 of 32 x BQ
    constexpr int WM = BQ == 128 ? 2 : 4, WN = 4 / WM;
    constexpr int MI = kBP / (16 * WM), NJ = BQ / (16 * WN);
    typedef typename V16<T>::t vec_t;
    typedef typename L::Acc Acc;

    __shared__ T Xs[2][kBP * LDK];
    __shared__ T Ys[2][BQ * LDK];

    int tp, tq;
    if (!tile_of(blockIdx.x, a.tiles_p, a.tiles_q, tp, tq)) return;
    if (a.upper && (int64_t)tp * kBP >= (int64_t)(tq + 1) * BQ) return;
    const int64_t p0 = (int64_t)tp * kBP;
    const int q0 = tq * BQ;
    const int64_t kbeg = (int64_t)blockIdx.y * a.kslice;
    int64_t kend = kbeg + a.kslice;
    if (kend > a.K) kend = a.K;

    int Qe = a.Q;
    const char* Yc = (const char*)a.Y;
    char* Oc = (char*)a.out;
    apply_desc(a, Qe, Yc, sizeof(T), Oc, sizeof(T));
    if (q0 >= Qe) return;
    const T* __restrict__ X = (const T*)a.X;
    const T* __restrict__ Y = (const T*)Yc;
    const int t = threadIdx.x;
    const int lr = t / VPR, lv = t % VPR;          // loader: row within pass, vector within row

    vec_t xr[PASSES], yr[YPASSES];
    auto gload = [&](int64_t k0) {
        const int64_t kk = k0 + lv * VN;
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int row = ps * ROWS_PER_PASS + lr;
            const int64_t pr = p0 + row;
            vec_t vx = {};
            if (kk + VN <= kend) {
                if (pr < a.P) vx = *(const vec_t*)(X + pr * a.ldx + kk);
            } else {
#pragma unroll
                for (int e = 0; e < VN; ++e)
                    if (kk + e < kend && pr < a.P) vx[e] = X[pr * a.ldx + kk + e];
            }
            if (a.maskx && kk < a.P) {
#pragma unroll
                for (int e = 0; e < VN; ++e) {
                    const int64_t k = kk + e;
                    vx[e] = k > pr ? vx[e] : (k == pr ? (T)1 : (T)0);
                }
            }
            xr[ps] = vx;
        }
#pragma unroll
        for (int ps = 0; ps < YPASSES; ++ps) {
            const int row = ps * ROWS_PER_PASS + lr;
            const int qr = q0 + row;
            vec_t vy = {};
            if (row < BQ) {
                if (kk + VN <= kend) {
                    if (qr < Qe) vy = *(const vec_t*)(Y + (int64_t)qr * a.ldy + kk);
                } else {
#pragma unroll
                    for (int e = 0; e < VN; ++e)
                        if (kk + e < kend && qr < Qe) vy[e] = Y[(int64_t)qr * a.ldy + kk + e];
                }
            }
            yr[ps] = vy;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int row = ps * ROWS_PER_PASS + lr;
            *(vec_t*)&Xs[buf][row * LDK + lv * VN] = xr[ps];
        }
#pragma unroll
        for (int ps = 0; ps < YPASSES; ++ps) {
            const int row = ps * ROWS_PER_PASS + lr;
            if (row < BQ) *(vec_t*)&Ys[buf][row * LDK + lv * VN] = yr[ps];
        }
    };

    const int lane = t & 63, wv = t >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int wp = (wv / WN) * (16 * MI), wq = (wv % WN) * (16 * NJ);

    Acc acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    constexpr bool F64 = sizeof(T) == 8;
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            T bf[NJ][4];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const T* src = &Ys[buf][(wq + 16 * j + c) * LDK + kk + 4 * g];
#pragma unroll
                for (int s = 0; s < 4; ++s) bf[j][s] = src[s];
            }
#pragma unroll
            for (int i = 0; i < MI; ++i) {
                T af[4];
                const T* src = &Xs[buf][(wp + 16 * i + c) * LDK + kk + 4 * g];
#pragma unroll
                for (int s = 0; s < 4; ++s) af[s] = src[s];
#pragma unroll
                for (int j = 0; j < NJ; ++j) mfma_nt<T>(acc[i][j], af, bf[j]);
            }
        }
    };
    // the subtracting epilogue's C tile is fetched during the last K step,
    // when the prefetch registers are free, so its latency hides behind it
    // (FP32 only: the FP64 accumulators already fill the register file)
    constexpr bool PRE = SUB && !F64;
    // FP32 accumulators hold rows 4g..4g+3 of one column: one 16-byte access
    typedef Acc accv_t;
    accv_t cpre[MI][NJ];
    auto load_c = [&]() {
        if constexpr (PRE) {
            const T* O = (const T*)Oc;
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const int q = q0 + wq + 16 * j + c;
                    const int64_t pb = p0 + wp + 16 * i + 4 * g;
                    accv_t v = {0, 0, 0, 0};
                    if (q < Qe) {
                        const T* d = O + pb + (int64_t)q * a.ldo;
                        if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) v = *(const accv_t*)d;
                        else
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (pb + r < a.P) v[r] = d[r];
                    }
                    cpre[i][j] = v;
                }
        }
    };

    if (kbeg < kend) {
        gload(kbeg);
        sstore(0);
        __syncthreads();
        int buf = 0;
        int64_t k0 = kbeg;
        for (; k0 + BK < kend; k0 += BK) {
            gload(k0 + BK);
            compute(buf);
            sstore(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
        if constexpr (SUB) load_c();
        compute(buf);
    } else if constexpr (SUB) {
        load_c();
    }

    T* O = (T*)Oc;
    if (!SUB) O += (int64_t)blockIdx.y * a.ostride;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int q = q0 + wq + 16 * j + c;
            if (q >= Qe) continue;
            if (!SUB && a.tout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = F64 ? p0 + wp + 16 * i + g + 4 * r : p0 + wp + 16 * i + 4 * g + r;
                    if (p < a.P) O[q + p * a.ldo] = (T)acc[i][j][r];
                }
            } else if constexpr (!F64) {
                const int64_t pb = p0 + wp + 16 * i + 4 * g;
                T* d = O + pb + (int64_t)q * a.ldo;
                accv_t v = acc[i][j];
                if constexpr (PRE) v = cpre[i][j] - v;
                if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) {
                    *(accv_t*)d = v;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (pb + r < a.P) d[r] = v[r];
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t p = p0 + wp + 16 * i + g + 4 * r;
                    if (p < a.P) {
                        T* d = O + p + (int64_t)q * a.ldo;
                        *d = SUB ? *d - (T)acc[i][j][r] : (T)acc[i][j][r];
                    }
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Masked copies of a reflector block V (mk x nb, column-major, ld ldv):
//   Vm (column-major, ld ldm): Vm[k][i] = V[k][i] for k > i, 1 for k == i, 0 above
//   Vt (row-major mk x nb, ld ldvt >= nb): Vt[k][i] = Vm[k][i], zero for i >= nb
// Tiles of 64 rows x 64 columns through LDS so both writes are coalesced.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) prep_v_kernel(const T* __restrict__ V, int64_t ldv, int64_t mk, int nb,
                                                     T* __restrict__ Vm, int64_t ldm, T* __restrict__ Vt, int64_t ldvt)
{
    __shared__ T tile[64][65];
    const int64_t k0 = (int64_t)blockIdx.x * 64;
    const int i0 = blockIdx.y * 64;
    const int t = threadIdx.x;
    for (int e = t; e < 64 * 64; e += 256) {
        const int ii = e / 64, kk = e % 64;            // kk fastest: coalesced along the column
        const int64_t k = k0 + kk;
        const int i = i0 + ii;
        T v = (T)0;
        if (k < mk && i < nb) {
            v = k > i ? V[k + (int64_t)i * ldv] : (k == i ? (T)1 : (T)0);
            Vm[k + (int64_t)i * ldm] = v;
        }
        tile[ii][kk] = v;
    }
    __syncthreads();
    if (!Vt) return;                                   // (the column-major copy only)
    for (int e = t; e < 64 * 64; e += 256) {
        const int kk = e / 64, ii = e % 64;            // ii fastest: coalesced along the row of Vt
        const int64_t k = k0 + kk;
        const int i = i0 + ii;
        if (k < mk && i < ldvt) Vt[k * ldvt + i] = i < nb ? tile[ii][kk] : (T)0;
    }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_prep_v(const T* V, int64_t ldv, int64_t mk, int nb, T* Vm, int64_t ldm, T* Vt, int64_t ldvt,
                         hipStream_t s)
{
    dim3 grid((unsigned)((mk + 63) / 64), (unsigned)((ldvt + 63) / 64));
    hipLaunchKernelGGL(prep_v_kernel<T>, grid, dim3(256), 0, s, V, ldv, mk, nb, Vm, ldm, Vt, ldvt);
    return hipGetLastError();
}

// out (P x Q) = X Y^T summed over K, split into slices; returns the slice count.
// Tile-width and split-K choices of the NT launches (set by the autotuner;
// the defaults suit the wide trailing updates).
NtPlan g_nt_default = {128, 1024};

template <typename T>
hipError_t launch_nt(const T* X, int64_t ldx, const T* Y, int64_t ldy, T* out, int64_t ldo, int64_t P, int Q,
                     int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s, const NtPlan* plan,
                     const int32_t* desc, int desc_y, int desc_out, int maskx, int tout, int upper)
{
    constexpr int BK = LdsTraits<T>::BK;
    const NtPlan pl = plan ? *plan : g_nt_default;
    const int bq = pl.bq;
    NtArgs a;
    a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy; a.out = out; a.ldo = ldo;
    a.P = P; a.Q = Q; a.K = K; a.sub = sub ? 1 : 0;
    a.desc = desc; a.desc_y = desc_y; a.desc_out = desc_out;
    a.maskx = maskx;
    a.tout = sub ? 0 : tout;
    a.upper = sub ? 0 : upper;
    a.tiles_p = (int)((P + kBP - 1) / kBP);
    a.tiles_q = (Q + bq - 1) / bq;
    a.ostride = a.tout ? ldo * P : ldo * (int64_t)Q;
    const int tiles = a.tiles_p * a.tiles_q;
    int nz = 1;
    if (!sub) {
        while (tiles * nz * 2 <= pl.split_target && K / (nz * 2) >= 8 * BK && nz < 256) nz *= 2;
        while (nz > 1 && (int64_t)nz * a.ostride > ocap) nz /= 2;
    }
    int64_t ks = (K + nz - 1) / nz;
    ks = (ks + BK - 1) / BK * BK;
    nz = (int)((K + ks - 1) / ks);
    if (nz < 1) nz = 1;
    a.kslice = ks;
    *nz_out = nz;
#define CT_NT_LAUNCH(BQV)                                                                   \
    if (sub)                                                                                \
        hipLaunchKernelGGL((gemm_nt_kernel<T, true, BQV>), dim3(padded_tiles(tiles), nz), dim3(256), 0, s, a); \
    else                                                                                    \
        hipLaunchKernelGGL((gemm_nt_kernel<T, false, BQV>), dim3(padded_tiles(tiles), nz), dim3(256), 0, s, a);
    switch (bq) {
        case 16: CT_NT_LAUNCH(16) break;
        case 32: CT_NT_LAUNCH(32) break;
        case 64: CT_NT_LAUNCH(64) break;
        default: CT_NT_LAUNCH(128) break;
    }
#undef CT_NT_LAUNCH
    return hipGetLastError();
}

template hipError_t launch_prep_v<float>(const float*, int64_t, int64_t, int, float*, int64_t, float*, int64_t,
                                         hipStream_t);
template hipError_t launch_prep_v<double>(const double*, int64_t, int64_t, int, double*, int64_t, double*, int64_t,
                                          hipStream_t);
template hipError_t launch_nt<float>(const float*, int64_t, const float*, int64_t, float*, int64_t, int64_t, int,
                                     int64_t, bool, int64_t, int*, hipStream_t, const NtPlan*, const int32_t*, int,
                                     int, int, int, int);
template hipError_t launch_nt<double>(const double*, int64_t, const double*, int64_t, double*, int64_t, int64_t, int,
                                      int64_t, bool, int64_t, int*, hipStream_t, const NtPlan*, const int32_t*, int,
                                      int, int, int, int);


// ---------------------------------------------------------------------------
// Low-precision variant of the NT update (same operands, FP32 in memory, FP32
// accumulation) on the 16x16x32 bf16 / f16 MFMA.  Each FP32 element is
// rounded once, when its tile is staged into LDS:
//   M_BF16 / M_F16: x -> bf16(x) / f16(x)                  (1 MFMA per block)
//   M_BF16X3: x -> hi = bf16(x), lo = bf16(x - hi); the product is formed as
//             lo*hi' + hi*lo' + hi*hi' (3 MFMA per block, about 16
//             significant bits, FP32 range)
// Tile 128 x 128, K step 64, one LDS buffer per operand half with register
// prefetch of the next K step; fragments are one ds_read_b128 per half.
// ---------------------------------------------------------------------------
template <int MODE> struct LpT;
template <> struct LpT<M_BF16> { typedef __bf16 e; typedef bf8_t v8; static constexpr bool X3 = false; };
template <> struct LpT<M_F16> { typedef _Float16 e; typedef h8_t v8; static constexpr bool X3 = false; };
template <> struct LpT<M_BF16X3> { typedef __bf16 e; typedef bf8_t v8; static constexpr bool X3 = true; };

template <int MODE>
__device__ __forceinline__ f4_t mfma_lp(const typename LpT<MODE>::v8& a, const typename LpT<MODE>::v8& b, f4_t acc)
{
    if constexpr (MODE == M_F16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// 16 bytes of bfloat16 (8 values)
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// 8 consecutive bfloat16 of row `row` from K index kk (zero past kend or the
// last row).
__device__ __forceinline__ u4v load_bf8(const __bf16* M, int64_t ld, int64_t row, int64_t rows, int64_t kk,
                                        int64_t kend)
{
    u4v v = {0, 0, 0, 0};
    if (row >= rows) return v;
    const __bf16* p = M + row * ld + kk;
    if (kk + 8 <= kend) return *(const u4v*)p;
    uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint16_t* q = (const uint16_t*)p;
    for (int i = 0; i < 8; ++i)
        if (kk + i < kend) e[i] = q[i];
    v[0] = e[0] | ((uint32_t)e[1] << 16);
    v[1] = e[2] | ((uint32_t)e[3] << 16);
    v[2] = e[4] | ((uint32_t)e[5] << 16);
    v[3] = e[6] | ((uint32_t)e[7] << 16);
    return v;
}

// PX / PY (BF16X3 only): the operand comes already split into bfloat16 high
// and low parts (Xlo / Ylo), so staging is a plain copy into LDS.
template <int MODE, bool SUB, bool PX = false, bool PY = false>
__global__ void __launch_bounds__(256, 2) gemm_nt_lp_kernel(NtArgs a)
{
    typedef typename LpT<MODE>::e E;
    typedef typename LpT<MODE>::v8 v8;
    constexpr bool X3 = LpT<MODE>::X3;
    constexpr int BK = 64, LDK = BK + 8;          // row stride 144 bytes
    constexpr int NH = X3 ? 2 : 1;                // hi (and lo) halves
    constexpr int VPR = BK / 4;                   // float4 per tile row
    constexpr int RPP = 256 / VPR;                // rows per pass
    constexpr int PASSES = kBP / RPP;             // 8

    __shared__ __attribute__((aligned(16))) E Xs[NH][kBP * LDK];
    __shared__ __attribute__((aligned(16))) E Ys[NH][kBQ * LDK];

    int tp, tq;
    if (!tile_of(blockIdx.x, a.tiles_p, a.tiles_q, tp, tq)) return;
    const int64_t p0 = (int64_t)tp * kBP;
    const int q0 = tq * kBQ;
    const int64_t kbeg = (int64_t)blockIdx.y * a.kslice;
    int64_t kend = kbeg + a.kslice;
    if (kend > a.K) kend = a.K;

    const float* __restrict__ X = (const float*)a.X;
    const float* __restrict__ Y = (const float*)a.Y;
    const int t = threadIdx.x;
    const int lr = t / VPR, lv = t % VPR;

    // FP32 operands: 16 float per thread-row vector, split when staged
    f4_t xr[PX ? 1 : PASSES], yr[PY ? 1 : PASSES];
    // split operands: 8 bfloat16 per 16-byte vector, 4 passes of 32 rows
    constexpr int VB = BK / 8, RB = 256 / VB, PB = kBP / RB;
    u4v xs[PX ? 2 * PB : 1], ys[PY ? 2 * PB : 1];
    const int lrb = t / VB, lvb = t % VB;
    auto gload = [&](int64_t k0) {
        // FP32 operands first: in W = V^T C the columns of C come fresh from
        // HBM while the split reflector block is mostly in L2, so C's loads
        // get the longest time in flight
        if constexpr (!PX || !PY) {
#pragma unroll
            for (int ps = 0; ps < PASSES; ++ps) {
                const int row = ps * RPP + lr;
                const int64_t kk = k0 + lv * 4;
                const int64_t pr = p0 + row;
                const int qr = q0 + row;
                f4_t vx = {0, 0, 0, 0}, vy = {0, 0, 0, 0};
                if (kk + 4 <= kend) {
                    if (!PX && pr < a.P) vx = *(const f4_t*)(X + pr * a.ldx + kk);
                    if (!PY && qr < a.Q) vy = *(const f4_t*)(Y + (int64_t)qr * a.ldy + kk);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (kk + e < kend) {
                            if (!PX && pr < a.P) vx[e] = X[pr * a.ldx + kk + e];
                            if (!PY && qr < a.Q) vy[e] = Y[(int64_t)qr * a.ldy + kk + e];
                        }
                }
                if constexpr (!PX) xr[ps] = vx;
                if constexpr (!PY) yr[ps] = vy;
            }
        }
        if constexpr (PX) {
            const __bf16* Xh = (const __bf16*)a.X;
            const __bf16* Xl = (const __bf16*)a.Xlo;
#pragma unroll
            for (int ps = 0; ps < PB; ++ps) {
                const int64_t pr = p0 + ps * RB + lrb, kk = k0 + lvb * 8;
                xs[ps] = load_bf8(Xh, a.ldx, pr, a.P, kk, kend);
                xs[PB + ps] = load_bf8(Xl, a.ldx, pr, a.P, kk, kend);
            }
        }
        if constexpr (PY) {
            const __bf16* Yh = (const __bf16*)a.Y;
            const __bf16* Yl = (const __bf16*)a.Ylo;
#pragma unroll
            for (int ps = 0; ps < PB; ++ps) {
                const int64_t qr = q0 + ps * RB + lrb, kk = k0 + lvb * 8;
                ys[ps] = load_bf8(Yh, a.ldy, qr, a.Q, kk, kend);
                ys[PB + ps] = load_bf8(Yl, a.ldy, qr, a.Q, kk, kend);
            }
        }
    };
    auto sstore = [&]() {
        if constexpr (PX) {
#pragma unroll
            for (int ps = 0; ps < PB; ++ps) {
                const int row = ps * RB + lrb;
                *(u4v*)&Xs[0][row * LDK + lvb * 8] = xs[ps];
                *(u4v*)&Xs[NH - 1][row * LDK + lvb * 8] = xs[PB + ps];
            }
        }
        if constexpr (PY) {
#pragma unroll
            for (int ps = 0; ps < PB; ++ps) {
                const int row = ps * RB + lrb;
                *(u4v*)&Ys[0][row * LDK + lvb * 8] = ys[ps];
                *(u4v*)&Ys[NH - 1][row * LDK + lvb * 8] = ys[PB + ps];
            }
        }
        if constexpr (!PX || !PY) {
#pragma unroll
            for (int ps = 0; ps < PASSES; ++ps) {
                const int row = ps * RPP + lr;
                typedef E e4 __attribute__((ext_vector_type(4)));
                e4 xh, yh, xl, yl;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if constexpr (!PX) xh[e] = (E)xr[ps][e];
                    if constexpr (!PY) yh[e] = (E)yr[ps][e];
                    if constexpr (X3) {
                        if constexpr (!PX) xl[e] = (E)(xr[ps][e] - (float)xh[e]);
                        if constexpr (!PY) yl[e] = (E)(yr[ps][e] - (float)yh[e]);
                    }
                }
                if constexpr (!PX) *(e4*)&Xs[0][row * LDK + lv * 4] = xh;
                if constexpr (!PY) *(e4*)&Ys[0][row * LDK + lv * 4] = yh;
                if constexpr (X3) {
                    if constexpr (!PX) *(e4*)&Xs[NH - 1][row * LDK + lv * 4] = xl;
                    if constexpr (!PY) *(e4*)&Ys[NH - 1][row * LDK + lv * 4] = yl;
                }
            }
        }
    };

    const int lane = t & 63, wv = t >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int wp = (wv >> 1) * 64, wq = (wv & 1) * 64;

    f4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

    // the wave raises its issue priority for its MFMAs, so that while one
    // workgroup of the CU stages its next K step the other keeps the matrix
    // cores fed (measured: W = V^T C 317 -> 343 TFLOP/s at the first trailing
    // update of the 256^2 factorization)
    auto compute = [&]() {
        __builtin_amdgcn_s_setprio(1);
        // scheduler hint: interleave the fragment reads with the MFMAs
        // (QR at 256^2 2.15 -> 2.12 s measured on one box)
        __builtin_amdgcn_iglp_opt(0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            v8 bh[4], bl[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                bh[j] = *(const v8*)&Ys[0][(wq + 16 * j + c) * LDK + kk + 8 * g];
                if constexpr (X3) bl[j] = *(const v8*)&Ys[NH - 1][(wq + 16 * j + c) * LDK + kk + 8 * g];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const v8 ah = *(const v8*)&Xs[0][(wp + 16 * i + c) * LDK + kk + 8 * g];
                v8 al;
                if constexpr (X3) al = *(const v8*)&Xs[NH - 1][(wp + 16 * i + c) * LDK + kk + 8 * g];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if constexpr (X3) {
                        acc[i][j] = mfma_lp<MODE>(al, bh[j], acc[i][j]);
                        acc[i][j] = mfma_lp<MODE>(ah, bl[j], acc[i][j]);
                    }
                    acc[i][j] = mfma_lp<MODE>(ah, bh[j], acc[i][j]);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // the subtracting epilogue's C tile is fetched during the last K step,
    // when the prefetch registers are free, so its latency hides behind it
    f4_t cpre[4][4];
    auto load_c = [&]() {
        const float* O = (const float*)a.out;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = q0 + wq + 16 * j + c;
                const int64_t pb = p0 + wp + 16 * i + 4 * g;
                f4_t v = {0, 0, 0, 0};
                if (q < a.Q) {
                    const float* d = O + pb + (int64_t)q * a.ldo;
                    if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) v = *(const f4_t*)d;
                    else
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (pb + r < a.P) v[r] = d[r];
                }
                cpre[i][j] = v;
            }
    };

    if (kbeg < kend) {
        gload(kbeg);
        sstore();
        __syncthreads();
        int64_t k0 = kbeg;
        for (; k0 + BK < kend; k0 += BK) {
            gload(k0 + BK);
            compute();
            __syncthreads();
            sstore();
            __syncthreads();
        }
        if constexpr (SUB) load_c();
        compute();
    } else if constexpr (SUB) {
        load_c();
    }

    float* O = (float*)a.out;
    if (!SUB) O += (int64_t)blockIdx.y * a.ostride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = q0 + wq + 16 * j + c;
            if (q >= a.Q) continue;
            const int64_t pb = p0 + wp + 16 * i + 4 * g;
            float* d = O + pb + (int64_t)q * a.ldo;
            f4_t v = acc[i][j];
            if constexpr (SUB) v = cpre[i][j] - v;
            if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) {
                *(f4_t*)d = v;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (pb + r < a.P) d[r] = v[r];
            }
        }
}

template <int MODE>
hipError_t launch_nt_lp(const void* X, int64_t ldx, const void* Y, int64_t ldy, float* out, int64_t ldo, int64_t P,
                        int Q, int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s, const void* Xlo,
                        const void* Ylo)
{
    constexpr int BK = 64;
    NtArgs a;
    a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy; a.out = out; a.ldo = ldo;
    a.P = P; a.Q = Q; a.K = K; a.sub = sub ? 1 : 0;
    a.desc = nullptr; a.desc_y = 0; a.desc_out = 0; a.maskx = 0; a.tout = 0; a.upper = 0;
    a.Xlo = Xlo; a.Ylo = Ylo;
    a.tiles_p = (int)((P + kBP - 1) / kBP);
    a.tiles_q = (Q + kBQ - 1) / kBQ;
    a.ostride = ldo * (int64_t)Q;
    const int tiles = a.tiles_p * a.tiles_q;
    int nz = 1;
    if (!sub) {
        while (tiles * nz * 2 <= 1024 && K / (nz * 2) >= 8 * BK && nz < 256) nz *= 2;
        while (nz > 1 && (int64_t)nz * a.ostride > ocap) nz /= 2;
    }
    int64_t ks = (K + nz - 1) / nz;
    ks = (ks + BK - 1) / BK * BK;
    nz = (int)((K + ks - 1) / ks);
    if (nz < 1) nz = 1;
    a.kslice = ks;
    *nz_out = nz;
    const dim3 grid(padded_tiles(tiles), nz);
    if constexpr (MODE == M_BF16X3) {
        if (Xlo && Ylo) {
            if (sub) hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, true, true, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, false, true, true>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
        if (Xlo) {
            if (sub) hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, true, true, false>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, false, true, false>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
    }
    if (sub)
        hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((gemm_nt_lp_kernel<MODE, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// hi = bf16(x), lo = bf16(x - hi) for a column-major rows x cols FP32 block
// (the same rounding as the BF16x3 kernel's staging).
__global__ void __launch_bounds__(256) split_x3_kernel(const float* __restrict__ src, int64_t lds,
                                                       __bf16* __restrict__ hi, __bf16* __restrict__ lo, int64_t ldd,
                                                       int64_t rows, int64_t cols)
{
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t c = e / rows, r = e - c * rows;
        const float x = src[r + c * lds];
        const __bf16 h = (__bf16)x;
        hi[r + c * ldd] = h;
        lo[r + c * ldd] = (__bf16)(x - (float)h);
    }
}

hipError_t launch_split_x3(const float* src, int64_t lds, void* hi, void* lo, int64_t ldd, int64_t rows, int64_t cols,
                           hipStream_t s)
{
    int64_t blocks = (rows * cols + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(split_x3_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, lds, (__bf16*)hi, (__bf16*)lo,
                       ldd, rows, cols);
    return hipGetLastError();
}

template hipError_t launch_nt_lp<M_BF16>(const void*, int64_t, const void*, int64_t, float*, int64_t, int64_t, int,
                                         int64_t, bool, int64_t, int*, hipStream_t, const void*, const void*);
template hipError_t launch_nt_lp<M_F16>(const void*, int64_t, const void*, int64_t, float*, int64_t, int64_t, int,
                                        int64_t, bool, int64_t, int*, hipStream_t, const void*, const void*);
template hipError_t launch_nt_lp<M_BF16X3>(const void*, int64_t, const void*, int64_t, float*, int64_t, int64_t, int,
                                           int64_t, bool, int64_t, int*, hipStream_t, const void*, const void*);


// ---------------------------------------------------------------------------
// BF16x3 NT product whose two operands both come split into bfloat16 high and
// low planes (the block-reflector update C -= V W' of the factorization, and
// W = V^T C when the trailing matrix is kept split as well), staged into LDS
// by direct global->LDS loads (global_load_lds_dwordx4): no staging
// registers and no conversion.
//
// A stage holds, for each half of each operand, the tile's rows as 64-byte
// records (K step 32) in 1 KB blocks of 16 rows; one load instruction of a
// wavefront fills one block (lane l writes bytes 16 l .. 16 l + 15), and lane
// l fetches chunk (l & 3) ^ dl_swz16(r) of row r = l >> 2, so that the
// sixteen rows a fragment read touches spread over all banks.  The stages
// form a ring: while one is multiplied the next ones are in flight, and one
// barrier per K step both publishes a landed stage and frees the stage read
// in the previous step.
template <int WTP_, int WTQ_, int WVP_, int WVQ_, int ST_, int CH_>
struct DlCfg {
    static constexpr int WTP = WTP_, WTQ = WTQ_;       // 16 x 16 blocks of one wavefront (P, Q)
    static constexpr int WVP = WVP_, WVQ = WVQ_;       // wavefronts along P, Q
    static constexpr int ST = ST_;                     // LDS stages
    static constexpr int CH = CH_;                     // row blocks per chunk of the subtracting epilogue
    static constexpr int NW = WVP * WVQ, NT = 64 * NW;
    static constexpr int BP = 16 * WTP * WVP, BQ = 16 * WTQ * WVQ, BK = 32;
    static constexpr int XHALF = BP * BK * 2, YHALF = BQ * BK * 2;
    static constexpr int STAGE = 2 * XHALF + 2 * YHALF;
    static constexpr int XBLK = 2 * BP / 16, YBLK = 2 * BQ / 16;   // 1 KB blocks per stage
    static constexpr int LPW = (XBLK + YBLK) / NW;                 // load instructions per wavefront per stage
    static_assert((XBLK + YBLK) % NW == 0, "stage blocks must split evenly over the wavefronts");
    static_assert(WTP % CH == 0, "epilogue chunks");
    static constexpr int LDS = ST * STAGE;
};
// 256 x 128 tile, 8 wavefronts of 64 x 64, 3 stages (144 KB of LDS)
using DlSmall = DlCfg<4, 4, 4, 2, 3, 4>;
// 256 x 256 tile, 8 wavefronts of 128 x 64, 2 stages (128 KB): a quarter less
// LDS traffic per MFMA than 64 x 64 wavefront tiles
using DlBig = DlCfg<8, 4, 2, 4, 2, 1>;

// Row records of a stage (the 16-byte chunks of a row are permuted by an XOR
// with a function of the row's place in its 16-row group, so that the rows a
// fragment read touches spread over all LDS banks):
//   bfloat16 halves: 64-byte rows, 16 rows per 1 KB block; chunk bit 0 flips
//     with row bit 0, chunk bit 1 with row bit 3 (chosen by timing every XOR
//     of row bits for the fragment read, 16 rows x 4 chunks per ds_read_b128:
//     1.5x faster than the XOR of row bits 1 and 3 with bit 2, which read no
//     faster than no permutation at all)
//   FP32 operand:   128-byte rows, 8 rows per 1 KB block
__device__ __forceinline__ int dl_swz16(int r) { return (r & 1) | ((r >> 2) & 2); }
__device__ __forceinline__ int dl_swz32(int r) { return (r ^ (r >> 3)) & 7; }

constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0xF70; }

// Split of 8 FP32 values (two 16-byte LDS reads) into bfloat16 halves,
// hi = bf16(y), lo = bf16(y - hi), round to nearest even, as everywhere; in
// pairs: one packed conversion gives both high halves, whose FP32 values are
// the packed word's halves moved into place.
__device__ __forceinline__ void split8(const f4_t& y0, const f4_t& y1, bf8_t& bh, bf8_t& bl)
{
    typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
    typedef float f2_t __attribute__((ext_vector_type(2)));
    u4v hp, lp;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const f2_t yv = e < 2 ? f2_t{y0[2 * e], y0[2 * e + 1]} : f2_t{y1[2 * e - 4], y1[2 * e - 3]};
        const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(yv, bf2_t));
        const f2_t hf = {__uint_as_float(h << 16), __uint_as_float(h & 0xffff0000u)};
        hp[e] = h;
        lp[e] = __builtin_bit_cast(uint32_t, __builtin_convertvector(yv - hf, bf2_t));
    }
    bh = __builtin_bit_cast(bf8_t, hp);
    bl = __builtin_bit_cast(bf8_t, lp);
}

// XF32 / YF32: that operand is FP32 (the trailing matrix in W = V^T C; the
// FP32 factor copies a solve reads), loaded into LDS as is and split into its
// bfloat16 halves when the fragments are read.
template <class CF, bool SUB, bool XF32, bool YF32>
__global__ void __launch_bounds__(CF::NT, 1) gemm_x3_dl_kernel(NtArgs a)
{
    extern __shared__ __attribute__((aligned(1024))) char dl_lds[];
    int tp, tq;
    if (!tile_of(blockIdx.x, a.tiles_p, a.tiles_q, tp, tq)) return;
    const int64_t p0 = (int64_t)tp * CF::BP;
    const int q0 = tq * CF::BQ;
    const int64_t kbeg = (int64_t)blockIdx.y * a.kslice;
    int64_t kend = kbeg + a.kslice;
    if (kend > a.K) kend = a.K;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);

    // this lane's part of the wavefront's load instructions (wavefront wv
    // fills blocks LPW wv .. LPW wv + LPW - 1 of the stage: X's high half,
    // X's low half, then Y); rows past P / Q read the last row (the products
    // they feed are not stored).  src: byte address at k = 0; ksh: log2 of
    // the element size; kk0: the first k of this lane's chunk.
    const char* src[CF::LPW];
    int dst[CF::LPW], ksh[CF::LPW], kk0[CF::LPW];
#pragma unroll
    for (int i = 0; i < CF::LPW; ++i) {
        const int idx = CF::LPW * wv + i;
        if (XF32 && idx < CF::XBLK) {
            const int blk = idx;                       // 8 rows of 128 bytes
            const int r = lane >> 3, ch = (lane & 7) ^ dl_swz32((blk & 1) * 8 + r);
            int64_t p = p0 + blk * 8 + r;
            if (p >= a.P) p = a.P - 1;
            src[i] = (const char*)a.X + (p * a.ldx + ch * 4) * 4;
            dst[i] = blk * 1024;
            ksh[i] = 2;
            kk0[i] = ch * 4;
        } else if (idx < CF::XBLK) {
            const int h = idx / (CF::BP / 16), rb = idx % (CF::BP / 16);
            const int r = lane >> 2, ch = (lane & 3) ^ dl_swz16(r);
            int64_t p = p0 + rb * 16 + r;
            if (p >= a.P) p = a.P - 1;
            src[i] = (const char*)(h ? a.Xlo : a.X) + (p * a.ldx + ch * 8) * 2;
            dst[i] = h * CF::XHALF + rb * 1024;
            ksh[i] = 1;
            kk0[i] = ch * 8;
        } else if constexpr (!YF32) {
            const int y = idx - CF::XBLK, h = y / (CF::BQ / 16), rb = y % (CF::BQ / 16);
            const int r = lane >> 2, ch = (lane & 3) ^ dl_swz16(r);
            int q = q0 + rb * 16 + r;
            if (q >= a.Q) q = a.Q - 1;
            src[i] = (const char*)(h ? a.Ylo : a.Y) + ((int64_t)q * a.ldy + ch * 8) * 2;
            dst[i] = 2 * CF::XHALF + h * CF::YHALF + rb * 1024;
            ksh[i] = 1;
            kk0[i] = ch * 8;
        } else {
            const int blk = idx - CF::XBLK;            // 8 rows of 128 bytes
            const int r = lane >> 3, ch = (lane & 7) ^ dl_swz32((blk & 1) * 8 + r);
            int q = q0 + blk * 8 + r;
            if (q >= a.Q) q = a.Q - 1;
            src[i] = (const char*)a.Y + ((int64_t)q * a.ldy + ch * 4) * 4;
            dst[i] = 2 * CF::XHALF + blk * 1024;
            ksh[i] = 2;
            kk0[i] = ch * 4;
        }
    }
    auto issue = [&](int stage, int64_t k0) {
        char* base = dl_lds + stage * CF::STAGE;
#pragma unroll
        for (int i = 0; i < CF::LPW; ++i)
            __builtin_amdgcn_global_load_lds((const void*)(src[i] + (k0 << ksh[i])),
                                             (__attribute__((address_space(3))) void*)(base + dst[i]), 16, 0, 0);
    };

    const int c = lane & 15, g = lane >> 4;
    const int wp = (wv / CF::WVQ) * 16 * CF::WTP, wq = (wv % CF::WVQ) * 16 * CF::WTQ;
    const int xfrag = XF32 ? (c >> 3) * 1024 + (c & 7) * 128 + 16 * ((2 * g) ^ dl_swz32(c))
                           : (c * 4 + (g ^ dl_swz16(c))) * 16;
    const int xfrag1 = XF32 ? (c >> 3) * 1024 + (c & 7) * 128 + 16 * ((2 * g + 1) ^ dl_swz32(c)) : 0;
    const int yfrag0 = YF32 ? (c >> 3) * 1024 + (c & 7) * 128 + 16 * ((2 * g) ^ dl_swz32(c))
                            : (c * 4 + (g ^ dl_swz16(c))) * 16;
    const int yfrag1 = YF32 ? (c >> 3) * 1024 + (c & 7) * 128 + 16 * ((2 * g + 1) ^ dl_swz32(c)) : 0;
    f4_t acc[CF::WTP][CF::WTQ];
#pragma unroll
    for (int i = 0; i < CF::WTP; ++i)
#pragma unroll
        for (int j = 0; j < CF::WTQ; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

    auto compute = [&](int stage) {
        const char* base = dl_lds + stage * CF::STAGE;
        __builtin_amdgcn_s_setprio(1);
        __builtin_amdgcn_iglp_opt(0);
        bf8_t bh[CF::WTQ], bl[CF::WTQ];
#pragma unroll
        for (int j = 0; j < CF::WTQ; ++j) {
            if constexpr (YF32) {
                const char* yb = base + 2 * CF::XHALF + (wq + 16 * j) * 128;
                // (the two reads into locals first: passed straight into the
                // call, this compiler version made the first LDS read wait for
                // every load in flight, the next stage's included)
                const f4_t y0 = *(const f4_t*)(yb + yfrag0);
                const f4_t y1 = *(const f4_t*)(yb + yfrag1);
                split8(y0, y1, bh[j], bl[j]);
            } else {
                const int rb = (wq >> 4) + j;
                bh[j] = *(const bf8_t*)(base + 2 * CF::XHALF + rb * 1024 + yfrag0);
                bl[j] = *(const bf8_t*)(base + 2 * CF::XHALF + CF::YHALF + rb * 1024 + yfrag0);
            }
        }
#pragma unroll
        for (int i = 0; i < CF::WTP; ++i) {
            const int rb = (wp >> 4) + i;
            bf8_t ah, al;
            if constexpr (XF32) {
                const char* xb = base + (wp + 16 * i) * 128;
                const f4_t x0 = *(const f4_t*)(xb + xfrag);
                const f4_t x1 = *(const f4_t*)(xb + xfrag1);
                split8(x0, x1, ah, al);
            } else {
                ah = *(const bf8_t*)(base + rb * 1024 + xfrag);
                al = *(const bf8_t*)(base + CF::XHALF + rb * 1024 + xfrag);
            }
#pragma unroll
            for (int j = 0; j < CF::WTQ; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
            }
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // a last K step shorter than 32: plain loads with zero fill, written to
    // the same layout by each lane for its own chunk
    auto tail_stage = [&](int stage, int64_t k0) {
        char* base = dl_lds + stage * CF::STAGE;
#pragma unroll
        for (int i = 0; i < CF::LPW; ++i) {
            const char* sp = src[i] + (k0 << ksh[i]);
            const int64_t kk = k0 + kk0[i];
            const int ne = 16 >> ksh[i];                // elements per chunk
            u4v v = {0, 0, 0, 0};
            if (kk + ne <= kend) {
                v = *(const u4v*)sp;
            } else if (kk < kend) {
                if (ksh[i] == 1) {
                    uint16_t e[8];
                    for (int u = 0; u < 8; ++u) e[u] = kk + u < kend ? ((const uint16_t*)sp)[u] : (uint16_t)0;
                    v[0] = e[0] | ((uint32_t)e[1] << 16);
                    v[1] = e[2] | ((uint32_t)e[3] << 16);
                    v[2] = e[4] | ((uint32_t)e[5] << 16);
                    v[3] = e[6] | ((uint32_t)e[7] << 16);
                } else {
                    for (int u = 0; u < 4; ++u) v[u] = kk + u < kend ? ((const uint32_t*)sp)[u] : 0u;
                }
            }
            *(u4v*)(base + dst[i] + lane * 16) = v;
        }
    };

    // the subtracting epilogue reads C in chunks of CH row blocks; the first
    // chunk is fetched during the last K step
    constexpr int CH = SUB ? CF::CH : 1;
    f4_t cpre[CH][CF::WTQ];
    auto load_c = [&](int i0) {
        if constexpr (SUB) {
            const float* O = (const float*)a.out;
#pragma unroll
            for (int ii = 0; ii < CH; ++ii)
#pragma unroll
                for (int j = 0; j < CF::WTQ; ++j) {
                    const int q = q0 + wq + 16 * j + c;
                    const int64_t pb = p0 + wp + 16 * (i0 + ii) + 4 * g;
                    f4_t v = {0, 0, 0, 0};
                    if (q < a.Q) {
                        const float* d = O + pb + (int64_t)q * a.ldo;
                        if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) v = *(const f4_t*)d;
                        else
                            for (int r = 0; r < 4; ++r)
                                if (pb + r < a.P) v[r] = d[r];
                    }
                    cpre[ii][j] = v;
                }
        }
    };

    const int64_t klen = kend > kbeg ? kend - kbeg : 0;
    const int nsteps = (int)(klen / CF::BK);
    const bool has_tail = klen % CF::BK != 0;
#pragma unroll
    for (int sgi = 0; sgi + 1 < CF::ST; ++sgi)
        if (sgi < nsteps) issue(sgi, kbeg + (int64_t)sgi * CF::BK);
    int stage = 0;
    for (int it = 0; it < nsteps; ++it) {
        // this wavefront's loads of step it have landed (with three stages,
        // those of step it + 1 may still be in flight); after the barrier
        // everyone's have, and every wavefront is done with step it - 1,
        // whose buffer is refilled next.  (An explicit wait and a bare
        // s_barrier: a workgroup fence would wait for every load in flight.)
        if (CF::ST >= 3 && it + 1 < nsteps) __builtin_amdgcn_s_waitcnt(vmcnt_imm(CF::LPW));
        else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (it + CF::ST - 1 < nsteps) {
            int nb = stage + CF::ST - 1;
            if (nb >= CF::ST) nb -= CF::ST;
            issue(nb, kbeg + (int64_t)(it + CF::ST - 1) * CF::BK);
        }
        if (SUB && it + 1 == nsteps && !has_tail) load_c(0);
        compute(stage);
        stage = stage + 1 == CF::ST ? 0 : stage + 1;
    }
    if (has_tail) {
        __syncthreads();
        tail_stage(stage, kbeg + (int64_t)nsteps * CF::BK);
        __syncthreads();
        if (SUB) load_c(0);
        compute(stage);
    } else if (SUB && nsteps == 0) {
        load_c(0);
    }

    float* O = (float*)a.out;
    if (!SUB) O += (int64_t)blockIdx.y * a.ostride;
#pragma unroll
    for (int i0 = 0; i0 < CF::WTP; i0 += CH) {
        if (SUB && i0 > 0) load_c(i0);
#pragma unroll
        for (int ii = 0; ii < CH; ++ii)
#pragma unroll
            for (int j = 0; j < CF::WTQ; ++j) {
                const int q = q0 + wq + 16 * j + c;
                const int64_t pb = p0 + wp + 16 * (i0 + ii) + 4 * g;
                if (q >= a.Q || pb >= a.P) continue;
                float* d = O + pb + (int64_t)q * a.ldo;
                f4_t v = acc[i0 + ii][j];
                if constexpr (SUB) v = cpre[ii][j] - v;
                if (pb + 3 < a.P && (((uintptr_t)d & 15) == 0)) {
                    *(f4_t*)d = v;
                } else {
                    for (int r = 0; r < 4; ++r)
                        if (pb + r < a.P) d[r] = v[r];
                }
            }
    }
}

template <class CF>
static hipError_t dl_set_lds()
{
    static bool done = false;
    if (done) return hipSuccess;
    const void* k[6] = {(const void*)gemm_x3_dl_kernel<CF, true, false, false>,
                        (const void*)gemm_x3_dl_kernel<CF, false, false, false>,
                        (const void*)gemm_x3_dl_kernel<CF, false, false, true>,
                        (const void*)gemm_x3_dl_kernel<CF, true, true, true>,
                        (const void*)gemm_x3_dl_kernel<CF, false, true, true>,
                        (const void*)gemm_x3_dl_kernel<CF, true, false, true>};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, CF::LDS);
        if (e != hipSuccess) return e;
    }
    done = true;
    return hipSuccess;
}

int g_x3dl_cfg = 1;   // 0: 256 x 128 tiles, 1: 256 x 256 tiles
static int g_nt_cus = 256;
void nt_set_cus(int cus) { if (cus > 0) g_nt_cus = cus; }

// Split-K factor for a launch of `tiles` tiles (one workgroup per CU): the
// smallest that fills the CUs' last round to at least 90 % (or the best one
// up to 64), keeping at least 16 K steps per slice.
static int dl_split(int tiles, int64_t K, int bk)
{
    int best = 1;
    double best_eff = 0.0;
    for (int nz = 1; nz <= 64 && K / nz >= 16 * bk; ++nz) {
        const int64_t w = (int64_t)tiles * nz;
        const int64_t rounds = (w + g_nt_cus - 1) / g_nt_cus;
        const double eff = (double)w / (double)(rounds * g_nt_cus);
        if (eff > best_eff + 1e-9) { best_eff = eff; best = nz; }
        if (eff >= 0.9) break;
    }
    return best;
}

template <class CF>
static hipError_t launch_x3dl_cfg(NtArgs& a, bool sub, bool xf32, bool yf32, int64_t ocap, int* nz_out,
                                  hipStream_t s)
{
    hipError_t e = dl_set_lds<CF>();
    if (e != hipSuccess) return e;
    a.tiles_p = (int)((a.P + CF::BP - 1) / CF::BP);
    a.tiles_q = (a.Q + CF::BQ - 1) / CF::BQ;
    a.ostride = a.ldo * (int64_t)a.Q;
    const int tiles = a.tiles_p * a.tiles_q;
    int nz = 1;
    if (!sub) {
        nz = dl_split(tiles, a.K, CF::BK);
        while (nz > 1 && (int64_t)nz * a.ostride > ocap) --nz;
    }
    int64_t ks = (a.K + nz - 1) / nz;
    ks = (ks + CF::BK - 1) / CF::BK * CF::BK;
    nz = (int)((a.K + ks - 1) / ks);
    if (nz < 1) nz = 1;
    a.kslice = ks;
    *nz_out = nz;
    const dim3 grid(padded_tiles(tiles), nz);
#define CT_X3DL(S_, X_, Y_) hipLaunchKernelGGL((gemm_x3_dl_kernel<CF, S_, X_, Y_>), grid, dim3(CF::NT), CF::LDS, s, a)
    if (xf32 && !yf32) return hipErrorInvalidValue;
    if (sub) {
        if (xf32) CT_X3DL(true, true, true);
        else if (yf32) CT_X3DL(true, false, true);
        else CT_X3DL(true, false, false);
    } else {
        if (xf32) CT_X3DL(false, true, true);
        else if (yf32) CT_X3DL(false, false, true);
        else CT_X3DL(false, false, false);
    }
#undef CT_X3DL
    return hipGetLastError();
}

// out (+)= X Y^T with X = Xhi + Xlo (P x K) and Y = Yhi + Ylo (Q x K), the
// planes bfloat16; a null low plane means that operand is FP32 (at Xh / Yh)
// and is split as it is read (X in FP32 only with Y in FP32 too).  All
// K-contiguous, leading dimensions multiples of 8 elements (4 for FP32),
// 16-byte aligned bases.  sub: out -= X Y^T (no split-K); otherwise split-K
// partials at out + z ldo Q, as launch_nt_lp.
hipError_t launch_nt_x3dl(const void* Xh, const void* Xl, int64_t ldx, const void* Yh, const void* Yl, int64_t ldy,
                          float* out, int64_t ldo, int64_t P, int Q, int64_t K, bool sub, int64_t ocap, int* nz_out,
                          hipStream_t s)
{
    NtArgs a;
    a.X = Xh; a.Xlo = Xl; a.ldx = ldx; a.Y = Yh; a.Ylo = Yl; a.ldy = ldy; a.out = out; a.ldo = ldo;
    a.P = P; a.Q = Q; a.K = K; a.sub = sub ? 1 : 0;
    a.desc = nullptr; a.desc_y = 0; a.desc_out = 0; a.maskx = 0; a.tout = 0; a.upper = 0;
    const bool xf32 = !Xl, yf32 = !Yl;
    if (g_x3dl_cfg == 1) return launch_x3dl_cfg<DlBig>(a, sub, xf32, yf32, ocap, nz_out, s);
    return launch_x3dl_cfg<DlSmall>(a, sub, xf32, yf32, ocap, nz_out, s);
}

}  // namespace ctqr
