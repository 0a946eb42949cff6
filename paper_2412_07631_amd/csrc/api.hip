// C-ABI of libctqr: argument checks, workspace layout, and the host-side
// schedule of the blocked Householder QR and of the solve (Eqs. (qr),
// (solve); the in-memory method of Sec. 2.1 with the blocked triangular
// solve of Sec. 2.2).
#include "ct_internal.h"
#include "../../include/ctqr.h"

#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <new>

namespace ctqr {
hipError_t launch_siddon_dense(const GeomDev& g, int dtype, void* A, int64_t lda, hipStream_t s);
hipError_t launch_siddon_csr(const GeomDev& g, int64_t* row_ptr, int32_t* col, double* val, int64_t cap,
                             hipStream_t s);
hipError_t launch_siddon_rows(const double* rays, int64_t r, int32_t N, double W, double* rows, hipStream_t s);
template <typename TS>
hipError_t launch_panel(TS* A, int64_t lda, int64_t mk, int nbp, int rw, double* tau, double* T, int64_t ldt,
                        double* part, double* gpart, uint64_t* counter, uint64_t* base, uint64_t* flag,
                        uint64_t* flag_base, int64_t* info, int64_t col0, int32_t* err, hipStream_t s);
size_t panel_lds_bytes(int nbp, int rw);
int panel_aux_words();
hipError_t panel_set_max_lds(size_t bytes);
hipError_t panel_max_active(int* per_cu, size_t shmem);
template <int MODE, typename TA, typename TB, typename TW, bool MA, bool MB_>
hipError_t launch_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, TW* W, int M, int N, int64_t K,
                     int64_t wcap, int* nz_out, hipStream_t s);
template <int MODE, typename TA, typename TB, typename TC, bool MA>
hipError_t launch_nn_sub(const TA* A, int64_t lda, const TB* Bhi, const TB* Blo, int64_t ldb, TC* C, int64_t ldc,
                         int64_t M, int N, int K, hipStream_t s);
template <typename TWp, typename TO, int OP, bool SPLIT>
hipError_t launch_tw(const TWp* Wp, int nz, int nbv, int N, const double* T, int64_t ldt, TO* out, TO* out_lo,
                     int64_t ldo, hipStream_t s);
hipError_t launch_t_from_gram(const double* G, int64_t ldg, const double* tau, int nb, double* T, int64_t ldt,
                              hipStream_t s);
hipError_t t_from_gram_set_max_lds(size_t bytes);
template <typename TWp, typename TS>
hipError_t launch_sum_slices(const TWp* Wp, int64_t wstride, int nz, int64_t count, TS* S, hipStream_t s);
template <typename T>
hipError_t launch_prep_v(const T* V, int64_t ldv, int64_t mk, int nb, T* Vm, int64_t ldm, T* Vt, int64_t ldvt,
                         hipStream_t s);
template <typename T>
hipError_t launch_nt(const T* X, int64_t ldx, const T* Y, int64_t ldy, T* out, int64_t ldo, int64_t P, int Q,
                     int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s);
template <int MODE>
hipError_t launch_nt_lp(const float* X, int64_t ldx, const float* Y, int64_t ldy, float* out, int64_t ldo, int64_t P,
                        int Q, int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s);
template <typename TS, bool UPPER>
hipError_t launch_trsm_diag(const TS* R, int64_t ldr, int bo, TS* B, int64_t ldb, int nrhs, hipStream_t s);
hipError_t trsm_set_max_lds(size_t bytes);
hipError_t launch_residual(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int nrhs,
                           hipStream_t s);
template <typename TI, typename TO>
hipError_t launch_convert(const TI* X, int64_t ldx, TO* Y, int64_t ldy, int64_t rows, int cols, hipStream_t s);
template <typename TD>
hipError_t launch_accumulate(double* X, int64_t ldx, const TD* D, int64_t ldd, int64_t rows, int cols,
                             hipStream_t s);
template <typename T>
hipError_t launch_zero_rows(T* Y, int64_t ldy, int64_t r0, int64_t r1, int cols, hipStream_t s);
hipError_t launch_colnorm(const double* X, int64_t ldx, int64_t rows, int cols, double* out, hipStream_t s);
hipError_t launch_residual_t(const int64_t* col_ptr, const int32_t* row, const double* cval, int64_t n,
                             const double* R, int64_t ldr, double* S, int64_t lds, int nrhs, hipStream_t s);
hipError_t launch_csc(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, int64_t n,
                      int64_t* col_ptr, int32_t* row, double* cval, int32_t* work, hipStream_t s);
hipError_t launch_spmv_rows_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows,
                              const double* Xt, const double* Bt, double* Rt, int64_t ld, int nrhs, hipStream_t s);
hipError_t launch_spmv_cols_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t cols,
                              const double* Rt, double* St, int64_t ld, int nrhs, hipStream_t s);
hipError_t launch_colnorm_t(const double* Zt, int64_t ld, int64_t rows, int nrhs, double* out, hipStream_t s);
template <typename TI, typename TO, bool TO_T, bool ACC>
hipError_t launch_transpose(const TI* in, TO* out, int64_t rows, int cols, int64_t ldc, int64_t ldt, hipStream_t s);
}  // namespace ctqr

using namespace ctqr;

// ------------------------------------------------------------ error handling
static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, const char* what)
{
    snprintf(g_err, sizeof g_err, fmt, what);
    return code;
}

#define CT_ARG(cond, idx, msg)                                                   \
    do {                                                                         \
        if (!(cond)) return fail(-(idx), "invalid argument %s", msg);            \
    } while (0)

#define CT_HIP(expr)                                                             \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            snprintf(g_err, sizeof g_err, "%s: %s", #expr, hipGetErrorString(e_)); \
            return -1000 - (int)e_;                                              \
        }                                                                        \
    } while (0)

static bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// ------------------------------------------------------------- device setup
struct DevInfo {
    int ok = 0;
    int cus = 0;
    size_t lds_max = 0;      // dynamic LDS bytes one workgroup may use
    int trsm_block = 64;     // diagonal block of the triangular solves (R_bb in LDS)
};
static DevInfo g_dev;

static int device_setup()
{
    if (g_dev.ok) return 0;
    int dev;
    CT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t p;
    CT_HIP(hipGetDeviceProperties(&p, dev));
    g_dev.cus = p.multiProcessorCount;
    size_t want = 160 * 1024;
    if (p.maxSharedMemoryPerMultiProcessor > 0 && (size_t)p.maxSharedMemoryPerMultiProcessor < want)
        want = p.maxSharedMemoryPerMultiProcessor;
    if (panel_set_max_lds(want) != hipSuccess || trsm_set_max_lds(want) != hipSuccess ||
        t_from_gram_set_max_lds(want) != hipSuccess) {
        (void)hipGetLastError();
        want = 64 * 1024;
    }
    g_dev.lds_max = want;
    g_dev.trsm_block = want >= (size_t)128 * 129 * 8 ? 128 : 64;
    g_dev.ok = 1;
    return 0;
}

// ------------------------------------------------------------ factor handle
struct ct_factor {
    void* A;
    int64_t m, n, lda;
    int prec;
    bool f64;          // storage FP64 (else FP32)
    double* tau;
    int nb_out, nb_in;
    int64_t nblocks;
    // workspace partition
    double* T_all;     // nblocks x nb_out x nb_out
    double* Tin;       // 32 x 32
    double* part;      // 2 x 256 x 64
    double* gpart;     // 256 x 1024
    uint64_t* counter;
    int64_t* info;
    int32_t* err;
    void* Wp;
    int64_t wp_elems;  // capacity in 8-byte elements
    void* Wq;
    int64_t wq_elems;
    double* G;
    void* Vm;          // masked copy of the current reflector block, column-major (ld ldvm)
    void* Vt;          // the same block transposed (row-major, ld ldvt)
    int64_t ldvm;
    void* Ws;          // split-K sums
    uint64_t barrier_base;
    uint64_t* flag;
    uint64_t flag_base;
    int rw;            // panel rows per workgroup
    int64_t max_nrhs;
};

static int nb_out_for(int prec) { (void)prec; return 128; }

struct Layout {
    size_t T_all, Tin, part, gpart, words, Wp, Wq, G, Vm, Vt, Ws, total;
    int64_t wp_elems, wq_elems;
};

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout layout(int64_t m, int64_t n, int prec, int64_t max_nrhs)
{
    Layout L;
    const int nbo = nb_out_for(prec);
    const int64_t nblocks = (n + nbo - 1) / nbo;
    const int64_t ncap = std::max<int64_t>(n, 64 * std::max<int64_t>(max_nrhs, 1));
    L.wp_elems = (int64_t)nbo * ncap;
    L.wq_elems = (int64_t)nbo * std::max<int64_t>(n, std::max<int64_t>(max_nrhs, 1));
    size_t off = 0;
    L.T_all = off; off += up256((size_t)nblocks * nbo * nbo * 8);
    L.Tin = off; off += up256(32 * 32 * 8);
    L.part = off; off += up256(2 * 256 * 64 * 8 + 2 * 64 * 8);
    L.gpart = off; off += up256(256 * 1024 * 8);
    L.words = off; off += 256;
    L.Wp = off; off += up256((size_t)L.wp_elems * 8);
    L.Wq = off; off += up256((size_t)L.wq_elems * 8);
    L.G = off; off += up256((size_t)nbo * nbo * 8);
    const int64_t ldm = (m + 15) / 16 * 16;
    L.Vm = off; off += up256((size_t)ldm * nbo * 8);
    L.Vt = off; off += up256((size_t)ldm * nbo * 8);
    L.Ws = off; off += up256((size_t)L.wq_elems * 8);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- profiling
#include <vector>
struct ProfRec {
    hipEvent_t a, b;
    int kind;
    double flop, bytes;
};
static struct {
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
} g_prof;

static hipEvent_t prof_event()
{
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    ProfRec r;
    hipStream_t s;
    bool active;
    ProfScope(int kind, double flop, double bytes, hipStream_t st) : s(st), active(g_prof.on && kind >= 0)
    {
        if (!active) return;
        r.kind = kind; r.flop = flop; r.bytes = bytes;
        r.a = prof_event();
        r.b = prof_event();
        active = r.a && r.b;
        if (active) (void)hipEventRecord(r.a, s);
    }
    ~ProfScope()
    {
        if (!active) return;
        (void)hipEventRecord(r.b, s);
        g_prof.recs.push_back(r);
    }
};

// --------------------------------------------------------------- larfb core
// C (mk x nc) <- (I - V op(T) V^T) C ; OPT 0: T^T (apply Q^T), 1: T (apply Q)
static int64_t ldvt_of(int nbv) { return (nbv + 15) / 16 * 16; }

// Masked copies of the reflector block into f->Vm / f->Vt
template <typename TS>
static int prep_block(ct_factor* f, const TS* V, int64_t ldv, int64_t mk, int nbv, hipStream_t s)
{
    CT_HIP(launch_prep_v<TS>(V, ldv, mk, nbv, (TS*)f->Vm, f->ldvm, (TS*)f->Vt, ldvt_of(nbv), s));
    return 0;
}

// Block-reflector update with the LDS-tiled NT kernel (FP32 / FP64 arithmetic
// equal to the storage type); the block must already be in f->Vm / f->Vt.
template <typename TS, int MODE>
static hipError_t nt_any(const TS* X, int64_t ldx, const TS* Y, int64_t ldy, TS* out, int64_t ldo, int64_t P, int Q,
                         int64_t K, bool sub, int64_t ocap, int* nz, hipStream_t s)
{
    if constexpr (MODE == M_F64 || MODE == M_F32)
        return launch_nt<TS>(X, ldx, Y, ldy, out, ldo, P, Q, K, sub, ocap, nz, s);
    else
        return launch_nt_lp<MODE>(X, ldx, Y, ldy, out, ldo, P, Q, K, sub, ocap, nz, s);
}

template <typename TS, int OPT, int MODE = (sizeof(TS) == 8 ? M_F64 : M_F32)>
static int larfb_nt(ct_factor* f, int64_t mk, int nbv, const double* T, int64_t ldt, TS* C, int64_t ldc, int nc,
                    hipStream_t s, bool timed)
{
    const double fl = 2.0 * (double)mk * nbv * nc;
    const int64_t ldw = ldvt_of(nbv);
    int nz = 1;
    {
        ProfScope ps(timed ? 0 : -1, fl, ((double)mk * nbv + (double)mk * nc) * sizeof(TS) + (double)nbv * nc * sizeof(TS), s);
        CT_HIP((nt_any<TS, MODE>((const TS*)f->Vm, f->ldvm, C, ldc, (TS*)f->Wp, nbv, nbv, nc, mk, false,
                                 f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s)));
    }
    const TS* Wsum = (const TS*)f->Wp;
    if (nz > 1) {
        CT_HIP((launch_sum_slices<TS, TS>((const TS*)f->Wp, (int64_t)nbv * nc, nz, (int64_t)nbv * nc, (TS*)f->Ws, s)));
        Wsum = (const TS*)f->Ws;
    }
    CT_HIP((launch_tw<TS, TS, OPT, false>(Wsum, 1, nbv, nc, T, ldt, (TS*)f->Wq, nullptr, ldw, s)));
    {
        ProfScope ps(timed ? 1 : -1, fl, (double)mk * nbv * sizeof(TS) + (double)nbv * nc * sizeof(TS) + 2.0 * mk * nc * sizeof(TS), s);
        int nz2;
        CT_HIP((nt_any<TS, MODE>((const TS*)f->Vt, ldw, (const TS*)f->Wq, ldw, C, ldc, mk, nc, nbv, true, 0, &nz2, s)));
    }
    return 0;
}


// prepared: the block is already in f->Vm / f->Vt
template <typename TS, int OPT>
static int larfb_mode(ct_factor* f, int mode, const TS* V, int64_t ldv, int64_t mk, int nbv, const double* T,
                      int64_t ldt, TS* C, int64_t ldc, int nc, hipStream_t s, bool timed = false, bool prepared = false)
{
    if (!prepared) {
        int r = prep_block<TS>(f, V, ldv, mk, nbv, s);
        if (r) return r;
    }
    if constexpr (sizeof(TS) == 8) {
        return larfb_nt<TS, OPT, M_F64>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed);
    } else {
        switch (mode) {
            case M_F32: return larfb_nt<TS, OPT, M_F32>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed);
            case M_BF16: return larfb_nt<TS, OPT, M_BF16>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed);
            case M_F16: return larfb_nt<TS, OPT, M_F16>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed);
            case M_BF16X3: return larfb_nt<TS, OPT, M_BF16X3>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed);
        }
    }
    return fail(-1, "%s", "unsupported precision");
}


static int trailing_mode(int prec)
{
    switch (prec) {
        case CT_PREC_F64: return M_F64;
        case CT_PREC_F32: return M_F32;
        case CT_PREC_BF16: return M_BF16;
        case CT_PREC_F16: return M_F16;
        default: return M_BF16X3;
    }
}

// Gram of the masked reflector block and its compact-WY factor
// Gram of the prepared (masked) block in f->Vm, in the storage precision, and
// the compact-WY factor from it.
template <typename TS>
static int block_t(ct_factor* f, int64_t mk, int bo, const double* tau, double* T, int64_t ldt, hipStream_t s)
{
    int nz = 1;
    CT_HIP(launch_nt<TS>((const TS*)f->Vm, f->ldvm, (const TS*)f->Vm, f->ldvm, (TS*)f->Wp, bo, bo, bo, mk, false,
                         f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s));
    CT_HIP((launch_sum_slices<TS, double>((const TS*)f->Wp, (int64_t)bo * bo, nz, (int64_t)bo * bo, f->G, s)));
    CT_HIP(launch_t_from_gram(f->G, bo, tau, bo, T, ldt, s));
    return 0;
}

template <typename TS>
static int factor_impl(ct_factor* f, hipStream_t s)
{
    TS* A = (TS*)f->A;
    const int64_t m = f->m, n = f->n, lda = f->lda;
    const int nbo = f->nb_out, nbi = f->nb_in;
    const int mode = trailing_mode(f->prec);
    const int inner_mode = sizeof(TS) == 8 ? M_F64 : M_F32;
    for (int64_t b = 0; b < f->nblocks; ++b) {
        const int64_t k0 = b * nbo;
        const int bo = (int)std::min<int64_t>(nbo, n - k0);
        const int64_t mk = m - k0;
        double* Tb = f->T_all + (size_t)b * nbo * nbo;
        for (int64_t p0 = k0; p0 < k0 + bo; p0 += nbi) {
            const int bi = (int)std::min<int64_t>(nbi, k0 + bo - p0);
            const int64_t mkp = m - p0;
            TS* Vp = A + p0 + p0 * lda;
            // the panel writes its T straight into the block's T when it is the only panel
            double* Tp = (bo == bi) ? Tb : f->Tin;
            const int64_t ldtp = (bo == bi) ? nbo : 32;
            CT_HIP(launch_panel<TS>(Vp, lda, mkp, bi, f->rw, f->tau + p0, Tp, ldtp, f->part, f->gpart, f->counter,
                                    &f->barrier_base, f->flag, &f->flag_base, f->info, p0, f->err, s));
            const int64_t rest = k0 + bo - (p0 + bi);
            if (rest > 0) {
                int r = larfb_mode<TS, 0>(f, inner_mode, Vp, lda, mkp, bi, Tp, ldtp, A + p0 + (p0 + bi) * lda, lda,
                                          (int)rest, s);
                if (r) return r;
            }
        }
        const int64_t nc = n - k0 - bo;
        if (bo > nbi || nc > 0) {
            int r = prep_block<TS>(f, A + k0 + k0 * lda, lda, mk, bo, s);
            if (r) return r;
        }
        if (bo > nbi) {
            int r = block_t<TS>(f, mk, bo, f->tau + k0, Tb, nbo, s);
            if (r) return r;
        }
        if (nc > 0) {
            int r = larfb_mode<TS, 0>(f, mode, A + k0 + k0 * lda, lda, mk, bo, Tb, nbo, A + k0 + (k0 + bo) * lda, lda,
                                      (int)nc, s, true, true);
            if (r) return r;
        }
    }
    return 0;
}

template <typename TS>
static int apply_qt_impl(const ct_factor* fc, TS* B, int64_t nrhs, int64_t ldb, hipStream_t s, bool transpose)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    const TS* A = (const TS*)f->A;
    const int nbo = f->nb_out;
    const int mode = f->f64 ? M_F64 : M_F32;
    for (int64_t bb = 0; bb < f->nblocks; ++bb) {
        const int64_t b = transpose ? bb : f->nblocks - 1 - bb;
        const int64_t k0 = b * nbo;
        const int bo = (int)std::min<int64_t>(nbo, f->n - k0);
        const double* Tb = f->T_all + (size_t)b * nbo * nbo;
        int r = transpose ? larfb_mode<TS, 0>(f, mode, A + k0 + k0 * f->lda, f->lda, f->m - k0, bo, Tb, nbo, B + k0,
                                              ldb, (int)nrhs, s)
                          : larfb_mode<TS, 1>(f, mode, A + k0 + k0 * f->lda, f->lda, f->m - k0, bo, Tb, nbo, B + k0,
                                              ldb, (int)nrhs, s);
        if (r) return r;
    }
    return 0;
}

template <typename TS>
static int trsm_impl(const ct_factor* fc, TS* B, int64_t nrhs, int64_t ldb, hipStream_t s)
{
    const TS* A = (const TS*)fc->A;
    const int64_t n = fc->n, lda = fc->lda;
    const int tb = g_dev.trsm_block;
    const int64_t nb = (n + tb - 1) / tb;
    for (int64_t b = nb - 1; b >= 0; --b) {
        const int64_t k0 = b * tb;
        const int bo = (int)std::min<int64_t>(tb, n - k0);
        CT_HIP((launch_trsm_diag<TS, true>(A + k0 + k0 * lda, lda, bo, B + k0, ldb, (int)nrhs, s)));
        if (k0 > 0) {
            if constexpr (sizeof(TS) == 8)
                CT_HIP((launch_nn_sub<M_F64, TS, TS, TS, false>(A + k0 * lda, lda, B + k0, nullptr, ldb, B, ldb, k0,
                                                                (int)nrhs, bo, s)));
            else
                CT_HIP((launch_nn_sub<M_F32, TS, TS, TS, false>(A + k0 * lda, lda, B + k0, nullptr, ldb, B, ldb, k0,
                                                                (int)nrhs, bo, s)));
        }
    }
    return 0;
}

// Y[0:n] <- R^{-T} Y[0:n]: forward substitution on the lower-triangular R^T,
// diagonal-block solves alternating with GEMM updates from the rows above.
template <typename TS>
static int trsm_lt_impl(const ct_factor* fc, TS* Y, int64_t k, int64_t ldy, hipStream_t s)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    const TS* A = (const TS*)f->A;
    const int64_t n = f->n, lda = f->lda;
    const int tb = g_dev.trsm_block;
    const int64_t nb = (n + tb - 1) / tb;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t k0 = b * tb;
        const int bo = (int)std::min<int64_t>(tb, n - k0);
        if (k0 > 0) {
            // Y[k0:k0+bo] -= R[0:k0, k0:k0+bo]^T Y[0:k0]  (columns of R are K-contiguous)
            int nz = 1;
            CT_HIP(launch_nt<TS>(A + k0 * lda, lda, Y, ldy, (TS*)f->Wp, bo, bo, (int)k, k0, false,
                                 f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s));
            const TS* Wsum = (const TS*)f->Wp;
            if (nz > 1) {
                CT_HIP((launch_sum_slices<TS, TS>((const TS*)f->Wp, (int64_t)bo * k, nz, (int64_t)bo * k, (TS*)f->Ws, s)));
                Wsum = (const TS*)f->Ws;
            }
            CT_HIP((launch_tw<TS, TS, 3, false>(Wsum, 1, bo, (int)k, nullptr, 0, Y + k0, nullptr, ldy, s)));
        }
        CT_HIP((launch_trsm_diag<TS, false>(A + k0 + k0 * lda, lda, bo, Y + k0, ldy, (int)k, s)));
    }
    return 0;
}

template <typename TS>
static int backward_impl(const ct_factor* fc, const TS* G, int64_t k, int64_t ldg, TS* Y, int64_t ldy, hipStream_t s)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    CT_HIP((launch_convert<TS, TS>(G, ldg, Y, ldy, f->n, (int)k, s)));
    CT_HIP((launch_zero_rows<TS>(Y, ldy, f->n, f->m, (int)k, s)));
    int r = trsm_lt_impl<TS>(f, Y, k, ldy, s);
    if (r) return r;
    return apply_qt_impl<TS>(f, Y, k, ldy, s, false);
}

template <typename TS>
static int refined_impl(const ct_factor* f, const ct_sparse* sp, const double* B, int64_t ldb, double* X,
                        int64_t ldx, int64_t nrhs, int steps, int method, char* scratch, double* rnorms,
                        double* gnorms, hipStream_t s)
{
    const int64_t m = f->m, n = f->n;
    const int64_t ld = (m + 15) / 16 * 16;             // column-major correction block
    const int64_t lt = (nrhs + 15) / 16 * 16;           // slice-contiguous blocks
    char* p = scratch;
    double* Bt = (double*)p; p += up256((size_t)m * lt * 8);
    double* Rt = (double*)p; p += up256((size_t)m * lt * 8);
    double* Xt = (double*)p; p += up256((size_t)n * lt * 8);
    double* St = (double*)p; p += up256((size_t)n * lt * 8);
    TS* C = (TS*)p;
    const bool have_csc = sp->col_ptr && sp->row && sp->cval;
    const int nr = (int)nrhs;
    CT_HIP((launch_transpose<double, double, true, false>(B, Bt, m, nr, ldb, lt, s)));
    // x_0 = R~^{-1} Q~^T b
    CT_HIP((launch_convert<double, TS>(B, ldb, C, ld, m, nr, s)));
    int r = ct_apply_qt(f, C, nrhs, ld, s);
    if (r) return r;
    r = ct_trsm_solve(f, C, nrhs, ld, s);
    if (r) return r;
    CT_HIP((launch_convert<TS, double>(C, ld, X, ldx, n, nr, s)));
    CT_HIP((launch_transpose<TS, double, true, false>(C, Xt, n, nr, ld, lt, s)));
    for (int st = 0; st <= steps; ++st) {
        // r_st = b - A x_st (FP64)
        CT_HIP(launch_spmv_rows_t(sp->row_ptr, sp->col, sp->val, m, Xt, Bt, Rt, lt, nr, s));
        if (rnorms) CT_HIP(launch_colnorm_t(Rt, lt, m, nr, rnorms + (size_t)st * nrhs, s));
        const bool need_grad = method == CT_REFINE_SNE ? st < steps : false;
        if (have_csc && (need_grad || gnorms)) {
            CT_HIP(launch_spmv_cols_t(sp->col_ptr, sp->row, sp->cval, n, Rt, St, lt, nr, s));
            if (gnorms) CT_HIP(launch_colnorm_t(St, lt, n, nr, gnorms + (size_t)st * nrhs, s));
        }
        if (st == steps) break;
        if (method == CT_REFINE_SNE) {
            // x += R~^{-1} R~^{-T} (A^T r)
            CT_HIP((launch_transpose<double, TS, false, false>(St, C, n, nr, ld, lt, s)));
            r = trsm_lt_impl<TS>(f, C, nrhs, ld, s);
            if (r) return r;
        } else {
            // x += R~^{-1} Q~^T r
            CT_HIP((launch_transpose<double, TS, false, false>(Rt, C, m, nr, ld, lt, s)));
            r = ct_apply_qt(f, C, nrhs, ld, s);
            if (r) return r;
        }
        r = ct_trsm_solve(f, C, nrhs, ld, s);
        if (r) return r;
        CT_HIP((launch_accumulate<TS>(X, ldx, C, ld, n, nr, s)));
        CT_HIP((launch_transpose<TS, double, true, true>(C, Xt, n, nr, ld, lt, s)));
    }
    return 0;
}

// ------------------------------------------------------------------- C ABI
extern "C" {

const char* ct_last_error(void) { return g_err; }

int ct_build_system(const ct_geometry* g, int dtype, void* A, int64_t lda, void* stream)
{
    CT_ARG(g != nullptr, 1, "g");
    CT_ARG(g->n_pix > 0 && g->n_angles > 0 && g->n_det > 0, 1, "g (sizes)");
    CT_ARG(g->grid_width > 0 && g->sdd > 0 && g->sid > 0.5 * g->grid_width * 1.4142135623730951, 1,
           "g (source must lie outside the image)");
    CT_ARG(dtype == CT_F64 || dtype == CT_F32, 2, "dtype");
    CT_ARG(A != nullptr && aligned(A), 3, "A");
    const int64_t m = (int64_t)g->n_angles * g->n_det;
    CT_ARG(lda >= m && lda % 16 == 0, 4, "lda");
    GeomDev gd{g->n_pix, g->n_angles, g->n_det, g->grid_width, g->sid, g->sdd, g->det_length, g->angle0};
    CT_HIP(launch_siddon_dense(gd, dtype, A, lda, (hipStream_t)stream));
    return 0;
}

int ct_build_csr(const ct_geometry* g, int64_t* row_ptr, int32_t* col, double* val, int64_t nnz_cap, void* stream)
{
    CT_ARG(g != nullptr && g->n_pix > 0 && g->n_angles > 0 && g->n_det > 0, 1, "g");
    CT_ARG(row_ptr != nullptr, 2, "row_ptr");
    CT_ARG((col == nullptr) == (val == nullptr), 3, "col/val (both or neither)");
    CT_ARG(col == nullptr || nnz_cap > 0, 5, "nnz_cap");
    GeomDev gd{g->n_pix, g->n_angles, g->n_det, g->grid_width, g->sid, g->sdd, g->det_length, g->angle0};
    CT_HIP(launch_siddon_csr(gd, row_ptr, col, val, nnz_cap, (hipStream_t)stream));
    return 0;
}

int ct_qr_workspace(int64_t m, int64_t n, int prec, int64_t max_nrhs, size_t* bytes)
{
    CT_ARG(m > 0, 1, "m");
    CT_ARG(n > 0 && n <= m, 2, "n (need 0 < n <= m)");
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 3, "prec");
    CT_ARG(max_nrhs >= 0, 4, "max_nrhs");
    CT_ARG(bytes != nullptr, 5, "bytes");
    *bytes = layout(m, n, prec, max_nrhs).total;
    return 0;
}

int ct_qr_factor(void* A, int64_t m, int64_t n, int64_t lda, int prec, double* tau, void* work, size_t work_bytes,
                 int64_t max_nrhs, ct_factor** f_out, void* stream)
{
    CT_ARG(A != nullptr && aligned(A), 1, "A");
    CT_ARG(m > 0, 2, "m");
    CT_ARG(n > 0 && n <= m, 3, "n (need 0 < n <= m)");
    CT_ARG(lda >= m && lda % 16 == 0, 4, "lda");
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 5, "prec");
    CT_ARG(tau != nullptr, 6, "tau");
    CT_ARG(work != nullptr && aligned(work), 7, "work");
    CT_ARG(max_nrhs >= 0, 9, "max_nrhs");
    CT_ARG(f_out != nullptr, 10, "f");
    const Layout L = layout(m, n, prec, max_nrhs);
    CT_ARG(work_bytes >= L.total, 8, "work_bytes (see ct_qr_workspace)");
    int r = device_setup();
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;

    ct_factor* f = new (std::nothrow) ct_factor();
    if (!f) return fail(-1001, "%s", "out of host memory");
    char* w = (char*)work;
    f->A = A; f->m = m; f->n = n; f->lda = lda; f->prec = prec; f->f64 = prec == CT_PREC_F64;
    f->tau = tau;
    f->nb_out = nb_out_for(prec);
    f->nblocks = (n + f->nb_out - 1) / f->nb_out;
    f->T_all = (double*)(w + L.T_all);
    f->Tin = (double*)(w + L.Tin);
    f->part = (double*)(w + L.part);
    f->gpart = (double*)(w + L.gpart);
    f->counter = (uint64_t*)(w + L.words);
    f->info = (int64_t*)(w + L.words + 64);
    f->err = (int32_t*)(w + L.words + 128);
    f->flag = (uint64_t*)(w + L.words + 192);
    f->flag_base = 0;
    f->Wp = w + L.Wp; f->wp_elems = L.wp_elems;
    f->Wq = w + L.Wq; f->wq_elems = L.wq_elems;
    f->G = (double*)(w + L.G);
    f->Vm = w + L.Vm;
    f->Vt = w + L.Vt;
    f->ldvm = (m + 15) / 16 * 16;
    f->Ws = w + L.Ws;
    f->barrier_base = 0;
    f->max_nrhs = max_nrhs;

    // panel geometry: rows per workgroup from the LDS budget; all workgroups
    // of a panel must be resident at once (one per CU at this LDS size)
    const size_t lds_words = g_dev.lds_max / 8 - panel_aux_words();
    int nbi = 32;
    int rw = (int)(lds_words / nbi);
    if ((rw & 1) == 0) --rw;
    if ((m + rw - 1) / rw > g_dev.cus) {
        nbi = 16;
        rw = (int)(lds_words / nbi);
        if ((rw & 1) == 0) --rw;
    }
    if ((m + rw - 1) / rw > g_dev.cus) {
        delete f;
        return fail(-2, "%s", "m too large for a resident panel on this device");
    }
    int per_cu = 0;
    CT_HIP(panel_max_active(&per_cu, panel_lds_bytes(nbi, rw)));
    if (per_cu < 1) {
        delete f;
        return fail(-1002, "%s", "panel kernel cannot be resident");
    }
    f->nb_in = nbi;
    f->rw = rw;

    CT_HIP(hipMemsetAsync(w + L.words, 0, 256, s));
    int rc = f->f64 ? factor_impl<double>(f, s) : factor_impl<float>(f, s);
    if (rc) {
        delete f;
        return rc;
    }
    *f_out = f;
    return 0;
}


int ct_apply_qt(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(B != nullptr && aligned(B), 2, "B");
    CT_ARG(nrhs >= 0 && nrhs <= f->max_nrhs, 3, "nrhs (0..max_nrhs)");
    CT_ARG(ldb >= f->m && ldb % 16 == 0, 4, "ldb");
    if (nrhs == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? apply_qt_impl<double>(f, (double*)B, nrhs, ldb, s, true)
                  : apply_qt_impl<float>(f, (float*)B, nrhs, ldb, s, true);
}


int ct_trsm_solve(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(B != nullptr && aligned(B), 2, "B");
    CT_ARG(nrhs >= 0, 3, "nrhs");
    CT_ARG(ldb >= f->n && ldb % 16 == 0, 4, "ldb");
    if (nrhs == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? trsm_impl<double>(f, (double*)B, nrhs, ldb, s) : trsm_impl<float>(f, (float*)B, nrhs, ldb, s);
}


int ct_solve_backward(const ct_factor* f, const void* G, int64_t k, int64_t ldg, void* gradB, int64_t ldgb,
                      void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(G != nullptr && aligned(G), 2, "G");
    CT_ARG(k >= 0 && k <= f->max_nrhs, 3, "k (0..max_nrhs)");
    CT_ARG(ldg >= f->n && ldg % 16 == 0, 4, "ldg");
    CT_ARG(gradB != nullptr && aligned(gradB), 5, "gradB");
    CT_ARG(ldgb >= f->m && ldgb % 16 == 0, 6, "ldgb");
    if (k == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? backward_impl<double>(f, (const double*)G, k, ldg, (double*)gradB, ldgb, s)
                  : backward_impl<float>(f, (const float*)G, k, ldg, (float*)gradB, ldgb, s);
}

int ct_residual(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, const double* X,
                int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs, void* stream)
{
    CT_ARG(row_ptr && col && val, 1, "CSR arrays");
    CT_ARG(m > 0, 4, "m");
    CT_ARG(X != nullptr, 5, "X");
    CT_ARG(B != nullptr && ldb >= m, 7, "B/ldb");
    CT_ARG(R != nullptr && ldr >= m, 9, "R/ldr");
    CT_ARG(nrhs >= 0, 11, "nrhs");
    if (nrhs == 0) return 0;
    CT_HIP(launch_residual(row_ptr, col, val, m, X, ldx, B, ldb, R, ldr, (int)nrhs, (hipStream_t)stream));
    return 0;
}

int ct_refine_workspace(int64_t m, int64_t n, int64_t nrhs, size_t* bytes)
{
    CT_ARG(m > 0, 1, "m");
    CT_ARG(n > 0, 2, "n");
    CT_ARG(nrhs >= 0, 3, "nrhs");
    CT_ARG(bytes != nullptr, 4, "bytes");
    const int64_t ld = (m + 15) / 16 * 16, lt = (nrhs + 15) / 16 * 16;
    *bytes = 2 * up256((size_t)m * lt * 8) + 2 * up256((size_t)n * lt * 8) + up256((size_t)ld * nrhs * 8);
    return 0;
}

int ct_build_csc(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                 int64_t* col_ptr, int32_t* row, double* cval, int32_t* work, void* stream)
{
    CT_ARG(m > 0, 1, "m");
    CT_ARG(n > 0, 2, "n");
    CT_ARG(row_ptr && col && val, 3, "CSR arrays");
    CT_ARG(col_ptr && row && cval, 6, "CSC arrays");
    CT_ARG(work != nullptr, 9, "work");
    CT_HIP(launch_csc(row_ptr, col, val, m, n, col_ptr, row, cval, work, (hipStream_t)stream));
    return 0;
}


int ct_solve_refined(const ct_factor* f, const ct_sparse* sp, const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, int32_t steps, int32_t method, void* scratch, size_t scratch_bytes,
                     double* res_norms, double* grad_norms, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(sp != nullptr && sp->row_ptr && sp->col && sp->val && sp->m == f->m && sp->n == f->n, 2,
           "A (CSR copy of the factored matrix)");
    CT_ARG(B != nullptr && ldb >= f->m, 3, "B/ldb");
    CT_ARG(X != nullptr && ldx >= f->n, 5, "X/ldx");
    CT_ARG(nrhs >= 0 && nrhs <= f->max_nrhs, 7, "nrhs (0..max_nrhs)");
    CT_ARG(steps >= 0 && steps <= 64, 8, "steps");
    CT_ARG(method == CT_REFINE_QR || method == CT_REFINE_SNE, 9, "method");
    CT_ARG(method != CT_REFINE_SNE || (sp->col_ptr && sp->row && sp->cval), 2, "A (CT_REFINE_SNE needs the CSC copy)");
    size_t need = 0;
    ct_refine_workspace(f->m, f->n, nrhs, &need);
    CT_ARG(scratch != nullptr && aligned(scratch) && scratch_bytes >= need, 10, "scratch");
    if (nrhs == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? refined_impl<double>(f, sp, B, ldb, X, ldx, nrhs, steps, method, (char*)scratch, res_norms,
                                         grad_norms, s)
                  : refined_impl<float>(f, sp, B, ldb, X, ldx, nrhs, steps, method, (char*)scratch, res_norms,
                                        grad_norms, s);
}

int ct_status(const ct_factor* f, int64_t* info, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(info != nullptr, 2, "info");
    hipStream_t s = (hipStream_t)stream;
    int64_t words[2] = {0, 0};
    int32_t err = 0;
    CT_HIP(hipMemcpyAsync(&words[0], f->info, 8, hipMemcpyDeviceToHost, s));
    CT_HIP(hipMemcpyAsync(&err, f->err, 4, hipMemcpyDeviceToHost, s));
    CT_HIP(hipStreamSynchronize(s));
    *info = words[0];
    if (err & 1) return fail(-2001, "%s", "a cross-workgroup wait timed out during the factorization");
    return 0;
}

int ct_factor_destroy(ct_factor* f)
{
    delete f;
    return 0;
}

int ct_profile_begin(void)
{
    for (auto& r : g_prof.recs) {
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
    g_prof.on = true;
    return 0;
}

int ct_profile_end(ct_profile* out)
{
    CT_ARG(out != nullptr, 1, "out");
    g_prof.on = false;
    memset(out, 0, sizeof *out);
    for (auto& r : g_prof.recs) {
        CT_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        CT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        out->launches[r.kind] += 1;
        out->ms[r.kind] += ms;
        out->flop[r.kind] += r.flop;
        out->bytes[r.kind] += r.bytes;
    }
    return 0;
}

int ct_siddon_rows(const double* rays_host, int64_t r, int32_t n_pix, double grid_width, double* rows_host)
{
    CT_ARG(rays_host != nullptr, 1, "rays_host");
    CT_ARG(r >= 0, 2, "r");
    CT_ARG(n_pix > 0, 3, "n_pix");
    CT_ARG(grid_width > 0, 4, "grid_width");
    CT_ARG(rows_host != nullptr, 5, "rows_host");
    if (r == 0) return 0;
    const size_t nr = (size_t)r * n_pix * n_pix;
    double *d_rays = nullptr, *d_rows = nullptr;
    CT_HIP(hipMalloc(&d_rays, (size_t)r * 4 * 8));
    hipError_t e = hipMalloc(&d_rows, nr * 8);
    if (e == hipSuccess) e = hipMemcpy(d_rays, rays_host, (size_t)r * 4 * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_siddon_rows(d_rays, r, n_pix, grid_width, d_rows, nullptr);
    if (e == hipSuccess) e = hipMemcpy(rows_host, d_rows, nr * 8, hipMemcpyDeviceToHost);
    (void)hipFree(d_rays);
    if (d_rows) (void)hipFree(d_rows);
    CT_HIP(e);
    return 0;
}

}  // extern "C"
