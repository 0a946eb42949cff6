// C-ABI of libctqr: argument checks, workspace layout, and the host-side
// schedule of the blocked Householder QR and of the solve (Eqs. (qr),
// (solve); the in-memory method of Sec. 2.1 with the blocked triangular
// solve of Sec. 2.2).
#include "ct_internal.h"
#include "../../include/ctqr.h"

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace ctqr {
hipError_t launch_siddon_dense(const GeomDev& g, int dtype, void* A, int64_t lda, hipStream_t s);
hipError_t launch_siddon_csr(const GeomDev& g, int64_t* row_ptr, int32_t* col, double* val, int64_t cap,
                             hipStream_t s);
hipError_t launch_siddon_rows(const double* rays, int64_t r, int32_t N, double W, double* rows, hipStream_t s);
template <typename TS>
hipError_t launch_panel(TS* A, int64_t lda, int64_t mk, int nbp, int rw, double* tau, double* T, int64_t ldt,
                        double* part, double* gpart, uint64_t* counter, uint64_t* base, uint64_t* col_base,
                        uint64_t* cq_count, int64_t* info, int64_t col0, int32_t* err, hipStream_t s);
hipError_t panel_reset(double* part, double* gpart, hipStream_t s);
void panel_set_cholesky(bool on);
hipError_t launch_quality(const double* X, int64_t ldx, const double* R, int64_t ldr, int N, int64_t k,
                          const int* crop, int win, double* out, hipStream_t s);
void panel_set_cus(int cus);
size_t panel_lds_bytes(int nbp, int rw);
int panel_aux_words();
size_t panel_scratch_words();
hipError_t panel_set_max_lds(size_t bytes);
hipError_t panel_max_active(int* per_cu, size_t shmem);
void panel_set_wait_limit(int64_t ticks);
template <int MODE, typename TA, typename TB, typename TW, bool MA, bool MB_>
hipError_t launch_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, TW* W, int M, int N, int64_t K,
                     int64_t wcap, int* nz_out, hipStream_t s);
template <int MODE, typename TA, typename TB, typename TC, bool MA>
hipError_t launch_nn_sub(const TA* A, int64_t lda, const TB* Bhi, const TB* Blo, int64_t ldb, TC* C, int64_t ldc,
                         int64_t M, int N, int K, hipStream_t s, const int32_t* desc = nullptr);
template <typename TWp, typename TO, int OP, bool SPLIT>
hipError_t launch_tw(const TWp* Wp, int nz, int nbv, int N, const double* T, int64_t ldt, TO* out, TO* out_lo,
                     int64_t ldo, hipStream_t s, const int32_t* desc = nullptr);
hipError_t launch_t_join(const double* G, int64_t ldg, double* T, int64_t ldt, double* M, int nb_panel, int bo,
                         hipStream_t s);
template <typename TWp, typename TS>
hipError_t launch_sum_slices(const TWp* Wp, int64_t wstride, int nz, int64_t count, TS* S, hipStream_t s,
                             const int32_t* desc = nullptr, int per_col = 1);
template <typename T>
hipError_t launch_prep_v(const T* V, int64_t ldv, int64_t mk, int nb, T* Vm, int64_t ldm, T* Vt, int64_t ldvt,
                         hipStream_t s);
template <typename T>
hipError_t launch_nt(const T* X, int64_t ldx, const T* Y, int64_t ldy, T* out, int64_t ldo, int64_t P, int Q,
                     int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s, const NtPlan* plan = nullptr,
                     const int32_t* desc = nullptr, int desc_y = 0, int desc_out = 0, int maskx = 0,
                     int tout = 0, int upper = 0);
extern NtPlan g_nt_default;
template <int MODE>
hipError_t launch_nt_lp(const void* X, int64_t ldx, const void* Y, int64_t ldy, float* out, int64_t ldo, int64_t P,
                        int Q, int64_t K, bool sub, int64_t ocap, int* nz_out, hipStream_t s,
                        const void* Xlo = nullptr, const void* Ylo = nullptr);
hipError_t launch_nt_x3dl(const void* Xh, const void* Xl, int64_t ldx, const void* Yh, const void* Yl, int64_t ldy,
                          float* out, int64_t ldo, int64_t P, int Q, int64_t K, bool sub, int64_t ocap, int* nz_out,
                          hipStream_t s);
// the direct-to-LDS BF16x3 products take blocks of at least this many
// reflectors (narrower ones would leave most of a 256-row tile empty)
constexpr int kX3dlMinWidth = 256;
// up to this many columns (the solves' right-hand sides) the FP32 operands
// are split as they are read instead of being split in a pass of their own
constexpr int kX3dlSplitAtRead = 2048;
void nt_set_cus(int cus);
hipError_t launch_split_x3(const float* src, int64_t lds, void* hi, void* lo, int64_t ldd, int64_t rows, int64_t cols,
                           hipStream_t s);
template <typename TS, bool UPPER>
hipError_t launch_trsm_diag(const TS* R, int64_t ldr, int bo, TS* B, int64_t ldb, int nrhs, hipStream_t s,
                            const int32_t* desc = nullptr);
hipError_t launch_begin_batch(const int32_t* desc, int32_t* rec, int max_cols, int64_t b_cols, int32_t* err,
                              hipStream_t s);
hipError_t launch_end_batch(int32_t* desc, hipStream_t s);
hipError_t trsm_set_max_lds(size_t bytes);
template <typename TS>
hipError_t launch_rinv(const TS* A, int64_t lda, int64_t n, TS* RiR, TS* RiC, double* Ri64, double* M, hipStream_t s);
template <typename TS>
hipError_t launch_rt(const TS* A, int64_t lda, int64_t n, int ob, TS* Rt, hipStream_t s);
size_t rt_elems(int64_t n, int ob);
template <typename TS>
hipError_t launch_eye(TS* C, int64_t ld, int64_t rows, int cols, int w, hipStream_t s);
template <typename TS>
hipError_t launch_copy_block(const TS* src, int64_t lds, TS* dst, int64_t ldd, int rows, int cols, hipStream_t s,
                             const int32_t* desc);
hipError_t rinv_set_max_lds(size_t bytes);
hipError_t launch_diag_x3(const float* Ri, float* B, int64_t ldb, int bo, int nrhs, hipStream_t s);
hipError_t launch_diag_f32(const float* Ri, float* B, int64_t ldb, int bo, int nrhs, const int32_t* desc,
                           hipStream_t s);
hipError_t launch_residual(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int nrhs,
                           hipStream_t s);
template <typename TI, typename TO>
hipError_t launch_convert(const TI* X, int64_t ldx, TO* Y, int64_t ldy, int64_t rows, int cols, hipStream_t s);
template <typename TD>
hipError_t launch_accumulate(double* X, int64_t ldx, const TD* D, int64_t ldd, int64_t rows, int cols,
                             hipStream_t s);
template <typename TD>
hipError_t launch_corr_ratio(const TD* D, int64_t ldd, const double* X, int64_t ldx, int64_t rows, int cols,
                             double* ratio, unsigned long long* maxw, hipStream_t s);
template <typename T>
hipError_t launch_zero_rows(T* Y, int64_t ldy, int64_t r0, int64_t r1, int cols, hipStream_t s);
hipError_t launch_colnorm(const double* X, int64_t ldx, int64_t rows, int cols, double* out, hipStream_t s);
template <typename T>
hipError_t launch_colsq(const T* C, int64_t ldc, int64_t rows, int cols, double* out, hipStream_t s);
template <typename TS>
hipError_t launch_fused_solve(const FusedArgs& a, int G, bool cooperative, hipStream_t s);
int fused_row_groups(int nbo, int64_t n, size_t es, size_t bytes, int kc, int cap);
uint64_t panel_wait_limit();
hipError_t launch_cg_update(const double* x, double* y, int64_t rows, int nrhs, int64_t ld, const double* num,
                            const double* den, int mode, hipStream_t s);
hipError_t launch_cg_ratio(const double* gam, const double* qn, const double* pn, const double* xn, int nrhs,
                           unsigned long long* maxw, hipStream_t s);
hipError_t launch_residual_t(const int64_t* col_ptr, const int32_t* row, const double* cval, int64_t n,
                             const double* R, int64_t ldr, double* S, int64_t lds, int nrhs, hipStream_t s);
hipError_t launch_csc(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, int64_t n,
                      int64_t* col_ptr, int32_t* row, double* cval, int32_t* work, hipStream_t s);
hipError_t launch_group_count(const int64_t* ptr, const int32_t* idx, int64_t rows, int group, int64_t* gptr,
                              int32_t* err, hipStream_t s);
hipError_t launch_group_fill(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, int group,
                             const int64_t* gptr, int32_t* gidx, double* gval, int64_t count, hipStream_t s);
hipError_t launch_group_spmm(const int64_t* gptr, const int32_t* gidx, const double* gval, int group, int64_t rows,
                             const double* Z, const double* B, double* out, int64_t ld, int nrhs, bool sub,
                             hipStream_t s);
hipError_t launch_spmv_rows_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows,
                              const double* Xt, const double* Bt, double* Rt, int64_t ld, int nrhs, hipStream_t s);
hipError_t launch_spmv_cols_t(const int64_t* ptr, const int32_t* idx, const double* val, int64_t cols,
                              const double* Rt, double* St, int64_t ld, int nrhs, hipStream_t s);
hipError_t launch_colnorm_t(const double* Zt, int64_t ld, int64_t rows, int nrhs, double* out, double* part,
                            hipStream_t s);
template <typename TI, typename TO, bool TO_T, bool ACC>
hipError_t launch_transpose(const TI* in, TO* out, int64_t rows, int cols, int64_t ldc, int64_t ldt, hipStream_t s);
}  // namespace ctqr

using namespace ctqr;

// ------------------------------------------------------------ error handling
static thread_local char g_err[512] = "";

__attribute__((format(printf, 2, 3))) static int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
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
    panel_set_cus(g_dev.cus);
    nt_set_cus(g_dev.cus);
    size_t want = 160 * 1024;
    if (p.maxSharedMemoryPerMultiProcessor > 0 && (size_t)p.maxSharedMemoryPerMultiProcessor < want)
        want = p.maxSharedMemoryPerMultiProcessor;
    if (panel_set_max_lds(want) != hipSuccess || trsm_set_max_lds(want) != hipSuccess ||
        rinv_set_max_lds(want) != hipSuccess) {
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
    double* part;      // 2 x 256 x 64
    double* gpart;     // the two-reduction panels' polled scratch
    uint64_t* counter;
    int64_t* info;
    int32_t* err;
    int32_t* batch_rec;   // (offset, count) of the current batch of a graph-captured solve
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
    uint64_t col_base;  // panel columns factored so far (parity of the panel's result slots)
    uint64_t cq_count;  // two-reduction panel launches so far (parity of their result slots)
    NtPlan solve_plan[5];   // per batch-size bucket (<=8, <=32, <=128, <=512, more)
    int rw;            // panel rows per workgroup
    int64_t max_nrhs;
    struct StreamState* st = nullptr;   // host-pinned streaming state (null: A is in device memory)
    // solve-side copies of R (in-memory factors): inverses of the 128 x 128
    // diagonal blocks, row- and column-major, and the row-major block columns
    void* RiR = nullptr;
    void* RiC = nullptr;
    void* Rt = nullptr;
    int rt_ob = 256;   // outer block of the two-level row-major R copy (see rt_kernel)
    // BF16x3 factors: inverses of the 1024 x 1024 diagonal blocks of R (FP32),
    // column-major (RiC4) and row-major (RiR4), for the refinement's solves
    void* RiC4 = nullptr;
    void* RiR4 = nullptr;
    // row-major copies of the outer reflector blocks (in-memory factors),
    // written by the factorization and reused by every solve
    void* VtAll = nullptr;
    // T of every outer block in the storage type (FP32 factors; FP64 ones use T_all)
    void* Tf = nullptr;
    // bfloat16 high / low parts of the current reflector block (BF16x3 updates)
    void* S3 = nullptr;
    // FP32 factors: blockdiag(R_qq^{-1}) R right of the 256 x 256 diagonal
    // blocks (fused_rh_off), built by the first fused solve and owned by the
    // factor (library allocation)
    mutable void* Rh = nullptr;
};

// Outer block width.  The trailing update of a block of nbo reflectors reads
// and writes the remaining columns once, so its arithmetic intensity grows
// with nbo (2 nbo / 8 flop per FP32 byte); the work inside a block (panels
// and their rank-32 updates, the block's Gram matrix) grows with it too.
// Measured on MI355X at 76800 x 65536: BF16x3 QR 3.46 s (256), 3.07 s (512),
// 3.02 s (768), 2.91 s (1024), 3.08 s (2048); at 23040 x 16384 the width
// changes little except in FP64 (494 ms at 256, 451 ms at 1024).  A streamed
// factor uses kNbStream when its column tiles allow, else 128.
constexpr int kNbStream = 256;

static int g_nb_force = 0;   // test hook: forced outer block width (0: by size)
static int g_nbi_force = 0;  // test hook: forced panel width (0: 32, or 16 for panels too tall for 32)
// BF16x3 products in the refinement of a BF16x3 factor: 0 never, 1 from
// kX3MinSlices slices (below that the extra launches cost more than the
// products save), 2 always
static int g_x3_refine = 1;
constexpr int64_t kX3MinSlices = 48;
static int64_t g_progress_blocks = 0;   // ct_debug_progress
static int nb_out_for(int64_t n) { return g_nb_force ? g_nb_force : (n >= 16384 ? 1024 : 256); }

struct Layout {
    size_t T_all, part, gpart, words, Wp, Wq, G, Vm, Vt, Ws, Ri, Ri64, Rt, Ri4, VtAll, Tf, S3, total;
    int64_t wp_elems, wq_elems;
};

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Outer block of the blocked triangular solves: the rows above an outer
// block of 1024 columns are updated once, by one product with K = 1024,
// instead of four times with K = 256 (each update reads and writes them).
static int rt_ob_for(int64_t n) { return n >= 2048 ? 1024 : 256; }

// Solve-side copies kept by a factorization: none (streamed factors), the
// diagonal-block inverses only (in-memory factors without the row-major
// copies, CT_QR_NO_SOLVE_COPIES), or all of them.
enum CopyLevel { kCopiesNone = 0, kCopiesInverses = 1, kCopiesAll = 2 };

// The FP64 scratch of the 256-block inverses borrows Wp when it is large enough
// (it is free once the factorization is done) in a factorization without the
// row-major copies.
static bool ri64_in_wp(const Layout& L, int64_t n) { return L.wp_elems >= ((n + 255) / 256) * 256 * 256; }

static Layout layout(int64_t m, int64_t n, int prec, int64_t max_nrhs, int nbo, int level = kCopiesAll)
{
    Layout L;
    const int64_t nblocks = (n + nbo - 1) / nbo;
    const int64_t ncap = std::max<int64_t>(n, 64 * std::max<int64_t>(max_nrhs, 1));
    L.wp_elems = (int64_t)nbo * ncap;
    L.wq_elems = (int64_t)nbo * std::max<int64_t>(n, std::max<int64_t>(max_nrhs, 1));
    size_t off = 0;
    L.T_all = off; off += up256((size_t)nblocks * nbo * nbo * 8);
    L.part = off; off += up256(2 * 256 * 64 * 8 + 2 * 64 * 8);
    L.gpart = off; off += up256(panel_scratch_words() * 8);
    L.words = off; off += 256;
    L.Wp = off; off += up256((size_t)L.wp_elems * 8);
    L.Wq = off; off += up256((size_t)L.wq_elems * 8);
    L.G = off; off += up256((size_t)nbo * nbo * 8);
    const int64_t ldm = (m + 15) / 16 * 16;
    L.Vm = off; off += up256((size_t)ldm * nbo * 8);
    L.Vt = off; off += up256((size_t)ldm * nbo * 8);
    L.Ws = off; off += up256((size_t)L.wq_elems * 8);
    // R copies for the solves: 2 inverses per 256-row block (and their FP64
    // scratch), and the block columns above the diagonal (256^2 nbt (nbt - 1)
    // / 2 elements)
    const size_t es = prec == CT_PREC_F64 ? 8 : 4;
    const int64_t nbt = (n + 255) / 256;
    const bool inv = level >= kCopiesInverses, all = level == kCopiesAll;
    L.Ri = off; off += inv ? up256((size_t)2 * nbt * 256 * 256 * es) : 0;
    L.Ri64 = off; off += (all || (inv && !ri64_in_wp(L, n))) ? up256((size_t)nbt * 256 * 256 * 8) : 0;
    L.Rt = off; off += all ? up256(rt_elems(n, rt_ob_for(n)) * es) : 0;
    // BF16x3: the inverses of the 1024-column diagonal blocks, two layouts
    const int64_t nb4 = (n + 1023) / 1024;
    L.Ri4 = off; off += (inv && prec == CT_PREC_BF16X3 && rt_ob_for(n) == 1024)
                            ? up256((size_t)2 * nb4 * 1024 * 1024 * 4) : 0;
    // reflector blocks, row-major: block b holds (m - b nbo) rows of nbo
    L.VtAll = off; off += all ? up256((size_t)(nblocks * m - nbo * (nblocks * (nblocks - 1) / 2)) * nbo * es) : 0;
    L.Tf = off; off += prec == CT_PREC_F64 ? 0 : up256((size_t)nblocks * nbo * nbo * 4);
    L.S3 = off; off += prec == CT_PREC_BF16X3 ? up256((size_t)ldm * nbo * 4) : 0;
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
static int prep_block(ct_factor* f, const TS* V, int64_t ldv, int64_t mk, int nbv, hipStream_t s,
                      TS* vt_dst = nullptr, bool with_vt = true)
{
    CT_HIP(launch_prep_v<TS>(V, ldv, mk, nbv, (TS*)f->Vm, f->ldvm,
                             with_vt ? (vt_dst ? vt_dst : (TS*)f->Vt) : nullptr, ldvt_of(nbv), s));
    return 0;
}

// Operands of a block-reflector update: the block K-contiguous by reflector
// (vm, ld ldvm; mask: read in place from the factored matrix, triangle
// masked by the kernel) and K-contiguous by row (vt, ld ldvt).
struct VOps {
    const void* vm;
    int64_t ldvm;
    int mask;
    const void* vt;
    int64_t ldvt;
    const void* tts;   // T in the storage type (column-major, ld as T, zero below
                       // the diagonal) for an MFMA T^T W; null: FP64 T through tw
};

// Offset (elements) of outer block b in the row-major reflector store.
static size_t vt_offset(const ct_factor* f, int64_t b)
{
    const int64_t nbo = f->nb_out;
    return (size_t)(b * f->m - nbo * (b * (b - 1) / 2)) * (size_t)ldvt_of(nbo);
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
                    hipStream_t s, bool timed, const NtPlan* plan = nullptr, const int32_t* desc = nullptr,
                    const VOps* ops = nullptr)
{
    const double fl = 2.0 * (double)mk * nbv * nc;
    const int64_t ldw = ldvt_of(nbv);
    const VOps o = ops ? *ops : VOps{f->Vm, f->ldvm, 0, f->Vt, ldw, nullptr};
    int nz = 1;
    {
        ProfScope ps(timed ? 0 : -1, fl, ((double)mk * nbv + (double)mk * nc) * sizeof(TS) + (double)nbv * nc * sizeof(TS), s);
        if constexpr (MODE == M_F64 || MODE == M_F32) {
            if (nbv <= 32 && !desc && !o.mask) {
                // narrow block: W^T = C^T V with C on the 128-row side of the
                // tile and the block on its 32-column side, stored transposed
                // (so W lands column-major as below)
                // (half the default split target: a narrow product has at
                // most 8 tiles, and its split-K sums cost a pass of their own)
                const NtPlan p32{32, plan ? plan->split_target : g_nt_default.split_target / 2};
                CT_HIP(launch_nt<TS>(C, ldc, (const TS*)o.vm, o.ldvm, (TS*)f->Wp, nbv, nc, nbv, mk, false,
                                     f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s, &p32, nullptr, 0, 0, 0, 1));
            } else {
                CT_HIP(launch_nt<TS>((const TS*)o.vm, o.ldvm, C, ldc, (TS*)f->Wp, nbv, nbv, nc, mk, false,
                                     f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s, plan, desc, 1, 0, o.mask));
            }
        } else {
            if (o.mask) return fail(-1, "%s", "internal: masked operand on the low-precision kernel");
            if (MODE == M_BF16X3 && f->S3 && nbv >= kX3dlMinWidth && nc <= kX3dlSplitAtRead) {
                // few columns (a solve): both operands split as they are read
                CT_HIP(launch_nt_x3dl(o.vm, nullptr, o.ldvm, C, nullptr, ldc, (float*)f->Wp, nbv, nbv, nc, mk, false,
                                      f->wp_elems * 2, &nz, s));
            } else if (MODE == M_BF16X3 && f->S3) {
                // the block's bfloat16 halves, column-major like Vm
                char* hi = (char*)f->S3;
                char* lo = hi + (size_t)o.ldvm * nbv * 2;
                CT_HIP(launch_split_x3((const float*)o.vm, o.ldvm, hi, lo, o.ldvm, mk, nbv, s));
                if (nbv >= kX3dlMinWidth)
                    CT_HIP(launch_nt_x3dl(hi, lo, o.ldvm, C, nullptr, ldc, (float*)f->Wp, nbv, nbv, nc, mk, false,
                                          f->wp_elems * 2, &nz, s));
                else
                    CT_HIP(launch_nt_lp<M_BF16X3>(hi, o.ldvm, C, ldc, (float*)f->Wp, nbv, nbv, nc, mk, false,
                                                  f->wp_elems * 2, &nz, s, lo, nullptr));
            } else {
                CT_HIP((nt_any<TS, MODE>((const TS*)o.vm, o.ldvm, C, ldc, (TS*)f->Wp, nbv, nbv, nc, mk, false,
                                         f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s)));
            }
        }
    }
    const TS* Wsum = (const TS*)f->Wp;
    if (nz > 1) {
        CT_HIP((launch_sum_slices<TS, TS>((const TS*)f->Wp, (int64_t)nbv * nc, nz, (int64_t)nbv * nc, (TS*)f->Ws, s,
                                          desc, nbv)));
        Wsum = (const TS*)f->Ws;
    }
    if (OPT == 0 && o.tts && MODE == M_BF16X3 && !desc) {
        // W' = T^T W in the update's own arithmetic (BF16x3, operands split
        // when staged): row p of T^T is column p of T
        int nz1;
        CT_HIP(launch_nt_lp<M_BF16X3>(o.tts, ldt, Wsum, nbv, (float*)f->Wq, ldw, nbv, nc, nbv, false, 0, &nz1, s,
                                      nullptr, nullptr));
    } else if (OPT == 0 && o.tts) {
        // W' = T^T W on the NT kernel: row p of T^T is column p of T
        int nz1;
        CT_HIP(launch_nt<TS>((const TS*)o.tts, ldt, Wsum, nbv, (TS*)f->Wq, ldw, nbv, nc, nbv, false, 0, &nz1, s, plan,
                             desc, 0, 0));
    } else if (OPT == 1 && o.tts) {
        // W' = T W on the NT kernel: T row-major (its transpose, built in the
        // Gram scratch, which the solves do not otherwise use)
        int nz1;
        TS* Tt = (TS*)f->G;
        CT_HIP((launch_transpose<TS, TS, true, false>((const TS*)o.tts, Tt, nbv, nbv, ldt, nbv, s)));
        CT_HIP(launch_nt<TS>(Tt, nbv, Wsum, nbv, (TS*)f->Wq, ldw, nbv, nc, nbv, false, 0, &nz1, s, plan, desc, 0, 0));
    } else {
        CT_HIP((launch_tw<TS, TS, OPT, false>(Wsum, 1, nbv, nc, T, ldt, (TS*)f->Wq, nullptr, ldw, s, desc)));
    }
    {
        ProfScope ps(timed ? 1 : -1, fl, (double)mk * nbv * sizeof(TS) + (double)nbv * nc * sizeof(TS) + 2.0 * mk * nc * sizeof(TS), s);
        int nz2;
        if constexpr (MODE == M_F64 || MODE == M_F32)
            CT_HIP(launch_nt<TS>((const TS*)o.vt, o.ldvt, (const TS*)f->Wq, ldw, C, ldc, mk, nc, nbv, true, 0, &nz2, s,
                                 plan, desc, 0, 1));
        else if (MODE == M_BF16X3 && f->S3 && nbv >= kX3dlMinWidth && nc <= kX3dlSplitAtRead)
            CT_HIP(launch_nt_x3dl(o.vt, nullptr, o.ldvt, f->Wq, nullptr, ldw, C, ldc, mk, nc, nbv, true, 0, &nz2, s));
        else if (MODE == M_BF16X3 && f->S3) {
            // V (row-major) and W' in bfloat16 halves: V to the split scratch,
            // W' to the split-K sum buffer, which is free by now
            char* vh = (char*)f->S3;
            char* vl = vh + (size_t)mk * o.ldvt * 2;
            char* wh = (char*)f->Ws;
            char* wl = wh + (size_t)ldw * nc * 2;
            CT_HIP(launch_split_x3((const float*)o.vt, o.ldvt, vh, vl, o.ldvt, o.ldvt, mk, s));
            CT_HIP(launch_split_x3((const float*)f->Wq, ldw, wh, wl, ldw, ldw, nc, s));
            if (nbv >= kX3dlMinWidth)
                CT_HIP(launch_nt_x3dl(vh, vl, o.ldvt, wh, wl, ldw, C, ldc, mk, nc, nbv, true, 0, &nz2, s));
            else
                CT_HIP(launch_nt_lp<M_BF16X3>(vh, o.ldvt, wh, ldw, C, ldc, mk, nc, nbv, true, 0, &nz2, s, vl, wl));
        } else
            CT_HIP((nt_any<TS, MODE>((const TS*)o.vt, o.ldvt, (const TS*)f->Wq, ldw, C, ldc, mk, nc, nbv, true, 0,
                                     &nz2, s)));
    }
    return 0;
}


// prepared: the block is already in f->Vm / f->Vt
template <typename TS, int OPT>
static int larfb_mode(ct_factor* f, int mode, const TS* V, int64_t ldv, int64_t mk, int nbv, const double* T,
                      int64_t ldt, TS* C, int64_t ldc, int nc, hipStream_t s, bool timed = false, bool prepared = false,
                      const VOps* ops = nullptr)
{
    if (!prepared) {
        int r = prep_block<TS>(f, V, ldv, mk, nbv, s);
        if (r) return r;
    }
    if constexpr (sizeof(TS) == 8) {
        return larfb_nt<TS, OPT, M_F64>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed, nullptr, nullptr, ops);
    } else {
        switch (mode) {
            case M_F32: return larfb_nt<TS, OPT, M_F32>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed, nullptr, nullptr, ops);
            case M_BF16: return larfb_nt<TS, OPT, M_BF16>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed, nullptr, nullptr, ops);
            case M_F16: return larfb_nt<TS, OPT, M_F16>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed, nullptr, nullptr, ops);
            case M_BF16X3:
                return larfb_nt<TS, OPT, M_BF16X3>(f, mk, nbv, T, ldt, C, ldc, nc, s, timed, nullptr, nullptr, ops);
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

// Compact-WY factor of an outer block whose panels have left their own
// factors on T's diagonal: the Gram matrix of the prepared (masked) block in
// f->Vm, in the storage precision, then pairwise joins of the panel factors.
// join0: width of the diagonal blocks of T that are already complete (the
// panels', or those of sub-blocks factored earlier).
template <typename TS>
static int block_t(ct_factor* f, int64_t mk, int bo, double* T, int64_t ldt, hipStream_t s, int join0)
{
    int nz = 1;
    // the joins read V1^T V2 blocks above the diagonal only
    CT_HIP(launch_nt<TS>((const TS*)f->Vm, f->ldvm, (const TS*)f->Vm, f->ldvm, (TS*)f->Wp, bo, bo, bo, mk, false,
                         f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s, nullptr, nullptr, 0, 0, 0, 0, 1));
    CT_HIP((launch_sum_slices<TS, double>((const TS*)f->Wp, (int64_t)bo * bo, nz, (int64_t)bo * bo, f->G, s)));
    CT_HIP(launch_t_join(f->G, bo, T, ldt, (double*)f->Wq, join0, bo, s));
    return 0;
}

// T of outer block b in the storage type, for the MFMA form of T^T W.
template <typename TS>
static const TS* t_storage(const ct_factor* f, int64_t b)
{
    const size_t off = (size_t)b * f->nb_out * f->nb_out;
    if constexpr (sizeof(TS) == 8) return (const TS*)(f->T_all + off);
    else return f->Tf ? (const TS*)f->Tf + off : nullptr;
}

// Factor the columns [c0, c1) of the matrix in place, assuming every earlier
// reflector block has already been applied to them: inner panels of nb_in
// columns with their updates inside the outer block, then the outer block's
// compact-WY factor and its update of the remaining columns up to c1.
// C points at column c0 (row 0); c0 is a multiple of nb_out.
template <typename TS>
static int factor_cols(ct_factor* f, TS* C, int64_t c0, int64_t c1, hipStream_t s)
{
    const int64_t m = f->m, lda = f->lda;
    const int nbo = f->nb_out, nbi = f->nb_in;
    const int mode = trailing_mode(f->prec);
    const int inner_mode = sizeof(TS) == 8 ? M_F64 : M_F32;
    for (int64_t k0 = c0; k0 < c1; k0 += nbo) {
        const int64_t b = k0 / nbo;
        const int bo = (int)std::min<int64_t>(nbo, c1 - k0);
        const int64_t mk = m - k0;
        TS* Ab = C + (k0 - c0) * lda + k0;      // diagonal entry of the block
        double* Tb = f->T_all + (size_t)b * nbo * nbo;
        for (int64_t p0 = k0; p0 < k0 + bo; p0 += nbi) {
            const int bi = (int)std::min<int64_t>(nbi, k0 + bo - p0);
            const int64_t mkp = m - p0;
            TS* Vp = Ab + (p0 - k0) * lda + (p0 - k0);
            // the panel writes its factor on the diagonal of the block's T
            double* Tp = Tb + (p0 - k0) * (1 + (int64_t)nbo);
            const int64_t ldtp = nbo;
            CT_HIP(launch_panel<TS>(Vp, lda, mkp, bi, f->rw, f->tau + p0, Tp, ldtp, f->part, f->gpart, f->counter,
                                    &f->barrier_base, &f->col_base, &f->cq_count, f->info, p0, f->err, s));
            const int64_t rest = k0 + bo - (p0 + bi);
            if (rest > 0) {
                int r = larfb_mode<TS, 0>(f, inner_mode, Vp, lda, mkp, bi, Tp, ldtp, Vp + bi * lda, lda, (int)rest, s);
                if (r) return r;
            }
        }
        const int64_t nc = c1 - k0 - bo;
        // the row-major copy of the block goes to its persistent place when
        // the solves keep one
        TS* vt_dst = f->VtAll ? (TS*)f->VtAll + vt_offset(f, b) : nullptr;
        if (bo > nbi || nc > 0 || vt_dst) {
            int r = prep_block<TS>(f, Ab, lda, mk, bo, s, vt_dst);
            if (r) return r;
        }
        if (bo > nbi) {
            int r = block_t<TS>(f, mk, bo, Tb, nbo, s, nbi);
            if (r) return r;
        }
        if constexpr (sizeof(TS) == 4)
            if (f->Tf) CT_HIP((launch_convert<double, float>(Tb, nbo, (float*)f->Tf + (size_t)b * nbo * nbo, nbo, bo, bo, s)));
        if (nc > 0) {
            const VOps ops{f->Vm, f->ldvm, 0, vt_dst ? (const void*)vt_dst : f->Vt, ldvt_of(bo), t_storage<TS>(f, b)};
            int r = larfb_mode<TS, 0>(f, mode, Ab, lda, mk, bo, Tb, nbo, Ab + bo * lda, lda, (int)nc, s, true, true,
                                      &ops);
            if (r) return r;
        }
        if (g_progress_blocks > 0 && !f->st && ((b + 1) % g_progress_blocks == 0 || k0 + bo >= c1)) {
            // progress line once the device has finished this block
            CT_HIP(hipStreamSynchronize(s));
            fprintf(stderr, "ct_qr_factor: %lld of %lld columns factored\n", (long long)(k0 + bo),
                    (long long)f->n);
            fflush(stderr);
        }
    }
    return 0;
}

template <typename TS>
static int factor_impl(ct_factor* f, hipStream_t s)
{
    return factor_cols<TS>(f, (TS*)f->A, 0, f->n, s);
}

static int bucket_of(int64_t nrhs) { return nrhs <= 8 ? 0 : nrhs <= 32 ? 1 : nrhs <= 128 ? 2 : nrhs <= 512 ? 3 : 4; }

// ------------------------------------------------------ host-pinned streaming
// A streamed factor keeps V\R in the caller's pinned host matrix, as column
// tiles of wt columns (wt a multiple of nb_out).  Tiles [0, nres) also stay in
// device memory as the leading columns of a device matrix f->A with the same
// leading dimension; the other tiles pass through kSlots staging slots, kept
// as a small cache.  Copies run on two streams of their own (host to device
// and device to host) and are ordered against the compute stream with events.
constexpr int kSlots = 4;

struct StreamState {
    char* Ah = nullptr;
    size_t es = 4;                 // bytes per element
    int64_t wt = 0, ntiles = 0, nres = 0;
    int64_t next_tile = 0;         // first tile not yet factored
    bool broken = false;           // a tile's write-back failed: no resume
    hipStream_t cin = nullptr, cout = nullptr;
    hipEvent_t done = nullptr;     // scratch event on the compute stream
    char* slot[kSlots] = {};
    int64_t held[kSlots] = {-1, -1, -1, -1};
    int64_t r0[kSlots] = {}, r1[kSlots] = {};
    uint64_t stamp[kSlots] = {};
    int pins[kSlots] = {};
    bool used_rec[kSlots] = {}, out_rec[kSlots] = {};
    hipEvent_t ready[kSlots] = {}, used[kSlots] = {}, out[kSlots] = {};
    std::vector<hipEvent_t> res_ready;   // resident tile t: its load from host
    std::vector<char> res_loaded;
    std::vector<hipEvent_t> d2h;          // tile t: its host copy is final
    std::vector<char> d2h_rec;
    uint64_t clock = 0;
    ~StreamState()
    {
        if (cin) (void)hipStreamSynchronize(cin);
        if (cout) (void)hipStreamSynchronize(cout);
        for (int k = 0; k < kSlots; ++k) {
            if (ready[k]) (void)hipEventDestroy(ready[k]);
            if (used[k]) (void)hipEventDestroy(used[k]);
            if (out[k]) (void)hipEventDestroy(out[k]);
        }
        for (hipEvent_t e : res_ready) if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : d2h) if (e) (void)hipEventDestroy(e);
        if (done) (void)hipEventDestroy(done);
        if (cin) (void)hipStreamDestroy(cin);
        if (cout) (void)hipStreamDestroy(cout);
    }
};

static int64_t tile_width(const ct_factor* f, int64_t t) { return std::min(f->st->wt, f->n - t * f->st->wt); }

static void stream_invalidate(StreamState* st)
{
    for (int k = 0; k < kSlots; ++k) st->held[k] = -1;
}

// Copy rows [r0, r1) of host tile t into slot k on the host-to-device stream.
static int stream_load(ct_factor* f, int k, int64_t t, int64_t r0, int64_t r1)
{
    StreamState* st = f->st;
    const size_t es = st->es, pitch = (size_t)f->lda * es;
    if (st->used_rec[k]) CT_HIP(hipStreamWaitEvent(st->cin, st->used[k], 0));
    if (st->out_rec[k]) CT_HIP(hipStreamWaitEvent(st->cin, st->out[k], 0));
    if (st->d2h_rec[t]) CT_HIP(hipStreamWaitEvent(st->cin, st->d2h[t], 0));
    const char* src = st->Ah + ((size_t)t * st->wt * f->lda + r0) * es;
    CT_HIP(hipMemcpy2DAsync(st->slot[k] + r0 * es, pitch, src, pitch, (size_t)(r1 - r0) * es, (size_t)tile_width(f, t),
                            hipMemcpyHostToDevice, st->cin));
    CT_HIP(hipEventRecord(st->ready[k], st->cin));
    st->held[k] = t;
    st->r0[k] = r0;
    st->r1[k] = r1;
    st->stamp[k] = ++st->clock;
    return 0;
}

static int find_slot(const StreamState* st, int64_t t, int64_t r0, int64_t r1)
{
    for (int k = 0; k < kSlots; ++k)
        if (st->held[k] == t && st->r0[k] <= r0 && st->r1[k] >= r1) return k;
    return -1;
}

static int victim_slot(const StreamState* st)
{
    int best = -1;
    for (int k = 0; k < kSlots; ++k) {
        if (st->pins[k]) continue;
        if (st->held[k] < 0) return k;
        if (best < 0 || st->stamp[k] < st->stamp[best]) best = k;
    }
    return best;
}

// First load of resident tile t (rows [0, m)), on the host-to-device stream.
static int stream_load_resident(ct_factor* f, int64_t t)
{
    StreamState* st = f->st;
    if (st->res_loaded[t]) return 0;
    const size_t es = st->es, pitch = (size_t)f->lda * es;
    const size_t off = (size_t)t * st->wt * f->lda * es;
    CT_HIP(hipMemcpy2DAsync((char*)f->A + off, pitch, st->Ah + off, pitch, (size_t)f->m * es, (size_t)tile_width(f, t),
                            hipMemcpyHostToDevice, st->cin));
    CT_HIP(hipEventRecord(st->res_ready[t], st->cin));
    st->res_loaded[t] = 1;
    return 0;
}

// Make rows [r0, r1) of tile t usable by work enqueued next on stream s.
// *ptr receives the device address of the tile's first column (row 0) and
// *k the slot to release afterwards (-1 for a resident tile).
static int stream_acquire(ct_factor* f, int64_t t, int64_t r0, int64_t r1, hipStream_t s, char** ptr, int* k)
{
    StreamState* st = f->st;
    if (t < st->nres) {
        int r = stream_load_resident(f, t);
        if (r) return r;
        CT_HIP(hipStreamWaitEvent(s, st->res_ready[t], 0));
        *ptr = (char*)f->A + (size_t)t * st->wt * f->lda * st->es;
        *k = -1;
        return 0;
    }
    int j = find_slot(st, t, r0, r1);
    if (j < 0) {
        j = victim_slot(st);
        if (j < 0) return fail(-1, "%s", "internal: no free staging slot");
        int r = stream_load(f, j, t, r0, r1);
        if (r) return r;
    }
    CT_HIP(hipStreamWaitEvent(s, st->ready[j], 0));
    st->pins[j]++;
    st->stamp[j] = ++st->clock;
    *ptr = st->slot[j];
    *k = j;
    return 0;
}

static int stream_release(ct_factor* f, int k, hipStream_t s)
{
    if (k < 0) return 0;
    StreamState* st = f->st;
    st->pins[k]--;
    CT_HIP(hipEventRecord(st->used[k], s));
    st->used_rec[k] = true;
    return 0;
}

// Start loading rows [r0, r1) of tile t if a slot is free for it.
static int stream_prefetch(ct_factor* f, int64_t t, int64_t r0, int64_t r1)
{
    StreamState* st = f->st;
    if (t < 0 || t >= st->ntiles) return 0;
    if (t < st->nres) return stream_load_resident(f, t);
    if (find_slot(st, t, r0, r1) >= 0) return 0;
    const int j = victim_slot(st);
    if (j < 0) return 0;
    return stream_load(f, j, t, r0, r1);
}

// Column access for one pass over the factor in a fixed direction.  vpart:
// the pass reads reflectors (rows [c0, m) of each tile), else it reads R
// (rows [0, c0 + w)).  In-memory factors return plain addresses.
template <typename TS>
struct ColWalk {
    ct_factor* f;
    hipStream_t s;
    int dir;
    bool vpart;
    int64_t cur = -1;
    int k = -1;
    char* base = nullptr;
    int rc = 0;
    ColWalk(ct_factor* f_, hipStream_t s_, int dir_, bool vpart_) : f(f_), s(s_), dir(dir_), vpart(vpart_) {}
    void rows(int64_t t, int64_t* a, int64_t* b) const
    {
        const int64_t c0 = t * f->st->wt;
        *a = vpart ? c0 : 0;
        *b = vpart ? f->m : c0 + tile_width(f, t);
    }
    // device address of column c (row 0); nullptr on failure (rc holds the code)
    TS* col(int64_t c)
    {
        if (!f->st) return (TS*)f->A + c * f->lda;
        const int64_t t = c / f->st->wt;
        if (t != cur) {
            if (cur >= 0 && (rc = stream_release(f, k, s))) return nullptr;
            cur = -1;
            int64_t a, b;
            rows(t, &a, &b);
            if ((rc = stream_acquire(f, t, a, b, s, &base, &k))) return nullptr;
            cur = t;
            const int64_t nx = t + dir;
            if (nx >= 0 && nx < f->st->ntiles) {
                rows(nx, &a, &b);
                if ((rc = stream_prefetch(f, nx, a, b))) return nullptr;
            }
        }
        return (TS*)base + (c - cur * f->st->wt) * f->lda;
    }
    int finish()
    {
        if (cur >= 0) {
            cur = -1;
            return stream_release(f, k, s);
        }
        return 0;
    }
    ~ColWalk() { finish(); }
};

// Left-looking factorization of a streamed matrix, tile by tile from
// st->next_tile: bring tile J in, apply every earlier reflector block to it
// (in order), factor it, and copy it back to the host matrix while the next
// tile is processed.
// Failure injection (tests): the factorization stops at tile g_inject_tile
// as if a copy had failed, before any work on the tile (g_inject_after < 0)
// or after g_inject_after of the earlier tiles' reflector blocks have been
// applied to it.
static int64_t g_inject_tile = -1, g_inject_after = -1;

// Undo a partly processed tile J after an error: wait for every stream, drop
// the staging cache and its pins, and forget that a resident tile J was
// loaded, so that a resume reloads it from the host matrix (whose copy of
// tile J is only written when the tile is finished).
static int stream_abort_tile(ct_factor* f, int64_t J, hipStream_t s, int code)
{
    StreamState* st = f->st;
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(st->cin);
    (void)hipStreamSynchronize(st->cout);
    stream_invalidate(st);
    for (int k = 0; k < kSlots; ++k) st->pins[k] = 0;
    if (J < st->nres) st->res_loaded[J] = 0;
    st->next_tile = J;
    return code;
}

template <typename TS>
static int stream_factor(ct_factor* f, hipStream_t s)
{
    StreamState* st = f->st;
    const int64_t m = f->m, lda = f->lda, wt = st->wt;
    const int nbo = f->nb_out;
    const int mode = trailing_mode(f->prec);
    auto injected = [&](int64_t J) {
        g_inject_tile = -1;
        g_inject_after = -1;
        const int r = fail(-2002, "%s", "tile copy failed (injected); ct_qr_resume continues from the failed tile");
        return stream_abort_tile(f, J, s, r);
    };
    for (int64_t J = st->next_tile; J < st->ntiles; ++J) {
        if (g_inject_tile == J && g_inject_after < 0) return injected(J);
        const int64_t c0 = J * wt, w = tile_width(f, J);
        char* Cb;
        int kc;
        int r = stream_acquire(f, J, 0, m, s, &Cb, &kc);
        if (r) return stream_abort_tile(f, J, s, r);
        TS* C = (TS*)Cb;
        if (J == 0) {
            r = stream_prefetch(f, 1, 0, m);
            if (r) return stream_abort_tile(f, J, s, r);
        }
        for (int64_t u = 0; u < J; ++u) {
            if (g_inject_tile == J && g_inject_after == u) return injected(J);
            const int64_t u0 = u * wt, uw = tile_width(f, u);
            char* Vb;
            int kv;
            r = stream_acquire(f, u, u0, m, s, &Vb, &kv);
            if (r) return stream_abort_tile(f, J, s, r);
            // overlap the next load with this tile's updates
            r = (u + 1 < J) ? stream_prefetch(f, u + 1, (u + 1) * wt, m) : stream_prefetch(f, J + 1, 0, m);
            if (r) return stream_abort_tile(f, J, s, r);
            const TS* V = (const TS*)Vb;
            for (int64_t k0 = u0; k0 < u0 + uw; k0 += nbo) {
                const int bo = (int)std::min<int64_t>(nbo, u0 + uw - k0);
                const double* Tb = f->T_all + (size_t)(k0 / nbo) * nbo * nbo;
                r = larfb_mode<TS, 0>(f, mode, V + (k0 - u0) * lda + k0, lda, m - k0, bo, Tb, nbo, C + k0, lda,
                                      (int)w, s, true);
                if (r) return stream_abort_tile(f, J, s, r);
            }
            r = stream_release(f, kv, s);
            if (r) return stream_abort_tile(f, J, s, r);
        }
        if (g_inject_tile == J && g_inject_after >= J) return injected(J);
        r = factor_cols<TS>(f, C, c0, c0 + w, s);
        if (r) return stream_abort_tile(f, J, s, r);
        // copy the finished tile back to the host matrix
        const size_t pitch = (size_t)lda * st->es;
        hipError_t e = hipEventRecord(st->done, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(st->cout, st->done, 0);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(st->Ah + (size_t)c0 * lda * st->es, pitch, C, pitch, (size_t)m * st->es, (size_t)w,
                                 hipMemcpyDeviceToHost, st->cout);
        if (e == hipSuccess) e = hipEventRecord(st->d2h[J], st->cout);
        if (e != hipSuccess) {
            // the host copy of tile J may be partly written, so the tile can
            // no longer be redone from it: the factorization cannot resume
            const int rc = fail(-1000 - (int)e, "tile write-back: %s", hipGetErrorString(e));
            (void)stream_abort_tile(f, J, s, rc);
            st->broken = true;
            return rc;
        }
        st->d2h_rec[J] = 1;
        if (kc >= 0) {
            CT_HIP(hipEventRecord(st->out[kc], st->cout));
            st->out_rec[kc] = true;
        }
        r = stream_release(f, kc, s);
        if (r) return stream_abort_tile(f, J + 1, s, r);
        st->next_tile = J + 1;
    }
    // the host matrix is complete once the compute stream passes this point
    CT_HIP(hipStreamWaitEvent(s, st->d2h[st->ntiles - 1], 0));
    return 0;
}

// B <- Q^T B (transpose) or B <- Q B, block by block, in the factor's storage
// precision.  desc: optional device batch descriptor (graph-captured solves).
// x3 (Q^T only, FP32 storage, no batch descriptor): both block products on
// the bfloat16 MFMA in BF16x3, the block first copied out of the factored
// matrix with its unit diagonal and zeros (that kernel reads no mask).
template <typename TS>
static int apply_qt_impl(const ct_factor* fc, TS* B, int64_t nrhs, int64_t ldb, hipStream_t s, bool transpose,
                         const int32_t* desc = nullptr, bool x3 = false)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    const int nbo = f->nb_out;
    const NtPlan* plan = &f->solve_plan[bucket_of(nrhs)];
    ColWalk<TS> walk(f, s, transpose ? 1 : -1, true);
    for (int64_t bb = 0; bb < f->nblocks; ++bb) {
        const int64_t b = transpose ? bb : f->nblocks - 1 - bb;
        const int64_t k0 = b * nbo;
        const int bo = (int)std::min<int64_t>(nbo, f->n - k0);
        const double* Tb = f->T_all + (size_t)b * nbo * nbo;
        const TS* Vb = walk.col(k0);
        if (!Vb) return walk.rc;
        int r;
        VOps ops;
        const VOps* op = nullptr;
        if (f->VtAll) {
            // the block read in place (masked) and its stored row-major copy
            ops = VOps{Vb + k0, f->lda, 1, (const TS*)f->VtAll + vt_offset(f, b), ldvt_of(bo), t_storage<TS>(f, b)};
        } else {
            r = prep_block<TS>(f, Vb + k0, f->lda, f->m - k0, bo, s);
            if (r) return r;
            ops = VOps{f->Vm, f->ldvm, 0, f->Vt, ldvt_of(bo), t_storage<TS>(f, b)};
        }
        op = &ops;
        if constexpr (sizeof(TS) == 4)
            if (x3 && transpose && !desc && f->VtAll) {
                // the masked column-major copy only: the row-major one is VtAll's
                r = prep_block<TS>(f, Vb + k0, f->lda, f->m - k0, bo, s, nullptr, false);
                if (r) return r;
                ops.vm = f->Vm;
                ops.ldvm = f->ldvm;
                ops.mask = 0;
                r = larfb_nt<TS, 0, M_BF16X3>(f, f->m - k0, bo, Tb, nbo, B + k0, ldb, (int)nrhs, s, false, nullptr,
                                              nullptr, op);
                if (r) return r;
                continue;
            }
        r = transpose ? larfb_nt<TS, 0>(f, f->m - k0, bo, Tb, nbo, B + k0, ldb, (int)nrhs, s, false, plan, desc, op)
                      : larfb_nt<TS, 1>(f, f->m - k0, bo, Tb, nbo, B + k0, ldb, (int)nrhs, s, false, plan, desc, op);
        if (r) return r;
    }
    return walk.finish();
}

// x3: the diagonal steps and block-column updates on the bfloat16 MFMA in
// BF16x3 (FP32 storage only, no batch descriptor).
// The diagonal block of outer block Bk in the blocked back-substitution:
// C[K0:K0+w] <- R[K0:K0+w, K0:K0+w]^{-1} C[K0:K0+w] for ncols columns, per
// 256-row block b, last first: X_b = R_bb^{-1} C_b (a product with the stored
// inverse), then C[K0:k0] -= R[K0:k0, b] X_b on the row-major copy of R.
template <typename TS>
static int inner_solve(ct_factor* f, TS* C, int64_t ldc, int64_t ncols, int64_t Bk, bool x3, const int32_t* desc,
                       hipStream_t s)
{
    const int64_t n = f->n;
    const int ob = f->rt_ob;
    const int64_t nbo = (n + ob - 1) / ob, q = ob / 256;
    const NtPlan* plan = &f->solve_plan[bucket_of(ncols)];
    const NtPlan diag_plan{32, 1024};     // 256-row products: narrow tiles for more workgroups
    TS* S = (TS*)f->Wq;
    const TS* Rin = f->Rt ? (const TS*)f->Rt + (size_t)ob * ob * (size_t)(nbo * (nbo - 1) / 2) : nullptr;
    const int64_t K0 = Bk * ob;
    const int64_t w = std::min<int64_t>(ob, n - K0);
    for (int64_t i = (w + 255) / 256 - 1; i >= 0; --i) {
        const int64_t k0 = K0 + 256 * i, b = k0 / 256;
        const int bo = (int)std::min<int64_t>(256, n - k0);
        int nz;
        bool done = false;
        if constexpr (sizeof(TS) == 4) {
            if (x3 && !desc)
                CT_HIP(launch_diag_x3((const float*)f->RiR + (size_t)b * 256 * 256, C + k0, ldc, bo, (int)ncols, s));
            else
                CT_HIP(launch_diag_f32((const float*)f->RiR + (size_t)b * 256 * 256, C + k0, ldc, bo, (int)ncols, desc,
                                       s));
            done = true;
        }
        if (!done) {
            CT_HIP((launch_copy_block<TS>(C + k0, ldc, S, 256, bo, (int)ncols, s, desc)));
            CT_HIP(launch_nt<TS>((const TS*)f->RiR + (size_t)b * 256 * 256, 256, S, 256, C + k0, ldc, bo, (int)ncols,
                                 bo, false, 0, &nz, s, &diag_plan, desc, 0, 1));
        }
        if (i == 0) continue;
        if (!Rin) {
            // C[K0:k0] -= R[K0:k0, k0:k0+bo] X_b with R read in place (column-major)
            const TS* Rc = (const TS*)f->A + K0 + k0 * f->lda;
            if constexpr (sizeof(TS) == 8)
                CT_HIP((launch_nn_sub<M_F64, TS, TS, TS, false>(Rc, f->lda, C + k0, nullptr, ldc, C + K0, ldc, 256 * i,
                                                                (int)ncols, bo, s, desc)));
            else
                CT_HIP((launch_nn_sub<M_F32, TS, TS, TS, false>(Rc, f->lda, C + k0, nullptr, ldc, C + K0, ldc, 256 * i,
                                                                (int)ncols, bo, s, desc)));
            continue;
        }
        const TS* Ri = Rin + (size_t)Bk * 256 * 256 * (size_t)(q * (q - 1) / 2) + (size_t)256 * 256 * (size_t)(i * (i - 1) / 2);
        if constexpr (sizeof(TS) == 4)
            if (x3 && !desc) {
                CT_HIP(launch_nt_lp<M_BF16X3>(Ri, 256, C + k0, ldc, C + K0, ldc, 256 * i, (int)ncols, bo, true, 0, &nz,
                                              s, nullptr, nullptr));
                continue;
            }
        CT_HIP(launch_nt<TS>(Ri, 256, C + k0, ldc, C + K0, ldc, 256 * i, (int)ncols, bo, true, 0, &nz, s, plan, desc,
                             1, 1));
    }
    return 0;
}

template <typename TS>
static int trsm_impl(const ct_factor* fc, TS* B, int64_t nrhs, int64_t ldb, hipStream_t s,
                     const int32_t* desc = nullptr, bool x3 = false)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    const int64_t n = f->n, lda = f->lda;
    const int tb = g_dev.trsm_block;
    const int64_t nb = (n + tb - 1) / tb;
    if (f->RiR && !f->st) {
        // two levels of blocks, last first: the diagonal block of each outer
        // block (inner_solve, or for BF16x3 one product with the stored
        // inverse of the whole 1024 x 1024 block), then B[0:K0] -= R[0:K0,
        // K0:K0+w] X_B, one product with K = w: on the row-major copy of R
        // (rt_kernel), an NT product with K-contiguous operands, or without
        // that copy an NN product reading R in place.
        const NtPlan* plan = &f->solve_plan[bucket_of(nrhs)];
        const int ob = f->rt_ob;
        const int64_t nbo = (n + ob - 1) / ob;
        const TS* Rt = (const TS*)f->Rt;
        const bool inv4 = x3 && !desc && f->RiR4 && (int64_t)ob * nrhs * (int64_t)sizeof(TS) <= f->wq_elems * 8;
        for (int64_t Bk = nbo - 1; Bk >= 0; --Bk) {
            const int64_t K0 = Bk * ob;
            const int64_t w = std::min<int64_t>(ob, n - K0);
            int nz;
            if constexpr (sizeof(TS) == 4) {
                if (inv4) {
                    TS* S = (TS*)f->Wq;
                    CT_HIP((launch_copy_block<TS>(B + K0, ldb, S, ob, (int)w, (int)nrhs, s, nullptr)));
                    CT_HIP(launch_nt_lp<M_BF16X3>((const float*)f->RiR4 + (size_t)Bk * ob * ob, ob, S, ob, B + K0, ldb,
                                                  w, (int)nrhs, w, false, 0, &nz, s, nullptr, nullptr));
                }
            }
            if (!inv4) {
                int r = inner_solve<TS>(f, B, ldb, nrhs, Bk, x3, desc, s);
                if (r) return r;
            }
            if (K0 == 0) continue;
            if (!Rt) {
                const TS* Rc = (const TS*)f->A + K0 * lda;
                if constexpr (sizeof(TS) == 8)
                    CT_HIP((launch_nn_sub<M_F64, TS, TS, TS, false>(Rc, lda, B + K0, nullptr, ldb, B, ldb, K0,
                                                                    (int)nrhs, (int)w, s, desc)));
                else
                    CT_HIP((launch_nn_sub<M_F32, TS, TS, TS, false>(Rc, lda, B + K0, nullptr, ldb, B, ldb, K0,
                                                                    (int)nrhs, (int)w, s, desc)));
                continue;
            }
            const TS* X = Rt + (size_t)ob * ob * (size_t)(Bk * (Bk - 1) / 2);
            if constexpr (sizeof(TS) == 4)
                if (x3 && !desc) {
                    CT_HIP(launch_nt_x3dl(X, nullptr, ob, B + K0, nullptr, ldb, B, ldb, K0, (int)nrhs, w, true, 0, &nz,
                                          s));
                    continue;
                }
            CT_HIP(launch_nt<TS>(X, ob, B + K0, ldb, B, ldb, K0, (int)nrhs, w, true, 0, &nz, s, plan, desc, 1, 1));
        }
        return 0;
    }
    ColWalk<TS> walk(f, s, -1, false);
    for (int64_t b = nb - 1; b >= 0; --b) {
        const int64_t k0 = b * tb;
        const int bo = (int)std::min<int64_t>(tb, n - k0);
        const TS* Rb = walk.col(k0);       // column k0 of R, row 0
        if (!Rb) return walk.rc;
        CT_HIP((launch_trsm_diag<TS, true>(Rb + k0, lda, bo, B + k0, ldb, (int)nrhs, s, desc)));
        if (k0 > 0) {
            if constexpr (sizeof(TS) == 8)
                CT_HIP((launch_nn_sub<M_F64, TS, TS, TS, false>(Rb, lda, B + k0, nullptr, ldb, B, ldb, k0,
                                                                (int)nrhs, bo, s, desc)));
            else
                CT_HIP((launch_nn_sub<M_F32, TS, TS, TS, false>(Rb, lda, B + k0, nullptr, ldb, B, ldb, k0,
                                                                (int)nrhs, bo, s, desc)));
        }
    }
    return walk.finish();
}

// Y[0:n] <- R^{-T} Y[0:n]: forward substitution on the lower-triangular R^T,
// diagonal-block solves alternating with GEMM updates from the rows above.
template <typename TS>
static int trsm_lt_impl(const ct_factor* fc, TS* Y, int64_t k, int64_t ldy, hipStream_t s, bool x3 = false)
{
    ct_factor* f = const_cast<ct_factor*>(fc);
    const int64_t n = f->n, lda = f->lda;
    const int tb = g_dev.trsm_block;
    const int64_t nb = (n + tb - 1) / tb;
    if (f->RiC && !f->st) {
        // right-looking, first block first, in two levels of blocks: inside an
        // outer block of ob columns, per 256-row block b: Z_b = R_bb^{-T} Y_b
        // with the stored inverse, then the outer block's later rows:
        // Y[k0+bo:K0+w] -= R[k0:k0+bo, k0+bo:K0+w]^T Z_b; after the outer block:
        // Y[K0+w:n] -= R[K0:K0+w, K0+w:n]^T Z_B, one product with K = w.  The X
        // rows of both are later columns of R read in place (K-contiguous
        // down a column).
        const NtPlan* plan = &f->solve_plan[bucket_of(k)];
        const NtPlan diag_plan{32, 1024};
        const TS* A = (const TS*)f->A;
        TS* S = (TS*)f->Wq;
        const int ob = f->rt_ob;
        const int64_t nbo = (n + ob - 1) / ob;
        auto update = [&](int64_t r0, int64_t c0, int64_t P, int K) -> int {
            // Y[c0 : c0 + P] -= R[r0 : r0 + K, c0 : c0 + P]^T Y[r0 : r0 + K]
            int nz;
            if constexpr (sizeof(TS) == 4)
                if (x3) {
                    if (K >= 256 && (r0 % 4) == 0)
                        CT_HIP(launch_nt_x3dl(A + r0 + c0 * lda, nullptr, lda, Y + r0, nullptr, ldy, Y + c0, ldy, P,
                                              (int)k, K, true, 0, &nz, s));
                    else
                        CT_HIP(launch_nt_lp<M_BF16X3>(A + r0 + c0 * lda, lda, Y + r0, ldy, Y + c0, ldy, P, (int)k, K,
                                                      true, 0, &nz, s, nullptr, nullptr));
                    return 0;
                }
            CT_HIP(launch_nt<TS>(A + r0 + c0 * lda, lda, Y + r0, ldy, Y + c0, ldy, P, (int)k, K, true, 0, &nz, s,
                                 plan));
            return 0;
        };
        const bool inv4 = x3 && f->RiC4 && (int64_t)ob * k * (int64_t)sizeof(TS) <= f->wq_elems * 8;
        for (int64_t Bk = 0; Bk < nbo; ++Bk) {
            const int64_t K0 = Bk * ob;
            const int64_t w = std::min<int64_t>(ob, n - K0);
            if constexpr (sizeof(TS) == 4)
                if (inv4) {
                    // Z_B = R_BB^{-T} Y_B with the stored inverse of the whole block
                    int nz;
                    CT_HIP((launch_copy_block<TS>(Y + K0, ldy, S, ob, (int)w, (int)k, s, nullptr)));
                    CT_HIP(launch_nt_lp<M_BF16X3>((const float*)f->RiC4 + (size_t)Bk * ob * ob, ob, S, ob, Y + K0, ldy,
                                                  w, (int)k, w, false, 0, &nz, s, nullptr, nullptr));
                }
            for (int64_t k0 = K0; !inv4 && k0 < K0 + w; k0 += 256) {
                const int64_t b = k0 / 256;
                const int bo = (int)std::min<int64_t>(256, n - k0);
                int nz;
                bool done = false;
                if constexpr (sizeof(TS) == 4) {
                    if (x3)
                        CT_HIP(launch_diag_x3((const float*)f->RiC + (size_t)b * 256 * 256, Y + k0, ldy, bo, (int)k, s));
                    else
                        CT_HIP(launch_diag_f32((const float*)f->RiC + (size_t)b * 256 * 256, Y + k0, ldy, bo, (int)k,
                                               nullptr, s));
                    done = true;
                }
                if (!done) {
                    CT_HIP((launch_copy_block<TS>(Y + k0, ldy, S, 256, bo, (int)k, s, nullptr)));
                    CT_HIP(launch_nt<TS>((const TS*)f->RiC + (size_t)b * 256 * 256, 256, S, 256, Y + k0, ldy, bo,
                                         (int)k, bo, false, 0, &nz, s, &diag_plan));
                }
                const int64_t rest_in = K0 + w - k0 - bo;
                if (rest_in > 0) {
                    int r = update(k0, k0 + bo, rest_in, bo);
                    if (r) return r;
                }
            }
            const int64_t rest = n - K0 - w;
            if (rest > 0) {
                int r = update(K0, K0 + w, rest, (int)w);
                if (r) return r;
            }
        }
        return 0;
    }
    ColWalk<TS> walk(f, s, 1, false);
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t k0 = b * tb;
        const int bo = (int)std::min<int64_t>(tb, n - k0);
        const TS* Rb = walk.col(k0);       // column k0 of R, row 0
        if (!Rb) return walk.rc;
        if (k0 > 0) {
            // Y[k0:k0+bo] -= R[0:k0, k0:k0+bo]^T Y[0:k0]  (columns of R are K-contiguous)
            int nz = 1;
            CT_HIP(launch_nt<TS>(Rb, lda, Y, ldy, (TS*)f->Wp, bo, bo, (int)k, k0, false,
                                 f->wp_elems * 8 / (int64_t)sizeof(TS), &nz, s));
            const TS* Wsum = (const TS*)f->Wp;
            if (nz > 1) {
                CT_HIP((launch_sum_slices<TS, TS>((const TS*)f->Wp, (int64_t)bo * k, nz, (int64_t)bo * k, (TS*)f->Ws, s)));
                Wsum = (const TS*)f->Ws;
            }
            CT_HIP((launch_tw<TS, TS, 3, false>(Wsum, 1, bo, (int)k, nullptr, 0, Y + k0, nullptr, ldy, s)));
        }
        CT_HIP((launch_trsm_diag<TS, false>(Rb + k0, lda, bo, Y + k0, ldy, (int)k, s)));
    }
    return walk.finish();
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
                        int64_t ldx, int64_t nrhs, int steps, int method, double tol, char* scratch, double* rnorms,
                        double* gnorms, int32_t* steps_done, hipStream_t s)
{
    const int64_t m = f->m, n = f->n;
    const int64_t ld = (m + 15) / 16 * 16;             // column-major correction block
    const int64_t lt = (nrhs + 15) / 16 * 16;           // slice-contiguous blocks
    char* p = scratch;
    double* Bt = (double*)p; p += up256((size_t)m * lt * 8);
    double* Rt = (double*)p; p += up256((size_t)m * lt * 8);
    double* Xt = (double*)p; p += up256((size_t)n * lt * 8);
    double* St = (double*)p; p += up256((size_t)n * lt * 8);
    TS* C = (TS*)p; p += up256((size_t)ld * nrhs * 8);
    double* Np = (double*)p; p += up256((size_t)256 * lt * 8);  // column-norm partials (256 x nrhs)
    const bool have_csc = sp->col_ptr && sp->row && sp->cval;
    const int nr = (int)nrhs;
    // a BF16x3 factor's corrections are solved with BF16x3 block updates:
    // the FP64 residual, not the correction's arithmetic, sets the accuracy
    const bool x3 = f->prec == CT_PREC_BF16X3 && (g_x3_refine == 2 || (g_x3_refine == 1 && nrhs >= kX3MinSlices));
    CT_HIP((launch_transpose<double, double, true, false>(B, Bt, m, nr, ldb, lt, s)));
    // x_0 = R~^{-1} Q~^T b
    CT_HIP((launch_convert<double, TS>(B, ldb, C, ld, m, nr, s)));
    int r = apply_qt_impl<TS>(f, C, nrhs, ld, s, true, nullptr, x3);
    if (r) return r;
    r = trsm_impl<TS>(f, C, nrhs, ld, s, nullptr, x3);
    if (r) return r;
    CT_HIP((launch_convert<TS, double>(C, ld, X, ldx, n, nr, s)));
    CT_HIP((launch_transpose<TS, double, true, false>(C, Xt, n, nr, ld, lt, s)));
    // A p (sign flipped: out = -A p) and A^T s over the sparse copies
    auto neg_a_times = [&](const double* Zt, const double* Bz, double* Out) {
        return sp->group_r > 0 ? launch_group_spmm(sp->grow_ptr, sp->grow_col, sp->grow_val, sp->group_r, m, Zt, Bz,
                                                   Out, lt, nr, true, s)
                               : launch_spmv_rows_t(sp->row_ptr, sp->col, sp->val, m, Zt, Bz, Out, lt, nr, s);
    };
    auto at_times = [&](const double* Zt, double* Out) {
        return sp->group_c > 0 ? launch_group_spmm(sp->gcol_ptr, sp->gcol_row, sp->gcol_val, sp->group_c, n, Zt,
                                                   nullptr, Out, lt, nr, false, s)
                               : launch_spmv_cols_t(sp->col_ptr, sp->row, sp->cval, n, Zt, Out, lt, nr, s);
    };
    if (method == CT_REFINE_PCGLS) {
        // Conjugate gradients on A^T A x = A^T b preconditioned with
        // (R~^T R~)^{-1} (CGLS on A R~^{-1}), from x_0 above.  The residual s
        // and the image x are FP64 and are updated with the same step c p and
        // the same FP64 product A p, so s stays b - A x to FP64 rounding; the
        // preconditioner runs in the factor's arithmetic.
        double* Pt = (double*)p; p += up256((size_t)n * lt * 8);
        double* gam = (double*)p;                       // gamma (two rows), ||A p||, ||p||, ||x||
        double* qn = gam + 2 * lt;
        double* pn = qn + lt;
        double* xn = pn + lt;
        double* Qt = Bt;                                // b is taken again from B at the end
        CT_HIP(neg_a_times(Xt, Bt, Rt));                // s_0 = b - A x_0
        if (rnorms) CT_HIP(launch_colnorm_t(Rt, lt, m, nr, rnorms, Np, s));
        CT_HIP(at_times(Rt, St));                       // A^T s_0
        if (gnorms) CT_HIP(launch_colnorm_t(St, lt, n, nr, gnorms, Np, s));
        int cur = 0, taken = 0;
        // z = (R~^T R~)^{-1} r for r in St, gamma = r^T z = ||R~^{-T} r||^2 into gam + row * lt
        auto precondition = [&](int row) -> int {
            CT_HIP((launch_transpose<double, TS, false, false>(St, C, n, nr, ld, lt, s)));
            int e = trsm_lt_impl<TS>(f, C, nrhs, ld, s, x3);
            if (e) return e;
            CT_HIP((launch_colsq<TS>(C, ld, n, nr, gam + (size_t)row * lt, s)));
            return trsm_impl<TS>(f, C, nrhs, ld, s, nullptr, x3);
        };
        if (steps > 0) {
            r = precondition(cur);
            if (r) return r;
            CT_HIP((launch_transpose<TS, double, true, false>(C, Pt, n, nr, ld, lt, s)));   // p_0 = z_0
        }
        bool last = steps == 0;
        while (!last) {
            CT_HIP(neg_a_times(Pt, nullptr, Qt));       // Qt = -A p
            CT_HIP(launch_colnorm_t(Qt, lt, m, nr, qn, Np, s));
            const double* g = gam + (size_t)cur * lt;
            CT_HIP(launch_cg_update(Pt, Xt, n, nr, lt, g, qn, 0, s));   // x += c p
            CT_HIP(launch_cg_update(Qt, Rt, m, nr, lt, g, qn, 0, s));   // s -= c A p
            ++taken;
            last = taken == steps;
            if (tol > 0.0) {
                unsigned long long* maxw = (unsigned long long*)(Np + 256 * lt - 1);
                CT_HIP(launch_colnorm_t(Pt, lt, n, nr, pn, Np, s));
                CT_HIP(launch_colnorm_t(Xt, lt, n, nr, xn, Np, s));
                CT_HIP(launch_cg_ratio(g, qn, pn, xn, nr, maxw, s));
                unsigned long long h = 0;
                CT_HIP(hipMemcpyAsync(&h, maxw, sizeof h, hipMemcpyDeviceToHost, s));
                CT_HIP(hipStreamSynchronize(s));
                double mx;
                memcpy(&mx, &h, sizeof mx);
                last = last || mx <= tol;
            }
            if (last) break;
            if (rnorms) CT_HIP(launch_colnorm_t(Rt, lt, m, nr, rnorms + (size_t)taken * nrhs, Np, s));
            CT_HIP(at_times(Rt, St));                   // r = A^T s
            if (gnorms) CT_HIP(launch_colnorm_t(St, lt, n, nr, gnorms + (size_t)taken * nrhs, Np, s));
            r = precondition(cur ^ 1);
            if (r) return r;
            CT_HIP((launch_transpose<TS, double, true, false>(C, St, n, nr, ld, lt, s)));   // z
            CT_HIP(launch_cg_update(St, Pt, n, nr, lt, gam + (size_t)(cur ^ 1) * lt, g, 1, s));  // p = z + beta p
            cur ^= 1;
        }
        if (taken > 0) {
            // the image, and the last residual recomputed from b (not the recurrence)
            CT_HIP((launch_transpose<double, double, false, false>(Xt, X, n, nr, ldx, lt, s)));
            CT_HIP((launch_transpose<double, double, true, false>(B, Bt, m, nr, ldb, lt, s)));
            if (rnorms || gnorms) {
                CT_HIP(neg_a_times(Xt, Bt, Rt));
                if (rnorms) CT_HIP(launch_colnorm_t(Rt, lt, m, nr, rnorms + (size_t)taken * nrhs, Np, s));
                if (gnorms && have_csc) {
                    CT_HIP(at_times(Rt, St));
                    CT_HIP(launch_colnorm_t(St, lt, n, nr, gnorms + (size_t)taken * nrhs, Np, s));
                }
            }
        }
        if (steps_done) *steps_done = taken;
        return 0;
    }
    int taken = 0;
    bool converged = false;
    for (int st = 0; st <= steps; ++st) {
        // r_st = b - A x_st (FP64)
        if (sp->group_r > 0)
            CT_HIP(launch_group_spmm(sp->grow_ptr, sp->grow_col, sp->grow_val, sp->group_r, m, Xt, Bt, Rt, lt, nr,
                                     true, s));
        else
            CT_HIP(launch_spmv_rows_t(sp->row_ptr, sp->col, sp->val, m, Xt, Bt, Rt, lt, nr, s));
        if (rnorms) CT_HIP(launch_colnorm_t(Rt, lt, m, nr, rnorms + (size_t)st * nrhs, Np, s));
        const bool need_grad = method == CT_REFINE_SNE ? st < steps : false;
        if (have_csc && (need_grad || gnorms)) {
            if (sp->group_c > 0)
                CT_HIP(launch_group_spmm(sp->gcol_ptr, sp->gcol_row, sp->gcol_val, sp->group_c, n, Rt, nullptr, St,
                                         lt, nr, false, s));
            else
                CT_HIP(launch_spmv_cols_t(sp->col_ptr, sp->row, sp->cval, n, Rt, St, lt, nr, s));
            if (gnorms) CT_HIP(launch_colnorm_t(St, lt, n, nr, gnorms + (size_t)st * nrhs, Np, s));
        }
        if (st == steps || converged) break;
        if (method == CT_REFINE_SNE) {
            // x += R~^{-1} R~^{-T} (A^T r)
            CT_HIP((launch_transpose<double, TS, false, false>(St, C, n, nr, ld, lt, s)));
            r = trsm_lt_impl<TS>(f, C, nrhs, ld, s, x3);
            if (r) return r;
        } else {
            // x += R~^{-1} Q~^T r
            CT_HIP((launch_transpose<double, TS, false, false>(Rt, C, m, nr, ld, lt, s)));
            r = apply_qt_impl<TS>(f, C, nrhs, ld, s, true, nullptr, x3);
            if (r) return r;
        }
        r = trsm_impl<TS>(f, C, nrhs, ld, s, nullptr, x3);
        if (r) return r;
        CT_HIP((launch_accumulate<TS>(X, ldx, C, ld, n, nr, s)));
        CT_HIP((launch_transpose<TS, double, true, true>(C, Xt, n, nr, ld, lt, s)));
        ++taken;
        if (tol > 0.0) {
            // stop rule: every slice's correction below tol relative to its
            // updated image; the next pass computes the final residual only
            unsigned long long* maxw = (unsigned long long*)(Np + 256 * lt - 1);
            CT_HIP((launch_corr_ratio<TS>(C, ld, X, ldx, n, nr, Np, maxw, s)));
            unsigned long long h = 0;
            CT_HIP(hipMemcpyAsync(&h, maxw, sizeof h, hipMemcpyDeviceToHost, s));
            CT_HIP(hipStreamSynchronize(s));
            double mx;
            memcpy(&mx, &h, sizeof mx);
            converged = mx <= tol;
        }
    }
    if (steps_done) *steps_done = taken;
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
    CT_ARG(g->projector == CT_PROJ_SIDDON || g->projector == CT_PROJ_JOSEPH, 1, "g (projector)");
    CT_ARG(dtype == CT_F64 || dtype == CT_F32, 2, "dtype");
    CT_ARG(A != nullptr && aligned(A), 3, "A");
    const int64_t m = (int64_t)g->n_angles * g->n_det;
    CT_ARG(lda >= m && lda % 16 == 0, 4, "lda");
    GeomDev gd{g->n_pix, g->n_angles, g->n_det, g->grid_width, g->sid, g->sdd, g->det_length, g->angle0,
               g->projector};
    CT_HIP(launch_siddon_dense(gd, dtype, A, lda, (hipStream_t)stream));
    return 0;
}

int ct_build_csr(const ct_geometry* g, int64_t* row_ptr, int32_t* col, double* val, int64_t nnz_cap, void* stream)
{
    CT_ARG(g != nullptr && g->n_pix > 0 && g->n_angles > 0 && g->n_det > 0, 1, "g");
    CT_ARG(g->projector == CT_PROJ_SIDDON || g->projector == CT_PROJ_JOSEPH, 1, "g (projector)");
    CT_ARG(row_ptr != nullptr, 2, "row_ptr");
    CT_ARG((col == nullptr) == (val == nullptr), 3, "col/val (both or neither)");
    CT_ARG(col == nullptr || nnz_cap > 0, 5, "nnz_cap");
    GeomDev gd{g->n_pix, g->n_angles, g->n_det, g->grid_width, g->sid, g->sdd, g->det_length, g->angle0,
               g->projector};
    CT_HIP(launch_siddon_csr(gd, row_ptr, col, val, nnz_cap, (hipStream_t)stream));
    return 0;
}

int ct_qr_workspace(int64_t m, int64_t n, int prec, int64_t max_nrhs, size_t* bytes)
{
    CT_ARG(m > 0, 1, "m");
    CT_ARG(n > 0 && n <= m, 2, "n (need 0 < n <= m)");
    const bool copies = !(prec & CT_QR_NO_SOLVE_COPIES);
    prec &= ~CT_QR_NO_SOLVE_COPIES;
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 3, "prec");
    CT_ARG(max_nrhs >= 0, 4, "max_nrhs");
    CT_ARG(bytes != nullptr, 5, "bytes");
    *bytes = layout(m, n, prec, max_nrhs, nb_out_for(n), copies ? kCopiesAll : kCopiesInverses).total;
    return 0;
}

}  // extern "C"

// Handle set-up shared by the in-memory and the streamed factorization:
// workspace partition and panel geometry (rows per workgroup from the LDS
// budget; all workgroups of a panel must be resident at once).
static int init_factor(ct_factor* f, void* A, int64_t m, int64_t n, int64_t lda, int prec, double* tau, char* w,
                       const Layout& L, int64_t max_nrhs, int nbo)
{
    f->A = A; f->m = m; f->n = n; f->lda = lda; f->prec = prec; f->f64 = prec == CT_PREC_F64;
    f->tau = tau;
    f->nb_out = nbo;
    f->nblocks = (n + f->nb_out - 1) / f->nb_out;
    f->T_all = (double*)(w + L.T_all);
    f->part = (double*)(w + L.part);
    f->gpart = (double*)(w + L.gpart);
    f->counter = (uint64_t*)(w + L.words);
    f->info = (int64_t*)(w + L.words + 64);
    f->err = (int32_t*)(w + L.words + 128);
    f->batch_rec = (int32_t*)(w + L.words + 192);
    f->col_base = 0;
    f->cq_count = 0;
    f->Wp = w + L.Wp; f->wp_elems = L.wp_elems;
    f->Wq = w + L.Wq; f->wq_elems = L.wq_elems;
    f->G = (double*)(w + L.G);
    f->Vm = w + L.Vm;
    f->Vt = w + L.Vt;
    f->ldvm = (m + 15) / 16 * 16;
    f->Ws = w + L.Ws;
    f->Tf = f->f64 ? nullptr : (void*)(w + L.Tf);
    // BF16x3 updates take the reflector block and W' already split into
    // bfloat16 halves (one split per block instead of one per tile)
    f->S3 = prec == CT_PREC_BF16X3 ? (void*)(w + L.S3) : nullptr;
    f->barrier_base = 0;
    f->max_nrhs = max_nrhs;
    for (int b = 0; b < 5; ++b) f->solve_plan[b] = NtPlan{b < 2 ? 32 : 128, 1024};

    const size_t lds_words = g_dev.lds_max / 8 - panel_aux_words();
    int nbi = g_nbi_force ? g_nbi_force : 32;
    int rw = (int)(lds_words / nbi);
    if ((rw & 1) == 0) --rw;
    if (!g_nbi_force && (m + rw - 1) / rw > g_dev.cus) {
        nbi = 16;
        rw = (int)(lds_words / nbi);
        if ((rw & 1) == 0) --rw;
    }
    if ((m + rw - 1) / rw > g_dev.cus) return fail(-2, "%s", "m too large for a resident panel on this device");
    int per_cu = 0;
    CT_HIP(panel_max_active(&per_cu, panel_lds_bytes(nbi, rw)));
    if (per_cu < 1) return fail(-1002, "%s", "panel kernel cannot be resident");
    f->nb_in = nbi;
    f->rw = rw;
    return 0;
}

// Device bytes of the streamed factorization: the in-memory workspace, then
// nres resident tiles, then the staging slots (none when every tile is resident).
static size_t tile_bytes(int64_t lda, int64_t wt, size_t es) { return up256((size_t)lda * wt * es); }

// Solve-side copies of R of an in-memory factor, from V\R in place: the
// diagonal-block inverses always, the row-major block columns of R when
// `row_major` (without them the solves read R in place).
static int r_copies(ct_factor* f, char* work, const Layout& L, hipStream_t s, bool row_major)
{
    if (g_dev.trsm_block != 128) return 0;
    const int64_t n = f->n, lda = f->lda;
    const size_t es = f->f64 ? 8 : 4;
    f->RiR = work + L.Ri;
    f->RiC = work + L.Ri + (size_t)((n + 255) / 256) * 256 * 256 * es;
    f->Rt = row_major ? work + L.Rt : nullptr;
    f->rt_ob = rt_ob_for(n);
    double* Ri64 = (double*)(row_major || !ri64_in_wp(L, n) ? work + L.Ri64 : (char*)f->Wp);
    double* M = (double*)f->Wq;      // free once the factorization is done
    hipError_t e;
    if (f->f64) {
        e = launch_rinv<double>((const double*)f->A, lda, n, (double*)f->RiR, (double*)f->RiC, Ri64, M, s);
        if (e == hipSuccess && row_major)
            e = launch_rt<double>((const double*)f->A, lda, n, f->rt_ob, (double*)f->Rt, s);
    } else {
        e = launch_rinv<float>((const float*)f->A, lda, n, (float*)f->RiR, (float*)f->RiC, Ri64, M, s);
        if (e == hipSuccess && row_major)
            e = launch_rt<float>((const float*)f->A, lda, n, f->rt_ob, (float*)f->Rt, s);
    }
    if (e != hipSuccess) return fail(-1000 - (int)e, "R copies: %s", hipGetErrorString(e));
    if (f->prec == CT_PREC_BF16X3 && f->rt_ob == 1024) {
        // inverses of the 1024 x 1024 diagonal blocks: R_BB^{-1} I by the
        // blocked substitution of the block itself (FP32 products), stored
        // column-major (RiC4) and transposed to row-major (RiR4)
        const int ob = 1024;
        const int64_t nbo = (n + ob - 1) / ob;
        float* Ic = (float*)(work + L.Ri4);
        float* Ir = Ic + (size_t)nbo * ob * ob;
        for (int64_t Bk = 0; Bk < nbo; ++Bk) {
            const int w = (int)std::min<int64_t>(ob, n - Bk * ob);
            float* C = Ic + (size_t)Bk * ob * ob;
            CT_HIP(launch_eye<float>(C, ob, ob, ob, w, s));
            int r = inner_solve<float>(f, C - Bk * ob, ob, w, Bk, false, nullptr, s);
            if (r) return r;
            CT_HIP((launch_transpose<float, float, true, false>(C, Ir + (size_t)Bk * ob * ob, ob, ob, ob, ob, s)));
        }
        f->RiC4 = Ic;
        f->RiR4 = Ir;
    }
    return 0;
}

// The per-block solve copies a factorization writes as it goes: the
// row-major reflector blocks and T in the storage type.
template <typename TS>
static int block_copies(ct_factor* f, hipStream_t s)
{
    const int nbo = f->nb_out;
    for (int64_t b = 0; b < f->nblocks; ++b) {
        const int64_t k0 = b * nbo;
        const int bo = (int)std::min<int64_t>(nbo, f->n - k0);
        TS* Ab = (TS*)f->A + k0 * f->lda + k0;
        int r = prep_block<TS>(f, Ab, f->lda, f->m - k0, bo, s, (TS*)f->VtAll + vt_offset(f, b));
        if (r) return r;
        if constexpr (sizeof(TS) == 4) {
            const double* Tb = f->T_all + (size_t)b * nbo * nbo;
            CT_HIP((launch_convert<double, float>(Tb, nbo, (float*)f->Tf + (size_t)b * nbo * nbo, nbo, bo, bo, s)));
        }
    }
    return 0;
}

// ------------------------------------------------------------- checkpoints
// File: a fixed header, the m x n matrix V\R column by column (m elements
// each, storage type), tau (n FP64), T of every outer block (nb_out^2 FP64
// each), then a 64-bit checksum of everything before it.
struct FactorFileHeader {
    char magic[8];          // "CTQRFAC1"
    int64_t m, n, prec, nb_out, nb_in, info, es, reserved;
};
static const char kFactorMagic[8] = {'C', 'T', 'Q', 'R', 'F', 'A', 'C', '1'};
constexpr size_t kChunk = (size_t)64 << 20;

// order-dependent 64-bit checksum of a byte stream (multiply-xorshift of
// 8-byte words, a tail padded with zeros)
struct Checksum {
    uint64_t h = 0x9E3779B97F4A7C15ull;
    void add(const void* p, size_t bytes)
    {
        const unsigned char* c = (const unsigned char*)p;
        size_t i = 0;
        for (; i + 8 <= bytes; i += 8) {
            uint64_t w;
            memcpy(&w, c + i, 8);
            mix(w);
        }
        if (i < bytes) {
            uint64_t w = 0;
            memcpy(&w, c + i, bytes - i);
            mix(w);
        }
    }
    void mix(uint64_t w)
    {
        h ^= w;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    }
};

static int read_header(FILE* fp, FactorFileHeader& hd)
{
    if (fread(&hd, sizeof hd, 1, fp) != 1) return fail(-1, "%s", "invalid argument path (not a factor file)");
    if (memcmp(hd.magic, kFactorMagic, 8) != 0) return fail(-1, "%s", "invalid argument path (not a factor file)");
    if (hd.m <= 0 || hd.n <= 0 || hd.n > hd.m || hd.prec < CT_PREC_F64 || hd.prec > CT_PREC_BF16X3 ||
        hd.nb_out < 32 || hd.nb_out > 2048 || hd.es != (hd.prec == CT_PREC_F64 ? 8 : 4))
        return fail(-1, "%s", "invalid argument path (inconsistent factor file header)");
    return 0;
}

extern "C" {

int ct_factor_save(const ct_factor* f, const char* path, void* stream)
{
    CT_ARG(f != nullptr && f->st == nullptr, 1, "f (a factor held in device memory)");
    CT_ARG(path != nullptr, 2, "path");
    hipStream_t s = (hipStream_t)stream;
    int64_t info = 0;
    int r = ct_status(f, &info, stream);
    if (r) return r;
    FILE* fp = fopen(path, "wb");
    if (!fp) return fail(-2, "invalid argument path (cannot open %s for writing)", path);
    FactorFileHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, kFactorMagic, 8);
    hd.m = f->m; hd.n = f->n; hd.prec = f->prec; hd.nb_out = f->nb_out; hd.nb_in = f->nb_in; hd.info = info;
    hd.es = f->f64 ? 8 : 4;
    Checksum ck;
    std::vector<char> buf;
    bool ok = fwrite(&hd, sizeof hd, 1, fp) == 1;
    ck.add(&hd, sizeof hd);
    hipError_t e = hipSuccess;
    auto put = [&](const void* dev, size_t bytes) {
        for (size_t o = 0; ok && o < bytes; o += kChunk) {
            const size_t nb = std::min(kChunk, bytes - o);
            buf.resize(nb);
            e = hipMemcpy(buf.data(), (const char*)dev + o, nb, hipMemcpyDeviceToHost);
            if (e != hipSuccess) { ok = false; break; }
            ck.add(buf.data(), nb);
            ok = fwrite(buf.data(), 1, nb, fp) == nb;
        }
    };
    // the matrix, column groups of at most kChunk bytes (m elements a column)
    const size_t colb = (size_t)f->m * hd.es;
    const int64_t cols = std::max<int64_t>(1, (int64_t)(kChunk / colb));
    for (int64_t j0 = 0; ok && j0 < f->n; j0 += cols) {
        const int64_t nc = std::min<int64_t>(cols, f->n - j0);
        buf.resize(nc * colb);
        e = hipMemcpy2D(buf.data(), colb, (const char*)f->A + (size_t)j0 * f->lda * hd.es, (size_t)f->lda * hd.es,
                        colb, nc, hipMemcpyDeviceToHost);
        if (e != hipSuccess) { ok = false; break; }
        ck.add(buf.data(), nc * colb);
        ok = fwrite(buf.data(), 1, nc * colb, fp) == nc * colb;
    }
    if (ok) put(f->tau, (size_t)f->n * 8);
    if (ok) put(f->T_all, (size_t)f->nblocks * f->nb_out * f->nb_out * 8);
    if (ok) ok = fwrite(&ck.h, 8, 1, fp) == 1;
    const bool closed = fclose(fp) == 0;
    (void)s;
    if (e != hipSuccess) return fail(-1000 - (int)e, "save: %s", hipGetErrorString(e));
    if (!ok || !closed) return fail(-2, "invalid argument path (write to %s failed)", path);
    return 0;
}

int ct_factor_file_info(const char* path, int64_t max_nrhs, int64_t* m, int64_t* n, int* prec, size_t* work_bytes)
{
    CT_ARG(path != nullptr, 1, "path");
    CT_ARG(max_nrhs >= 0, 2, "max_nrhs");
    FILE* fp = fopen(path, "rb");
    if (!fp) return fail(-1, "invalid argument path (cannot open %s)", path);
    FactorFileHeader hd;
    const int r = read_header(fp, hd);
    fclose(fp);
    if (r) return r;
    if (m) *m = hd.m;
    if (n) *n = hd.n;
    if (prec) *prec = (int)hd.prec;
    if (work_bytes) *work_bytes = layout(hd.m, hd.n, (int)hd.prec, max_nrhs, (int)hd.nb_out).total;
    return 0;
}

int ct_factor_load(const char* path, void* A, int64_t lda, double* tau, void* work, size_t work_bytes,
                   int64_t max_nrhs, ct_factor** f_out, void* stream)
{
    CT_ARG(path != nullptr, 1, "path");
    CT_ARG(A != nullptr && aligned(A), 2, "A");
    CT_ARG(tau != nullptr, 4, "tau");
    CT_ARG(work != nullptr && aligned(work), 5, "work");
    CT_ARG(max_nrhs >= 0, 7, "max_nrhs");
    CT_ARG(f_out != nullptr, 8, "f");
    FILE* fp = fopen(path, "rb");
    if (!fp) return fail(-1, "invalid argument path (cannot open %s)", path);
    FactorFileHeader hd;
    int r = read_header(fp, hd);
    if (r) {
        fclose(fp);
        return r;
    }
    const Layout L = layout(hd.m, hd.n, (int)hd.prec, max_nrhs, (int)hd.nb_out);
    if (!(lda >= hd.m && lda % 16 == 0)) {
        fclose(fp);
        return fail(-3, "%s", "invalid argument lda (need >= m of the file, a multiple of 16)");
    }
    if (work_bytes < L.total) {
        fclose(fp);
        return fail(-6, "%s", "invalid argument work_bytes (see ct_factor_file_info)");
    }
    r = device_setup();
    if (r) {
        fclose(fp);
        return r;
    }
    hipStream_t s = (hipStream_t)stream;
    ct_factor* f = new (std::nothrow) ct_factor();
    if (!f) {
        fclose(fp);
        return fail(-1001, "%s", "out of host memory");
    }
    r = init_factor(f, A, hd.m, hd.n, lda, (int)hd.prec, tau, (char*)work, L, max_nrhs, (int)hd.nb_out);
    if (!r && f->nb_in != hd.nb_in)
        r = fail(-1, "invalid argument path (saved with panels of %lld columns, this device uses %d)",
                 (long long)hd.nb_in, f->nb_in);
    Checksum ck;
    ck.add(&hd, sizeof hd);
    std::vector<char> buf;
    hipError_t e = hipSuccess;
    bool ok = r == 0;
    auto get = [&](void* dev, size_t bytes) {
        for (size_t o = 0; ok && o < bytes; o += kChunk) {
            const size_t nb = std::min(kChunk, bytes - o);
            buf.resize(nb);
            ok = fread(buf.data(), 1, nb, fp) == nb;
            if (!ok) break;
            ck.add(buf.data(), nb);
            e = hipMemcpy((char*)dev + o, buf.data(), nb, hipMemcpyHostToDevice);
            if (e != hipSuccess) ok = false;
        }
    };
    const size_t colb = (size_t)hd.m * hd.es;
    const int64_t cols = std::max<int64_t>(1, (int64_t)(kChunk / colb));
    for (int64_t j0 = 0; ok && j0 < hd.n; j0 += cols) {
        const int64_t nc = std::min<int64_t>(cols, hd.n - j0);
        buf.resize(nc * colb);
        ok = fread(buf.data(), 1, nc * colb, fp) == nc * colb;
        if (!ok) break;
        ck.add(buf.data(), nc * colb);
        e = hipMemcpy2D((char*)A + (size_t)j0 * lda * hd.es, (size_t)lda * hd.es, buf.data(), colb, colb, nc,
                        hipMemcpyHostToDevice);
        if (e != hipSuccess) ok = false;
    }
    if (ok) get(tau, (size_t)hd.n * 8);
    if (ok) get(f->T_all, (size_t)f->nblocks * f->nb_out * f->nb_out * 8);
    uint64_t want = 0;
    if (ok) ok = fread(&want, 8, 1, fp) == 1 && want == ck.h;
    fclose(fp);
    if (r || e != hipSuccess || !ok) {
        delete f;
        if (r) return r;
        if (e != hipSuccess) return fail(-1000 - (int)e, "load: %s", hipGetErrorString(e));
        return fail(-1, "%s", "invalid argument path (truncated or corrupted factor file)");
    }
    // status words: info from the file, no failed wait
    int64_t words[2] = {hd.info, 0};
    CT_HIP(hipMemsetAsync((char*)work + L.words, 0, 256, s));
    CT_HIP(hipMemcpyAsync(f->info, words, 8, hipMemcpyHostToDevice, s));
    CT_HIP(panel_reset(f->part, f->gpart, s));
    f->VtAll = (char*)work + L.VtAll;
    int rc = f->f64 ? block_copies<double>(f, s) : block_copies<float>(f, s);
    if (!rc) rc = r_copies(f, (char*)work, L, s, true);
    if (!rc) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(-1000 - (int)e, "load: %s", hipGetErrorString(e));
    }
    if (rc) {
        delete f;
        return rc;
    }
    *f_out = f;
    return 0;
}

int ct_qr_factor(void* A, int64_t m, int64_t n, int64_t lda, int prec, double* tau, void* work, size_t work_bytes,
                 int64_t max_nrhs, ct_factor** f_out, void* stream)
{
    CT_ARG(A != nullptr && aligned(A), 1, "A");
    CT_ARG(m > 0, 2, "m");
    CT_ARG(n > 0 && n <= m, 3, "n (need 0 < n <= m)");
    CT_ARG(lda >= m && lda % 16 == 0, 4, "lda");
    const bool copies = !(prec & CT_QR_NO_SOLVE_COPIES);
    prec &= ~CT_QR_NO_SOLVE_COPIES;
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 5, "prec");
    CT_ARG(tau != nullptr, 6, "tau");
    CT_ARG(work != nullptr && aligned(work), 7, "work");
    CT_ARG(max_nrhs >= 0, 9, "max_nrhs");
    CT_ARG(f_out != nullptr, 10, "f");
    const Layout L = layout(m, n, prec, max_nrhs, nb_out_for(n), copies ? kCopiesAll : kCopiesInverses);
    CT_ARG(work_bytes >= L.total, 8, "work_bytes (see ct_qr_workspace)");
    int r = device_setup();
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;

    ct_factor* f = new (std::nothrow) ct_factor();
    if (!f) return fail(-1001, "%s", "out of host memory");
    r = init_factor(f, A, m, n, lda, prec, tau, (char*)work, L, max_nrhs, nb_out_for(n));
    if (r) {
        delete f;
        return r;
    }
    CT_HIP(hipMemsetAsync((char*)work + L.words, 0, 256, s));
    CT_HIP(panel_reset(f->part, f->gpart, s));
    f->VtAll = copies ? (char*)work + L.VtAll : nullptr;
    int rc = f->f64 ? factor_impl<double>(f, s) : factor_impl<float>(f, s);
    if (!rc) rc = r_copies(f, (char*)work, L, s, copies);
    if (rc) {
        delete f;
        return rc;
    }
    *f_out = f;
    return 0;
}

int ct_qr_stream_workspace(int64_t m, int64_t n, int64_t lda, int prec, int64_t max_nrhs, int64_t tile_cols,
                           size_t* min_bytes, size_t* all_resident_bytes)
{
    CT_ARG(m > 0, 1, "m");
    CT_ARG(n > 0 && n <= m, 2, "n (need 0 < n <= m)");
    CT_ARG(lda >= m && lda % 16 == 0, 3, "lda");
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 4, "prec");
    CT_ARG(max_nrhs >= 0, 5, "max_nrhs");
    CT_ARG(tile_cols > 0 && tile_cols % 128 == 0, 6, "tile_cols (a positive multiple of 128)");
    CT_ARG(min_bytes != nullptr, 7, "min_bytes");
    const size_t es = prec == CT_PREC_F64 ? 8 : 4;
    const int64_t nt = (n + tile_cols - 1) / tile_cols;
    const size_t base = layout(m, n, prec, max_nrhs, kNbStream, kCopiesNone).total, tb = tile_bytes(lda, tile_cols, es);
    *min_bytes = base + std::min<int64_t>(nt, kSlots) * tb;
    if (all_resident_bytes) *all_resident_bytes = base + nt * tb;
    return 0;
}

int ct_qr_factor_streamed(void* A_host, int64_t m, int64_t n, int64_t lda, int prec, double* tau, void* work,
                          size_t work_bytes, int64_t max_nrhs, int64_t tile_cols, ct_factor** f_out, void* stream)
{
    CT_ARG(A_host != nullptr, 1, "A_host");
    CT_ARG(m > 0, 2, "m");
    CT_ARG(n > 0 && n <= m, 3, "n (need 0 < n <= m)");
    CT_ARG(lda >= m && lda % 16 == 0, 4, "lda");
    CT_ARG(prec >= CT_PREC_F64 && prec <= CT_PREC_BF16X3, 5, "prec");
    CT_ARG(tau != nullptr, 6, "tau");
    CT_ARG(work != nullptr && aligned(work), 7, "work");
    CT_ARG(max_nrhs >= 0, 9, "max_nrhs");
    CT_ARG(tile_cols > 0 && tile_cols % 128 == 0, 10, "tile_cols (a positive multiple of 128)");
    CT_ARG(f_out != nullptr, 11, "f");
    size_t need = 0, full = 0;
    ct_qr_stream_workspace(m, n, lda, prec, max_nrhs, tile_cols, &need, &full);
    CT_ARG(work_bytes >= need, 8, "work_bytes (see ct_qr_stream_workspace)");
    int r = device_setup();
    if (r) return r;
    {
        hipPointerAttribute_t at;
        const hipError_t e = hipPointerGetAttributes(&at, A_host);
        if (e != hipSuccess || at.type != hipMemoryTypeHost) {
            (void)hipGetLastError();
            return fail(-1, "%s", "invalid argument A_host (must be pinned host memory from hipHostMalloc)");
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const Layout L = layout(m, n, prec, max_nrhs, kNbStream, kCopiesNone);
    const size_t es = prec == CT_PREC_F64 ? 8 : 4;
    const size_t tb = tile_bytes(lda, tile_cols, es);
    const int64_t nt = (n + tile_cols - 1) / tile_cols;
    char* w = (char*)work;

    ct_factor* f = new (std::nothrow) ct_factor();
    StreamState* st = f ? new (std::nothrow) StreamState() : nullptr;
    if (!st) {
        delete f;
        return fail(-1001, "%s", "out of host memory");
    }
    f->st = st;
    st->Ah = (char*)A_host;
    st->es = es;
    st->wt = tile_cols;
    st->ntiles = nt;
    if (work_bytes >= full) {
        st->nres = nt;
    } else {
        st->nres = (int64_t)((work_bytes - L.total - kSlots * tb) / tb);
        for (int k = 0; k < kSlots; ++k) st->slot[k] = w + L.total + (size_t)st->nres * tb + (size_t)k * tb;
    }
    r = init_factor(f, w + L.total, m, n, lda, prec, tau, w, L, max_nrhs, tile_cols % kNbStream == 0 ? kNbStream : 128);
    if (r) {
        delete st;
        delete f;
        return r;
    }
    auto cleanup = [&](int code) {
        delete st;
        f->st = nullptr;
        delete f;
        return code;
    };
    hipError_t e = hipStreamCreateWithFlags(&st->cin, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->cout, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->done, hipEventDisableTiming);
    for (int k = 0; k < kSlots && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&st->ready[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st->used[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st->out[k], hipEventDisableTiming);
    }
    st->res_ready.assign(st->nres, nullptr);
    st->res_loaded.assign(st->nres, 0);
    st->d2h.assign(nt, nullptr);
    st->d2h_rec.assign(nt, 0);
    for (int64_t t = 0; t < st->nres && e == hipSuccess; ++t)
        e = hipEventCreateWithFlags(&st->res_ready[t], hipEventDisableTiming);
    for (int64_t t = 0; t < nt && e == hipSuccess; ++t)
        e = hipEventCreateWithFlags(&st->d2h[t], hipEventDisableTiming);
    if (e != hipSuccess) {
        snprintf(g_err, sizeof g_err, "stream set-up: %s", hipGetErrorString(e));
        return cleanup(-1000 - (int)e);
    }
    e = hipMemsetAsync(w + L.words, 0, 256, s);
    if (e == hipSuccess) e = panel_reset(f->part, f->gpart, s);
    if (e != hipSuccess) {
        snprintf(g_err, sizeof g_err, "hipMemsetAsync: %s", hipGetErrorString(e));
        return cleanup(-1000 - (int)e);
    }
    const int rc = f->f64 ? stream_factor<double>(f, s) : stream_factor<float>(f, s);
    if (rc == -2002) {
        *f_out = f;     // resumable
        return rc;
    }
    if (rc) return cleanup(rc);
    *f_out = f;
    return 0;
}

int ct_qr_resume(ct_factor* f, void* stream)
{
    CT_ARG(f != nullptr && f->st != nullptr, 1, "f (a streamed factor)");
    CT_ARG(!f->st->broken, 1, "f (a tile's write-back to the host matrix failed; the factorization cannot resume)");
    if (f->st->next_tile >= f->st->ntiles) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? stream_factor<double>(f, s) : stream_factor<float>(f, s);
}

int ct_stream_info(const ct_factor* f, int64_t* tiles, int64_t* resident, int64_t* next_tile)
{
    CT_ARG(f != nullptr, 1, "f");
    const StreamState* st = f->st;
    if (tiles) *tiles = st ? st->ntiles : 0;
    if (resident) *resident = st ? st->nres : 0;
    if (next_tile) *next_tile = st ? st->next_tile : 0;
    return 0;
}

int ct_debug_wait_limit(int64_t ticks)
{
    panel_set_wait_limit(ticks);
    return 0;
}

int ct_quality(const double* X, int64_t ldx, const double* ref, int64_t ldr, int32_t n_pix, int64_t k,
               const int32_t* crop_host, int32_t window, double* out, void* stream)
{
    CT_ARG(X != nullptr || k == 0, 1, "X");
    CT_ARG(n_pix > 0 && ldx >= (int64_t)n_pix * n_pix, 2, "ldx");
    CT_ARG(ref != nullptr || k == 0, 3, "ref");
    CT_ARG(ldr >= (int64_t)n_pix * n_pix, 4, "ldr");
    CT_ARG(n_pix > 0, 5, "n_pix");
    CT_ARG(k >= 0 && k <= 2147483647, 6, "k");
    int crop[4] = {0, 0, 0, 0};
    if (crop_host)
        for (int i = 0; i < 4; ++i) crop[i] = crop_host[i];
    CT_ARG(window >= 2, 8, "window");
    CT_ARG(crop[0] >= 0 && crop[1] >= 0 && crop[2] >= 0 && crop[3] >= 0 && n_pix - crop[0] - crop[1] >= window &&
               n_pix - crop[2] - crop[3] >= window,
           7, "crop_host (non-negative margins leaving at least window x window pixels)");
    CT_ARG(out != nullptr || k == 0, 9, "out");
    if (k == 0) return 0;
    CT_HIP(launch_quality(X, ldx, ref, ldr, n_pix, k, crop, window, out, (hipStream_t)stream));
    return 0;
}

int ct_debug_panel_width(int nbi)
{
    if (nbi != 0 && nbi != 16 && nbi != 32) return fail(-1, "%s", "invalid argument nbi (0, 16 or 32)");
    g_nbi_force = nbi;
    return 0;
}

int ct_debug_progress(int64_t blocks)
{
    if (blocks < 0) return fail(-1, "%s", "invalid argument blocks (>= 0)");
    g_progress_blocks = blocks;
    return 0;
}

int ct_debug_refine_x3(int mode)
{
    if (mode < 0 || mode > 2) return fail(-1, "%s", "invalid argument mode (0, 1 or 2)");
    const int was = g_x3_refine;
    g_x3_refine = mode;
    return was;
}

int ct_debug_panel_cholesky(int enable)
{
    panel_set_cholesky(enable != 0);
    return 0;
}

int ct_debug_block_width(int nb_out)
{
    CT_ARG(nb_out == 0 || (nb_out >= 32 && nb_out <= 2048 && nb_out % 32 == 0), 1, "nb_out (0, or a multiple of 32 up to 2048)");
    g_nb_force = nb_out;
    return 0;
}

int ct_stream_inject_failure(int64_t tile, int64_t after_updates)
{
    g_inject_tile = tile;
    g_inject_after = tile < 0 ? -1 : after_updates;
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
    *bytes = 2 * up256((size_t)m * lt * 8) + 2 * up256((size_t)n * lt * 8) + up256((size_t)ld * nrhs * 8) +
             up256((size_t)256 * lt * 8);
    return 0;
}

int ct_refine_workspace_for(int64_t m, int64_t n, int64_t nrhs, int32_t method, size_t* bytes)
{
    CT_ARG(method == CT_REFINE_QR || method == CT_REFINE_SNE || method == CT_REFINE_PCGLS, 4, "method");
    CT_ARG(bytes != nullptr, 5, "bytes");
    int r = ct_refine_workspace(m, n, nrhs, bytes);
    if (r) return r;
    const int64_t lt = (nrhs + 15) / 16 * 16;
    if (method == CT_REFINE_PCGLS) *bytes += up256((size_t)n * lt * 8) + up256((size_t)5 * lt * 8);
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


int ct_group_sparse(int64_t rows, const int64_t* ptr, const int32_t* idx, const double* val, int32_t group,
                    int64_t* gptr, int32_t* gidx, double* gval, int64_t* count, int32_t* work, void* stream)
{
    CT_ARG(rows > 0, 1, "rows");
    CT_ARG(ptr && idx && val, 2, "sparse arrays");
    CT_ARG(group == 1 || group == 2 || group == 4 || group == 8, 5, "group (1, 2, 4 or 8)");
    CT_ARG(gptr != nullptr, 6, "gptr");
    CT_ARG((gidx == nullptr) == (gval == nullptr), 7, "gidx/gval (both or neither)");
    CT_ARG(count != nullptr, 9, "count");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ng = (rows + group - 1) / group;
    if (gidx == nullptr) {
        CT_ARG(work != nullptr, 10, "work");
        CT_HIP(launch_group_count(ptr, idx, rows, group, gptr, work, s));
        int32_t err = 0;
        CT_HIP(hipMemcpyAsync(count, gptr + ng, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CT_HIP(hipMemcpyAsync(&err, work, sizeof err, hipMemcpyDeviceToHost, s));
        CT_HIP(hipStreamSynchronize(s));
        if (err) return fail(-2005, "a group of %d rows stores more than 8192 entries; use a smaller group", group);
        return 0;
    }
    CT_ARG(*count >= 0, 9, "count");
    CT_HIP(launch_group_fill(ptr, idx, val, rows, group, gptr, gidx, gval, *count, s));
    return 0;
}

int ct_solve_refined(const ct_factor* f, const ct_sparse* sp, const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, int32_t steps, int32_t method, double tol, void* scratch, size_t scratch_bytes,
                     double* res_norms, double* grad_norms, int32_t* steps_done, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(sp != nullptr && sp->row_ptr && sp->col && sp->val && sp->m == f->m && sp->n == f->n, 2,
           "A (CSR copy of the factored matrix)");
    CT_ARG(B != nullptr && ldb >= f->m, 3, "B/ldb");
    CT_ARG(X != nullptr && ldx >= f->n, 5, "X/ldx");
    CT_ARG(nrhs >= 0 && nrhs <= f->max_nrhs, 7, "nrhs (0..max_nrhs)");
    CT_ARG(steps >= 0 && steps <= 64, 8, "steps");
    CT_ARG(method == CT_REFINE_QR || method == CT_REFINE_SNE || method == CT_REFINE_PCGLS, 9, "method");
    CT_ARG(tol >= 0.0, 10, "tol");
    CT_ARG(method == CT_REFINE_QR || (sp->col_ptr && sp->row && sp->cval), 2,
           "A (CT_REFINE_SNE and CT_REFINE_PCGLS need the CSC copy)");
    size_t need = 0;
    ct_refine_workspace_for(f->m, f->n, nrhs, method, &need);
    CT_ARG(scratch != nullptr && aligned(scratch) && scratch_bytes >= need, 11, "scratch");
    if (steps_done) *steps_done = 0;
    if (nrhs == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    return f->f64 ? refined_impl<double>(f, sp, B, ldb, X, ldx, nrhs, steps, method, tol, (char*)scratch,
                                         res_norms, grad_norms, steps_done, s)
                  : refined_impl<float>(f, sp, B, ldb, X, ldx, nrhs, steps, method, tol, (char*)scratch,
                                        res_norms, grad_norms, steps_done, s);
}

}  // extern "C"

// Scratch of ct_solve_refined_noalloc: one statically allocated array per
// device (the loader reserves it with the code object; it lives until the
// process ends).  Host code never uses the symbol itself as an address: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int static_scratch(void** out)
{
    int dev = 0;
    CT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(-2004, "device %d beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        CT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(-2004, "%s", "static scratch has no device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

extern "C" {

int ct_solve_refined_noalloc(const ct_factor* f, const ct_sparse* sp, const double* B, int64_t ldb, double* X,
                             int64_t ldx, int64_t nrhs, int32_t steps, int32_t method, double tol,
                             double* res_norms, double* grad_norms, int32_t* steps_done, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(nrhs >= 0 && nrhs <= f->max_nrhs, 7, "nrhs (0..max_nrhs)");
    CT_ARG(method == CT_REFINE_QR || method == CT_REFINE_SNE || method == CT_REFINE_PCGLS, 9, "method");
    size_t need = 0;
    ct_refine_workspace_for(f->m, f->n, nrhs, method, &need);
    if (need > kStaticScratchBytes)
        return fail(-7, "invalid argument nrhs: %lld slices need %zu bytes of scratch, above the %zu-byte static "
                        "scratch of ct_solve_refined_noalloc", (long long)nrhs, need, kStaticScratchBytes);
    void* ptr = nullptr;
    int r = static_scratch(&ptr);
    if (r) return r;
    // every word of the scratch is written before it is read (the slice
    // blocks by transposes and products, the norm partials by their first
    // pass), so nothing left by an earlier call needs clearing
    return ct_solve_refined(f, sp, B, ldb, X, ldx, nrhs, steps, method, tol, ptr, kStaticScratchBytes, res_norms,
                            grad_norms, steps_done, stream);
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
    if (err & 4) {
        // reported once: the word is cleared for later launches
        CT_HIP(hipMemsetAsync(f->err, 0, 4, s));
        CT_HIP(hipStreamSynchronize(s));
        return fail(-2003, "%s", "a graph-captured solve met an invalid batch descriptor entry and solved nothing");
    }
    if (err & 8) {
        CT_HIP(hipMemsetAsync(f->err, 0, 4, s));
        CT_HIP(hipStreamSynchronize(s));
        return fail(-2006, "%s", "a cross-workgroup wait of the fused solve timed out; its result is incomplete");
    }
    return 0;
}

int ct_factor_destroy(ct_factor* f)
{
    if (f) {
        delete f->st;
        if (f->Rh) (void)hipFree(f->Rh);
    }
    delete f;
    return 0;
}

// ------------------------------------------------------------- fused solve
// One persistent launch for B <- R^{-1} Q^T B (fused.hip): needs an in-memory
// factor with its solve-side copies (row-major reflector blocks, inverses of
// R's 256 x 256 diagonal blocks); its scratch is the factor's update buffer.
// The fused solve's Rh for an FP32 factor: blockdiag(R_qq^{-1}) R right of
// the diagonal blocks, one product of R_qq^{-1} (row-major copy) with R's block
// row q read in place (K = 256) per block row.  Built once, by the first fused
// solve or graph; if the allocation fails the solves go without it (the
// back-substitution then multiplies by each inverse on the chain).
static int fused_prepare(const ct_factor* f, hipStream_t s)
{
    const int64_t n = f->n, nbq = (n + 255) / 256;
    if (f->f64 || f->Rh || f->st || !f->RiR || nbq < 2) return 0;
    void* p = nullptr;
    if (hipMalloc(&p, fused_rh_off(nbq - 1, n) * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    for (int64_t q = 0; q + 1 < nbq; ++q) {
        int nz;
        hipError_t e = launch_nt<float>((const float*)f->RiR + (size_t)q * 256 * 256, 256,
                                        (const float*)f->A + 256 * q + 256 * (q + 1) * f->lda, f->lda,
                                        (float*)p + fused_rh_off(q, n), 256, 256, (int)(n - 256 * (q + 1)), 256, false,
                                        0, &nz, s);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
            return fail(-1000 - (int)e, "fused solve, R_qq^{-1} R: %s", hipGetErrorString(e));
        }
    }
    f->Rh = p;
    return 0;
}

static int fused_solve(const ct_factor* f, void* B, int64_t ldb, int64_t nrhs, const int32_t* rec, bool coop,
                       hipStream_t s)
{
    if (f->st || !f->VtAll || !f->RiC)
        return fail(-2007, "%s", "the fused solve needs an in-memory factor with its solve-side copies");
    if (f->nb_out > 1024) return fail(-2007, "%s", "the fused solve takes outer blocks of at most 1024 columns");
    int r = device_setup();
    if (r) return r;
    const int G = g_dev.cus;
    const int64_t nbq = (f->n + 255) / 256;
    if (nbq > (int64_t)2 * G) return fail(-2007, "%s", "the fused solve takes at most 512 x CUs columns");
    const size_t es = f->f64 ? 8 : 4;
    const int nrg = fused_row_groups(f->nb_out, f->n, es, (size_t)f->wp_elems * 8, es == 4 ? 32 : 16, 32);
    const int nrw = fused_row_groups(f->nb_out, f->n, es, (size_t)f->wp_elems * 8, 8, G);
    if (nrg < 1 || nrw < 1) return fail(-2007, "%s", "the factor's update buffer is too small for the fused solve");
    FusedArgs a;
    if (!rec) {
        r = fused_prepare(f, s);
        if (r) return r;
    }
    a.A = f->A; a.lda = f->lda; a.Vt = f->VtAll; a.T = f->T_all; a.RiC = f->RiC; a.Rh = f->Rh;
    a.m = f->m; a.n = f->n; a.nbo = f->nb_out; a.nblocks = (int)f->nblocks;
    a.B = B; a.ldb = ldb; a.nrhs = (int)nrhs; a.rec = rec;
    a.scratch = (char*)f->Wp; a.nrg_cap = nrg; a.nrw = nrw; a.err = f->err; a.wait_ticks = panel_wait_limit();
    hipError_t e = f->f64 ? launch_fused_solve<double>(a, G, coop, s) : launch_fused_solve<float>(a, G, coop, s);
    if (e != hipSuccess) return fail(-1000 - (int)e, "fused solve launch: %s", hipGetErrorString(e));
    return 0;
}

extern "C" {

int ct_solve_fused(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(B != nullptr && aligned(B), 2, "B");
    CT_ARG(nrhs >= 0 && nrhs <= (int64_t)1 << 30, 3, "nrhs");
    CT_ARG(ldb >= f->m && ldb % 16 == 0, 4, "ldb");
    if (nrhs == 0) return 0;
    return fused_solve(f, B, ldb, nrhs, nullptr, true, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------- graph solves
struct ct_solve_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

static int graph_create(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols, int32_t* desc,
                        void* stream, ct_solve_graph** out, bool fused);

int ct_solve_graph_create(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols, int32_t* desc,
                          void* stream, ct_solve_graph** out)
{
    return graph_create(f, B, ldb, b_cols, max_cols, desc, stream, out, false);
}

int ct_solve_graph_create_fused(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols,
                                int32_t* desc, void* stream, ct_solve_graph** out)
{
    return graph_create(f, B, ldb, b_cols, max_cols, desc, stream, out, true);
}

}  // extern "C"

static int graph_create(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols, int32_t* desc,
                        void* stream, ct_solve_graph** out, bool fused)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(B != nullptr && aligned(B), 2, "B");
    CT_ARG(ldb >= f->m && ldb % 16 == 0, 3, "ldb");
    CT_ARG(b_cols > 0, 4, "b_cols");
    CT_ARG(max_cols > 0 && max_cols <= f->max_nrhs && max_cols <= b_cols, 5, "max_cols (1..min(max_nrhs, b_cols))");
    CT_ARG(desc != nullptr, 6, "desc");
    CT_ARG(stream != nullptr, 7, "stream (capture needs a created stream)");
    CT_ARG(out != nullptr, 8, "g");
    CT_ARG(f->st == nullptr, 1, "f (graph-captured solves need a factor held in device memory)");
    hipStream_t s = (hipStream_t)stream;
    if (fused) {
        // built outside the capture: the graph only reads it
        int r = fused_prepare(f, s);
        if (r) return r;
    }
    ct_solve_graph* g = new (std::nothrow) ct_solve_graph();
    if (!g) return fail(-1001, "%s", "out of host memory");
    CT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int32_t* rec = f->batch_rec;
    int r = 0;
    {
        hipError_t e = launch_begin_batch(desc, f->batch_rec, (int)max_cols, b_cols, f->err, s);
        if (e != hipSuccess) r = fail(-1000 - (int)e, "begin batch: %s", hipGetErrorString(e));
    }
    if (!r && fused) r = fused_solve(f, B, ldb, max_cols, rec, true, s);
    if (!r && !fused)
        r = f->f64 ? apply_qt_impl<double>(f, (double*)B, max_cols, ldb, s, true, rec)
                   : apply_qt_impl<float>(f, (float*)B, max_cols, ldb, s, true, rec);
    if (!r && !fused)
        r = f->f64 ? trsm_impl<double>(f, (double*)B, max_cols, ldb, s, rec)
                   : trsm_impl<float>(f, (float*)B, max_cols, ldb, s, rec);
    if (!r) {
        hipError_t e = launch_end_batch(desc, s);
        if (e != hipSuccess) r = fail(-1000 - (int)e, "end batch: %s", hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(s, &graph);
    if (r || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        if (r) return r;
        CT_HIP(ee);
    }
    g->graph = graph;
    hipError_t ie = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        CT_HIP(ie);
    }
    *out = g;
    return 0;
}

extern "C" {

int ct_solve_graph_launch(ct_solve_graph* g, void* stream)
{
    CT_ARG(g != nullptr, 1, "g");
    CT_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return 0;
}

int ct_solve_graph_destroy(ct_solve_graph* g)
{
    if (!g) return 0;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return 0;
}

// --------------------------------------------------------------- autotuner

static std::string tune_key(const ct_factor* f, int bucket)
{
    char buf[160];
    snprintf(buf, sizeof buf, "gfx950/%s/%lld/%lld/%d", f->f64 ? "f64" : "f32", (long long)f->m, (long long)f->n,
             bucket);
    return buf;
}

// the cache is a flat JSON object {"key": [bq, split_target], ...}
static std::map<std::string, NtPlan> read_cache(const char* path)
{
    std::map<std::string, NtPlan> out;
    FILE* fp = path ? fopen(path, "r") : nullptr;
    if (!fp) return out;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, k);
    fclose(fp);
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        int bq = 0, sp = 0;
        if (sscanf(text.c_str() + end + 1, " : [ %d , %d ]", &bq, &sp) == 2 &&
            (bq == 16 || bq == 32 || bq == 64 || bq == 128) && sp > 0)
            out[key] = NtPlan{bq, sp};
        pos = end + 1;
    }
    return out;
}

static void write_cache(const char* path, const std::map<std::string, NtPlan>& m)
{
    if (!path) return;
    FILE* fp = fopen(path, "w");
    if (!fp) return;
    fprintf(fp, "{\n");
    size_t i = 0;
    for (auto& kv : m)
        fprintf(fp, "  \"%s\": [%d, %d]%s\n", kv.first.c_str(), kv.second.bq, kv.second.split_target,
                ++i < m.size() ? "," : "");
    fprintf(fp, "}\n");
    fclose(fp);
}

int ct_autotune_solve(ct_factor* f, void* B, int64_t ldb, int64_t max_nrhs, const char* cache_path, void* stream)
{
    CT_ARG(f != nullptr, 1, "f");
    CT_ARG(B != nullptr && aligned(B), 2, "B");
    CT_ARG(ldb >= f->m && ldb % 16 == 0, 3, "ldb");
    CT_ARG(max_nrhs > 0 && max_nrhs <= f->max_nrhs, 4, "max_nrhs (1..factor max_nrhs)");
    hipStream_t s = (hipStream_t)stream;
    std::map<std::string, NtPlan> cache = read_cache(cache_path);
    static const int sizes[4] = {8, 32, 128, 512};
    static const int splits[3] = {512, 1024, 2048};
    hipEvent_t e0, e1;
    CT_HIP(hipEventCreate(&e0));
    CT_HIP(hipEventCreate(&e1));
    int rc = 0;
    for (int b = 0; b < 4 && !rc; ++b) {
        const int64_t cols = std::min<int64_t>(sizes[b], max_nrhs);
        if (b > 0 && sizes[b - 1] >= max_nrhs) break;
        const std::string key = tune_key(f, b);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            f->solve_plan[b] = hit->second;
            continue;
        }
        float best = 1e30f;
        NtPlan best_plan = f->solve_plan[b];
        for (int bq : {16, 32, 64, 128}) {
            if (bq > 2 * cols && bq > 16) continue;
            for (int sp : splits) {
                f->solve_plan[b] = NtPlan{bq, sp};
                float tmin = 1e30f;
                for (int rep = 0; rep < 3 && !rc; ++rep) {
                    hipError_t e = hipEventRecord(e0, s);
                    if (e == hipSuccess) {
                        rc = f->f64 ? apply_qt_impl<double>(f, (double*)B, cols, ldb, s, true)
                                    : apply_qt_impl<float>(f, (float*)B, cols, ldb, s, true);
                        if (!rc)
                            rc = f->f64 ? trsm_impl<double>(f, (double*)B, cols, ldb, s)
                                        : trsm_impl<float>(f, (float*)B, cols, ldb, s);
                        e = hipEventRecord(e1, s);
                    }
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) rc = -1000 - (int)e;
                    if (rep > 0 && ms < tmin) tmin = ms;   // first run warms up
                }
                if (!rc && tmin < best) {
                    best = tmin;
                    best_plan = f->solve_plan[b];
                }
            }
        }
        f->solve_plan[b] = best_plan;
        cache[key] = best_plan;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) {
        for (int b = 4; b < 5; ++b) f->solve_plan[b] = f->solve_plan[3];
        write_cache(cache_path, cache);
    }
    return rc;
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
