// Native driver of libctqr (C-ABI only, no Python): assembles the Siddon
// system matrix of a fan-beam scanner, factors it once at the chosen
// precision and solves one block of right-hand sides, timing each phase with
// HIP events.  Used for profiler runs (hardware counters) where a Python
// process would add its own dispatches, and as a minimal example of the
// interface.  An optional plain device-to-device copy of known size runs
// first, so that the byte counters of a profiler can be calibrated on it.
//
//   ctqr_bench [--n-pix 256] [--views 120] [--bins 640]
//              [--prec f64|f32|bf16|f16|bf16x3] [--nrhs 16] [--copy-mib 0]
//              [--stream-gib G --tile-cols 1024] [--nb-out 0] [--refine S]
// With --stream-gib the matrix is factored from pinned host memory
// (ct_qr_factor_streamed) with a device buffer of G GiB, and the time
// includes every host<->device transfer.  With --refine S the in-memory run
// also solves the nrhs right-hand sides with S steps of FP64-residual
// refinement (ct_solve_refined, semi-normal-equations steps) and times it;
// --group G (default 8, 0: none) sets the grouping of its sparse products.
// --adjoint K times ct_solve_backward on K gradients (K <= nrhs) next to a
// forward solve of K slices.
//
// Scanner: grid width 1, source-isocentre distance 2, source-detector 4, flat
// detector whose fan covers the circle inscribed in the image (the reading of
// the paper's Table 1 geometry used throughout the library's tests).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/ctqr.h"

#define HIP_OK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));              \
            exit(1);                                                                    \
        }                                                                               \
    } while (0)
#define CT_OK(x)                                                                        \
    do {                                                                                \
        int r_ = (x);                                                                   \
        if (r_ != 0) {                                                                  \
            fprintf(stderr, "%s returned %d: %s\n", #x, r_, ct_last_error());           \
            exit(1);                                                                    \
        }                                                                               \
    } while (0)

static int prec_of(const char* s)
{
    if (!strcmp(s, "f64")) return CT_PREC_F64;
    if (!strcmp(s, "f32")) return CT_PREC_F32;
    if (!strcmp(s, "bf16")) return CT_PREC_BF16;
    if (!strcmp(s, "f16")) return CT_PREC_F16;
    if (!strcmp(s, "bf16x3")) return CT_PREC_BF16X3;
    fprintf(stderr, "unknown precision %s\n", s);
    exit(2);
}

int main(int argc, char** argv)
{
    int n_pix = 256, views = 120, bins = 640, nrhs = 16;
    long copy_mib = 0;
    double stream_gib = 0.0;
    long tile_cols = 1024;
    int nb_out = 0, refine = -1, group = 8, adjoint = 0;
    const char* pname = "bf16x3";
    for (int i = 1; i + 1 < argc; i += 2) {
        if (!strcmp(argv[i], "--n-pix")) n_pix = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--views")) views = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--bins")) bins = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--prec")) pname = argv[i + 1];
        else if (!strcmp(argv[i], "--nrhs")) nrhs = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--copy-mib")) copy_mib = atol(argv[i + 1]);
        else if (!strcmp(argv[i], "--stream-gib")) stream_gib = atof(argv[i + 1]);
        else if (!strcmp(argv[i], "--tile-cols")) tile_cols = atol(argv[i + 1]);
        else if (!strcmp(argv[i], "--nb-out")) nb_out = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--refine")) refine = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--group")) group = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--adjoint")) adjoint = atoi(argv[i + 1]);
        else {
            fprintf(stderr, "unknown option %s\n", argv[i]);
            return 2;
        }
    }
    const int prec = prec_of(pname);
    CT_OK(ct_debug_block_width(nb_out));
    ct_geometry g;
    memset(&g, 0, sizeof g);
    g.n_pix = n_pix;
    g.n_angles = views;
    g.n_det = bins;
    g.grid_width = 1.0;
    g.sid = 2.0;
    g.sdd = 4.0;
    g.det_length = 2.0 * g.sdd * tan(asin(g.grid_width / (2.0 * g.sid)));
    g.angle0 = 0.0;
    const int64_t m = (int64_t)views * bins, n = (int64_t)n_pix * n_pix;
    const int64_t lda = (m + 15) / 16 * 16;
    const size_t es = prec == CT_PREC_F64 ? 8 : 4;
    printf("m %lld n %lld prec %s nrhs %d\n", (long long)m, (long long)n, pname, nrhs);
    fflush(stdout);

    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    if (copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void *a, *b;
        HIP_OK(hipMalloc(&a, bytes));
        HIP_OK(hipMalloc(&b, bytes));
        HIP_OK(hipMemsetAsync(a, 1, bytes, s));
        HIP_OK(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
        HIP_OK(hipFree(a));
        HIP_OK(hipFree(b));
        printf("copy probe: %ld MiB read, %ld MiB written\n", copy_mib, copy_mib);
        fflush(stdout);
    }

    if (stream_gib > 0.0) {
        // out-of-core: A built on the device, moved to pinned host memory,
        // then factored from there through a device buffer of stream_gib GiB
        size_t lo = 0, full = 0;
        CT_OK(ct_qr_stream_workspace(m, n, lda, prec, nrhs, tile_cols, &lo, &full));
        size_t wb = (size_t)(stream_gib * (double)(1ull << 30));
        if (wb < lo) wb = lo;
        if (wb > full) wb = full;
        void *Ad, *Ah, *work;
        double* tau;
        HIP_OK(hipMalloc(&Ad, (size_t)n * lda * es));
        CT_OK(ct_build_system(&g, prec == CT_PREC_F64 ? CT_F64 : CT_F32, Ad, lda, s));
        HIP_OK(hipHostMalloc(&Ah, (size_t)n * lda * es, hipHostMallocDefault));
        HIP_OK(hipMemcpyAsync(Ah, Ad, (size_t)n * lda * es, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        HIP_OK(hipFree(Ad));
        HIP_OK(hipMalloc(&tau, (size_t)n * sizeof(double)));
        HIP_OK(hipMalloc(&work, wb));
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        ct_factor* f = nullptr;
        HIP_OK(hipEventRecord(e0, s));
        CT_OK(ct_qr_factor_streamed(Ah, m, n, lda, prec, tau, work, wb, nrhs, tile_cols, &f, s));
        HIP_OK(hipEventRecord(e1, s));
        int64_t info = 0, tiles = 0, res = 0;
        CT_OK(ct_status(f, &info, s));
        CT_OK(ct_stream_info(f, &tiles, &res, nullptr));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        const double fl = 2.0 * m * (double)n * n - 2.0 * (double)n * n * n / 3.0;
        printf("streamed: info %lld tiles %lld resident %lld device %.2f GiB of %.2f (A %.2f GiB) qr_ms %.1f "
               "qr_tflops %.2f\n", (long long)info, (long long)tiles, (long long)res, wb / 1073741824.0,
               full / 1073741824.0, (double)n * lda * es / 1073741824.0, ms, fl / (ms * 1e-3) / 1e12);
        fflush(stdout);
        CT_OK(ct_factor_destroy(f));
        HIP_OK(hipFree(work));
        HIP_OK(hipFree(tau));
        HIP_OK(hipHostFree(Ah));
        HIP_OK(hipStreamDestroy(s));
        return info == 0 ? 0 : 3;
    }

    void *A, *work, *B;
    double* tau;
    size_t wbytes = 0;
    CT_OK(ct_qr_workspace(m, n, prec, nrhs, &wbytes));
    HIP_OK(hipMalloc(&A, (size_t)n * lda * es));
    HIP_OK(hipMalloc(&tau, (size_t)n * sizeof(double)));
    HIP_OK(hipMalloc(&work, wbytes));
    HIP_OK(hipMalloc(&B, (size_t)nrhs * lda * es));
    {
        // right-hand sides: a fixed pseudo-random pattern (the factorization
        // and the solve do not depend on the values)
        std::vector<char> h((size_t)nrhs * lda * es);
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (size_t i = 0; i < (size_t)nrhs * lda; ++i) {
            x ^= x << 13; x ^= x >> 7; x ^= x << 17;
            const double v = (double)(x >> 11) / 9007199254740992.0;
            if (es == 8) ((double*)h.data())[i] = v;
            else ((float*)h.data())[i] = (float)v;
        }
        HIP_OK(hipMemcpy(B, h.data(), h.size(), hipMemcpyHostToDevice));
    }
    hipEvent_t ev[4];
    for (auto& e : ev) HIP_OK(hipEventCreate(&e));
    CT_OK(ct_build_system(&g, prec == CT_PREC_F64 ? CT_F64 : CT_F32, A, lda, s));
    ct_factor* f = nullptr;
    HIP_OK(hipEventRecord(ev[0], s));
    CT_OK(ct_qr_factor(A, m, n, lda, prec, tau, work, wbytes, nrhs, &f, s));
    HIP_OK(hipEventRecord(ev[1], s));
    HIP_OK(hipEventRecord(ev[2], s));
    CT_OK(ct_apply_qt(f, B, nrhs, lda, s));
    CT_OK(ct_trsm_solve(f, B, nrhs, lda, s));
    HIP_OK(hipEventRecord(ev[3], s));
    int64_t info = 0;
    CT_OK(ct_status(f, &info, s));
    float qr_ms = 0, sol_ms = 0;
    HIP_OK(hipEventElapsedTime(&qr_ms, ev[0], ev[1]));
    HIP_OK(hipEventElapsedTime(&sol_ms, ev[2], ev[3]));
    const double fl = 2.0 * m * (double)n * n - 2.0 * (double)n * n * n / 3.0;
    printf("info %lld qr_ms %.1f qr_tflops %.2f solve_ms %.2f\n", (long long)info, qr_ms, fl / (qr_ms * 1e-3) / 1e12,
           sol_ms);
    fflush(stdout);
    if (adjoint > 0 && adjoint <= nrhs) {
        // gradB = Q R^{-T} G for K columns of the right-hand sides as G, and
        // the forward solve of the same K columns, each timed twice
        void* Gb;
        HIP_OK(hipMalloc(&Gb, (size_t)adjoint * lda * es));
        HIP_OK(hipMemcpy(Gb, B, (size_t)adjoint * lda * es, hipMemcpyDeviceToDevice));
        float fms = 0, bms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_OK(hipEventRecord(ev[0], s));
            CT_OK(ct_apply_qt(f, Gb, adjoint, lda, s));
            CT_OK(ct_trsm_solve(f, Gb, adjoint, lda, s));
            HIP_OK(hipEventRecord(ev[1], s));
            HIP_OK(hipEventRecord(ev[2], s));
            CT_OK(ct_solve_backward(f, B, adjoint, lda, Gb, lda, s));
            HIP_OK(hipEventRecord(ev[3], s));
            HIP_OK(hipEventSynchronize(ev[3]));
            HIP_OK(hipEventElapsedTime(&fms, ev[0], ev[1]));
            HIP_OK(hipEventElapsedTime(&bms, ev[2], ev[3]));
        }
        printf("adjoint: %d gradients %.2f ms, forward solve of %d slices %.2f ms\n", adjoint, bms, adjoint, fms);
        fflush(stdout);
        HIP_OK(hipFree(Gb));
    }
    if (refine >= 0) {
        // FP64 CSR and CSC copies of A, FP64 right-hand sides (the same
        // pattern), then the refined solve twice (the second one timed)
        int64_t *row_ptr, *col_ptr;
        HIP_OK(hipMalloc(&row_ptr, (size_t)(m + 1) * 8));
        CT_OK(ct_build_csr(&g, row_ptr, nullptr, nullptr, 0, s));
        int64_t nnz = 0;
        HIP_OK(hipMemcpy(&nnz, row_ptr + m, 8, hipMemcpyDeviceToHost));
        int32_t *col, *row, *cwork;
        double *val, *cval, *Bd, *Xd;
        HIP_OK(hipMalloc(&col, (size_t)nnz * 4));
        HIP_OK(hipMalloc(&val, (size_t)nnz * 8));
        HIP_OK(hipMalloc(&row, (size_t)nnz * 4));
        HIP_OK(hipMalloc(&cval, (size_t)nnz * 8));
        HIP_OK(hipMalloc(&col_ptr, (size_t)(n + 1) * 8));
        HIP_OK(hipMalloc(&cwork, (size_t)n * 4));
        CT_OK(ct_build_csr(&g, row_ptr, col, val, nnz, s));
        CT_OK(ct_build_csc(m, n, row_ptr, col, val, col_ptr, row, cval, cwork, s));
        const int64_t ldx = (n + 15) / 16 * 16;
        HIP_OK(hipMalloc(&Bd, (size_t)nrhs * lda * 8));
        HIP_OK(hipMalloc(&Xd, (size_t)nrhs * ldx * 8));
        {
            std::vector<double> h((size_t)nrhs * lda);
            uint64_t x = 0x2545F4914F6CDD1Dull;
            for (auto& v : h) {
                x ^= x << 13; x ^= x >> 7; x ^= x << 17;
                v = (double)(x >> 11) / 9007199254740992.0;
            }
            HIP_OK(hipMemcpy(Bd, h.data(), h.size() * 8, hipMemcpyHostToDevice));
        }
        size_t rbytes = 0;
        CT_OK(ct_refine_workspace(m, n, nrhs, &rbytes));
        void* rw;
        HIP_OK(hipMalloc(&rw, rbytes));
        ct_sparse sp{m, n, nnz, row_ptr, col, val, col_ptr, row, cval};
        // grouped copies of the CSR and CSC matrices (ct_group_sparse)
        std::vector<void*> gbufs;
        auto grouped = [&](int64_t rows, const int64_t* ptr, const int32_t* idx, const double* v, int32_t& g,
                           const int64_t*& gp, const int32_t*& gi, const double*& gv) {
            int32_t* w;
            HIP_OK(hipMalloc(&w, 4));
            gbufs.push_back(w);
            for (g = group; g >= 1; g /= 2) {
                int64_t* gptr;
                HIP_OK(hipMalloc(&gptr, (size_t)((rows + g - 1) / g + 1) * 8));
                int64_t cnt = 0;
                int rc = ct_group_sparse(rows, ptr, idx, v, g, gptr, nullptr, nullptr, &cnt, w, s);
                if (rc == -2005) {
                    HIP_OK(hipFree(gptr));
                    continue;
                }
                CT_OK(rc);
                int32_t* gidx;
                double* gval;
                HIP_OK(hipMalloc(&gidx, (size_t)cnt * 4));
                HIP_OK(hipMalloc(&gval, (size_t)cnt * g * 8));
                CT_OK(ct_group_sparse(rows, ptr, idx, v, g, gptr, gidx, gval, &cnt, w, s));
                gbufs.push_back(gptr);
                gbufs.push_back(gidx);
                gbufs.push_back(gval);
                gp = gptr;
                gi = gidx;
                gv = gval;
                printf("grouped %lld rows by %d: %lld columns stored (%.2f per row entry)\n", (long long)rows, g,
                       (long long)cnt, (double)cnt * g / (double)nnz);
                return;
            }
            g = 0;
        };
        if (group > 0) {
            grouped(m, row_ptr, col, val, sp.group_r, sp.grow_ptr, sp.grow_col, sp.grow_val);
            grouped(n, col_ptr, row, cval, sp.group_c, sp.gcol_ptr, sp.gcol_row, sp.gcol_val);
        }
        float rms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_OK(hipEventRecord(ev[0], s));
            CT_OK(ct_solve_refined(f, &sp, Bd, lda, Xd, ldx, nrhs, refine, CT_REFINE_SNE, 0.0, rw, rbytes, nullptr,
                                   nullptr, nullptr, s));
            HIP_OK(hipEventRecord(ev[1], s));
            HIP_OK(hipEventSynchronize(ev[1]));
            HIP_OK(hipEventElapsedTime(&rms, ev[0], ev[1]));
        }
        printf("refined: nnz %lld steps %d solve_ms %.2f slices_per_s %.1f\n", (long long)nnz, refine, rms,
               nrhs / (rms * 1e-3));
        fflush(stdout);
        for (void* p : {(void*)row_ptr, (void*)col_ptr, (void*)col, (void*)row, (void*)cwork, (void*)val,
                        (void*)cval, (void*)Bd, (void*)Xd, rw})
            HIP_OK(hipFree(p));
        for (void* p : gbufs) HIP_OK(hipFree(p));
    }
    CT_OK(ct_factor_destroy(f));
    HIP_OK(hipFree(A));
    HIP_OK(hipFree(tau));
    HIP_OK(hipFree(work));
    HIP_OK(hipFree(B));
    HIP_OK(hipStreamDestroy(s));
    return info == 0 ? 0 : 3;
}
