// Profiling probe of libctqr's hot kernels at the shapes of a factorization
// and a refined solve, for hardware-counter passes of a profiler.  It runs no
// cooperative launch (the Householder panels use one; the counter mode of a
// profiler did not survive those), so it calls the library's kernel
// launchers directly on synthetic operands of the same sizes -- the traffic
// of a product does not depend on the values it multiplies.
//
//   kernel_probe [--n-pix 256] [--views 120] [--bins 640] [--nrhs 512]
//                [--nb 1024] [--copy-mib 1024] [--phases copy,update,vtc,solve,spmm]
//
//   copy:   one plain device-to-device copy of --copy-mib MiB (calibrates the
//           byte counters: it reads and writes exactly that many bytes)
//   update: C -= V W' of every outer block of the BF16x3 factorization, in
//           order (m_k = m - nb b rows, n_c = n - nb (b + 1) columns, K = nb;
//           V and W' as bfloat16 halves)
//   vtc:    W = V^T C of every outer block (V split, C FP32 split when read)
//   solve:  the BF16x3 products of one Q^T B of nrhs slices (X and Y FP32)
//   spmm:   the refinement's grouped FP64 products r = b - A x and A^T r on
//           the scanner's Siddon matrix (8 rays / 8 pixels per group)
// Each launch is timed with HIP events; the per-phase totals are printed.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/ctqr.h"

namespace ctqr {
hipError_t launch_nt_x3dl(const void* Xh, const void* Xl, int64_t ldx, const void* Yh, const void* Yl, int64_t ldy,
                          float* out, int64_t ldo, int64_t P, int Q, int64_t K, bool sub, int64_t ocap, int* nz_out,
                          hipStream_t s);
hipError_t launch_group_spmm(const int64_t* gptr, const int32_t* gidx, const double* gval, int group, int64_t rows,
                             const double* Z, const double* B, double* out, int64_t ld, int nrhs, bool sub,
                             hipStream_t s);
}  // namespace ctqr

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

__global__ void fill_u16(uint16_t* p, size_t n, uint16_t base)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = (uint16_t)(base + (uint16_t)(i % 61));
}
__global__ void fill_f32(float* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = 1e-3f * (float)(i % 97);
}
__global__ void fill_f64(double* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = 1e-3 * (double)(i % 89);
}

int main(int argc, char** argv)
{
    int n_pix = 256, views = 120, bins = 640, nrhs = 512, nb = 1024;
    long copy_mib = 1024;
    std::string phases = "copy,update,vtc,solve,spmm";
    for (int i = 1; i + 1 < argc; i += 2) {
        if (!strcmp(argv[i], "--n-pix")) n_pix = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--views")) views = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--bins")) bins = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--nrhs")) nrhs = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--nb")) nb = atoi(argv[i + 1]);
        else if (!strcmp(argv[i], "--copy-mib")) copy_mib = atol(argv[i + 1]);
        else if (!strcmp(argv[i], "--phases")) phases = argv[i + 1];
        else {
            fprintf(stderr, "unknown option %s\n", argv[i]);
            return 2;
        }
    }
    auto want = [&](const char* p) { return phases.find(p) != std::string::npos; };
    const int64_t m = (int64_t)views * bins, n = (int64_t)n_pix * n_pix;
    const int64_t ldc = (m + 15) / 16 * 16;
    if (nb % 256 != 0 || nb <= 0 || n <= nb) {
        fprintf(stderr, "--nb must be a positive multiple of 256 below n\n");
        return 2;
    }
    const int64_t nblocks = (n + nb - 1) / nb;
    printf("kernel probe: m %lld n %lld nb %d nrhs %d phases %s\n", (long long)m, (long long)n, nb, nrhs,
           phases.c_str());
    fflush(stdout);
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    auto timed = [&](auto&& launch) {
        HIP_OK(hipEventRecord(e0, s));
        launch();
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms;
    };
    std::vector<void*> keep;   // everything stays allocated until the end
    auto dalloc = [&](size_t bytes) {
        void* p;
        HIP_OK(hipMalloc(&p, bytes));
        keep.push_back(p);
        return p;
    };

    if (want("copy") && copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void* a = dalloc(bytes);
        void* b = dalloc(bytes);
        HIP_OK(hipMemsetAsync(a, 1, bytes, s));
        const double ms = timed([&] { HIP_OK(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, s)); });
        printf("copy: %ld MiB read, %ld MiB written, %.3f ms\n", copy_mib, copy_mib, ms);
        fflush(stdout);
    }

    if (want("update") || want("vtc") || want("solve")) {
        // operands of the largest (first) block, reused by every later one
        const int64_t mk0 = m, nc0 = n - nb;
        float* C = (float*)dalloc((size_t)ldc * nc0 * 4);
        uint16_t* Vh = (uint16_t*)dalloc((size_t)ldc * nb * 2);
        uint16_t* Vl = (uint16_t*)dalloc((size_t)ldc * nb * 2);
        uint16_t* Wh = (uint16_t*)dalloc((size_t)nb * nc0 * 2);
        uint16_t* Wl = (uint16_t*)dalloc((size_t)nb * nc0 * 2);
        const int64_t ocap = (int64_t)2 * nb * std::max<int64_t>(n, 64 * (int64_t)std::max(nrhs, 1));
        float* Wp = (float*)dalloc((size_t)ocap * 4);
        hipLaunchKernelGGL(fill_f32, dim3(8192), dim3(256), 0, s, C, (size_t)ldc * nc0);
        hipLaunchKernelGGL(fill_u16, dim3(8192), dim3(256), 0, s, Vh, (size_t)ldc * nb, (uint16_t)0x3c00);
        hipLaunchKernelGGL(fill_u16, dim3(8192), dim3(256), 0, s, Vl, (size_t)ldc * nb, (uint16_t)0x3400);
        hipLaunchKernelGGL(fill_u16, dim3(8192), dim3(256), 0, s, Wh, (size_t)nb * nc0, (uint16_t)0x3c00);
        hipLaunchKernelGGL(fill_u16, dim3(8192), dim3(256), 0, s, Wl, (size_t)nb * nc0, (uint16_t)0x3400);
        HIP_OK(hipStreamSynchronize(s));
        (void)mk0;
        if (want("update")) {
            double ms = 0, fl = 0;
            for (int64_t b = 0; b + 1 < nblocks; ++b) {
                const int64_t mk = m - nb * b;
                const int nc = (int)(n - nb * (b + 1));
                int nz;
                ms += timed([&] {
                    HIP_OK(ctqr::launch_nt_x3dl(Vh, Vl, nb, Wh, Wl, nb, C, ldc, mk, nc, nb, true, 0, &nz, s));
                });
                fl += 2.0 * mk * nb * nc;
            }
            printf("update (C -= V W'): %lld launches, %.2f ms, %.1f TFLOP/s\n", (long long)(nblocks - 1), ms,
                   fl / (ms * 1e-3) / 1e12);
            fflush(stdout);
        }
        if (want("vtc")) {
            double ms = 0, fl = 0;
            for (int64_t b = 0; b + 1 < nblocks; ++b) {
                const int64_t mk = m - nb * b;
                const int nc = (int)(n - nb * (b + 1));
                int nz;
                ms += timed([&] {
                    HIP_OK(ctqr::launch_nt_x3dl(Vh, Vl, ldc, C, nullptr, ldc, Wp, nb, nb, nc, mk, false, ocap, &nz,
                                                s));
                });
                fl += 2.0 * mk * nb * nc;
            }
            printf("vtc (W = V^T C): %lld launches, %.2f ms, %.1f TFLOP/s\n", (long long)(nblocks - 1), ms,
                   fl / (ms * 1e-3) / 1e12);
            fflush(stdout);
        }
        if (want("solve")) {
            // one Q^T B of nrhs slices: per block, W = V^T B and B -= V W'
            // with FP32 operands (the reflector block, B and W' read as FP32)
            float* Bs = (float*)dalloc((size_t)ldc * nrhs * 4);
            float* Vf = C;                          // any FP32 block of the right size
            float* Wf = (float*)dalloc((size_t)nb * nrhs * 4);
            hipLaunchKernelGGL(fill_f32, dim3(4096), dim3(256), 0, s, Bs, (size_t)ldc * nrhs);
            hipLaunchKernelGGL(fill_f32, dim3(1024), dim3(256), 0, s, Wf, (size_t)nb * nrhs);
            double ms = 0, fl = 0;
            for (int64_t b = 0; b < nblocks; ++b) {
                const int64_t mk = m - nb * b;
                int nz;
                ms += timed([&] {
                    HIP_OK(ctqr::launch_nt_x3dl(Vf, nullptr, ldc, Bs + nb * b, nullptr, ldc, Wp, nb, nb, nrhs, mk,
                                                false, ocap, &nz, s));
                    HIP_OK(ctqr::launch_nt_x3dl(Vf, nullptr, nb, Wf, nullptr, nb, Bs + nb * b, ldc, mk, nrhs, nb,
                                                true, 0, &nz, s));
                });
                fl += 4.0 * mk * nb * nrhs;
            }
            printf("solve (Q^T B, %d slices): %lld block pairs, %.2f ms, %.1f TFLOP/s\n", nrhs, (long long)nblocks, ms,
                   fl / (ms * 1e-3) / 1e12);
            fflush(stdout);
        }
    }

    if (want("spmm")) {
        ct_geometry g;
        memset(&g, 0, sizeof g);
        g.n_pix = n_pix;
        g.n_angles = views;
        g.n_det = bins;
        g.grid_width = 1.0;
        g.sid = 2.0;
        g.sdd = 4.0;
        g.det_length = 2.0 * g.sdd * tan(asin(g.grid_width / (2.0 * g.sid)));
        int64_t* row_ptr = (int64_t*)dalloc((size_t)(m + 1) * 8);
        CT_OK(ct_build_csr(&g, row_ptr, nullptr, nullptr, 0, s));
        int64_t nnz = 0;
        HIP_OK(hipMemcpy(&nnz, row_ptr + m, 8, hipMemcpyDeviceToHost));
        int32_t* col = (int32_t*)dalloc((size_t)nnz * 4);
        double* val = (double*)dalloc((size_t)nnz * 8);
        int32_t* row = (int32_t*)dalloc((size_t)nnz * 4);
        double* cval = (double*)dalloc((size_t)nnz * 8);
        int64_t* col_ptr = (int64_t*)dalloc((size_t)(n + 1) * 8);
        int32_t* work = (int32_t*)dalloc((size_t)n * 4);
        CT_OK(ct_build_csr(&g, row_ptr, col, val, nnz, s));
        CT_OK(ct_build_csc(m, n, row_ptr, col, val, col_ptr, row, cval, work, s));
        struct Grp { int g; int64_t* ptr; int32_t* idx; double* val; };
        auto grouped = [&](int64_t rows, const int64_t* p, const int32_t* ix, const double* v) {
            for (int gs = 8; gs >= 1; gs /= 2) {
                int64_t* gp = (int64_t*)dalloc((size_t)((rows + gs - 1) / gs + 1) * 8);
                int64_t cnt = 0;
                const int rc = ct_group_sparse(rows, p, ix, v, gs, gp, nullptr, nullptr, &cnt, work, s);
                if (rc == -2005) continue;
                CT_OK(rc);
                int32_t* gi = (int32_t*)dalloc((size_t)cnt * 4);
                double* gv = (double*)dalloc((size_t)cnt * gs * 8);
                CT_OK(ct_group_sparse(rows, p, ix, v, gs, gp, gi, gv, &cnt, work, s));
                return Grp{gs, gp, gi, gv};
            }
            fprintf(stderr, "no group size fits\n");
            exit(1);
        };
        const Grp gr = grouped(m, row_ptr, col, val), gc = grouped(n, col_ptr, row, cval);
        const int64_t lt = (nrhs + 15) / 16 * 16;
        double* Xt = (double*)dalloc((size_t)n * lt * 8);
        double* Bt = (double*)dalloc((size_t)m * lt * 8);
        double* Rt = (double*)dalloc((size_t)m * lt * 8);
        double* St = (double*)dalloc((size_t)n * lt * 8);
        hipLaunchKernelGGL(fill_f64, dim3(4096), dim3(256), 0, s, Xt, (size_t)n * lt);
        hipLaunchKernelGGL(fill_f64, dim3(4096), dim3(256), 0, s, Bt, (size_t)m * lt);
        double msr = 0, msc = 0;
        for (int rep = 0; rep < 3; ++rep) {
            msr += timed([&] {
                HIP_OK(ctqr::launch_group_spmm(gr.ptr, gr.idx, gr.val, gr.g, m, Xt, Bt, Rt, lt, nrhs, true, s));
            });
            msc += timed([&] {
                HIP_OK(ctqr::launch_group_spmm(gc.ptr, gc.idx, gc.val, gc.g, n, Rt, nullptr, St, lt, nrhs, false, s));
            });
        }
        printf("spmm: nnz %lld, residual %.3f ms, A^T r %.3f ms (%d slices, averages of 3)\n", (long long)nnz,
               msr / 3, msc / 3, nrhs);
        fflush(stdout);
    }
    for (void* p : keep) HIP_OK(hipFree(p));
    HIP_OK(hipStreamDestroy(s));
    printf("kernel probe done\n");
    fflush(stdout);
    return 0;
}
