// Image quality of reconstructed slices against reference images (Sec. 3.1,
// Eqs. (snr), (mse), (psnr), (ssim)), in FP64: one workgroup per slice, every
// reduction in a fixed order (the same numbers on every run).
//   SNR  = 10 log10(sum I0^2 / sum (I0 - I)^2)
//   MSE  = mean (I0 - I)^2,  PSNR = 10 log10(MAX^2 / MSE), MAX the largest
//          reference pixel
//   SSIM = mean over every w x w window of the (cropped) image of
//          (2 mu_x mu_y + c1)(2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1)(s_x^2 + s_y^2 + c2)),
//          sample (co)variances, c1 = (0.01 L)^2, c2 = (0.03 L)^2, L the
//          reference's max - min over the crop.
#include "ct_internal.h"

#include <math.h>

namespace ctqr {

struct QualityArgs {
    const double* X;
    int64_t ldx;
    const double* R;
    int64_t ldr;
    int N;
    int bottom, top, left, right;   // crop margins in pixels
    int win;
    double* out;                    // k x 4: SNR, MSE, PSNR, SSIM
};

// op 0: sum, 1: max, 2: min; a fixed pairing tree over the 256 lanes
__device__ double block_reduce(double v, double* red, int t, int op)
{
    red[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            const double a = red[t], b = red[t + s];
            red[t] = op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
        }
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) quality_kernel(QualityArgs a)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int64_t k = blockIdx.x;
    const double* x = a.X + k * a.ldx;
    const double* r = a.R + k * a.ldr;
    const int N = a.N;
    const int H = N - a.bottom - a.top, Wd = N - a.left - a.right;
    double s2 = 0.0, e2 = 0.0, mx = -INFINITY, mn = INFINITY;
    for (int p = t; p < H * Wd; p += 256) {
        const int iy = a.bottom + p / Wd, ix = a.left + p % Wd;
        const double rv = r[iy * N + ix], d = rv - x[iy * N + ix];
        s2 += rv * rv;
        e2 += d * d;
        mx = fmax(mx, rv);
        mn = fmin(mn, rv);
    }
    const double S2 = block_reduce(s2, red, t, 0);
    const double E2 = block_reduce(e2, red, t, 0);
    const double MX = block_reduce(mx, red, t, 1);
    const double MN = block_reduce(mn, red, t, 2);
    const double mse = E2 / ((double)H * Wd);
    const double L = MX - MN;
    const double c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
    const int w = a.win, nwx = Wd - w + 1, nwy = H - w + 1;
    const double n = (double)w * w;
    double acc = 0.0;
    for (int q = t; q < nwx * nwy; q += 256) {
        const int y0 = a.bottom + q / nwx, x0 = a.left + q % nwx;
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < w; ++i)
            for (int j = 0; j < w; ++j) {
                sa += r[(y0 + i) * N + x0 + j];
                sb += x[(y0 + i) * N + x0 + j];
            }
        const double ma = sa / n, mb = sb / n;
        double va = 0.0, vb = 0.0, cab = 0.0;
        for (int i = 0; i < w; ++i)
            for (int j = 0; j < w; ++j) {
                const double da = r[(y0 + i) * N + x0 + j] - ma, db = x[(y0 + i) * N + x0 + j] - mb;
                va += da * da;
                vb += db * db;
                cab += da * db;
            }
        va /= n - 1.0;
        vb /= n - 1.0;
        cab /= n - 1.0;
        acc += ((2.0 * ma * mb + c1) * (2.0 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2));
    }
    const double SS = block_reduce(acc, red, t, 0);
    if (t == 0) {
        double* o = a.out + 4 * k;
        o[0] = E2 > 0.0 ? 10.0 * log10(S2 / E2) : INFINITY;
        o[1] = mse;
        o[2] = mse > 0.0 ? 10.0 * log10(MX * MX / mse) : INFINITY;
        o[3] = SS / ((double)nwx * nwy);
    }
}

hipError_t launch_quality(const double* X, int64_t ldx, const double* R, int64_t ldr, int N, int64_t k,
                          const int* crop, int win, double* out, hipStream_t s)
{
    QualityArgs a;
    a.X = X; a.ldx = ldx; a.R = R; a.ldr = ldr; a.N = N;
    a.bottom = crop[0]; a.top = crop[1]; a.left = crop[2]; a.right = crop[3];
    a.win = win; a.out = out;
    hipLaunchKernelGGL(quality_kernel, dim3((unsigned)k), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqr
