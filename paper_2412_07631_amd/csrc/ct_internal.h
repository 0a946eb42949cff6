// Internal definitions shared by the HIP kernels and the host driver of
// libctqr.  Not installed; the public interface is include/ctqr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace ctqr {

// ----------------------------------------------------------------------------
// Arithmetic modes of the block-reflector GEMMs (trailing update, solve).
//   F64    : FP64 operands, v_mfma_f64_16x16x4 (FP64 accumulate)
//   F32    : FP32 operands, v_mfma_f32_16x16x4 (FP32 accumulate)
//   BF16   : operands rounded to bfloat16, v_mfma_f32_16x16x32_bf16
//   F16    : operands rounded to half, v_mfma_f32_16x16x32_f16
//   BF16X3 : each FP32 operand split as hi + lo bfloat16 pair; the product is
//            hi*hi + hi*lo + lo*hi on the bf16 MFMA (about 16 significant bits)
// ----------------------------------------------------------------------------
enum Mode : int { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_F16 = 3, M_BF16X3 = 4 };

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

// Lane layouts of the 16x16 MFMA tiles used here (wavefront of 64 lanes,
// g = lane / 16, c = lane % 16):
//   A operand: lane holds A[c][k] for the k slots of its group g
//   B operand: lane holds B[k][c] for the k slots of its group g
//   D (FP32 accumulating forms): value q of lane is D[4 g + q][c]
//   D (FP64 form):               value q of lane is D[g + 4 q][c]
// The sum over k does not care which physical k a (group, slot) pair carries
// as long as A and B agree, so loaders assign k = group * S + slot with S
// consecutive k per lane, which turns every fragment load into one vector load.
__device__ __forceinline__ int d_row(int mode, int g, int q) { return mode == M_F64 ? g + 4 * q : 4 * g + q; }

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4_t v; };
template <> struct Acc<float> { typedef f4_t v; };

// Time limit of one cross-workgroup wait, in ticks of the 100 MHz real-time
// counter (0.5 s; a normal wait takes microseconds).  A wait that reaches it
// sets bit 0 of the error word; every other wait, in this launch and in later
// ones, sees the bit and ends at once, so a launch whose workgroups are not
// all resident ends with an error instead of waiting without bound.
constexpr uint64_t kWaitTicks = 50000000ull;

// Device-side copy of the scanner description (see ct_geometry).
struct GeomDev {
    int32_t n_pix, n_angles, n_det;
    double W, sid, sdd, det_length, angle0;
    int32_t proj;      // 0: Siddon's exact lengths, 1: Joseph's interpolation
};

// Launch plan of the LDS-tiled NT update kernel: tile width along the
// right-hand-side / trailing-column dimension (16, 32, 64 or 128) and the
// workgroup count the split-K heuristic aims for.
struct NtPlan {
    int bq;
    int split_target;
};

// Batch record of a graph-captured solve: the graph's first node checks the
// caller's descriptor entry of the current batch and writes rec[0] = column
// offset, rec[1] = column count (0 for an invalid entry or a launch past the
// last batch); every solve kernel of the graph reads only this record.
__device__ __forceinline__ int desc_count(const int32_t* rec, int n)
{
    if (!rec) return n;
    const int c = rec[1];
    return c < n ? c : n;
}
__device__ __forceinline__ int desc_offset(const int32_t* rec) { return rec ? rec[0] : 0; }

// Output tile of workgroup b in the NT update kernels.  The hardware places
// workgroup b on XCD b % 8; with the grid padded to a multiple of 8, each XCD
// takes a contiguous range of the tile sequence.  The sequence walks bands of
// kBand tile columns row by row (columns fastest), so the tiles that run at
// the same time on one XCD share their row and column operand blocks in L2.
// Returns false for the padding workgroups.
constexpr int kBand = 4;
__device__ __forceinline__ bool tile_of(int b, int tiles_p, int tiles_q, int& tp, int& tq)
{
    const int nt = tiles_p * tiles_q;
    const int per = (nt + 7) / 8;
    const int L = (b % 8) * per + b / 8;
    if (L >= nt) return false;
    const int band = L / (kBand * tiles_p);
    const int rest = tiles_q - band * kBand;
    const int gq = rest < kBand ? rest : kBand;
    const int local = L - band * kBand * tiles_p;
    tq = band * kBand + local % gq;
    tp = local / gq;
    return true;
}
__host__ __forceinline__ int padded_tiles(int nt) { return (nt + 7) / 8 * 8; }

struct ErrWord {
    // bit 0: barrier spin limit hit; bit 1: CSR capacity exceeded; bit 2: invalid batch descriptor entry
    int32_t flags;
};

// Arguments of the persistent fused solve (fused.hip), filled by api.hip.
struct FusedArgs {
    const void* A;        // V\R in place, column-major
    int64_t lda;
    const void* Vt;       // row-major reflector blocks: block b at vt_off(b), ld round16(width)
    const double* T;      // T of block b at b nbo^2, column-major, upper triangular
    const void* RiC;      // inverses of the 256 x 256 diagonal blocks of R, column-major, block q at q 256^2
    const void* Rh;       // FP32 factors: blockdiag(R_qq^{-1}) R right of the diagonal blocks (fused_rh_off), or null
    int64_t m, n;
    int nbo, nblocks;
    void* B;
    int64_t ldb;
    int nrhs;             // columns (eager), or the largest batch (graph)
    const int32_t* rec;   // batch record (offset, count) of a graph-captured solve, or null
    char* scratch;
    int nrg_cap;          // row groups of the W partials at most (wide chunks)
    int nrw;              // row ranges of the narrow FP32 chunks (one per workgroup at most)
    int32_t* err;
    uint64_t wait_ticks;
};

// Element offset of block row q in the fused solve's Rh (block row q: the
// 256 x (n - 256(q+1)) part of blockdiag(R_qq^{-1}) R right of the diagonal
// block, column-major with leading dimension 256); fused_rh_off(nbq - 1, n) is
// the whole size.
__host__ __device__ inline size_t fused_rh_off(int64_t q, int64_t n)
{
    return (size_t)256 * (size_t)(q * n - 256 * (q * (q + 1) / 2));
}

}  // namespace ctqr
