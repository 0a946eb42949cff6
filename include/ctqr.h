/*
 * ctqr -- direct algebraic CT reconstruction on AMD Instinct MI355X (gfx950).
 *
 * The method (paper: "Direct Low-Dose CT Image Reconstruction on GPU using
 * Out-Of-Core: Precision and Quality Study", Sec. 2, Eqs. (system), (qr),
 * (solve)): model the scanner as A X = B, with A the M x N weights matrix
 * (a_ij = contribution of ray i to pixel j), B one sinogram per column and X
 * one image per column; factor A = Q R once and reconstruct every set of
 * sinograms sharing A by X = R^{-1} (Q^T B), with Q kept as Householder
 * reflectors and R^{-1} never formed.  Sec. 2.1 names the three library calls
 * this interface mirrors: geqrf (ct_qr_factor), ormqr (ct_apply_qt) and trsm
 * (ct_trsm_solve).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers unless the name ends in _host.
 *    Matrices are column-major with an explicit leading dimension, which must
 *    be a multiple of 16 elements; device arrays must be 256-byte aligned.
 *  - The caller allocates and frees all memory.  The library never frees a
 *    caller buffer and allocates device memory only in ct_siddon_rows and
 *    in the first fused solve (or fused graph) of an FP32-storage factor,
 *    whose Rh the factor then owns (freed by ct_factor_destroy).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work and return without waiting, except ct_status and ct_siddon_rows.
 *    Calls that share a factor must be ordered on one stream.
 *  - Return value: 0 on success; -i when argument i (1-based) is invalid;
 *    -1000 - e for a HIP error e.  ct_last_error() gives the message
 *    (thread-local, valid until the next call from the same thread).
 *  - Numerical status never stalls the stream: it goes to a device word read
 *    by ct_status.
 */
#ifndef CTQR_H
#define CTQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fan-beam scanner (Table 1 lists the same parameters: circular 360-degree
 * scan, source-to-isocentre and source-to-detector distances, detector
 * count, image size, number of projections).  The image is an n_pix x n_pix
 * grid of side grid_width centred at the isocentre; pixel (ix, iy) is column
 * j = iy * n_pix + ix.  View k is at angle angle0 + 2 pi k / n_angles; the
 * flat detector of length det_length is centred on the line through the
 * isocentre at distance sdd from the source; ray i = k * n_det + d runs from
 * the source to the centre of bin d.
 * projector: CT_PROJ_SIDDON (0) -- a_ij is the exact length of ray i inside
 * pixel j (Siddon 1985); CT_PROJ_JOSEPH (1) -- Joseph's interpolating
 * projector (Joseph 1982), which the paper builds A with (Sec. 3.1): the ray
 * is sampled once per pixel-centre line across its dominant axis, the image
 * there is linearly interpolated between the two pixels whose centres
 * bracket the ray (zero outside the grid), and each sample weighs one pixel
 * width along the dominant axis, h |p1 - p0| / |d_dominant|. */
typedef struct ct_geometry {
    int32_t n_pix, n_angles, n_det, projector;
    double grid_width, sid, sdd, det_length, angle0;
} ct_geometry;

enum { CT_PROJ_SIDDON = 0, CT_PROJ_JOSEPH = 1 };

/* Storage types of A and of the sinogram blocks */
enum { CT_F64 = 0, CT_F32 = 1 };

/* Factorization precisions (the arithmetic of the trailing-matrix updates).
 * Householder column norms, tau and the reflector scaling are FP64 in all of
 * them.  CT_PREC_F64 stores A in FP64; all others store A in FP32.
 *   CT_PREC_F32    FP32 MFMA
 *   CT_PREC_BF16   bfloat16 operands, FP32 accumulation
 *   CT_PREC_F16    half operands, FP32 accumulation
 *   CT_PREC_BF16X3 each FP32 operand split into two bfloat16 halves, three
 *                  bf16 MFMA products per pair, FP32 accumulation           */
enum { CT_PREC_F64 = 0, CT_PREC_F32 = 1, CT_PREC_BF16 = 2, CT_PREC_F16 = 3, CT_PREC_BF16X3 = 4 };

typedef struct ct_factor ct_factor; /* opaque, host-side */

/* Assemble the dense system matrix (Eq. (system)) with the geometry's
 * projector (Siddon's exact ray-pixel intersection lengths, or Joseph's
 * interpolation weights).  A: m x n (m = n_angles * n_det, n = n_pix^2),
 * dtype CT_F64 or CT_F32 (FP64 weights rounded to nearest), leading
 * dimension lda >= m.  Every entry of A[0:m, 0:n] is written.  An unknown
 * projector is argument error -1. */
int ct_build_system(const ct_geometry* g, int dtype, void* A, int64_t lda, void* stream);

/* FP64 CSR copy of the same matrix, used for FP64 residuals.  row_ptr has
 * m + 1 entries.  With col == NULL and val == NULL only row_ptr is filled
 * (row_ptr[m] = nnz, read it to size col/val); otherwise col/val (capacity
 * nnz_cap) receive the entries of each row in ray order.  If nnz_cap is
 * smaller than nnz, col and val are left untouched (check row_ptr[m]). */
int ct_build_csr(const ct_geometry* g, int64_t* row_ptr, int32_t* col, double* val, int64_t nnz_cap,
                 void* stream);

/* Flag OR'ed into prec for ct_qr_workspace and ct_qr_factor: keep no
 * row-major solve-side copies (of the reflector blocks and of R above its
 * diagonal), which at 512^2 would take about 275 GB next to the 278 GB FP32
 * matrix.  The factor is the same; the inverses of R's 256 x 256 diagonal
 * blocks (and for CT_PREC_BF16X3 of its 1024 x 1024 ones) are still kept, and
 * the solves read V and R in place, R's off-diagonal blocks in NN products.
 * The workspace is about 16.5 GB at 512^2 with 1024-column blocks. */
#define CT_QR_NO_SOLVE_COPIES 0x100

/* Workspace bytes for ct_qr_factor of an m x n matrix at precision prec that
 * will later solve up to max_nrhs right-hand sides per call. */
int ct_qr_workspace(int64_t m, int64_t n, int prec, int64_t max_nrhs, size_t* bytes);

/* Householder QR, A = Q R (Eq. (qr)), in place: on return A holds R in its
 * upper triangle and the reflectors v_j (implicit unit diagonal) below it,
 * tau (n doubles) the reflector scalars, with the LAPACK sign convention
 * beta = -sign(a_jj) ||a_j||.  Requires m >= n.  A is FP64 for CT_PREC_F64 and
 * FP32 otherwise.  work (work_bytes from ct_qr_workspace) keeps the
 * compact-WY factors used by the solve and must stay alive, unmodified, with
 * A and tau until ct_factor_destroy.  *f receives the host handle. */
int ct_qr_factor(void* A, int64_t m, int64_t n, int64_t lda, int prec, double* tau, void* work,
                 size_t work_bytes, int64_t max_nrhs, ct_factor** f, void* stream);

/* Out-of-core factorization (Sec. 2.2: the matrix is split into blocks kept
 * outside device memory, part of a faster tier caches them, and transfers
 * overlap the GPU's computation, so the problem size is not bounded by
 * device memory).  Here the outer tier is
 * pinned host memory: A_host (m x n, column-major, leading dimension lda,
 * FP64 for CT_PREC_F64 else FP32) must come from hipHostMalloc and is
 * factored in place, with the same layout and results as ct_qr_factor.  The
 * matrix is processed left-looking in column tiles of tile_cols columns (a
 * multiple of 128): each tile is copied to the device, updated by every
 * earlier reflector block, factored, and copied back while the next tile is
 * processed.  Device memory is the caller's `work` buffer of work_bytes:
 * beyond the minimum from ct_qr_stream_workspace, whole tiles stay resident
 * (the leading ones first); the others are re-read from A_host when a later
 * tile or a solve needs them, so a larger buffer means less host traffic.
 * The host matrix is complete once `stream` reaches the end of the call's
 * work.  The handle works with every solve call except the graph-captured
 * ones; A_host, tau and work must stay alive until ct_factor_destroy.
 * Returns -2002 after an injected copy failure (see ct_stream_inject_failure)
 * with *f set: ct_qr_resume then continues from the failed tile.  Any error
 * inside a tile leaves the handle at that tile with the tile's host copy
 * untouched, so a resume redoes it; only a failed write-back of a finished
 * tile makes the handle unresumable (ct_qr_resume then returns -1). */
int ct_qr_stream_workspace(int64_t m, int64_t n, int64_t lda, int prec, int64_t max_nrhs, int64_t tile_cols,
                           size_t* min_bytes, size_t* all_resident_bytes);
int ct_qr_factor_streamed(void* A_host, int64_t m, int64_t n, int64_t lda, int prec, double* tau, void* work,
                          size_t work_bytes, int64_t max_nrhs, int64_t tile_cols, ct_factor** f, void* stream);
/* Continue a streamed factorization from its first unfinished tile (no-op if
 * it is complete). */
int ct_qr_resume(ct_factor* f, void* stream);
/* Tile count, resident tile count and first unfinished tile of a streamed
 * factor (all 0 for an in-memory factor). */
int ct_stream_info(const ct_factor* f, int64_t* tiles, int64_t* resident, int64_t* next_tile);
/* Failure injection for tests: the next streamed factorization (or resume)
 * stops at tile `tile` as if a copy had failed and returns -2002 -- before
 * any work on the tile (after_updates < 0), or after the reflector blocks of
 * the first after_updates earlier tiles have been applied to it (a value of
 * `tile` or more: after all of them, just before the tile's own panels).  A
 * failed tile is redone from its host copy by ct_qr_resume, which gives
 * bitwise the uninterrupted result.  tile = -1 disables. */
int ct_stream_inject_failure(int64_t tile, int64_t after_updates);

/* The Householder panels wait for each other's column reductions (their
 * workgroups must all be resident; the handle checks the occupancy).  A wait
 * longer than its limit (default 0.5 s; normal waits take microseconds) sets
 * the error word that ct_status reports as -2001, and every later wait of the
 * same factorization ends at once, so a factorization whose workgroups could
 * not all be resident fails in bounded time instead of waiting forever.  For
 * tests: set the limit in 100 MHz ticks for later factorizations and fused
 * solves (ct_solve_fused, whose time-outs ct_status reports as -2006; ticks
 * < 0 restores the default; 0 makes every wait give up). */
int ct_debug_wait_limit(int64_t ticks);
/* A Householder panel (Sec. 2.1, the geqrf step) is factored first from two
 * Gram reductions (CholeskyQR2 followed by reconstruction of the Householder
 * vectors, the same V, T, R and tau in exact arithmetic); a rank-deficient or
 * badly conditioned panel falls back, on the device, to one reduction per
 * column.  For tests: enable != 0 (default) allows the two-reduction form for
 * later factorizations, 0 forces the column-wise form.  Always returns 0. */
int ct_debug_panel_cholesky(int enable);
/* The factorization groups reflectors in outer blocks of nb_out columns (its
 * trailing update is one compact-WY block product, Sec. 2.1); nb_out is 1024
 * from 16384 columns up, else 256.  For tests: force nb_out (a multiple of 32 up to 2048) for
 * later workspace queries and factorizations, or restore the default with 0.
 * A factor must be created and used under the same setting.  Returns -1
 * (argument 1 invalid) for other values. */
int ct_debug_block_width(int nb_out);
/* ct_solve_refined on a CT_PREC_BF16X3 factor runs the products of its
 * solves (Q^T blocks, the triangular solves' diagonal steps and 256-row
 * block-column updates) in BF16x3, the precision of the factor's own trailing
 * updates, when it solves 48 slices or more (fewer: FP32 products, whose
 * fewer launches cost less there); the FP64 residual sets the final
 * accuracy.  For tests and comparisons, mode 0 makes later calls always use
 * FP32 products, 2 always BF16x3, 1 restores the default.  Returns the
 * previous mode, or -1 (argument 1 invalid) for another value. */
int ct_debug_refine_x3(int mode);

/* Test hook: width of the Householder panels (0: 32 columns, or 16 when a
 * 32-column panel of the matrix's height does not fit in the LDS of all CUs;
 * 16 or 32 forces it).  Returns -1 for other values. */
int ct_debug_panel_width(int nbi);

/* Progress of long in-memory factorizations: with blocks > 0, ct_qr_factor
 * waits for its stream after every `blocks` outer blocks (and the last) and
 * writes "ct_qr_factor: <j> of <n> columns factored" to stderr; 0 (the
 * default) turns this off.  Returns -1 for blocks < 0. */
int ct_debug_progress(int64_t blocks);

/* B <- Q^T B (Eq. (solve), first half; ormqr).  B: m x nrhs, same storage
 * type as the factor's A, nrhs <= max_nrhs.  Rows n..m-1 of the result hold
 * the least-squares residual components. */
int ct_apply_qt(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream);

/* B[0:n] <- R^{-1} B[0:n] (Eq. (solve), second half; trsm), by blocked
 * back-substitution: diagonal-block solves alternating with GEMM updates of
 * the rows above (Sec. 2.2). */
int ct_trsm_solve(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream);

/* Adjoint of the solve map of Eq. (solve), b -> x = R^{-1} Q^T b (linear in
 * b, so its transpose is the gradient map): gradB <- Q [R^{-T} G; 0], by a
 * forward substitution with R^T followed by the reflectors applied in reverse
 * order.
 * G: n x k (ldg), gradB: m x k (ldgb), both of the factor's storage type. */
int ct_solve_backward(const ct_factor* f, const void* G, int64_t k, int64_t ldg, void* gradB, int64_t ldgb,
                      void* stream);

/* R = B - A X in FP64 with the CSR copy of A (m rows); X: n x nrhs. */
int ct_residual(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t m, const double* X,
                int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs, void* stream);

/* CSC copy of A (the rows of A^T) from its CSR copy, for FP64 products A^T r.
 * col_ptr: n + 1 entries; row/cval: nnz entries each; work: n int32 scratch.
 * Entries of each column are sorted by row (the result is deterministic). */
int ct_build_csc(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                 int64_t* col_ptr, int32_t* row, double* cval, int32_t* work, void* stream);

/* Grouped copy of a sparse matrix (CSR, or CSC as the rows of A^T) for FP64
 * products with many slices: consecutive rows taken `group` at a time (1, 2,
 * 4 or 8; adjacent rays of a view cross nearly the same pixels, adjacent
 * pixels of an image row are crossed by nearly the same rays), each group
 * storing the sorted distinct column indices of its rows once and, for each
 * of them, `group` weights (zero where a row has no entry; repeated entries
 * summed).  A product then reads each slice row of the dense operand once per
 * group instead of once per stored entry.
 *   gptr: ceil(rows / group) + 1 entries; gidx: count entries; gval:
 *   count * group, weight of row g * group + r at gval[(gptr[g] + k) * group + r]
 *   for the k-th column of group g.
 * Two calls: with gidx = gval = NULL it fills gptr, waits for the stream and
 * sets *count (work: one device int32 of scratch); then with gidx / gval of
 * count (and count * group) entries it fills them.  Returns -2005 if a group
 * holds more than 8192 stored entries (use a smaller group). */
int ct_group_sparse(int64_t rows, const int64_t* ptr, const int32_t* idx, const double* val, int32_t group,
                    int64_t* gptr, int32_t* gidx, double* gval, int64_t* count, int32_t* work, void* stream);

/* The FP64 sparse copies of A used by the refinement (device arrays).  The
 * grouped copies are optional (group_r / group_c = 0: the products use the
 * CSR / CSC copies entry by entry). */
typedef struct ct_sparse {
    int64_t m, n, nnz;
    const int64_t* row_ptr; const int32_t* col; const double* val;   /* CSR of A  */
    const int64_t* col_ptr; const int32_t* row; const double* cval;  /* CSC of A (may be NULL for CT_REFINE_QR) */
    int32_t group_r, group_c;                                         /* rows per group of the grouped copies */
    const int64_t* grow_ptr; const int32_t* grow_col; const double* grow_val;  /* grouped CSR (rays) */
    const int64_t* gcol_ptr; const int32_t* gcol_row; const double* gcol_val;  /* grouped CSC (pixels) */
} ct_sparse;

/* Refinement steps (the correction is computed with the factor Q~ R~ in its
 * own precision; residuals and the accumulated solution are FP64):
 *   CT_REFINE_QR:  x += R~^{-1} Q~^T (b - A x)
 *     Its fixed point satisfies Q~^T (b - A x) = 0, which differs from the
 *     least-squares solution by O(kappa^2 u ||r||) when b is not in range(A).
 *   CT_REFINE_SNE: x += R~^{-1} R~^{-T} A^T (b - A x)   (corrected semi-normal
 *     equations, Bjorck 1987).  Its fixed point is A^T (b - A x) = 0, the
 *     least-squares solution itself; each step contracts the error by about
 *     kappa(A) u_factor.  Needs the CSC copy.
 *   CT_REFINE_PCGLS: conjugate gradients on A^T A x = A^T b with the
 *     preconditioner (R~^T R~)^{-1}, i.e. CGLS on A R~^{-1} (Bjorck,
 *     Numerical Methods for Least Squares Problems, 1996, ch. 7), started
 *     from x_0.  Each step costs what an SNE step costs (A p, A^T s, one
 *     solve with R~^T and one with R~) plus per-slice dot products; the
 *     residual s and x are FP64 and take the same step, so s = b - A x to FP64
 *     rounding.  Where kappa(A) u_factor is near or above 1 the stationary
 *     SNE step stops contracting, while the Krylov iteration still converges
 *     (the singular values of A R~^{-1} stay clustered near 1 but for a few).
 *     Needs the CSC copy and ct_refine_workspace_for's larger scratch. */
enum { CT_REFINE_QR = 0, CT_REFINE_SNE = 1, CT_REFINE_PCGLS = 2 };

/* Scratch bytes for ct_solve_refined with nrhs right-hand sides and method
 * CT_REFINE_QR or CT_REFINE_SNE. */
int ct_refine_workspace(int64_t m, int64_t n, int64_t nrhs, size_t* bytes);

/* Scratch bytes for ct_solve_refined with nrhs right-hand sides and the given
 * method (CT_REFINE_PCGLS adds n x nrhs FP64 for the search directions).
 * Returns -4 for an unknown method. */
int ct_refine_workspace_for(int64_t m, int64_t n, int64_t nrhs, int32_t method, size_t* bytes);

/* Reconstruction with iterative refinement on the FP64 residual r = b - A x:
 *   x_0 = R~^{-1} Q~^T b, then up to `steps` refinement steps of kind `method`.
 * B: m x nrhs FP64 (unchanged), X: n x nrhs FP64 (output).
 * Stop rule: with tol > 0, after each step the correction d of every slice is
 * compared with the updated image, and the refinement ends once
 * max_j ||d_j||_2 / ||x_j||_2 <= tol (each step contracts the error by
 * roughly kappa(A) u_factor, so the image error after that step is a small
 * fraction of tol).  Checking it waits for the stream once per step.
 * tol = 0 runs all `steps` without waiting.  steps_done (host, may be NULL)
 * receives the number of steps taken.  If not NULL, res_norms receives
 * ||r_s||_2 and grad_norms ||A^T r_s||_2 (the latter needs the CSC copy) for
 * s = 0..steps_done, (steps + 1) x nrhs, step-major; later rows are not
 * written.  With CT_REFINE_PCGLS the correction is the step c_j p_j and
 * res_norms rows 1..steps_done-1 hold the norms of the recurred residual
 * (equal to ||b - A x|| up to rounding); row steps_done is recomputed from b.
 * On a CT_PREC_BF16X3 factor the solves inside use BF16x3 products
 * from 48 slices up (see ct_debug_refine_x3); other factors use their
 * storage precision. */
int ct_solve_refined(const ct_factor* f, const ct_sparse* A, const double* B, int64_t ldb, double* X,
                     int64_t ldx, int64_t nrhs, int32_t steps, int32_t method, double tol, void* scratch,
                     size_t scratch_bytes, double* res_norms, double* grad_norms, int32_t* steps_done, void* stream);

/* ct_solve_refined without a scratch argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * ct_solve_refined, whose kernels it runs; its scratch is a statically
 * allocated 128 MiB device array, one per GPU, held until the process ends
 * (up to 40 slices at 256^2 with 76800 rays, 160 at 128^2 with 23040).
 * A call whose ct_refine_workspace_for size exceeds 128 MiB returns -7 (nrhs) and
 * launches nothing.  The call itself allocates nothing (no hipMalloc, no
 * library allocation).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams or host threads without
 * ordering) race on it and must be serialized by the caller. */
int ct_solve_refined_noalloc(const ct_factor* f, const ct_sparse* A, const double* B, int64_t ldb, double* X,
                             int64_t ldx, int64_t nrhs, int32_t steps, int32_t method, double tol,
                             double* res_norms, double* grad_norms, int32_t* steps_done, void* stream);

/* Waits for `stream`, then reports the factor's numerical status: *info = 0
 * for full column rank, j + 1 if column j had a zero Householder norm.
 * Returns -2001 if a cross-workgroup wait of the factorization timed out, and
 * -2003 (once; the flag is then cleared) if a graph-captured solve met an
 * invalid batch descriptor entry. */
int ct_status(const ct_factor* f, int64_t* info, void* stream);

int ct_factor_destroy(ct_factor* f);

/* Checkpoint of a factor held in device memory (the factor is reused for
 * every later batch of sinograms, Sec. 2): ct_factor_save waits for the
 * stream, then writes V\R (m x n, without the lda padding), tau, the
 * compact-WY factor T of every outer block and a 64-bit checksum to the host
 * file `path` (overwritten).  A factor whose factorization failed (ct_status
 * < 0) is not saved.  Returns -2 when the file cannot be written.
 * ct_factor_file_info reads a file's header: m, n, prec and the work bytes a
 * load with max_nrhs needs (any pointer may be NULL except path); -1 for a
 * file that is not a factor file.
 * ct_factor_load reads the file into the caller's A (lda >= m, a multiple of
 * 16), tau (n) and work (work_bytes from ct_factor_file_info), rebuilds the
 * solve-side copies, waits for the stream and returns a handle equivalent to
 * the saved one: the solves give bitwise the same results.  -1 for a
 * missing, truncated or corrupted file (checksum) or one saved on a device
 * with another panel width. */
int ct_factor_save(const ct_factor* f, const char* path, void* stream);
int ct_factor_file_info(const char* path, int64_t max_nrhs, int64_t* m, int64_t* n, int* prec, size_t* work_bytes);
int ct_factor_load(const char* path, void* A, int64_t lda, double* tau, void* work, size_t work_bytes,
                   int64_t max_nrhs, ct_factor** f, void* stream);

/* Graph-captured solve over a device batch descriptor, for many batches of
 * uneven size sharing one factor (Sec. 2: one factorization serves every
 * later set of sinograms; Eq. (solve) per batch).  desc is a device int32
 * array [cur, nbatch, off_0, cnt_0, off_1, cnt_1, ...]: cur is the index of
 * the batch the next launch solves, nbatch the number of batches, and batch k
 * occupies columns off_k .. off_k + cnt_k - 1 of B (m x b_cols, ldb, the
 * factor's storage type).  The whole solve (Q^T then R^{-1}) is captured once
 * into a hipGraph with the launch plan of the max_cols size bucket.  The
 * graph's first node checks the entry of batch cur (0 <= cur < nbatch,
 * off_k >= 0, 0 <= cnt_k <= max_cols, off_k + cnt_k <= b_cols); an invalid
 * entry, or a launch past the last batch, leaves B untouched and makes the
 * next ct_status return -2003.  The last node advances cur (never past
 * nbatch), so consecutive launches walk the batch list with no host work.
 * `stream` must not be the legacy default stream during creation (capture).
 * The caller sets desc before the first launch and keeps B, desc and the
 * factor alive until ct_solve_graph_destroy.  Graphs and solve calls sharing
 * a factor must be ordered on one stream (they share the factor's scratch). */
typedef struct ct_solve_graph ct_solve_graph;
int ct_solve_graph_create(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols, int32_t* desc,
                          void* stream, ct_solve_graph** g);
int ct_solve_graph_launch(ct_solve_graph* g, void* stream);
int ct_solve_graph_destroy(ct_solve_graph* g);

/* B[0:n] <- R^{-1} Q^T B (Eq. (solve)) in one persistent launch: one
 * workgroup per CU (a cooperative launch, refused rather than run with part
 * of the grid waiting), Sec. 2.1's ormqr and trsm in one kernel.  Per outer
 * reflector block, W = V^T B is summed over row ranges, W' = T^T W, and
 * B -= V W', with a grid-wide barrier between the phases; then the
 * back-substitution over R's 256-row blocks, whose results are published to
 * the other workgroups through flags as soon as every later block has been
 * applied.  A batch of at most 8 columns of an FP32-storage factor takes the
 * latency path: R_qq^{-1} folded into R (Rh = blockdiag(R_qq^{-1}) R), each
 * block split over four workgroups.  The first fused solve (or fused
 * graph) of an FP32-storage factor allocates and computes Rh (4 (n^2/2 -
 * 128 n) bytes for n a multiple of 256, about 8.6 GB at n = 65536; freed by
 * ct_factor_destroy; if the allocation fails the solves run without it,
 * slower), so that every later fused solve of the factor, eager or
 * captured, runs the same arithmetic.  Larger batches go 32 columns at a time (16 for an
 * FP64 factor), faster through ct_apply_qt + ct_trsm_solve above 8 columns.
 * Needs an in-memory factor with its solve-side copies (not
 * CT_QR_NO_SOLVE_COPIES, not streamed) and n <= 512 x CUs; otherwise returns
 * -2007.  Uses the factor's update buffer as scratch, so it is ordered with
 * the factor's other solves like them.  A cross-workgroup wait that times out
 * (0.5 s) makes the launch end early and the next ct_status return -2006.
 * B: m x nrhs (ldb), the factor's storage type, any nrhs >= 0. */
int ct_solve_fused(const ct_factor* f, void* B, int64_t nrhs, int64_t ldb, void* stream);

/* ct_solve_graph_create with the solve captured as the single launch of
 * ct_solve_fused (plus its reset node): the graph is the batch check, one
 * fused solve of the current batch and the advance of the cursor.  Same
 * arguments, descriptor rules and errors as ct_solve_graph_create, plus
 * ct_solve_fused's requirements on the factor; Rh (see ct_solve_fused) is
 * built before the capture. */
int ct_solve_graph_create_fused(const ct_factor* f, void* B, int64_t ldb, int64_t b_cols, int64_t max_cols,
                                int32_t* desc, void* stream, ct_solve_graph** g);

/* Autotuner of the solve kernels: for each batch-size bucket (<= 8, <= 32,
 * <= 128, <= 512 columns, up to max_nrhs) it times every candidate launch
 * plan -- tile width 16/32/64/128 along the slices and the split-K workgroup
 * target -- on a full Q^T + R^{-1} solve, and keeps the fastest in the factor
 * (used by ct_apply_qt, ct_trsm_solve, ct_solve_refined and graphs created
 * afterwards).  Results are merged into the JSON file cache_path (may be
 * NULL), keyed by architecture, storage type, m, n and bucket; cached buckets
 * are not re-timed.  B: scratch of at least m x max_nrhs (ldb), overwritten.
 * Synchronous. */
int ct_autotune_solve(ct_factor* f, void* B, int64_t ldb, int64_t max_nrhs, const char* cache_path, void* stream);

/* Live timing of the trailing-matrix update GEMMs of ct_qr_factor (the
 * dominant kernels): while enabled, every launch of the two update kernels
 * (W = V^T C, and C -= V W) is bracketed by HIP events on the stream it runs
 * on.  ct_profile_begin clears and enables; ct_profile_end waits for the
 * recorded events, disables, and returns per-kernel totals: launches, summed
 * event time (ms), algorithmic flops (2 M N K per launch) and algorithmic
 * bytes (operands read once, results written once).  Host-side state, one
 * process-wide recorder; not for concurrent factorizations. */
typedef struct ct_profile {
    int64_t launches[2];   /* [0]: W = V^T C kernel, [1]: C -= V W kernel */
    double ms[2];
    double flop[2];
    double bytes[2];
} ct_profile;
int ct_profile_begin(void);
int ct_profile_end(ct_profile* out);

const char* ct_last_error(void);

/* Image quality of k reconstructed slices against reference images
 * (Sec. 3.1, Eqs. (snr), (mse), (psnr), (ssim)), FP64 on the device.  X and
 * ref: slice s at X + s * ldx (ref + s * ldr), n_pix^2 pixels each, pixel
 * (ix, iy) at iy * n_pix + ix (iy = 0 the bottom row).  crop_host: NULL, or
 * 4 host margins in pixels (bottom, top, left, right) that leave at least
 * window x window pixels (the paper's cropped variant drops the image's
 * edges).  out (device, k x 4): SNR (dB); MSE; PSNR (dB, MAX = the largest
 * reference pixel of the crop); SSIM, the mean over every window x window
 * window of the crop with window means, sample (co)variances (divisor
 * window^2 - 1), c1 = (0.01 L)^2 and c2 = (0.03 L)^2, L the reference's
 * max - min over the crop.  An exact reconstruction gives SNR = PSNR = inf.
 * k = 0 does nothing (the pointers may then be NULL).  Bad arguments return
 * their 1-based position (negated) and launch nothing. */
int ct_quality(const double* X, int64_t ldx, const double* ref, int64_t ldr, int32_t n_pix, int64_t k,
               const int32_t* crop_host, int32_t window, double* out, void* stream);

/* Rows of A for explicit rays (host arrays): rays_host r x 4 (x0, y0, x1, y1)
 * row-major, rows_host r x n_pix^2 row-major.  Synchronous; computed on the
 * GPU with the same Siddon walk as ct_build_system. */
int ct_siddon_rows(const double* rays_host, int64_t r, int32_t n_pix, double grid_width, double* rows_host);

#ifdef __cplusplus
}
#endif
#endif /* CTQR_H */
