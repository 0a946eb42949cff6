"""Python binding of libctqr (include/ctqr.h): argument marshalling only.

Every computation happens in the HIP library; torch provides device memory
and streams.  Importing this module loads ``libctqr.so`` from the package
directory and raises ImportError if it has not been built
(``python -m paper_2412_07631_amd.build``) -- there is no fallback.

Matrix convention: a column-major matrix with leading dimension ``ld`` and
``cols`` columns is a contiguous torch tensor of shape ``(cols, ld)`` (row c
of the tensor is column c of the matrix).  ``colmajor(rows, cols, dtype)``
allocates one with ``ld`` rounded up to a multiple of 16.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctqr.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libctqr.so is not built (run: python -m paper_2412_07631_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)

F64, F32 = 0, 1
QR_NO_SOLVE_COPIES = 0x100    # flag OR'ed into prec: no solve-side copies (lean workspace)
REFINE_QR, REFINE_SNE, REFINE_PCGLS = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16, PREC_F16, PREC_BF16X3 = 0, 1, 2, 3, 4
PREC_NAMES = {"f64": PREC_F64, "f32": PREC_F32, "bf16": PREC_BF16, "f16": PREC_F16, "bf16x3": PREC_BF16X3}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


class Geometry(ctypes.Structure):
    _fields_ = [("n_pix", _i32), ("n_angles", _i32), ("n_det", _i32), ("projector", _i32),
                ("grid_width", ctypes.c_double), ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
                ("det_length", ctypes.c_double), ("angle0", ctypes.c_double)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("ct_build_system", [ctypes.POINTER(Geometry), ctypes.c_int, _vp, _i64, _vp])
_sig("ct_build_csr", [ctypes.POINTER(Geometry), _vp, _vp, _vp, _i64, _vp])
_sig("ct_qr_workspace", [_i64, _i64, ctypes.c_int, _i64, ctypes.POINTER(_sz)])
_sig("ct_qr_factor", [_vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp, _sz, _i64, ctypes.POINTER(_vp), _vp])
_sig("ct_qr_stream_workspace", [_i64, _i64, _i64, ctypes.c_int, _i64, _i64, ctypes.POINTER(_sz), ctypes.POINTER(_sz)])
_sig("ct_qr_factor_streamed", [_vp, _i64, _i64, _i64, ctypes.c_int, _vp, _vp, _sz, _i64, _i64, ctypes.POINTER(_vp),
                               _vp])
_sig("ct_qr_resume", [_vp, _vp])
_sig("ct_stream_info", [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("ct_stream_inject_failure", [_i64, _i64])
_sig("ct_debug_wait_limit", [_i64])
_sig("ct_debug_panel_cholesky", [ctypes.c_int])
_sig("ct_debug_block_width", [ctypes.c_int])
_sig("ct_debug_refine_x3", [ctypes.c_int])
_sig("ct_debug_progress", [_i64])
_sig("ct_debug_panel_width", [ctypes.c_int])
_sig("ct_quality", [_vp, _i64, _vp, _i64, _i32, _i64, _vp, _i32, _vp, _vp])
_sig("ct_factor_save", [_vp, ctypes.c_char_p, _vp])
_sig("ct_factor_file_info", [ctypes.c_char_p, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_sz)])
_sig("ct_factor_load", [ctypes.c_char_p, _vp, _i64, _vp, _vp, _sz, _i64, ctypes.POINTER(_vp), _vp])
_sig("ct_apply_qt", [_vp, _vp, _i64, _i64, _vp])
_sig("ct_trsm_solve", [_vp, _vp, _i64, _i64, _vp])
_sig("ct_solve_backward", [_vp, _vp, _i64, _i64, _vp, _i64, _vp])
_sig("ct_residual", [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _i64, _vp])
_sig("ct_refine_workspace", [_i64, _i64, _i64, ctypes.POINTER(_sz)])
_sig("ct_refine_workspace_for", [_i64, _i64, _i64, _i32, ctypes.POINTER(_sz)])
_sig("ct_build_csc", [_i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("ct_group_sparse", [_i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, ctypes.POINTER(_i64), _vp, _vp])


class Sparse(ctypes.Structure):
    _fields_ = [("m", _i64), ("n", _i64), ("nnz", _i64), ("row_ptr", _vp), ("col", _vp), ("val", _vp),
                ("col_ptr", _vp), ("row", _vp), ("cval", _vp), ("group_r", _i32), ("group_c", _i32),
                ("grow_ptr", _vp), ("grow_col", _vp), ("grow_val", _vp),
                ("gcol_ptr", _vp), ("gcol_row", _vp), ("gcol_val", _vp)]


_sig("ct_solve_refined", [_vp, ctypes.POINTER(Sparse), _vp, _i64, _vp, _i64, _i64, _i32, _i32, ctypes.c_double,
                          _vp, _sz, _vp, _vp, ctypes.POINTER(_i32), _vp])
_sig("ct_solve_refined_noalloc", [_vp, ctypes.POINTER(Sparse), _vp, _i64, _vp, _i64, _i64, _i32, _i32,
                                  ctypes.c_double, _vp, _vp, ctypes.POINTER(_i32), _vp])


class Profile(ctypes.Structure):
    _fields_ = [("launches", _i64 * 2), ("ms", ctypes.c_double * 2), ("flop", ctypes.c_double * 2),
                ("bytes", ctypes.c_double * 2)]


_sig("ct_profile_begin", [])
_sig("ct_profile_end", [ctypes.POINTER(Profile)])
_sig("ct_status", [_vp, ctypes.POINTER(_i64), _vp])
_sig("ct_solve_graph_create", [_vp, _vp, _i64, _i64, _i64, _vp, _vp, ctypes.POINTER(_vp)])
_sig("ct_solve_graph_create_fused", [_vp, _vp, _i64, _i64, _i64, _vp, _vp, ctypes.POINTER(_vp)])
_sig("ct_solve_fused", [_vp, _vp, _i64, _i64, _vp])
_sig("ct_solve_graph_launch", [_vp, _vp])
_sig("ct_solve_graph_destroy", [_vp])
_sig("ct_autotune_solve", [_vp, _vp, _i64, _i64, ctypes.c_char_p, _vp])
_sig("ct_factor_destroy", [_vp])
_sig("ct_last_error", [], ctypes.c_char_p)
_sig("ct_siddon_rows", [_vp, _i64, _i32, ctypes.c_double, _vp])


class CtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ctqr error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != 0:
        raise CtError(rc, (_lib.ct_last_error() or b"").decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def ld16(rows: int) -> int:
    return (int(rows) + 15) // 16 * 16


def colmajor(rows: int, cols: int, dtype, device="cuda", zero=False):
    """Column-major (rows x cols) matrix as a (cols, ld) tensor."""
    shape = (int(cols), ld16(rows))
    return torch.zeros(shape, dtype=dtype, device=device) if zero else torch.empty(shape, dtype=dtype, device=device)


def geometry(s) -> Geometry:
    """Geometry from any object with the ct_geometry fields (e.g. synth.Scanner)."""
    return Geometry(int(s.n_pix), int(s.n_angles), int(s.n_det), int(getattr(s, "projector", 0)),
                    float(s.grid_width), float(s.sid),
                    float(s.sdd), float(s.det_length), float(s.angle0))


# -------------------------------------------------------------------- calls
def build_system(geom, A: torch.Tensor, stream=None):
    """A: (n, lda) tensor, float64 or float32; filled with the system matrix."""
    g = geometry(geom)
    dt = F64 if A.dtype == torch.float64 else F32
    _check(_lib.ct_build_system(ctypes.byref(g), dt, _ptr(A), A.shape[1], _stream(stream)))
    return A


def build_csr(geom, device="cuda", stream=None):
    """(row_ptr int64[m+1], col int32[nnz], val float64[nnz]) on the device."""
    g = geometry(geom)
    m = int(geom.n_angles) * int(geom.n_det)
    row_ptr = torch.empty(m + 1, dtype=torch.int64, device=device)
    _check(_lib.ct_build_csr(ctypes.byref(g), _ptr(row_ptr), None, None, 0, _stream(stream)))
    nnz = int(row_ptr[m].item())
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=device)
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=device)
    _check(_lib.ct_build_csr(ctypes.byref(g), _ptr(row_ptr), _ptr(col), _ptr(val), nnz, _stream(stream)))
    return row_ptr, col[:nnz], val[:nnz]


def qr_workspace(m: int, n: int, prec: int, max_nrhs: int) -> int:
    b = _sz(0)
    _check(_lib.ct_qr_workspace(m, n, prec, max_nrhs, ctypes.byref(b)))
    return b.value


class Factor:
    """Host handle of a factorization; keeps the device buffers it borrows alive."""

    def __init__(self, handle, A, tau, work, m, n, prec, max_nrhs):
        self.handle, self.A, self.tau, self.work = handle, A, tau, work
        self.m, self.n, self.prec, self.max_nrhs = m, n, prec, max_nrhs
        self.dtype = torch.float64 if prec == PREC_F64 else torch.float32

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            _lib.ct_factor_destroy(h)
            self.handle = None


def qr_factor(A: torch.Tensor, m: int, n: int, prec: int, max_nrhs: int = 512, stream=None,
              solve_copies: bool = True) -> Factor:
    """Factor A (an (n, lda) tensor holding the m x n matrix) in place
    (solve_copies=False: the lean workspace of CT_QR_NO_SOLVE_COPIES)."""
    want = torch.float64 if prec == PREC_F64 else torch.float32
    if A.dtype != want:
        raise TypeError("A must be %s for this precision" % want)
    p = prec if solve_copies else prec | QR_NO_SOLVE_COPIES
    tau = torch.zeros(n, dtype=torch.float64, device=A.device)
    work = torch.empty(qr_workspace(m, n, p, max_nrhs), dtype=torch.uint8, device=A.device)
    h = _vp()
    _check(_lib.ct_qr_factor(_ptr(A), m, n, A.shape[1], p, _ptr(tau), _ptr(work), work.numel(), max_nrhs,
                             ctypes.byref(h), _stream(stream)))
    return Factor(h, A, tau, work, m, n, prec, max_nrhs)


def factor_save(f: Factor, path: str, stream=None):
    """Write the factor (V\\R, tau, T, checksum) to a host file."""
    _check(_lib.ct_factor_save(f.handle, os.fsencode(path), _stream(stream)))


def factor_file_info(path: str, max_nrhs: int = 512):
    """(m, n, prec, work bytes for max_nrhs) of a saved factor."""
    m, n, p, b = _i64(0), _i64(0), ctypes.c_int(0), _sz(0)
    _check(_lib.ct_factor_file_info(os.fsencode(path), max_nrhs, ctypes.byref(m), ctypes.byref(n), ctypes.byref(p),
                                    ctypes.byref(b)))
    return m.value, n.value, p.value, b.value


def factor_load(path: str, max_nrhs: int = 512, device="cuda", stream=None) -> Factor:
    """Load a saved factor into new device buffers."""
    m, n, prec, wb = factor_file_info(path, max_nrhs)
    dt = torch.float64 if prec == PREC_F64 else torch.float32
    A = torch.empty((n, ld16(m)), dtype=dt, device=device)
    tau = torch.zeros(n, dtype=torch.float64, device=device)
    work = torch.empty(wb, dtype=torch.uint8, device=device)
    h = _vp()
    _check(_lib.ct_factor_load(os.fsencode(path), _ptr(A), A.shape[1], _ptr(tau), _ptr(work), work.numel(),
                               max_nrhs, ctypes.byref(h), _stream(stream)))
    return Factor(h, A, tau, work, m, n, prec, max_nrhs)


def qr_stream_workspace(m: int, n: int, lda: int, prec: int, max_nrhs: int, tile_cols: int):
    """(minimum, all-tiles-resident) device bytes of a streamed factorization."""
    a, b = _sz(0), _sz(0)
    _check(_lib.ct_qr_stream_workspace(m, n, lda, prec, max_nrhs, tile_cols, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def qr_factor_streamed(A_host: torch.Tensor, m: int, n: int, prec: int, tile_cols: int = 1024,
                       device_bytes: int = None, max_nrhs: int = 512, device="cuda", stream=None) -> Factor:
    """Out-of-core factorization of a pinned host matrix (an (n, lda) tensor
    holding the m x n matrix), in place.  device_bytes caps the device buffer
    (default: enough to keep every tile resident).  A copy failure injected
    with inject_failure() raises CtError(-2002) carrying the resumable factor
    as its .factor attribute."""
    want = torch.float64 if prec == PREC_F64 else torch.float32
    if A_host.dtype != want or A_host.device.type != "cpu" or not A_host.is_pinned():
        raise TypeError("A_host must be a pinned CPU tensor of %s" % want)
    lda = A_host.shape[1]
    lo, full = qr_stream_workspace(m, n, lda, prec, max_nrhs, tile_cols)
    nbytes = full if device_bytes is None else max(lo, min(full, int(device_bytes)))
    tau = torch.zeros(n, dtype=torch.float64, device=device)
    work = torch.empty(nbytes, dtype=torch.uint8, device=device)
    h = _vp()
    rc = _lib.ct_qr_factor_streamed(_ptr(A_host), m, n, lda, prec, _ptr(tau), _ptr(work), work.numel(), max_nrhs,
                                    tile_cols, ctypes.byref(h), _stream(stream))
    f = Factor(h, A_host, tau, work, m, n, prec, max_nrhs) if h.value else None
    if rc != 0:
        err = CtError(rc, (_lib.ct_last_error() or b"").decode())
        err.factor = f
        raise err
    return f


def qr_resume(f: Factor, stream=None):
    _check(_lib.ct_qr_resume(f.handle, _stream(stream)))
    return f


def stream_info(f: Factor):
    """(tiles, resident tiles, first unfinished tile) of a streamed factor."""
    a, b, c = _i64(0), _i64(0), _i64(0)
    _check(_lib.ct_stream_info(f.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def inject_failure(tile: int, after_updates: int = -1):
    """Make the next streamed factorization stop at `tile` as if a copy had
    failed: before the tile's work (after_updates < 0) or after the reflector
    blocks of that many earlier tiles have been applied to it."""
    _check(_lib.ct_stream_inject_failure(tile, after_updates))


def debug_wait_limit(ticks: int):
    """Time limit (100 MHz ticks) of one cross-workgroup wait of the panels;
    negative restores the default."""
    _check(_lib.ct_debug_wait_limit(ticks))


def debug_panel_cholesky(enable: bool):
    """Allow (default) or forbid the two-reduction panel form for later
    factorizations; forbidden, every panel takes one reduction per column."""
    _check(_lib.ct_debug_panel_cholesky(1 if enable else 0))


def debug_block_width(nb_out: int):
    """Force the outer block width of later factorizations (0 restores the
    size-based default)."""
    _check(_lib.ct_debug_block_width(nb_out))


def debug_panel_width(nbi: int):
    """Force the panel width (16 or 32; 0: by the matrix's height)."""
    _check(_lib.ct_debug_panel_width(int(nbi)))


def debug_progress(blocks: int):
    """Progress lines on stderr every `blocks` outer blocks of a factorization (0: off)."""
    _check(_lib.ct_debug_progress(int(blocks)))


def debug_refine_x3(mode: int) -> int:
    """BF16x3 products in the refinement of a BF16x3 factor: 0 never, 1 from
    48 slices (default), 2 always; returns the previous mode."""
    r = _lib.ct_debug_refine_x3(int(mode))
    if r < 0:
        _check(r)
    return r


def quality(X: torch.Tensor, ref: torch.Tensor, n_pix: int, crop=None, window: int = 7, stream=None) -> torch.Tensor:
    """(k, 4) FP64 tensor of SNR (dB), MSE, PSNR (dB), SSIM of the k slices
    (rows) of X against those of ref; crop = (bottom, top, left, right)."""
    if X.dtype != torch.float64 or ref.dtype != torch.float64:
        raise TypeError("X and ref must be float64")
    k = X.shape[0]
    out = torch.empty((max(k, 1), 4), dtype=torch.float64, device=X.device)
    c = None
    if crop is not None:
        c = (ctypes.c_int32 * 4)(*[int(v) for v in crop])
    _check(_lib.ct_quality(_ptr(X), X.shape[1], _ptr(ref), ref.shape[1], n_pix, k, c, window, _ptr(out),
                           _stream(stream)))
    return out[:k]


def apply_qt(f: Factor, B: torch.Tensor, nrhs: int = None, stream=None):
    nrhs = B.shape[0] if nrhs is None else nrhs
    _check(_lib.ct_apply_qt(f.handle, _ptr(B), nrhs, B.shape[1], _stream(stream)))
    return B


def solve_fused(f: Factor, B: torch.Tensor, nrhs: int = None, stream=None):
    """B[:, :n] <- R^{-1} Q^T B in one persistent launch (ct_solve_fused)."""
    nrhs = B.shape[0] if nrhs is None else nrhs
    _check(_lib.ct_solve_fused(f.handle, _ptr(B), nrhs, B.shape[1], _stream(stream)))
    return B


def trsm_solve(f: Factor, B: torch.Tensor, nrhs: int = None, stream=None):
    nrhs = B.shape[0] if nrhs is None else nrhs
    _check(_lib.ct_trsm_solve(f.handle, _ptr(B), nrhs, B.shape[1], _stream(stream)))
    return B


def solve_backward(f: Factor, G: torch.Tensor, gradB: torch.Tensor, k: int = None, stream=None):
    k = G.shape[0] if k is None else k
    _check(_lib.ct_solve_backward(f.handle, _ptr(G), k, G.shape[1], _ptr(gradB), gradB.shape[1], _stream(stream)))
    return gradB


def residual(csr, m: int, X: torch.Tensor, B: torch.Tensor, R: torch.Tensor, nrhs: int = None, stream=None):
    row_ptr, col, val = csr
    nrhs = X.shape[0] if nrhs is None else nrhs
    _check(_lib.ct_residual(_ptr(row_ptr), _ptr(col), _ptr(val), m, _ptr(X), X.shape[1], _ptr(B), B.shape[1],
                            _ptr(R), R.shape[1], nrhs, _stream(stream)))
    return R


def refine_workspace(m: int, n: int, nrhs: int, method: int = REFINE_SNE) -> int:
    b = _sz(0)
    _check(_lib.ct_refine_workspace_for(m, n, nrhs, int(method), ctypes.byref(b)))
    return b.value


def group_sparse(rows: int, ptr, idx, val, group: int = 8, device="cuda", stream=None):
    """Grouped copy (ct_group_sparse) of a CSR-like matrix; the group shrinks
    (8, 4, 2, 1) while a group holds more entries than the builder takes."""
    work = torch.zeros(1, dtype=torch.int32, device=device)
    g = group
    while True:
        ng = (rows + g - 1) // g
        gptr = torch.empty(ng + 1, dtype=torch.int64, device=device)
        cnt = _i64(0)
        rc = _lib.ct_group_sparse(rows, _ptr(ptr), _ptr(idx), _ptr(val), g, _ptr(gptr), None, None,
                                  ctypes.byref(cnt), _ptr(work), _stream(stream))
        if rc == -2005 and g > 1:
            g //= 2
            continue
        _check(rc)
        break
    gidx = torch.empty(max(cnt.value, 1), dtype=torch.int32, device=device)
    gval = torch.empty(max(cnt.value, 1) * g, dtype=torch.float64, device=device)
    _check(_lib.ct_group_sparse(rows, _ptr(ptr), _ptr(idx), _ptr(val), g, _ptr(gptr), _ptr(gidx), _ptr(gval),
                                ctypes.byref(cnt), _ptr(work), _stream(stream)))
    return g, gptr, gidx, gval


class SparseA:
    """FP64 CSR and CSC copies of A on the device (kept alive with the struct),
    and their grouped copies for the refinement's products (group 0: none)."""

    def __init__(self, geom, device="cuda", stream=None, group: int = 8):
        self.m = int(geom.n_angles) * int(geom.n_det)
        self.n = int(geom.n_pix) ** 2
        self.row_ptr, self.col, self.val = build_csr(geom, device, stream)
        self.nnz = int(self.val.numel())
        self.col_ptr = torch.empty(self.n + 1, dtype=torch.int64, device=device)
        self.row = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=device)
        self.cval = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=device)
        work = torch.empty(self.n, dtype=torch.int32, device=device)
        _check(_lib.ct_build_csc(self.m, self.n, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val),
                                 _ptr(self.col_ptr), _ptr(self.row), _ptr(self.cval), _ptr(work), _stream(stream)))
        self.group_r = self.group_c = 0
        self.grouped_r = self.grouped_c = (None, None, None)
        if group:
            self.group_r, *self.grouped_r = group_sparse(self.m, self.row_ptr, self.col, self.val, group, device,
                                                         stream)
            self.group_c, *self.grouped_c = group_sparse(self.n, self.col_ptr, self.row, self.cval, group, device,
                                                         stream)
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        p = lambda t: None if t is None else t.data_ptr()
        self.struct = Sparse(self.m, self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                             self.val.data_ptr(), self.col_ptr.data_ptr(), self.row.data_ptr(), self.cval.data_ptr(),
                             self.group_r, self.group_c, *[p(t) for t in self.grouped_r],
                             *[p(t) for t in self.grouped_c])

    @property
    def csr(self):
        return self.row_ptr, self.col, self.val


def solve_refined(f: Factor, sp: SparseA, B: torch.Tensor, X: torch.Tensor, steps: int, method: int = REFINE_SNE,
                  nrhs: int = None, scratch: torch.Tensor = None, res_norms: torch.Tensor = None,
                  grad_norms: torch.Tensor = None, stream=None, tol: float = 0.0) -> int:
    """X (FP64) <- refined least-squares solution for the FP64 sinograms B;
    returns the number of refinement steps taken (all `steps` unless tol > 0
    stops earlier)."""
    nrhs = B.shape[0] if nrhs is None else nrhs
    if scratch is None:
        scratch = torch.empty(refine_workspace(f.m, f.n, nrhs, method), dtype=torch.uint8, device=B.device)
    done = _i32(0)
    _check(_lib.ct_solve_refined(f.handle, ctypes.byref(sp.struct), _ptr(B), B.shape[1], _ptr(X), X.shape[1], nrhs,
                                 int(steps), int(method), float(tol), _ptr(scratch), scratch.numel(), _ptr(res_norms),
                                 _ptr(grad_norms), ctypes.byref(done), _stream(stream)))
    return done.value


def solve_refined_noalloc(f: Factor, sp: SparseA, B: torch.Tensor, X: torch.Tensor, steps: int,
                          method: int = REFINE_SNE, nrhs: int = None, res_norms: torch.Tensor = None,
                          grad_norms: torch.Tensor = None, stream=None, tol: float = 0.0) -> int:
    """solve_refined with the library's static scratch (allocates nothing)."""
    nrhs = B.shape[0] if nrhs is None else nrhs
    done = _i32(0)
    _check(_lib.ct_solve_refined_noalloc(f.handle, ctypes.byref(sp.struct), _ptr(B), B.shape[1], _ptr(X), X.shape[1],
                                         nrhs, int(steps), int(method), float(tol), _ptr(res_norms),
                                         _ptr(grad_norms), ctypes.byref(done), _stream(stream)))
    return done.value


def batch_descriptor(sizes, device="cuda"):
    """Device descriptor for a list of batch sizes laid out back to back:
    [current batch, batch count, offset_0, count_0, offset_1, count_1, ...]
    (int32)."""
    d = [0, len(sizes)]
    off = 0
    for c in sizes:
        d += [off, int(c)]
        off += int(c)
    return torch.tensor(d, dtype=torch.int32, device=device)


class SolveGraph:
    """A captured solve (Q^T then R^{-1}) over the batch descriptor `desc` of
    columns inside B; each launch solves the current batch and advances it."""

    def __init__(self, f: Factor, B: torch.Tensor, max_cols: int, desc: torch.Tensor, stream=None,
                 fused: bool = False):
        self.f, self.B, self.desc = f, B, desc
        st = stream if stream is not None else torch.cuda.Stream()
        self.stream = st
        h = _vp()
        create = _lib.ct_solve_graph_create_fused if fused else _lib.ct_solve_graph_create
        with torch.cuda.stream(st):
            _check(create(f.handle, _ptr(B), B.shape[1], B.shape[0], int(max_cols), _ptr(desc),
                          _vp(st.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(_lib.ct_solve_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            _lib.ct_solve_graph_destroy(h)
            self.handle = None


def autotune_solve(f: Factor, B: torch.Tensor, max_nrhs: int, cache_path: str = None, stream=None):
    """Time the candidate launch plans of the solve kernels per batch bucket and
    keep the fastest in the factor (B is scratch, overwritten)."""
    _check(_lib.ct_autotune_solve(f.handle, _ptr(B), B.shape[1], int(max_nrhs),
                                  cache_path.encode() if cache_path else None, _stream(stream)))


def profile_begin():
    _check(_lib.ct_profile_begin())


def profile_end() -> dict:
    """Event-timed totals of the trailing-update kernels since profile_begin."""
    p = Profile()
    _check(_lib.ct_profile_end(ctypes.byref(p)))
    names = ("update_vtc", "update_cvw")
    return {names[k]: {"launches": int(p.launches[k]), "ms": float(p.ms[k]), "flop": float(p.flop[k]),
                       "bytes": float(p.bytes[k])} for k in range(2)}


def status(f: Factor, stream=None) -> int:
    info = _i64(0)
    _check(_lib.ct_status(f.handle, ctypes.byref(info), _stream(stream)))
    return info.value


def siddon_rows(rays, n_pix: int, grid_width: float = 1.0):
    """Host numpy in/out: dense rows (r x n_pix^2) for r x 4 ray end points."""
    import numpy as np
    r = np.ascontiguousarray(np.asarray(rays, dtype=np.float64).reshape(-1, 4))
    out = np.empty((r.shape[0], int(n_pix) ** 2), dtype=np.float64)
    _check(_lib.ct_siddon_rows(r.ctypes.data_as(_vp), r.shape[0], int(n_pix), float(grid_width),
                               out.ctypes.data_as(_vp)))
    return out


# ------------------------------------------------------------ differentiation
class QRSolve(torch.autograd.Function):
    """x = R^{-1} Q^T b for a batch of sinograms, differentiable in b.

    forward(B, factor): B is (nrhs, m) -- one sinogram per row -- in the
    factor's storage dtype; returns X (nrhs, n).  backward(G) returns
    grad_B = (Q [R^{-T} g; 0])^T per row, computed by ct_solve_backward; the
    factor receives no gradient.
    """

    @staticmethod
    def forward(ctx, B, factor):
        m, n = factor.m, factor.n
        nrhs = B.shape[0]
        C = torch.zeros((nrhs, ld16(m)), dtype=factor.dtype, device=B.device)
        C[:, :m] = B
        apply_qt(factor, C)
        trsm_solve(factor, C)
        ctx.factor = factor
        return C[:, :n].clone()

    @staticmethod
    def backward(ctx, G):
        f = ctx.factor
        k = G.shape[0]
        Gd = torch.zeros((k, ld16(f.n)), dtype=f.dtype, device=G.device)
        Gd[:, :f.n] = G
        Y = torch.empty((k, ld16(f.m)), dtype=f.dtype, device=G.device)
        solve_backward(f, Gd, Y)
        return Y[:, :f.m].clone(), None


def qr_solve(B, factor):
    """Differentiable reconstruction X = R^{-1} Q^T B (rows of B are sinograms)."""
    return QRSolve.apply(B, factor)
