"""Python face of the FP64 CPU oracle (ctqr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg, never by the product path.  It
does not import the HIP package either; both sides meet only in the seeded
input generators (``paper_2412_07631_amd.synth``, which holds no method
arithmetic).

Functions and the passages they follow:
  rays / system_dense / system_csr / siddon_rows -- the weights matrix A of
      Eq. (system): a_ij = length of ray i inside pixel j (Siddon's exact
      intersection lengths; the fan-beam scan of Table 1); with a scanner's
      projector = 1, system_dense / system_csr use joseph_ray / joseph_rows,
      Joseph's interpolating projector (the one Sec. 3.1 builds A with).
  householder_qr -- Eq. (qr), unblocked Householder with the LAPACK sign rule.
  apply_qt / back_substitute / solve -- Eq. (solve): C = Q^T B, X = R^{-1} C.
  apply_q / forward_substitute_rt / adjoint -- the transpose of the solve map,
      grad_b = Q [R^{-T} g; 0].
  rank_report -- the full-column-rank condition of Sec. 3.1.
  snr / mse / psnr / ssim -- the image-quality metrics of Sec. 3.1,
      Eqs. (snr), (mse), (psnr), (ssim), with an optional crop.

Every function here has a pin in tests/test_oracle_*.py (values fixed by the
paper, closed forms, brute force at tiny sizes, exact rational arithmetic or
library special cases); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctqr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Geom(ctypes.Structure):
    _fields_ = [("n_pix", _i32), ("n_angles", _i32), ("n_det", _i32), ("projector", _i32),
                ("grid_width", ctypes.c_double), ("sid", ctypes.c_double),
                ("sdd", ctypes.c_double), ("det_length", ctypes.c_double),
                ("angle0", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.orc_ray_endpoints.argtypes = [ctypes.POINTER(_Geom), _dp]
            lib.orc_siddon_ray.argtypes = [ctypes.c_double] * 4 + [_i32, ctypes.c_double, _i32p, _dp, _dp]
            lib.orc_siddon_ray.restype = _i64
            lib.orc_siddon_rows.argtypes = [_dp, _i64, _i32, ctypes.c_double, _dp]
            lib.orc_joseph_ray.argtypes = [ctypes.c_double] * 4 + [_i32, ctypes.c_double, _i32p, _dp]
            lib.orc_joseph_ray.restype = _i64
            lib.orc_joseph_rows.argtypes = [_dp, _i64, _i32, ctypes.c_double, _dp]
            lib.orc_system_dense.argtypes = [ctypes.POINTER(_Geom), _dp, _i64]
            lib.orc_system_csr.argtypes = [ctypes.POINTER(_Geom), _i64p, _i32p, _dp, _i64]
            lib.orc_system_csr.restype = _i64
            lib.orc_householder_qr.argtypes = [_i64, _i64, _dp, _i64, _dp]
            lib.orc_householder_qr.restype = _i64
            for name in ("orc_apply_qt", "orc_apply_q"):
                getattr(lib, name).argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _i64, _i64]
            for name in ("orc_back_substitute", "orc_forward_substitute_rt"):
                getattr(lib, name).argtypes = [_i64, _dp, _i64, _dp, _i64, _i64]
                getattr(lib, name).restype = _i64
            lib.orc_csr_matvec.argtypes = [_i64, _i64p, _i32p, _dp, _dp, _dp]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _geom(s) -> _Geom:
    return _Geom(int(s.n_pix), int(s.n_angles), int(s.n_det), int(getattr(s, "projector", 0)),
                 float(s.grid_width), float(s.sid), float(s.sdd), float(s.det_length), float(s.angle0))


def _f64_colmajor(a) -> np.ndarray:
    return np.require(np.asarray(a, dtype=np.float64), requirements=["F", "A", "W", "O"])


# ----------------------------------------------------------------- geometry
def rays(scanner) -> np.ndarray:
    """m x 4 ray end points (source x, y; bin-centre x, y), rows i = k*n_det + d."""
    lib = _load()
    m = int(scanner.n_angles) * int(scanner.n_det)
    out = np.empty((m, 4), dtype=np.float64)
    g = _geom(scanner)
    lib.orc_ray_endpoints(ctypes.byref(g), _ptr(out))
    return out


def siddon_ray(x0, y0, x1, y1, n_pix: int, grid_width: float = 1.0):
    """(pixel indices, lengths) of one ray, in order along the ray."""
    lib = _load()
    cap = 2 * n_pix + 8
    pix = np.empty(cap, dtype=np.int32)
    ln = np.empty(cap, dtype=np.float64)
    work = np.empty(cap, dtype=np.float64)
    c = lib.orc_siddon_ray(float(x0), float(y0), float(x1), float(y1), int(n_pix),
                           float(grid_width), _ptr(pix, _i32p), _ptr(ln), _ptr(work))
    return pix[:c].copy(), ln[:c].copy()


def siddon_rows(ray_list, n_pix: int, grid_width: float = 1.0) -> np.ndarray:
    """Dense rows (r x N^2) of A for explicit rays given as r x 4 end points."""
    lib = _load()
    r = np.ascontiguousarray(np.asarray(ray_list, dtype=np.float64).reshape(-1, 4))
    out = np.empty((r.shape[0], n_pix * n_pix), dtype=np.float64)
    lib.orc_siddon_rows(_ptr(r), r.shape[0], int(n_pix), float(grid_width), _ptr(out))
    return out


def joseph_ray(x0, y0, x1, y1, n_pix: int, grid_width: float = 1.0):
    """(pixel indices, weights) of one ray under Joseph's projector."""
    lib = _load()
    cap = 2 * n_pix + 8
    pix = np.empty(cap, dtype=np.int32)
    wt = np.empty(cap, dtype=np.float64)
    c = lib.orc_joseph_ray(float(x0), float(y0), float(x1), float(y1), int(n_pix), float(grid_width),
                           _ptr(pix, _i32p), _ptr(wt))
    return pix[:c].copy(), wt[:c].copy()


def joseph_rows(ray_list, n_pix: int, grid_width: float = 1.0) -> np.ndarray:
    """Dense rows (r x N^2) of Joseph's A for explicit rays (r x 4 end points)."""
    lib = _load()
    r = np.ascontiguousarray(np.asarray(ray_list, dtype=np.float64).reshape(-1, 4))
    out = np.empty((r.shape[0], n_pix * n_pix), dtype=np.float64)
    lib.orc_joseph_rows(_ptr(r), r.shape[0], int(n_pix), float(grid_width), _ptr(out))
    return out


def system_dense(scanner) -> np.ndarray:
    """Dense FP64 A (m x n, Fortran order)."""
    lib = _load()
    m, n = scanner.m, scanner.n
    A = np.empty((m, n), dtype=np.float64, order="F")
    g = _geom(scanner)
    lib.orc_system_dense(ctypes.byref(g), _ptr(A), m)
    return A


def system_csr(scanner):
    """(row_ptr int64[m+1], col int32[nnz], val float64[nnz]) of A."""
    lib = _load()
    m = scanner.m
    cap = m * (2 * scanner.n_pix + 2)
    row_ptr = np.empty(m + 1, dtype=np.int64)
    col = np.empty(cap, dtype=np.int32)
    val = np.empty(cap, dtype=np.float64)
    g = _geom(scanner)
    nnz = lib.orc_system_csr(ctypes.byref(g), _ptr(row_ptr, _i64p), _ptr(col, _i32p), _ptr(val), cap)
    if nnz < 0:
        raise RuntimeError("CSR capacity exceeded")
    return row_ptr, col[:nnz].copy(), val[:nnz].copy()


def csr_matvec(csr, x) -> np.ndarray:
    """A x in FP64 from the CSR copy; x may be n or n x k."""
    lib = _load()
    row_ptr, col, val = csr
    m = row_ptr.shape[0] - 1
    X = np.asarray(x, dtype=np.float64)
    vec = X.ndim == 1
    X = X.reshape(X.shape[0], -1)
    Y = np.empty((m, X.shape[1]), dtype=np.float64)
    for c in range(X.shape[1]):
        xc = np.ascontiguousarray(X[:, c])
        yc = np.empty(m, dtype=np.float64)
        lib.orc_csr_matvec(m, _ptr(row_ptr, _i64p), _ptr(col, _i32p), _ptr(val), _ptr(xc), _ptr(yc))
        Y[:, c] = yc
    return Y[:, 0] if vec else Y


# ----------------------------------------------------------------- QR / solve
def householder_qr(A):
    """Returns (VR, tau, info): R in the upper triangle of VR, the reflectors
    v_j (implicit unit leading entry) below it; info = first zero-norm column + 1."""
    lib = _load()
    VR = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = VR.shape
    tau = np.zeros(min(m, n), dtype=np.float64)
    info = lib.orc_householder_qr(m, n, _ptr(VR), m, _ptr(tau))
    return VR, tau, int(info)


def _rhs(B):
    Bm = np.array(B, dtype=np.float64, order="F", copy=True)
    vec = Bm.ndim == 1
    if vec:
        Bm = Bm.reshape(-1, 1, order="F")
    return Bm, vec


def apply_qt(VR, tau, B) -> np.ndarray:
    lib = _load()
    VR = _f64_colmajor(VR)
    Bm, vec = _rhs(B)
    m = VR.shape[0]
    lib.orc_apply_qt(m, tau.shape[0], _ptr(VR), m, _ptr(np.ascontiguousarray(tau)),
                     _ptr(Bm), Bm.shape[1], Bm.shape[0])
    return Bm[:, 0] if vec else Bm


def apply_q(VR, tau, B) -> np.ndarray:
    lib = _load()
    VR = _f64_colmajor(VR)
    Bm, vec = _rhs(B)
    m = VR.shape[0]
    lib.orc_apply_q(m, tau.shape[0], _ptr(VR), m, _ptr(np.ascontiguousarray(tau)),
                    _ptr(Bm), Bm.shape[1], Bm.shape[0])
    return Bm[:, 0] if vec else Bm


def back_substitute(VR, C) -> np.ndarray:
    """X = R^{-1} C[0:n] with R = triu(VR[0:n, 0:n])."""
    lib = _load()
    VR = _f64_colmajor(VR)
    n = VR.shape[1]
    Cm, vec = _rhs(np.asarray(C)[:n])
    info = lib.orc_back_substitute(n, _ptr(VR), VR.shape[0], _ptr(Cm), Cm.shape[1], Cm.shape[0])
    if info:
        raise ZeroDivisionError("R[%d, %d] == 0" % (info - 1, info - 1))
    return Cm[:, 0] if vec else Cm


def forward_substitute_rt(VR, G) -> np.ndarray:
    """Z = R^{-T} G."""
    lib = _load()
    VR = _f64_colmajor(VR)
    n = VR.shape[1]
    Gm, vec = _rhs(G)
    info = lib.orc_forward_substitute_rt(n, _ptr(VR), VR.shape[0], _ptr(Gm), Gm.shape[1], Gm.shape[0])
    if info:
        raise ZeroDivisionError("R[%d, %d] == 0" % (info - 1, info - 1))
    return Gm[:, 0] if vec else Gm


def solve(VR, tau, B) -> np.ndarray:
    """X = R^{-1} (Q^T B) (Eq. (solve))."""
    return back_substitute(VR, apply_qt(VR, tau, B))


def adjoint(VR, tau, G) -> np.ndarray:
    """grad_b = Q [R^{-T} g; 0]: the transpose of the map b -> R^{-1} Q^T b."""
    m, n = VR.shape
    Z = forward_substitute_rt(VR, G)
    Zm = Z.reshape(n, -1)
    Y = np.zeros((m, Zm.shape[1]), dtype=np.float64, order="F")
    Y[:n] = Zm
    Y = apply_q(VR, tau, Y)
    return Y[:, 0] if np.asarray(G).ndim == 1 else Y


def lstsq(A, B):
    """Least-squares solution through the oracle's own QR (factor + solve)."""
    VR, tau, info = householder_qr(A)
    if info:
        raise np.linalg.LinAlgError("rank deficient at column %d" % (info - 1))
    return solve(VR, tau, B)


def rank_report(VR) -> dict:
    """min |R_jj| / max |R_jj| and the rank-deficiency test of the full-column-
    rank condition (rows >= columns alone does not guarantee it)."""
    d = np.abs(np.diag(np.asarray(VR)[: VR.shape[1], : VR.shape[1]]))
    m, n = VR.shape
    ratio = float(d.min() / d.max()) if d.max() > 0 else 0.0
    return {"min_rjj": float(d.min()), "max_rjj": float(d.max()), "ratio": ratio,
            "numerically_deficient": bool(d.min() <= n * np.finfo(np.float64).eps * d.max())}


# ----------------------------------------------------------- image quality
# Sec. 3.1 "Image quality metrics", Eqs. (snr), (mse), (psnr), (ssim).  Images
# are N x N with pixel (ix, iy) at index iy * N + ix (iy = 0 is the bottom row,
# y = -W/2).  Readings where the paper is silent: MAX of Eq. (psnr) is the
# largest pixel of the reference image; SSIM uses every 7 x 7 window of the
# image (no padding), window means and sample (co)variances (divisor 48), and
# c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L the reference's dynamic range
# (max - min); the image's SSIM is the mean over its windows.  A crop keeps
# the pixels iy in [bottom, N - top), ix in [left, N - right).

def _crop(img, N, crop):
    a = np.asarray(img, dtype=np.float64).reshape(N, N)          # [iy, ix]
    if crop is None:
        return a
    bottom, top, left, right = (int(v) for v in crop)
    return a[bottom:N - top, left:N - right]


def snr(ref, img, N, crop=None) -> float:
    """Eq. (snr): 10 log10 (sum I0^2 / sum (I0 - I)^2), in dB."""
    r, x = _crop(ref, N, crop), _crop(img, N, crop)
    num = sum(float(v) ** 2 for v in r.ravel())
    den = sum(float(a - b) ** 2 for a, b in zip(r.ravel(), x.ravel()))
    return 10.0 * np.log10(num / den) if den > 0 else float("inf")


def mse(ref, img, N, crop=None) -> float:
    """Eq. (mse): mean of (I0 - I)^2 over the (cropped) image."""
    r, x = _crop(ref, N, crop), _crop(img, N, crop)
    return sum(float(a - b) ** 2 for a, b in zip(r.ravel(), x.ravel())) / r.size


def psnr(ref, img, N, crop=None) -> float:
    """Eq. (psnr): 10 log10 (MAX_I0^2 / MSE), MAX_I0 the reference's largest pixel."""
    e = mse(ref, img, N, crop)
    mx = float(np.max(_crop(ref, N, crop)))
    return 10.0 * np.log10(mx * mx / e) if e > 0 else float("inf")


def ssim(ref, img, N, crop=None, window: int = 7) -> float:
    """Eq. (ssim) per window x (reference) and y (image), averaged over all
    window positions; written out window by window."""
    r, x = _crop(ref, N, crop), _crop(img, N, crop)
    L = float(np.max(r) - np.min(r))
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    k = window
    total, count = 0.0, 0
    for i in range(r.shape[0] - k + 1):
        for j in range(r.shape[1] - k + 1):
            a = r[i:i + k, j:j + k].ravel()
            b = x[i:i + k, j:j + k].ravel()
            mu_a, mu_b = sum(a) / a.size, sum(b) / b.size
            va = sum((v - mu_a) ** 2 for v in a) / (a.size - 1)
            vb = sum((v - mu_b) ** 2 for v in b) / (b.size - 1)
            cov = sum((u - mu_a) * (v - mu_b) for u, v in zip(a, b)) / (a.size - 1)
            total += ((2 * mu_a * mu_b + c1) * (2 * cov + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (va + vb + c2))
            count += 1
    return total / count
