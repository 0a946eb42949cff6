"""CPU-side checks of the C-ABI library: it loads, and it exports every entry
point the public header declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctqr.h")
LIB = os.path.join(ROOT, "paper_2412_07631_amd", "libctqr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("ct_build_system", "ct_qr_factor", "ct_apply_qt", "ct_trsm_solve", "ct_solve_backward"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python -m paper_2412_07631_amd.build"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu():
    """Argument validation runs before any device work: -i for argument i."""
    lib = ctypes.CDLL(LIB)
    lib.ct_qr_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.ct_last_error.restype = ctypes.c_char_p
    b = ctypes.c_size_t(0)
    assert lib.ct_qr_workspace(100, 200, 0, 1, ctypes.byref(b)) == -2      # n > m
    assert b"n" in lib.ct_last_error()
    assert lib.ct_qr_workspace(100, 50, 9, 1, ctypes.byref(b)) == -3       # bad precision
    assert lib.ct_qr_workspace(1920, 1024, 0, 4, ctypes.byref(b)) == 0 and b.value > 1920 * 8
    lib.ct_factor_destroy.argtypes = [ctypes.c_void_p]
    assert lib.ct_factor_destroy(None) == 0
    # the block-width hook takes 0 or a multiple of 32 up to 2048, and the
    # workspace follows the width (T of every outer block grows with it)
    for bad in (16, 100, 4096, -32):
        assert lib.ct_debug_block_width(bad) == -1
    ws = {}
    for nb in (256, 1024):
        assert lib.ct_debug_block_width(nb) == 0
        assert lib.ct_qr_workspace(4096, 2048, 1, 4, ctypes.byref(b)) == 0
        ws[nb] = b.value
    assert lib.ct_debug_block_width(0) == 0
    assert ws[1024] > ws[256]
    # the refinement-precision hook takes modes 0..2 and returns the previous one
    assert lib.ct_debug_refine_x3(3) == -1 and lib.ct_debug_refine_x3(-1) == -1
    assert lib.ct_debug_refine_x3(2) == 1
    assert lib.ct_debug_refine_x3(0) == 2
    assert lib.ct_debug_refine_x3(1) == 0


def test_binding_marshals_without_gpu():
    from paper_2412_07631_amd import ctqr
    assert ctqr.ld16(1920) == 1920 and ctqr.ld16(1401) == 1408
    assert ctqr.qr_workspace(76800, 65536, ctqr.PREC_BF16X3, 512) > 65536 * 256 * 8
    try:
        ctqr.qr_workspace(10, 20, ctqr.PREC_F64, 1)
    except ctqr.CtError as e:
        assert e.code == -2
    else:
        raise AssertionError("expected an argument error")


def test_refine_workspace_by_method():
    """The Krylov refinement needs n x lt FP64 more (its search directions)
    plus five rows of per-slice scalars; the other methods share one size;
    an unknown method is argument 4."""
    from paper_2412_07631_amd import ctqr
    up = lambda x: (x + 255) // 256 * 256
    m, n = 3360, 2304
    for nrhs in (1, 16, 37):
        lt = (nrhs + 15) // 16 * 16
        base = ctqr.refine_workspace(m, n, nrhs, ctqr.REFINE_SNE)
        assert base == ctqr.refine_workspace(m, n, nrhs, ctqr.REFINE_QR)
        assert base == 2 * up(m * lt * 8) + 2 * up(n * lt * 8) + up(m * nrhs * 8) + up(256 * lt * 8)
        assert ctqr.refine_workspace(m, n, nrhs, ctqr.REFINE_PCGLS) == base + up(n * lt * 8) + up(5 * lt * 8)
    try:
        ctqr.refine_workspace(m, n, 4, 7)
    except ctqr.CtError as e:
        assert e.code == -4
    else:
        raise AssertionError("expected an argument error")


def test_stream_workspace_arithmetic():
    """Streamed factorization: the minimum device buffer is the in-memory
    workspace without its solve-side copies (the diagonal-block inverses of R,
    2 x 128 x 128 per 128-row block; the row-major block columns of R above the
    diagonal, 128^2 b (b - 1) / 2 elements for b blocks; the row-major
    reflector blocks, (m - 256 k) x 256 elements for outer block k) plus four
    staging tiles; keeping every tile resident needs that workspace plus all
    tiles (tile = lda x tile_cols elements, 256-B rounded).  Below 16384
    columns both factorizations use outer blocks of 256 columns, so their
    other buffers coincide."""
    from paper_2412_07631_amd import ctqr
    m, n, lda = 3360, 2304, 3360
    nbt = (n + 255) // 256
    nbo = (n + 255) // 256
    up = lambda x: (x + 255) // 256 * 256
    # row-major copies of R above its diagonal in two levels (outer blocks of
    # 1024 columns from n >= 2048, 256-column blocks inside)
    ob = 1024
    nro, q = (n + ob - 1) // ob, ob // 256
    rt = ob * ob * (nro * (nro - 1) // 2) + nro * 256 * 256 * (q * (q - 1) // 2)
    rcopies = (up(2 * nbt * 256 * 256 * 8) + up(nbt * 256 * 256 * 8) + up(rt * 8)
               + up((nbo * m - 256 * (nbo * (nbo - 1) // 2)) * 256 * 8))
    base = ctqr.qr_workspace(m, n, ctqr.PREC_F64, 8) - rcopies
    lo, full = ctqr.qr_stream_workspace(m, n, lda, ctqr.PREC_F64, 8, 256)
    tile = (lda * 256 * 8 + 255) // 256 * 256
    assert lo == base + 4 * tile and full == base + 9 * tile
    lo32, full32 = ctqr.qr_stream_workspace(m, n, lda, ctqr.PREC_BF16X3, 8, 1024)
    # (plus, for BF16x3, the inverses of the 1024-column diagonal blocks in two layouts)
    rc32 = (up(2 * nbt * 256 * 256 * 4) + up(nbt * 256 * 256 * 8) + up(rt * 4) + up(2 * nro * 1024 * 1024 * 4)
            + up((nbo * m - 256 * (nbo * (nbo - 1) // 2)) * 256 * 4))
    base32 = ctqr.qr_workspace(m, n, ctqr.PREC_BF16X3, 8) - rc32
    assert full32 == base32 + 3 * ((lda * 1024 * 4 + 255) // 256 * 256)
    assert lo32 == full32          # three tiles: fewer than the staging slots
    for bad_tile in (0, 100, -128):
        try:
            ctqr.qr_stream_workspace(m, n, lda, ctqr.PREC_F64, 8, bad_tile)
        except ctqr.CtError as e:
            assert e.code == -6
        else:
            raise AssertionError("expected an argument error")


def test_streamed_factor_argument_errors_without_gpu():
    from paper_2412_07631_amd import ctqr
    lib = ctqr._lib
    h = ctypes.c_void_p()
    # tile_cols not a multiple of 128 (argument 10), n > m (argument 3)
    assert lib.ct_qr_factor_streamed(ctypes.c_void_p(256), 100, 50, 112, ctqr.PREC_F64, ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), 1 << 30, 1, 100, ctypes.byref(h), None) == -10
    assert lib.ct_qr_factor_streamed(ctypes.c_void_p(256), 100, 150, 112, ctqr.PREC_F64, ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), 1 << 30, 1, 128, ctypes.byref(h), None) == -3
    # a buffer below the minimum (argument 8)
    assert lib.ct_qr_factor_streamed(ctypes.c_void_p(256), 100, 50, 112, ctqr.PREC_F64, ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), 1024, 1, 128, ctypes.byref(h), None) == -8
    assert lib.ct_qr_resume(None, None) == -1
    with __import__("pytest").raises(TypeError):
        import torch
        ctqr.qr_factor_streamed(torch.zeros((4, 16)), 16, 4, ctqr.PREC_F32, tile_cols=128)


def test_factor_file_header_checks_without_gpu(tmp_path):
    """ct_factor_file_info / ct_factor_load refuse what is not a factor file,
    and report the workspace of a well-formed header before any device work."""
    import struct
    lib = ctypes.CDLL(LIB)
    lib.ct_factor_file_info.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_size_t)]
    lib.ct_factor_load.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
    lib.ct_qr_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_size_t)]
    m, n, p, b = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0), ctypes.c_size_t(0)
    info = lambda path: lib.ct_factor_file_info(path.encode(), 8, ctypes.byref(m), ctypes.byref(n),
                                                ctypes.byref(p), ctypes.byref(b))
    assert info(str(tmp_path / "missing.bin")) == -1
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a factor file at all, just text" * 4)
    assert info(str(junk)) == -1
    # header: magic, m, n, prec, nb_out, nb_in, info, element size, reserved
    hdr = tmp_path / "hdr.bin"
    hdr.write_bytes(b"CTQRFAC1" + struct.pack("<8q", 3360, 2304, 1, 256, 32, 0, 4, 0))
    assert info(str(hdr)) == 0 and (m.value, n.value, p.value) == (3360, 2304, 1)
    w = ctypes.c_size_t(0)
    assert lib.ct_qr_workspace(3360, 2304, 1, 8, ctypes.byref(w)) == 0
    assert b.value == w.value          # the same blocking as a fresh factorization
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"CTQRFAC1" + struct.pack("<8q", 3360, 2304, 1, 256, 32, 0, 8, 0))   # wrong element size
    assert info(str(bad)) == -1
    h = ctypes.c_void_p(0)
    # too small a workspace and a bad lda are refused before any device work
    assert lib.ct_factor_load(str(hdr).encode(), ctypes.c_void_p(256), 3360, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), 1024, 8, ctypes.byref(h), None) == -6
    assert lib.ct_factor_load(str(hdr).encode(), ctypes.c_void_p(256), 3000, ctypes.c_void_p(256),
                              ctypes.c_void_p(256), 1 << 40, 8, ctypes.byref(h), None) == -3


def test_fused_solve_argument_errors_without_gpu():
    """ct_solve_fused and its graph form validate their arguments before any
    device work."""
    lib = ctypes.CDLL(LIB)
    lib.ct_solve_fused.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    assert lib.ct_solve_fused(None, ctypes.c_void_p(256), 4, 64, None) == -1
    lib.ct_solve_graph_create_fused.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert lib.ct_solve_graph_create_fused(None, ctypes.c_void_p(256), 64, 4, 4, ctypes.c_void_p(256),
                                           ctypes.c_void_p(256), ctypes.byref(h)) == -1
