"""Pins of the stored oracle reference of the 128x128 workload
(tests/golden/c2_oracle_reference.npz, written by the script beside it), on
the CPU: the stored solutions are least-squares solutions of the stored
sinograms (A^T (b - A x) = 0 to FP64 rounding, Eq. (solve)), and the stored
reflector scalars and diagonal of R over the first 1024 columns are bitwise
those of the oracle's QR of A's leading 1024 columns (Eq. (qr): the first k
Householder steps read and write only the first k columns' history)."""
import hashlib
import os

import numpy as np

from oracle import oracle as O
from paper_2412_07631_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_reference.npz")


def test_c2_reference_is_least_squares_and_matches_leading_qr():
    g = np.load(GOLDEN)
    sc = synth.workload_scanner("c2_128")
    w = synth.WORKLOADS["c2_128"]
    ids = [int(s) for s in g["slice_ids"]]
    csr = O.system_csr(sc)
    B = synth.noisy_sinograms(w["cfg"], O.csr_matvec(csr, synth.phantoms(w["cfg"], sc.n_pix, ids)), w["I0"], ids)
    assert hashlib.sha256(np.asfortranarray(B).tobytes(order="F")).hexdigest() == str(g["b_sha256"])
    X = g["x"]
    row_ptr, col, val = csr
    rows = np.repeat(np.arange(sc.m), np.diff(row_ptr))
    R = B - O.csr_matvec(csr, X)
    for c in range(X.shape[1]):
        gr = np.bincount(col, weights=val * R[rows, c], minlength=sc.n)
        gb = np.bincount(col, weights=val * B[rows, c], minlength=sc.n)
        rel = np.linalg.norm(gr) / np.linalg.norm(gb)
        # backward-stable FP64 Householder least squares; measured ~1e-16
        assert rel <= 1e-12, (c, rel)
    k = 1024
    sel = col < k
    Alead = np.zeros((sc.m, k), order="F")
    Alead[rows[sel], col[sel]] = val[sel]
    VR, tau, info = O.householder_qr(Alead)
    assert info == 0
    assert np.array_equal(tau, g["tau"][:k])
    assert np.array_equal(np.diag(VR[:k]), g["r_diag"][:k])
