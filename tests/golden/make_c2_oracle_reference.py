"""Write tests/golden/c2_oracle_reference.npz: the FP64 oracle's solution of
the 128x128 workload (90 views x 256 bins, A = 23040 x 16384, Siddon lengths)
for four of its noisy slices, plus samples of its factor.

It calls only the oracle (unblocked FP64 Householder QR, Eq. (qr); Q^T b and
back substitution, Eq. (solve)) and the seeded input generators; nothing here
touches the HIP library.  The factorization takes several minutes on the
host, which is why its result is stored instead of recomputed by the GPU
test that compares against it (tests/test_gpu_c2_oracle.py).

    python tests/golden/make_c2_oracle_reference.py

Stored arrays:
  slice_ids         the slice numbers of the c2 workload (config 2) solved
  b_sha256          SHA-256 of the FP64 sinograms B (m x 4, column-major
                    bytes), so a test can tell that it rebuilt the same B
  x                 n x 4 oracle solutions x* = R^-1 Q^T b
  tau               all n reflector scalars
  r_diag            the n diagonal entries of R
  cols, vr_cols     whole columns j of V\\R (R above and on the diagonal,
                    the Householder vector below it) for the listed j
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2412_07631_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "c2_oracle_reference.npz")
SLICES = [0, 21, 42, 63]
COLS = [1025, 8191, 16383]


def sinograms(sc, csr):
    """The c2 workload's noisy sinograms for SLICES (config 2, I0 = 5e4)."""
    w = synth.WORKLOADS["c2_128"]
    X_true = synth.phantoms(w["cfg"], sc.n_pix, SLICES)
    return synth.noisy_sinograms(w["cfg"], O.csr_matvec(csr, X_true), w["I0"], SLICES)


def b_digest(B):
    return hashlib.sha256(np.asfortranarray(B, dtype=np.float64).tobytes(order="F")).hexdigest()


def main():
    sc = synth.workload_scanner("c2_128")
    csr = O.system_csr(sc)
    B = sinograms(sc, csr)
    t0 = time.time()
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    del A
    assert info == 0, info
    X = O.solve(VR, tau, B)
    print("oracle QR + solve of %d x %d in %.0f s" % (sc.m, sc.n, time.time() - t0))
    np.savez_compressed(OUT, slice_ids=np.array(SLICES), b_sha256=np.array(b_digest(B)), x=X,
                        tau=tau, r_diag=np.diag(VR[: sc.n, :]).copy(), cols=np.array(COLS),
                        vr_cols=VR[:, COLS].copy())
    print("wrote", OUT)


if __name__ == "__main__":
    main()
