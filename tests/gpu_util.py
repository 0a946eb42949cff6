"""Helpers shared by the GPU tests: moving column-major matrices between numpy
(rows x cols) and the binding's (cols, ld) device tensors, and the seeded
problems the parity tests use."""
import numpy as np
import torch

from paper_2412_07631_amd import synth


def ld16(rows):
    return (int(rows) + 15) // 16 * 16


def to_dev(M, dtype, ld=None):
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 1:
        M = M[:, None]
    rows, cols = M.shape
    ld = ld16(rows) if ld is None else ld
    host = np.zeros((cols, ld), dtype=np.float64)
    host[:, :rows] = M.T
    return torch.from_numpy(host).to(device="cuda", dtype=dtype).contiguous()


def from_dev(T, rows):
    return T[:, :rows].double().cpu().numpy().T.copy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_col_rel(X, Xs):
    return max(float(np.linalg.norm(X[:, c] - Xs[:, c]) / np.linalg.norm(Xs[:, c])) for c in range(Xs.shape[1]))


def sinograms(sc, A64, cfg, slices, I0):
    """Phantoms, noiseless line integrals A x and their noisy counterparts."""
    ids = list(range(slices))
    X = synth.phantoms(cfg, sc.n_pix, ids)
    P = A64 @ X
    B = synth.noisy_sinograms(cfg, P, I0, ids)
    return X, P, B
