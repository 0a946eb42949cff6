#!/usr/bin/env python3
"""Reconstruction throughput against the number of slices solved together
(the experiment of Sec. 3.1, Fig. 1: slices per second grows with the number
of simultaneous slices until the solve is compute-bound).

For each precision the system matrix of a workload is built and factored
once; then batches of 1, 2, 4, ... up to --max-nrhs noisy sinograms are
reconstructed by X = R^-1 Q^T B (FP64 and FP32 factors) or by the BF16x3
factor followed by FP64-residual refinement (semi-normal correction steps),
and the batch's event time gives slices/s.  Every step runs in the library's
kernels; the inputs are seeded synthetic phantoms and Poisson noise.

    python -m paper_2412_07631_amd.sweep [--workload c3_256] [--max-nrhs 2048]

Prints one JSON object per (precision, batch size) and a summary table.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import ctqr, synth


def sinogram_batch(sc, sp, k, dev):
    """k noisy sinograms (FP64, slice-major rows) from seeded phantoms: the
    projections come from the library's own FP64 sparse product."""
    X = synth.phantoms(1, sc.n_pix, range(k))                    # n x k
    Xd = torch.zeros((k, ctqr.ld16(sc.n)), dtype=torch.float64, device=dev)
    Xd[:, : sc.n] = torch.from_numpy(np.ascontiguousarray(X.T)).to(dev)
    Z = torch.zeros((k, ctqr.ld16(sc.m)), dtype=torch.float64, device=dev)
    P = torch.empty_like(Z)
    ctqr.residual((sp.row_ptr, sp.col, sp.val), sc.m, Xd, Z, P)  # P = 0 - A X
    p = (-P[:, : sc.m]).cpu().numpy().T
    B = synth.noisy_sinograms(1, p, 5e4, range(k))
    Bd = torch.zeros((k, ctqr.ld16(sc.m)), dtype=torch.float64, device=dev)
    Bd[:, : sc.m] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    return Bd


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="c3_256")
    ap.add_argument("--max-nrhs", type=int, default=2048)
    ap.add_argument("--precs", default="f64,f32,bf16x3")
    ap.add_argument("--refine", type=int, default=4, help="refinement steps of the BF16x3 path")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    dev = "cuda"
    sc = synth.workload_scanner(args.workload)
    m, n = sc.m, sc.n
    sizes = []
    k = 1
    while k <= args.max_nrhs:
        sizes.append(k)
        k *= 2
    sp = ctqr.SparseA(sc)
    Ball = sinogram_batch(sc, sp, args.max_nrhs, dev)
    flop = 4.0 * m * n - float(n) * n
    table = {}
    for prec in args.precs.split(","):
        p = ctqr.PREC_NAMES[prec]
        dt = torch.float64 if p == ctqr.PREC_F64 else torch.float32
        A = torch.empty((n, ctqr.ld16(m)), dtype=dt, device=dev)
        ctqr.build_system(sc, A)
        f = ctqr.qr_factor(A, m, n, p, max_nrhs=args.max_nrhs)
        assert ctqr.status(f) == 0
        refined = prec == "bf16x3"
        for k in sizes:
            best = None
            for _ in range(args.reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                if refined:
                    Xd = torch.zeros((k, ctqr.ld16(n)), dtype=torch.float64, device=dev)
                    Bk = Ball[:k].clone()
                    torch.cuda.synchronize()
                    e0.record()
                    ctqr.solve_refined(f, sp, Bk, Xd, args.refine, ctqr.REFINE_SNE)
                else:
                    Bk = Ball[:k].to(dt)
                    torch.cuda.synchronize()
                    e0.record()
                    ctqr.apply_qt(f, Bk)
                    ctqr.trsm_solve(f, Bk)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
            rate = k / (best * 1e-3)
            rec = {"workload": args.workload, "prec": prec + ("+%d sne" % args.refine if refined else ""),
                   "nrhs": k, "ms": best, "slices_per_s": rate, "solve_tflops": flop * rate / 1e12}
            print(json.dumps(rec), flush=True)
            table.setdefault(k, {})[rec["prec"]] = rate
        del f, A
        torch.cuda.empty_cache()
    precs = sorted({p for v in table.values() for p in v})
    print("%8s " % "nrhs" + " ".join("%16s" % p for p in precs), file=sys.stderr)
    for k in sizes:
        print("%8d " % k + " ".join("%16.1f" % table[k].get(p, float("nan")) for p in precs), file=sys.stderr)


if __name__ == "__main__":
    main()
