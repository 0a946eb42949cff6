#!/usr/bin/env python3
"""Reconstruction throughput against the number of slices solved together
(the experiment of Sec. 3.1, Fig. 1: slices per second grows with the number
of simultaneous slices until the solve is compute-bound).

For each precision the system matrix of a workload is built and factored
once; then batches of 1, 2, 4, ... up to --max-nrhs noisy sinograms are
reconstructed by X = R^-1 Q^T B (FP64 and FP32 factors) or by the BF16x3
factor followed by FP64-residual refinement (semi-normal steps, or the
preconditioned conjugate-gradient steps with --method pcgls, up to --refine
steps under the stop rule --tol), and the batch's event time gives slices/s.
The precisions named by --fused are timed a second time through the one-launch
fused solve (ct_solve_fused).  Every step runs in the library's
kernels; the inputs are seeded synthetic phantoms and Poisson noise.

    python -m paper_2412_07631_amd.sweep [--workload c3_256] [--max-nrhs 2048]

Every timed batch is checked: its images against the FP64 path's images of
the same slices (solved once as one batch of --max-nrhs), each precision
within its stated bound (FP64 1e-10; FP32 1e-2, the kappa(A) u32 level of an
unrefined FP32 solve at 256^2, where kappa(A) is about 1e4 and the error
2.5e-3; BF16x3 with refinement to the stop rule 1e-6).  A batch outside its bound is reported and makes the run
exit with status 1.

Prints one JSON object per (precision, batch size) and a summary table; with
--out, also writes the table as markdown (with the command) to that file.
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


BOUND = {"f64": 1e-10, "f32": 1e-2, "bf16x3": 1e-6}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="c3_256")
    ap.add_argument("--max-nrhs", type=int, default=2048)
    ap.add_argument("--precs", default="f64,f32,bf16x3")
    ap.add_argument("--refine", type=int, default=6, help="refinement steps of the BF16x3 path at most")
    ap.add_argument("--tol", type=float, default=1e-6, help="stop rule of the refinement")
    ap.add_argument("--method", default="sne", choices=["sne", "pcgls"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="markdown summary file")
    ap.add_argument("--fused", default="f32", help="precisions also timed through the one-launch fused solve "
                                                 "(comma-separated, empty for none)")
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
    method = {"sne": ctqr.REFINE_SNE, "pcgls": ctqr.REFINE_PCGLS}[args.method]
    precs = args.precs.split(",")
    if "f64" in precs:
        precs = ["f64"] + [p for p in precs if p != "f64"]
    table, worst, failed = {}, {}, []
    Xref = None
    for prec in precs:
        p = ctqr.PREC_NAMES[prec]
        dt = torch.float64 if p == ctqr.PREC_F64 else torch.float32
        A = torch.empty((n, ctqr.ld16(m)), dtype=dt, device=dev)
        ctqr.build_system(sc, A)
        f = ctqr.qr_factor(A, m, n, p, max_nrhs=args.max_nrhs)
        assert ctqr.status(f) == 0
        refined = prec == "bf16x3"
        variants = [(prec + ("+%s" % args.method if refined else ""), False)]
        if prec in args.fused.split(","):
            variants.append((prec + " fused", True))

        def solve(k, fused=False):
            if refined:
                Xd = torch.zeros((k, ctqr.ld16(n)), dtype=torch.float64, device=dev)
                steps = ctqr.solve_refined(f, sp, Ball[:k], Xd, args.refine, method, tol=args.tol)
                return Xd[:, :n], steps
            Bk = Ball[:k].to(dt, copy=True)          # the solves work in place
            if fused:
                ctqr.solve_fused(f, Bk)
            else:
                ctqr.apply_qt(f, Bk)
                ctqr.trsm_solve(f, Bk)
            return Bk[:, :n].double(), 0

        if prec == "f64":
            Xref, _ = solve(args.max_nrhs)
            Xref = Xref.clone()
        for (label, fused), k in ((v, k) for v in variants for k in sizes):
            best, X, steps = None, None, 0
            for _ in range(args.reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                X, steps = solve(k, fused)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
            rate = k / (best * 1e-3)
            rec = {"workload": args.workload, "prec": label, "nrhs": k, "ms": best, "slices_per_s": rate,
                   "solve_tflops": flop * rate / 1e12}
            if refined:
                rec["refine_steps"] = steps
            if Xref is not None:
                R = Xref[:k]
                err = ((X - R).norm(dim=1) / R.norm(dim=1)).max().item()
                rec["max_rel_err_vs_fp64"] = err
                rec["bound"] = BOUND[prec]
                rec["check"] = "ok" if err <= BOUND[prec] else "FAIL"
                rec["status"] = ctqr.status(f)
                worst[label] = max(worst.get(label, 0.0), err)
                if err > BOUND[prec]:
                    failed.append((label, k, err))
            print(json.dumps(rec), flush=True)
            table.setdefault(k, {})[label] = rate
        del f, A
        torch.cuda.empty_cache()
    labels = list(dict.fromkeys(l for v in table.values() for l in v))
    print("%8s " % "nrhs" + " ".join("%16s" % p for p in labels), file=sys.stderr)
    for k in sizes:
        print("%8d " % k + " ".join("%16.1f" % table[k].get(p, float("nan")) for p in labels), file=sys.stderr)
    if args.out:
        with open(args.out, "w") as fo:
            fo.write("# Slices/s against slices per batch, %s (%d x %d)\n\n" % (args.workload, m, n))
            fo.write("Command: `python -m paper_2412_07631_amd.sweep %s`\n\n" % " ".join(sys.argv[1:]))
            fo.write("Best of %d batches per size; every batch checked against the FP64 path's images of the same "
                     "slices (one batch of %d).\n\n" % (args.reps, args.max_nrhs))
            fo.write("| slices | " + " | ".join(labels) + " |\n|---|" + "---|" * len(labels) + "\n")
            for k in sizes:
                fo.write("| %d | " % k + " | ".join("%.1f" % table[k].get(p, float("nan")) for p in labels) + " |\n")
            fo.write("\nLargest relative image error against the FP64 path over all batch sizes: " +
                     ", ".join("%s %.2e (bound %.0e)" % (l, worst[l], BOUND[l.split("+")[0].split(" ")[0]])
                               for l in worst) + "\n")
    if failed:
        print("outside the bound: %s" % failed, file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
