"""The largest workload on one GPU: the 512 x 512 image (180 views x 1472
bins, A = 264960 x 262144, 278 GB in FP32) factored in device memory.

    python -m paper_2412_07631_amd.large [--workload c5_512] [--slices 1024]
                                         [--batch 128] [--tol 1e-6]

On a 288 GiB device the FP32 matrix fits beside the factorization's lean
workspace (ct_qr_factor with CT_QR_NO_SOLVE_COPIES: no solve-side copies, the
solves read V and R in place), so the out-of-core path the paper needs for this
size on a 40 GB device is not needed here; it stays exercised, at smaller
sizes, by the streamed factorization.  BF16x3 factorization, then batches of
noisy sinograms through the FP64-residual refinement with the stop rule.  The
FP64 oracle of this size does not exist (556 GB, 2.4e16 flop), so correctness
is checked by what holds at any size: recovery of the phantoms from noiseless
sinograms, the least-squares optimality of the noisy solutions in FP64
(||A^T r|| / (||A||_F ||r||)), and the step-by-step fall of ||A^T r||.
Prints progress to stderr and one JSON line to stdout.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="c5_512")
    ap.add_argument("--slices", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--refine", type=int, default=6, help="refinement steps at most")
    ap.add_argument("--tol", type=float, default=1e-6, help="stop rule of the refinement")
    ap.add_argument("--prec", default="bf16x3", choices=["f32", "bf16x3"], help="arithmetic of the factorization")
    ap.add_argument("--method", default="pcgls", choices=["sne", "pcgls"],
                    help="refinement: stationary semi-normal steps or preconditioned conjugate gradients")
    ap.add_argument("--check-columns", type=int, default=16, help="sampled columns of the Q^T a_j check")
    ap.add_argument("--geometry", default=None,
                    help="N,views,bins: the workload's seeds and dose with another scanner (same proportions "
                         "at a smaller size, say)")
    args = ap.parse_args()

    import torch
    from paper_2412_07631_amd import ctqr, synth

    w = synth.WORKLOADS[args.workload]
    sc = synth.workload_scanner(args.workload)
    if args.geometry:
        N, views, bins = (int(v) for v in args.geometry.split(","))
        sc = synth.scanner(N, views, bins)
    m, n = sc.m, sc.n
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    free, total = torch.cuda.mem_get_info(0)
    log("%s: m=%d n=%d, device memory %.1f of %.1f GiB free" % (args.workload, m, n, free / 2**30, total / 2**30))

    A = torch.empty((n, ctqr.ld16(m)), dtype=torch.float32, device=dev)
    e0, e1 = ev(), ev()
    e0.record(stream)
    ctqr.build_system(sc, A)
    e1.record(stream)
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    log("A built: %.1f GiB in %.1f ms" % (A.numel() * 4 / 2**30, build_ms))

    ctqr.debug_progress(16)                                 # a line every 16384 columns
    e0.record(stream)
    f = ctqr.qr_factor(A, m, n, ctqr.PREC_NAMES[args.prec], max_nrhs=args.batch, solve_copies=False)
    e1.record(stream)
    info = ctqr.status(f)
    qr_ms = e0.elapsed_time(e1)
    ctqr.debug_progress(0)
    flops = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    log("QR (%s): %.1f s, %.1f TFLOP/s, info %d" % (args.prec, qr_ms / 1e3, flops / (qr_ms * 1e-3) / 1e12, info))
    if info != 0:
        raise RuntimeError("rank deficiency reported at column %d" % (info - 1))
    # a lower bound of kappa(A) = kappa(R): the spread of R's diagonal
    ld = A.shape[1]
    diag = A.view(-1)[torch.arange(n, device=dev) * (ld + 1)].abs().double()
    rdiag = {"max": float(diag.max().item()), "min": float(diag.min().item())}
    rdiag["ratio"] = rdiag["max"] / rdiag["min"]
    log("|R_jj|: max %.4g min %.4g ratio %.4g (a lower bound of kappa(A))" % (rdiag["max"], rdiag["min"],
                                                                            rdiag["ratio"]))
    del diag

    free, _ = torch.cuda.mem_get_info(0)
    log("device memory free after the factorization: %.1f GiB (workspace %.1f GiB)" % (
        free / 2**30, f.work.numel() / 2**30))
    sp = ctqr.SparseA(sc, group=0)
    a_fro = float(torch.linalg.vector_norm(sp.val).item())
    log("sparse copies: nnz %d, ||A||_F %.6g" % (sp.nnz, a_fro))

    # the factorization itself, column by column: Q^T a_j = [R_{0:j, j}; 0]
    # for sampled columns j (a_j the FP32 column that was factored, from the
    # CSC copy; R_{0:j, j} read from the factored matrix)
    cols = sorted(set(int(c) for c in np.linspace(0, n - 1, args.check_columns)))
    cp = sp.col_ptr.cpu().numpy()
    Bc = torch.zeros((len(cols), ctqr.ld16(m)), dtype=torch.float32, device=dev)
    for i, j in enumerate(cols):
        rows = sp.row[cp[j]:cp[j + 1]].long()
        Bc[i, rows] = sp.cval[cp[j]:cp[j + 1]].float()
    anorm = Bc[:, :m].double().norm(dim=1)
    ctqr.apply_qt(f, Bc)
    col_err = []
    for i, j in enumerate(cols):
        want = torch.zeros(m, dtype=torch.float64, device=dev)
        want[: j + 1] = A[j, : j + 1].double()
        col_err.append(float(((Bc[i, :m].double() - want).norm() / anorm[i]).item()))
    log("Q^T a_j = [r_j; 0] on %d columns: worst %.3g at column %d" % (
        len(cols), max(col_err), cols[int(np.argmax(col_err))]))
    del Bc

    out_batches = []
    solve_ms = 0.0
    done = 0
    method = {"sne": ctqr.REFINE_SNE, "pcgls": ctqr.REFINE_PCGLS}[args.method]
    scratch = torch.empty(ctqr.refine_workspace(m, n, args.batch, method), dtype=torch.uint8, device=dev)
    while done < args.slices:
        k = min(args.batch, args.slices - done)
        ids = list(range(done, done + k))
        Xtrue = synth.phantoms(w["cfg"], sc.n_pix, ids)
        Xtd = torch.zeros((k, ctqr.ld16(n)), dtype=torch.float64, device=dev)
        Xtd[:, :n] = torch.from_numpy(np.ascontiguousarray(Xtrue.T)).to(dev)
        zero = torch.zeros((k, ctqr.ld16(m)), dtype=torch.float64, device=dev)
        Pnl = torch.empty_like(zero)
        ctqr.residual(sp.csr, m, Xtd, zero, Pnl)             # -A x
        Pnl.neg_()
        del zero
        B = synth.noisy_sinograms(w["cfg"], Pnl[:, :m].cpu().numpy().T, w["I0"], ids)
        Bd = torch.zeros_like(Pnl)
        Bd[:, :m] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
        X = torch.zeros((k, ctqr.ld16(n)), dtype=torch.float64, device=dev)
        rn = torch.zeros((args.refine + 1) * k, dtype=torch.float64, device=dev)
        gn = torch.zeros((args.refine + 1) * k, dtype=torch.float64, device=dev)
        e0.record(stream)
        steps = ctqr.solve_refined(f, sp, Bd, X, args.refine, method, nrhs=k, scratch=scratch, res_norms=rn,
                                   grad_norms=gn, tol=args.tol)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        solve_ms += ms
        rnv = rn.view(args.refine + 1, k).cpu().numpy()[: steps + 1]
        gnv = gn.view(args.refine + 1, k).cpu().numpy()[: steps + 1]
        eta = float(np.max(gnv[-1] / (a_fro * rnv[-1])))
        # noiseless sinograms: the phantoms themselves come back
        Xn = torch.zeros_like(X)
        ctqr.solve_refined(f, sp, Pnl, Xn, args.refine, method, nrhs=k, scratch=scratch, tol=args.tol)
        e = ((Xn[:, :n] - Xtd[:, :n]).norm(dim=1) / Xtd[:, :n].norm(dim=1)).max().item()
        rec = {"slices": k, "solve_ms": ms, "steps": steps, "ls_optimality_max": eta,
               "grad_norm_by_step_max": [float(np.max(g)) for g in gnv], "noiseless_rel_err_max": e}
        out_batches.append(rec)
        done += k
        log("batch of %d: %d steps, %.1f ms (%.1f slices/s), LS optimality %.2e, noiseless recovery %.2e" % (
            k, steps, ms, k / (ms * 1e-3), eta, e))
        del Xtd, Pnl, Bd, X, Xn, rn, gn

    res = {"workload": args.workload, "precision": args.prec, "refinement": args.method, "m": m, "n": n,
           "r_diag": rdiag,
           "qt_column_check": {"columns": cols, "rel_err": col_err},
           "matrix_gib_fp32": A.numel() * 4 / 2**30,
           "workspace_gib": f.work.numel() / 2**30, "build_ms": build_ms, "qr_ms": qr_ms,
           "qr_tflops": flops / (qr_ms * 1e-3) / 1e12, "slices": done, "slices_per_s": done / (solve_ms * 1e-3),
           "refine_tol": args.tol, "batches": out_batches}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
