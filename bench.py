#!/usr/bin/env python3
"""Benchmark of the direct algebraic CT reconstruction path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
Siddon assembly of A (dense FP32 + FP64 CSR/CSC copies), Householder QR at the
chosen precision, reconstruction of the batch by X = R^-1 Q^T B followed by
FP64-residual refinement, and the residual report.  Inputs (phantoms, noisy
sinograms) are built before the timed region and are resident in HBM.

Printed: one JSON line with QR TFLOP/s (value), slices/s, error against the
plain FP64 GPU path on the same problem, the live roofline of the dominant
kernel, and the CPU oracle's rate on a bounded sample of the same work.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "QR TFLOP/s + slices/s at 256^2: FP32/BF16+refine vs FP64 on MI355X, rel err"
# MFMA peak of the arithmetic each path's trailing update runs on: BF16x3
# runs on the bfloat16 MFMA, so its method flops are measured against the
# bfloat16 peak (it issues three MFMA products per method product, reported
# separately as the issue rate)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "bf16x3": 2500.0}
ISSUE_FACTOR = {"f64": 1, "f32": 1, "bf16": 1, "f16": 1, "bf16x3": 3}
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def qr_flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def solve_flops(m, n):
    return 4.0 * m * n - float(n) * n


def batched_leg(ctqr, synth, torch, f, sc, Bd, dev, total, sp, X64=None):
    """Uneven batches (seeded sizes 1..512) of sinograms through the
    graph-captured solve, then the adjoint on 64 upstream gradients with a
    central finite-difference check (step 1e-3) on the same factor.  The
    finite differences use refined (FP64-residual) solves, so that their own
    rounding (about kappa(A) u32 / h for plain FP32 solves) does not swamp
    the comparison."""
    m, n = sc.m, sc.n
    sizes = synth.uneven_batches(total, 1, 512, cfg=4)
    nr = Bd.shape[0]
    idx = torch.arange(total, device=dev) % nr
    src = Bd[idx, :].to(f.dtype)                           # (total, ld) storage-typed sinograms
    Bb = torch.zeros_like(src)
    desc = ctqr.batch_descriptor(sizes, device=dev)
    caps = (8, 16, 32, 64, 96, 128, 192, 256, 320, 384, 448, 512)
    cap_of = lambda c: next(x for x in caps if c <= x)
    graphs = {c: ctqr.SolveGraph(f, Bb, c, desc) for c in sorted({cap_of(c) for c in sizes})}
    gs = torch.cuda.Stream()
    torch.cuda.synchronize()

    def run_graphs():
        Bb.copy_(src)
        desc[0] = 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(gs)
        for c in sizes:
            graphs[cap_of(c)].launch(gs)
        e1.record(gs)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run_graphs()                                           # first replay (untimed)
    g_ms = run_graphs()
    Xg = Bb[:, :n].clone()
    # the same batches solved eagerly, for time and agreement
    Bb.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    off = 0
    for c in sizes:
        blk = Bb[off:off + c]
        ctqr.apply_qt(f, blk)
        ctqr.trsm_solve(f, blk)
        off += c
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1)
    agree = float(((Xg - Bb[:, :n]).abs().max() / Bb[:, :n].abs().max()).item())
    vs64 = None
    if X64 is not None:
        Xr = X64[idx, :n]
        e = (Xg.double() - Xr).norm(dim=1) / Xr.norm(dim=1)
        vs64 = {"rel_err_max": float(e.max().item()), "rel_err_median": float(e.median().item())}

    # adjoint: 64 FP32 upstream gradients; FD check along seeded directions
    k = 64
    G = torch.from_numpy(np.ascontiguousarray(synth.gradients(n, k).T)).to(dev, f.dtype)
    B0 = src[:k, :m].clone().requires_grad_(True)
    X0 = ctqr.qr_solve(B0, f)
    (gB,) = torch.autograd.grad(X0, B0, G, retain_graph=True)    # warm-up (first launches of its kernels)
    torch.cuda.synchronize()
    e0.record()
    (gB,) = torch.autograd.grad(X0, B0, G)
    e1.record()
    torch.cuda.synchronize()
    bwd_ms = e0.elapsed_time(e1)
    # the forward solve of the same 64 sinograms, for comparison
    with torch.no_grad():
        e0.record()
        ctqr.qr_solve(B0.detach(), f)
        e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    nd = 4
    D = torch.from_numpy(np.ascontiguousarray(synth.directions(m, nd).T)).to(dev, torch.float64)
    h = 1e-3
    Bpm = torch.zeros((2 * nd, ctqr.ld16(m)), dtype=torch.float64, device=dev)
    with torch.no_grad():
        Bpm[:nd, :m] = B0[:nd].double() + h * D
        Bpm[nd:, :m] = B0[:nd].double() - h * D
    Xpm = torch.zeros((2 * nd, ctqr.ld16(n)), dtype=torch.float64, device=dev)
    ctqr.solve_refined(f, sp, Bpm, Xpm, 4, ctqr.REFINE_SNE)
    torch.cuda.synchronize()
    dx = (Xpm[:nd, :n] - Xpm[nd:, :n]) / (2 * h)
    fd = (dx * G[:nd].double()).sum(dim=1)
    an = (gB[:nd].double() * D).sum(dim=1)
    # errors of <g, S d> and <S^T g, d> scale with ||S^T g|| ||d||, not with
    # the inner product itself (random directions can cancel)
    scale = gB[:nd].double().norm(dim=1) * D.norm(dim=1)
    fd_err = float(((fd - an).abs() / scale).max().item())
    small = small_batch_leg(ctqr, torch, f, src, n)
    return {"sinograms": total, "batches": len(sizes), "graph_slices_per_s": total / (g_ms * 1e-3),
            "eager_slices_per_s": total / (eager_ms * 1e-3), "graph_vs_eager_max_rel_diff": agree,
            "graph_vs_fp64": vs64,
            "adjoint_gradients": k, "adjoint_ms": bwd_ms, "forward_same_slices_ms": fwd_ms, "fd_step": h,
            "fd_err_by_norms": fd_err, "small_batch": small}


def small_batch_leg(ctqr, torch, f, src, n):
    """Latency of a small batch (1 and 8 slices) on the same factor: the
    multi-kernel solve (apply_qt + trsm), the one-launch fused solve, and the
    fused solve captured in a graph over a one-batch descriptor; best of 3,
    after one untimed call (the factor's first fused solve also builds the
    blockdiag(R_qq^-1) R copy its back-substitution reads)."""
    out = {}
    for k in (1, 8):
        B0 = src[:k].clone()
        ws = ctqr.solve_fused(f, B0.clone())
        desc = ctqr.batch_descriptor([k], device=B0.device)
        Bg = B0.clone()
        g = ctqr.SolveGraph(f, Bg, k, desc, fused=True)
        torch.cuda.synchronize()

        def timed(fn):
            best = 1e30
            for _ in range(3):
                B = B0.clone()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn(B)
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1))
            return best, B

        multi_ms, Bm = timed(lambda B: (ctqr.apply_qt(f, B), ctqr.trsm_solve(f, B)))
        fused_ms, Bf = timed(lambda B: ctqr.solve_fused(f, B))
        best = 1e30
        for _ in range(3):
            Bg.copy_(B0)
            desc[0] = 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(g.stream)
            g.launch(g.stream)
            e1.record(g.stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        Xm = Bm[:, :n].double()
        diff = max(float(((X[:, :n].double() - Xm).norm(dim=1) / Xm.norm(dim=1)).max().item()) for X in (Bf, Bg))
        out[str(k)] = {"multi_kernel_ms": multi_ms, "fused_ms": fused_ms, "fused_graph_ms": best,
                       "fused_vs_multi_max_rel_diff": diff}
        del ws, g
    return out


def code_hash(path):
    """SHA-256 prefix of a source file's code: comments and blank lines
    removed, so that editing a comment does not invalidate counters taken
    on the same code."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [l.rstrip() for l in text.split("\n") if l.strip()]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def counted_traffic(prec, dom):
    """HBM bytes per launch of the roofline kernel from the committed
    hardware-counter summary (FETCH_SIZE and WRITE_SIZE passes, scaled by the
    same counters on a plain copy), or None when there is none for this
    kernel or the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "x3dl_update_c3_256_traffic.json")
    if prec != "bf16x3" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2412_07631_amd", "csrc", "gemm_lds.hip")
    if code_hash(src) != rec.get("code_sha256_16"):
        return None
    k = rec.get("sub" if dom == "update_cvw" else "vtc")
    if not k:
        return None
    return {"bytes_per_launch": k["traffic_bytes_per_launch"], "fetch_bytes_per_launch": k["fetch_bytes_per_launch"],
            "write_bytes_per_launch": k["write_bytes_per_launch"], "over_algorithmic":
            k["traffic_bytes_per_launch"] / k["algorithmic_bytes_per_launch"],
            "source": "profiles/x3dl_update_c3_256_traffic.json"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_256")
    ap.add_argument("--prec", default="bf16x3", choices=["f64", "f32", "bf16", "f16", "bf16x3"])
    ap.add_argument("--refine", type=int, default=6, help="refinement steps at most")
    ap.add_argument("--tol", type=float, default=1e-6,
                    help="stop rule: end the refinement once every slice's correction is at most tol relative to "
                         "its image (0: always run --refine steps); the stated bound of the mixed path's image "
                         "error against the FP64 path")
    ap.add_argument("--method", default="sne", choices=["sne", "pcgls", "qr"],
                    help="refinement: semi-normal steps, preconditioned conjugate gradients, or Q^T corrections")
    ap.add_argument("--nrhs", type=int, default=None, help="slices per batch (default: the workload's)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference path")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=2048, help="leading columns in the CPU oracle sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB device copy first (calibrates profiler byte counters)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the uneven-batch graph solve and the adjoint leg on the same factor")
    ap.add_argument("--batched-total", type=int, default=4096, help="sinograms in the uneven-batch leg")
    ap.add_argument("--projector", default="siddon", choices=["siddon", "joseph"],
                    help="system matrix: Siddon's exact lengths or Joseph's interpolation")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_07631_amd import ctqr, synth

    w = synth.WORKLOADS[args.workload]
    sc = synth.workload_scanner(args.workload)
    if args.projector == "joseph":
        import dataclasses
        sc = dataclasses.replace(sc, projector=1)
    m, n = sc.m, sc.n
    nrhs = args.nrhs or w["slices"]
    prec = ctqr.PREC_NAMES[args.prec]
    method = {"sne": ctqr.REFINE_SNE, "pcgls": ctqr.REFINE_PCGLS, "qr": ctqr.REFINE_QR}[args.method]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    log("workload %s: m=%d n=%d nrhs=%d prec=%s refine=%d(%s)" % (args.workload, m, n, nrhs, args.prec,
                                                                  args.refine, args.method))

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    sp = ctqr.SparseA(sc)
    ids = list(range(nrhs))
    Xtrue = synth.phantoms(w["cfg"], sc.n_pix, ids)
    Xt = torch.from_numpy(np.ascontiguousarray(Xtrue.T)).to(dev)
    Xtd = torch.zeros((nrhs, ctqr.ld16(n)), dtype=torch.float64, device=dev)
    Xtd[:, :n] = Xt
    zero = torch.zeros((nrhs, ctqr.ld16(m)), dtype=torch.float64, device=dev)
    Pd = torch.empty_like(zero)
    ctqr.residual(sp.csr, m, Xtd, zero, Pd)          # P = 0 - A x  (noiseless line integrals, negated)
    P = (-Pd[:, :m]).cpu().numpy().T
    B = synth.noisy_sinograms(w["cfg"], P, w["I0"], ids)
    Bd = torch.zeros((nrhs, ctqr.ld16(m)), dtype=torch.float64, device=dev)
    Bd[:, :m] = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    Pnl = torch.zeros_like(Pd)                         # the noiseless sinograms A x (consistent data)
    Pnl[:, :m] = -Pd[:, :m]
    del zero, Pd, P, Xt
    torch.cuda.synchronize()
    log("inputs ready in %.1fs" % (time.time() - t0))

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 1 GiB read + 1 GiB written")

    dt_store = torch.float64 if prec == ctqr.PREC_F64 else torch.float32
    A = torch.empty((n, ctqr.ld16(m)), dtype=dt_store, device=dev)
    X = torch.zeros((nrhs, ctqr.ld16(n)), dtype=torch.float64, device=dev)
    scratch = torch.empty(ctqr.refine_workspace(m, n, nrhs, method), dtype=torch.uint8, device=dev)
    rn = torch.zeros((args.refine + 1) * nrhs, dtype=torch.float64, device=dev)
    gn = torch.zeros((args.refine + 1) * nrhs, dtype=torch.float64, device=dev)

    steps_taken = []

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ctqr.build_system(sc, A)
        sp_step = ctqr.SparseA(sc)
        e[0].record(stream)
        f = ctqr.qr_factor(A, m, n, prec, max_nrhs=nrhs)
        e[1].record(stream)
        e[2].record(stream)
        taken = ctqr.solve_refined(f, sp_step, Bd, X, args.refine, method, scratch=scratch, res_norms=rn,
                                   grad_norms=gn, tol=args.tol)
        e[3].record(stream)
        steps_taken.append(taken)
        info = ctqr.status(f)
        if info != 0:
            raise RuntimeError("factorization reports rank deficiency at column %d" % (info - 1))
        record.append((e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3])))
        return f

    for i in range(args.warmup):
        tw = time.time()
        step([])
        torch.cuda.synchronize()
        log("warmup step %d: %.1fs" % (i, time.time() - tw))

    times = []
    ctqr.profile_begin()
    torch.cuda.synchronize()
    t_start = time.time()
    for i in range(args.steps):
        f = step(times)
        log("step %d: qr %.1f ms, solve+refine %.1f ms" % (i, times[-1][0], times[-1][1]))
    torch.cuda.synchronize()
    wall = time.time() - t_start
    prof = ctqr.profile_end()

    qr_ms = sum(t[0] for t in times)
    sol_ms = sum(t[1] for t in times)
    qr_tflops = qr_flops(m, n) * args.steps / (qr_ms * 1e-3) / 1e12
    slices_per_s = nrhs * args.steps / (sol_ms * 1e-3)
    taken = steps_taken[-1]
    rnorm = rn.view(args.refine + 1, nrhs).cpu().numpy()[: taken + 1]
    gnorm = gn.view(args.refine + 1, nrhs).cpu().numpy()[: taken + 1]
    bnorm = np.linalg.norm(B, axis=0)
    Xm = X[:, :n].cpu().numpy().T.copy()

    def ev_pair():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def paper_residual(Xd, Bsrc):
        """||A X - B||_F / ||B||_F in FP64 with the CSR copy of A (Tables 2, 6, 8)."""
        R = torch.empty_like(Bsrc)
        ctqr.residual(sp.csr, m, Xd, Bsrc, R)
        return float((R[:, :m].norm() / Bsrc[:, :m].norm()).item())

    def errs_vs(Xa, Xref):
        """Per-slice relative image error and max pixel error (Sec. 3.1)."""
        d = (Xa[:, :n] - Xref[:, :n])
        e = d.norm(dim=1) / Xref[:, :n].norm(dim=1)
        return {"rel_err_max": float(e.max().item()), "rel_err_median": float(e.median().item()),
                "max_abs_pixel_err": float(d.abs().max().item())}

    def plain_solve(fac, Bsrc):
        """X = R^-1 Q^T B in the factor's storage precision (Eq. (solve)); ms."""
        Bs = Bsrc.to(fac.dtype, copy=True)
        e0, e1 = ev_pair()
        e0.record(stream)
        ctqr.apply_qt(fac, Bs)
        ctqr.trsm_solve(fac, Bs)
        e1.record(stream)
        torch.cuda.synchronize()
        Xo = torch.zeros((Bs.shape[0], ctqr.ld16(n)), dtype=torch.float64, device=dev)
        Xo[:, :n] = Bs[:, :n].double()
        return Xo, e0.elapsed_time(e1)

    # refined headline path on the noiseless sinograms (consistent data, as
    # the paper's projected references): the paper-style residual
    Xnl = torch.zeros_like(X)
    ctqr.solve_refined(f, sp, Pnl, Xnl, args.refine, method, scratch=scratch, tol=args.tol)
    torch.cuda.synchronize()
    headline_residual_noiseless = paper_residual(Xnl, Pnl)

    # -------------------------------------------------- plain FP64 GPU path
    fp64 = None
    X64d = None
    if not args.no_fp64 and prec != ctqr.PREC_F64:
        A64 = torch.empty((n, ctqr.ld16(m)), dtype=torch.float64, device=dev)
        ctqr.build_system(sc, A64)
        e0, e1 = ev_pair()
        e0.record(stream)
        f64 = ctqr.qr_factor(A64, m, n, ctqr.PREC_F64, max_nrhs=nrhs)
        e1.record(stream)
        torch.cuda.synchronize()
        qr64_ms = e0.elapsed_time(e1)
        X64d, sol64_ms = plain_solve(f64, Bd)
        X64nl, _ = plain_solve(f64, Pnl)
        fp64 = {"qr_tflops": qr_flops(m, n) / (qr64_ms * 1e-3) / 1e12, "qr_ms": qr64_ms,
                "qr_tflops_frac_of_peak": qr_flops(m, n) / (qr64_ms * 1e-3) / 1e12 / PEAK_TFLOPS["f64"],
                "slices_per_s": nrhs / (sol64_ms * 1e-3), "solve_ms": sol64_ms,
                "residual_noiseless": paper_residual(X64nl, Pnl),
                "noiseless_rel_err_vs_phantom": errs_vs(X64nl, Xtd)["rel_err_max"]}
        del A64, f64, X64nl
        torch.cuda.empty_cache()
        log("fp64 path: qr %.1f ms (%.2f TFLOP/s), solve %.1f slices/s, noiseless residual %.3g" % (
            fp64["qr_ms"], fp64["qr_tflops"], fp64["slices_per_s"], fp64["residual_noiseless"]))

    headline_vs_fp64 = errs_vs(X, X64d) if X64d is not None else None
    # the headline path's error against the FP64 path after each number of
    # refinement steps (untimed; s = 0 is the plain low-precision solve)
    err_by_step = None
    if X64d is not None:
        err_by_step = []
        Xs_ = torch.zeros_like(X)
        for s_ in range(args.refine + 1):
            ctqr.solve_refined(f, sp, Bd, Xs_, s_, method, scratch=scratch)
            err_by_step.append(errs_vs(Xs_, X64d)["rel_err_max"])
        del Xs_
        log("error against the FP64 path by refinement step: " + " ".join("%.2e" % v for v in err_by_step))
    noiseless_vs_fp64 = None

    # ------------------------------------------------------ plain FP32 path
    fp32 = None
    f32 = None
    if not args.no_fp32 and prec != ctqr.PREC_F32:
        A32 = torch.empty((n, ctqr.ld16(m)), dtype=torch.float32, device=dev)
        ctqr.build_system(sc, A32)
        e0, e1 = ev_pair()
        e0.record(stream)
        f32 = ctqr.qr_factor(A32, m, n, ctqr.PREC_F32, max_nrhs=nrhs)
        e1.record(stream)
        torch.cuda.synchronize()
        qr32_ms = e0.elapsed_time(e1)
        X32, sol32_ms = plain_solve(f32, Bd)
        X32nl, _ = plain_solve(f32, Pnl)
        X32r = torch.zeros_like(X)
        e0, e1 = ev_pair()
        e0.record(stream)
        ctqr.solve_refined(f32, sp, Bd, X32r, 3, ctqr.REFINE_SNE, scratch=scratch)
        e1.record(stream)
        torch.cuda.synchronize()
        ref32_ms = e0.elapsed_time(e1)
        fp32 = {"qr_tflops": qr_flops(m, n) / (qr32_ms * 1e-3) / 1e12, "qr_ms": qr32_ms,
                "qr_tflops_frac_of_peak": qr_flops(m, n) / (qr32_ms * 1e-3) / 1e12 / PEAK_TFLOPS["f32"],
                "slices_per_s": nrhs / (sol32_ms * 1e-3), "solve_ms": sol32_ms,
                "residual_noiseless": paper_residual(X32nl, Pnl),
                "refined3_slices_per_s": nrhs / (ref32_ms * 1e-3)}
        if X64d is not None:
            fp32["vs_fp64"] = errs_vs(X32, X64d)
            fp32["refined3_vs_fp64"] = errs_vs(X32r, X64d)
        del X32, X32nl, X32r
        log("fp32 path: qr %.1f ms (%.2f TFLOP/s), solve %.1f slices/s, noiseless residual %.3g" % (
            fp32["qr_ms"], fp32["qr_tflops"], fp32["slices_per_s"], fp32["residual_noiseless"]))

    # ------------- the same solve with B handed over in pinned host memory
    # (the timed region starts with B in host RAM: its H2D copy is included)
    Bh = torch.empty(Bd.shape, dtype=Bd.dtype, pin_memory=True)
    Bh.copy_(Bd)
    Bd2 = torch.empty_like(Bd)
    hev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    hev[0].record(stream)
    Bd2.copy_(Bh, non_blocking=True)
    ctqr.solve_refined(f, sp, Bd2, X, args.refine, method, scratch=scratch, tol=args.tol)
    hev[1].record(stream)
    torch.cuda.synchronize()
    h2d_ms = hev[0].elapsed_time(hev[1])
    slices_per_s_h2d = nrhs / (h2d_ms * 1e-3)
    del Bh, Bd2
    log("with B from pinned host memory: %.1f slices/s (%.1f ms)" % (slices_per_s_h2d, h2d_ms))

    # -------------------------------- image quality against the phantoms
    # full image and the edge crop (the 512^2 margins of 130 rows at the
    # bottom and 100 pixels elsewhere, scaled to the image size)
    Np = sc.n_pix
    crop = (round(130 * Np / 512), round(100 * Np / 512), round(100 * Np / 512), round(100 * Np / 512))
    qev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def metrics(Xd, c):
        q = ctqr.quality(Xd, Xtd, Np, crop=c).cpu().numpy()
        return {"snr_db": float(q[:, 0].mean()), "mse": float(q[:, 1].mean()), "psnr_db": float(q[:, 2].mean()),
                "ssim": float(q[:, 3].mean())}

    qev[0].record(stream)
    ctqr.quality(X, Xtd, Np)
    qev[1].record(stream)
    torch.cuda.synchronize()
    quality = {"crop_bottom_top_left_right": list(crop), "kernel_ms": qev[0].elapsed_time(qev[1]),
               "slices": nrhs, "refined": metrics(X, None), "refined_cropped": metrics(X, crop),
               "noiseless_refined": metrics(Xnl, None), "noiseless_refined_cropped": metrics(Xnl, crop)}
    if X64d is not None:
        quality["fp64"] = metrics(X64d, None)
        quality["fp64_cropped"] = metrics(X64d, crop)
    log("quality (mean over %d slices): refined SNR %.2f dB, SSIM %.4f; cropped SSIM %.4f; noiseless SNR %.1f dB, "
        "SSIM %.6f; %.2f ms" % (nrhs, quality["refined"]["snr_db"], quality["refined"]["ssim"],
                                quality["refined_cropped"]["ssim"], quality["noiseless_refined"]["snr_db"],
                                quality["noiseless_refined"]["ssim"], quality["kernel_ms"]))
    del Xnl, Pnl

    # ------------------------------------- uneven batches and the adjoint
    # (on the FP32 factor: a plain FP32 solve meets the FP32 path's
    # tolerance, which a plain solve on a bfloat16-based factor does not)
    batched = None
    if not args.no_batched:
        fb = f32 if f32 is not None else f
        batched = batched_leg(ctqr, synth, torch, fb, sc, Bd, dev, args.batched_total, sp, X64d)
        batched["factor"] = "f32" if f32 is not None else args.prec
        for k, v in batched["small_batch"].items():
            log("%s slice(s): multi-kernel solve %.2f ms, fused %.2f ms, fused graph %.2f ms (max rel diff %.1e)" % (
                k, v["multi_kernel_ms"], v["fused_ms"], v["fused_graph_ms"], v["fused_vs_multi_max_rel_diff"]))
    del f32

    # ------------------------------------------------------ roofline (live)
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    achieved = d["flop"] / (d["ms"] * 1e-3) / 1e12 if d["ms"] > 0 else 0.0
    peak = PEAK_TFLOPS[args.prec]
    tname = {"f64": "gemm_nt_kernel<double, %s, 128>", "f32": "gemm_nt_kernel<float, %s, 128>",
             "bf16": "gemm_nt_lp_kernel<2, %s, false, false>", "f16": "gemm_nt_lp_kernel<3, %s, false, false>",
             "bf16x3": "gemm_nt_lp_kernel<4, %s>"}[args.prec]
    if args.prec == "bf16x3":
        # 1024-wide blocks: the direct-to-LDS kernel on 256 x 256 tiles; both
        # operands of C -= V W' arrive split into bfloat16 halves, V of
        # W = V^T C too, while C is split as it is read
        tname = "gemm_x3_dl_kernel<DlCfg<8, 4, 2, 4, 2, 1>, %s>"
        kname = (tname % "true, false, false") + " (C -= V W')" if dom == "update_cvw" else \
            (tname % "false, false, true") + " (W = V^T C)"
    else:
        kname = (tname % "true") + " (C -= V W')" if dom == "update_cvw" else (tname % "false") + " (W = V^T C)"
    # the kernel's own bound: its algorithmic flop per algorithmic byte
    # against the balance of the MFMA rate it can reach (the dtype's peak over
    # the MFMA products it issues per method product) and 8 TB/s of HBM; the
    # fraction is always taken against the dtype's own MFMA peak
    issue = ISSUE_FACTOR[args.prec]
    intensity = d["flop"] / d["bytes"] if d["bytes"] > 0 else float("inf")
    ridge = peak / issue * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity >= ridge:
        bound = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        bound = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    if issue > 1:
        bound["mfma_issue"] = {"products_per_method_product": issue, "tflops": achieved * issue,
                               "frac_of_peak": achieved * issue / peak}
    roofline = {**bound, "kernel": kname, "flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                "launches": d["launches"], "avg_launch_ms": d["ms"] / max(d["launches"], 1),
                "algorithmic_bytes_per_launch": d["bytes"] / max(d["launches"], 1),
                "algorithmic_gbs": d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0,
                "traffic": counted_traffic(args.prec, dom),
                "other_kernel": {k: {"tflops": prof[k]["flop"] / (prof[k]["ms"] * 1e-3) / 1e12 if prof[k]["ms"] else 0,
                                     "ms": prof[k]["ms"]} for k in prof if k != dom}}

    # --------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        k = min(args.cpu_cols, n)
        row_ptr, col, val = O.system_csr(sc)
        Ablk = np.zeros((m, k), dtype=np.float64, order="F")
        rows = np.repeat(np.arange(m), np.diff(row_ptr))
        sel = col < k
        Ablk[rows[sel], col[sel]] = val[sel]
        tc = time.time()
        O.householder_qr(Ablk)
        tcpu = time.time() - tc
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": qr_flops(m, k) / tcpu / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
               "sample": "unblocked FP64 Householder QR of the leading %d x %d column block of the same A (%.1f s)"
                         % (m, k, tcpu)}
        log("cpu oracle sample: %.3g TFLOP/s on %d cores (%.1fs)" % (cpu["value"], cores, tcpu))

    out = {
        "metric": METRIC,
        "value": qr_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic (seeded random-ellipse phantoms, Poisson noise)",
        "config": {"workload": "%s: %dx%d image, %d views x %d bins (m=%d, n=%d), %d noisy slices, I0=%g"
                               % (args.workload, sc.n_pix, sc.n_pix, sc.n_angles, sc.n_det, m, n, nrhs, w["I0"]),
                   "global_batch": nrhs, "precision": args.prec, "refine_steps_max": args.refine,
                   "refine_tol": args.tol, "refine_method": args.method, "projector": args.projector},
        "qr_ms": qr_ms / args.steps,
        "qr_tflops_frac_of_peak": qr_tflops / peak,
        "slices_per_s": slices_per_s,
        "solve_ms": sol_ms / args.steps,
        "slices_per_s_incl_h2d": slices_per_s_h2d,
        "refine_steps_taken": steps_taken,
        "vs_fp64": headline_vs_fp64,
        "vs_fp64_rel_err_by_step": err_by_step,
        "slices_per_s_vs_fp64_path": slices_per_s / fp64["slices_per_s"] if fp64 else None,
        "residual_noiseless": headline_residual_noiseless,
        "residual_rel_final": float(np.max(rnorm[-1] / bnorm)),
        "ls_grad_norm_by_step": [float(np.max(gnorm[s])) for s in range(len(gnorm))],
        "fp64_path": fp64,
        "fp32_path": fp32,
        "quality": quality,
        "batched": batched,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
