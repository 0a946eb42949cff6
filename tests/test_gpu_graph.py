"""Graph-captured solves over a device batch descriptor (uneven batches) and
the solve autotuner.  Every replay is checked; eager work and host
synchronisation run between replays."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import ld16, max_col_rel

pytestmark = pytest.mark.gpu

SIZES = [1, 17, 5, 33, 8, 36, 2, 64]            # uneven batches, 166 columns


@pytest.fixture(scope="module")
def setup():
    from paper_2412_07631_amd import ctqr
    sc = synth.scanner(48, 40, 84)
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ctqr.build_system(sc, Ad)
    f = ctqr.qr_factor(Ad, sc.m, sc.n, ctqr.PREC_F32, max_nrhs=64)
    total = sum(SIZES)
    B = synth.noisy_sinograms(6, A @ synth.phantoms(6, sc.n_pix, range(total)), 5e4, range(total))
    return ctqr, sc, A, VR, tau, f, B


def bucket_max(c):
    return 8 if c <= 8 else 32 if c <= 32 else 64


def test_graph_uneven_batches(setup):
    ctqr, sc, A, VR, tau, f, B = setup
    total = B.shape[1]
    Bd = torch.zeros((total, ld16(sc.m)), dtype=torch.float32, device="cuda")
    src = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda", torch.float32)
    desc = ctqr.batch_descriptor(SIZES)
    graphs = {mc: ctqr.SolveGraph(f, Bd, mc, desc) for mc in (8, 32, 64)}
    Xs = O.solve(VR, tau, B)
    # eager reference, batch by batch
    ref = torch.zeros_like(Bd)
    ref[:, :sc.m] = src
    off = 0
    for c in SIZES:
        blk = ref[off:off + c].clone()
        ctqr.apply_qt(f, blk)
        ctqr.trsm_solve(f, blk)
        ref[off:off + c] = blk
        off += c
    eager = ref[:, :sc.n].double().cpu().numpy().T
    junk = torch.randn(512, 512, device="cuda")
    for replay in range(2):
        Bd[:, :sc.m] = src
        desc[0] = 0
        torch.cuda.synchronize()
        for k, c in enumerate(SIZES):
            graphs[bucket_max(c)].launch(graphs[bucket_max(c)].stream)
            graphs[bucket_max(c)].stream.synchronize()
            junk = junk @ junk.T * 1e-3            # unrelated eager work between replays
            torch.cuda.synchronize()
        X = Bd[:, :sc.n].double().cpu().numpy().T
        assert int(desc[0].item()) == len(SIZES)
        assert max_col_rel(X, eager) <= 1e-5, replay
        assert max_col_rel(X, Xs) <= 1e-4, replay


def test_autotuner_keeps_results_correct(setup, tmp_path):
    ctqr, sc, A, VR, tau, f, B = setup
    scratch = torch.zeros((64, ld16(sc.m)), dtype=torch.float32, device="cuda")
    cache = str(tmp_path / "tune.json")
    ctqr.autotune_solve(f, scratch, 64, cache)
    with open(cache) as fh:
        entries = json.load(fh)
    assert len(entries) >= 3
    for key, (bq, split) in entries.items():
        assert key.startswith("gfx950/f32/%d/%d/" % (sc.m, sc.n))
        assert bq in (16, 32, 64, 128) and split > 0
    ctqr.autotune_solve(f, scratch, 64, cache)          # cached: no re-timing, same file
    with open(cache) as fh:
        assert json.load(fh) == entries
    Bd = torch.zeros((9, ld16(sc.m)), dtype=torch.float32, device="cuda")
    Bd[:, :sc.m] = torch.from_numpy(np.ascontiguousarray(B[:, :9].T)).to("cuda", torch.float32)
    ctqr.apply_qt(f, Bd)
    ctqr.trsm_solve(f, Bd)
    X = Bd[:, :sc.n].double().cpu().numpy().T
    assert max_col_rel(X, O.solve(VR, tau, B[:, :9])) <= 1e-4


def test_graph_launch_past_end_and_invalid_entry_solve_nothing(setup):
    """A launch after the last batch, and one whose entry lies outside B or
    exceeds the graph's column cap, leave B untouched; ct_status then reports
    -2003 once.  The cursor never moves past the batch count."""
    ctqr, sc, A, VR, tau, f, B = setup
    cols = 12
    Bd = torch.zeros((cols, ld16(sc.m)), dtype=torch.float32, device="cuda")
    Bd[:, :sc.m] = torch.from_numpy(np.ascontiguousarray(B[:, :cols].T)).to("cuda", torch.float32)
    desc = ctqr.batch_descriptor([4, 8])
    g = ctqr.SolveGraph(f, Bd, 8, desc)
    for _ in range(2):
        g.launch(g.stream)
    g.stream.synchronize()
    assert int(desc[0].item()) == 2
    assert ctqr.status(f) == 0
    solved = Bd.clone()
    # two launches past the end: nothing changes, the cursor stays at 2
    for _ in range(2):
        g.launch(g.stream)
    g.stream.synchronize()
    assert int(desc[0].item()) == 2
    assert torch.equal(Bd, solved)
    with pytest.raises(ctqr.CtError) as ei:
        ctqr.status(f)
    assert ei.value.code == -2003
    assert ctqr.status(f) == 0                     # reported once
    # entries outside B (offset + count > columns) or above the cap of 8
    for bad in ([[6, 7]], [[0, 9]], [[-1, 2]]):
        d = torch.tensor([0, 1] + bad[0], dtype=torch.int32, device="cuda")
        gb = ctqr.SolveGraph(f, Bd, 8, d)
        gb.launch(gb.stream)
        gb.stream.synchronize()
        assert torch.equal(Bd, solved), bad
        assert int(d[0].item()) == 1
        with pytest.raises(ctqr.CtError) as ei:
            ctqr.status(f)
        assert ei.value.code == -2003
