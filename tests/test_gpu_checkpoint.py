"""Checkpoint of a factor: save, load into new buffers, and the loaded factor
gives bitwise the solves of the saved one; damaged files are refused."""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import to_dev, from_dev, max_col_rel, sinograms, ld16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct():
    from paper_2412_07631_amd import ctqr
    return ctqr


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_save_load_round_trip(ct, prec, tmp_path):
    sc = synth.scanner(48, 40, 84)
    A = O.system_dense(sc)
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=dt, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=16)
    assert ct.status(f) == 0
    path = str(tmp_path / ("factor_%s.bin" % prec))
    ct.factor_save(f, path)
    m, n, p, wb = ct.factor_file_info(path, 16)
    assert (m, n, p) == (sc.m, sc.n, ct.PREC_NAMES[prec])
    g = ct.factor_load(path, max_nrhs=16)
    assert ct.status(g) == 0
    assert torch.equal(g.A[:, : sc.m], f.A[:, : sc.m]) and torch.equal(g.tau, f.tau)
    _, P, B = sinograms(sc, A, 1, 5, 1e5)
    outs = []
    for h in (f, g):
        Bd = to_dev(B, dt)
        ct.apply_qt(h, Bd)
        ct.trsm_solve(h, Bd)
        outs.append(Bd.clone())
    assert torch.equal(outs[0], outs[1])
    # and the loaded factor solves the least-squares problem like the oracle
    VR, tau, _ = O.householder_qr(A)
    err = max_col_rel(from_dev(outs[1], sc.n), O.solve(VR, tau, B))
    assert err <= (1e-10 if prec == "f64" else 1e-3)
    # the adjoint uses the same copies
    G = torch.from_numpy(np.ascontiguousarray(synth.gradients(sc.n, 3).T)).to("cuda", dt)
    Gd = torch.zeros((3, ld16(sc.n)), dtype=dt, device="cuda")
    Gd[:, : sc.n] = G
    ys = []
    for h in (f, g):
        Y = torch.empty((3, ld16(sc.m)), dtype=dt, device="cuda")
        ct.solve_backward(h, Gd, Y)
        ys.append(Y[:, : sc.m].clone())
    assert torch.equal(ys[0], ys[1])


def test_damaged_files_are_refused(ct, tmp_path):
    sc = synth.scanner(32, 30, 64)
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F32, max_nrhs=4)
    path = str(tmp_path / "f.bin")
    ct.factor_save(f, path)
    raw = open(path, "rb").read()
    flipped = bytearray(raw)
    flipped[len(raw) // 2] ^= 0x10                      # one bit in V\R
    bad = str(tmp_path / "flipped.bin")
    open(bad, "wb").write(bytes(flipped))
    short = str(tmp_path / "short.bin")
    open(short, "wb").write(raw[:-9])                   # truncated checksum
    for p in (bad, short):
        with pytest.raises(ct.CtError) as ei:
            ct.factor_load(p, max_nrhs=4)
        assert ei.value.code == -1
    # a good file still loads after the refusals
    g = ct.factor_load(path, max_nrhs=4)
    assert torch.equal(g.A[:, : sc.m], f.A[:, : sc.m])
