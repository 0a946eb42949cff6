"""ct_solve_refined_noalloc: the refined solve on the library's static scratch
gives what ct_solve_refined gives with a caller workspace, on consecutive
calls whose sizes shrink (the static array keeps the previous call's data)."""
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
    assert torch.cuda.is_available()
    return ctqr


def _solve_both(ct, f, sp, Bd, nrhs, steps, method):
    n = f.n
    out = []
    for noalloc in (True, False):
        Xd = torch.full((nrhs, ld16(n)), float("nan"), dtype=torch.float64, device="cuda")
        rn = torch.zeros((steps + 1) * nrhs, dtype=torch.float64, device="cuda")
        gn = torch.zeros((steps + 1) * nrhs, dtype=torch.float64, device="cuda")
        if noalloc:
            ct.solve_refined_noalloc(f, sp, Bd, Xd, steps, method, nrhs=nrhs, res_norms=rn, grad_norms=gn)
        else:
            ct.solve_refined(f, sp, Bd, Xd, steps, method, nrhs=nrhs, res_norms=rn, grad_norms=gn)
        torch.cuda.synchronize()
        out.append((Xd[:, :n].clone(), rn.clone(), gn.clone()))
    return out


@pytest.mark.parametrize("prec,steps,method", [("bf16x3", 4, 1), ("f32", 3, 0)])
def test_noalloc_matches_workspace_entry_point(ct, prec, steps, method):
    sc = synth.scanner(48, 40, 84)                       # 3360 x 2304
    A64 = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A64)
    assert info == 0
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=64)
    assert ct.status(f) == 0
    sp = ct.SparseA(sc)
    _, _, B = sinograms(sc, A64, 5, 52, 5e4)
    Bd = to_dev(B, torch.float64)
    # 52 slices (the BF16x3 block products of the refinement), then 5 on the
    # same static scratch, which then still holds the first call's vectors
    for nrhs in (52, 5):
        (Xa, rna, gna), (Xb, rnb, gnb) = _solve_both(ct, f, sp, Bd[:nrhs], nrhs, steps, method)
        assert ct.status(f) == 0
        assert torch.equal(Xa, Xb), "static-scratch solve differs from the workspace solve"
        assert torch.equal(rna, rnb) and torch.equal(gna, gnb)
        Xs = O.solve(VR, tau, B[:, :nrhs])
        err = max_col_rel(from_dev(Xa, sc.n), Xs)
        print(prec, "nrhs", nrhs, "max rel err vs oracle %.3g" % err)
        assert err <= (1e-10 if method == 1 else 1e-4)


def test_noalloc_rejects_sizes_beyond_the_static_scratch(ct):
    sc = synth.scanner(32, 30, 64)                       # 1920 x 1024: 2080 slices fit in 128 MiB
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F32, max_nrhs=2100)
    sp = ct.SparseA(sc)
    assert ct.refine_workspace(sc.m, sc.n, 2080) <= (128 << 20) < ct.refine_workspace(sc.m, sc.n, 2081)
    Bd = torch.zeros((2081, ld16(sc.m)), dtype=torch.float64, device="cuda")
    Xd = torch.full((2081, ld16(sc.n)), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ct.CtError) as e:
        ct.solve_refined_noalloc(f, sp, Bd, Xd, 2, ct.REFINE_SNE, nrhs=2081)
    assert e.value.code == -7 and "static" in str(e.value)
    torch.cuda.synchronize()
    assert bool((Xd == 7.0).all()), "a rejected call must launch nothing"
