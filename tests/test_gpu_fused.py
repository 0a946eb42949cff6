"""The persistent fused solve (one launch: Q^T, then R^{-1} by published
256-row blocks) against the FP64 oracle and against the multi-kernel solve of
the same factor, eager and graph-captured over uneven batches."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import to_dev, from_dev, max_col_rel, sinograms, ld16

pytestmark = pytest.mark.gpu

# (N, views, bins): ragged is 1400 x 900 (last outer block 132 columns, last
# 256-row block of R 132 rows), multi 3360 x 2304
GEOMS = {"ragged": (30, 28, 50), "multi": (48, 40, 84)}
_cache = {}


@pytest.fixture(scope="module")
def ct():
    from paper_2412_07631_amd import ctqr
    assert torch.cuda.is_available()
    return ctqr


def problem(name):
    if name not in _cache:
        sc = synth.scanner(*GEOMS[name])
        A = O.system_dense(sc)
        VR, tau, info = O.householder_qr(A)
        assert info == 0
        _cache[name] = (sc, A, VR, tau)
    return _cache[name]


def factor(ct, sc, prec, max_nrhs, block_width=0):
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=dt, device="cuda")
    ct.build_system(sc, Ad)
    ct.debug_block_width(block_width)
    try:
        f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=max_nrhs)
    finally:
        ct.debug_block_width(0)
    assert ct.status(f) == 0
    return f, dt


@pytest.mark.parametrize("name", ["ragged", "multi"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("nrhs", [1, 17, 37])
def test_fused_solve_matches_oracle(ct, name, prec, nrhs):
    """One launch gives the oracle's least-squares images (FP64 1e-10, FP32
    storage 1e-4) and agrees with the multi-kernel solve of the same factor
    (FP64 1e-12; FP32 storage 5e-5: two FP32 solves, each about 1e-5 from
    the oracle at these sizes); 37 columns take two chunks (three for FP64)."""
    sc, A, VR, tau = problem(name)
    _, P, B = sinograms(sc, A, 3, nrhs, 5e4)
    Xs = O.solve(VR, tau, B)
    f, dt = factor(ct, sc, prec, max(8, nrhs))
    Bd = to_dev(B, dt)
    ct.solve_fused(f, Bd)
    assert ct.status(f) == 0
    X = from_dev(Bd, sc.n)
    err = max_col_rel(X, Xs)
    B2 = to_dev(B, dt)
    ct.apply_qt(f, B2)
    ct.trsm_solve(f, B2)
    diff = max_col_rel(X, from_dev(B2, sc.n))
    print(name, prec, nrhs, "fused vs oracle %.3g, vs multi-kernel %.3g" % (err, diff))
    assert err <= (1e-10 if prec == "f64" else 1e-4)
    assert diff <= (1e-12 if prec == "f64" else 5e-5)
    # rows n..m-1 hold the least-squares residual components, like ct_apply_qt's
    assert np.allclose(from_dev(Bd, sc.m)[sc.n:], from_dev(B2, sc.m)[sc.n:], rtol=0,
                       atol=(1e-12 if prec == "f64" else 5e-5) * np.abs(B).max())


@pytest.mark.parametrize("bw", [96, 1024])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_solve_block_widths(ct, bw, prec):
    """Outer blocks of 96 columns (one partial column group) and of 1024
    (eight column groups, a 256-wide last block), as at 256^2."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 3, 6, 5e4)
    Xs = O.solve(VR, tau, B)
    f, dt = factor(ct, sc, prec, 8, bw)
    Bd = to_dev(B, dt)
    ct.solve_fused(f, Bd)
    assert ct.status(f) == 0
    err = max_col_rel(from_dev(Bd, sc.n), Xs)
    print("block width", bw, prec, "fused vs oracle %.3g" % err)
    assert err <= (1e-10 if prec == "f64" else 1e-4)


def test_fused_solve_refuses_lean_factor(ct):
    sc, A, VR, tau = problem("ragged")
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F32, max_nrhs=8, solve_copies=False)
    Bd = torch.zeros((2, ld16(sc.m)), dtype=torch.float32, device="cuda")
    with pytest.raises(ct.CtError) as e:
        ct.solve_fused(f, Bd)
    assert e.value.code == -2007
    assert ct.status(f) == 0


SIZES = [1, 17, 5, 33, 8, 36, 2, 64]            # uneven batches, 166 columns


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_graph_uneven_batches(ct, prec):
    """The graph of one fused launch per batch walks the descriptor: every
    replay (two, with unrelated eager work in between) matches the eager fused
    solve batch by batch bitwise and the oracle; a launch past the last batch
    solves nothing and is reported by ct_status."""
    sc, A, VR, tau = problem("multi")
    total = sum(SIZES)
    B = synth.noisy_sinograms(6, A @ synth.phantoms(6, sc.n_pix, range(total)), 5e4, range(total))
    Xs = O.solve(VR, tau, B)
    f, dt = factor(ct, sc, prec, 64)
    src = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda", dt)
    ref = torch.zeros((total, ld16(sc.m)), dtype=dt, device="cuda")
    ref[:, :sc.m] = src
    off = 0
    for c in SIZES:
        blk = ref[off:off + c].clone()
        ct.solve_fused(f, blk)
        ref[off:off + c] = blk
        off += c
    eager = ref[:, :sc.n].double().cpu().numpy().T
    Bd = torch.zeros_like(ref)
    desc = ct.batch_descriptor(SIZES)
    g = ct.SolveGraph(f, Bd, 64, desc, fused=True)
    junk = torch.randn(256, 256, device="cuda")
    for replay in range(2):
        Bd[:, :sc.m] = src
        desc[0] = 0
        torch.cuda.synchronize()
        for _ in SIZES:
            g.launch(g.stream)
            g.stream.synchronize()
            junk = junk @ junk.T * 1e-3
            torch.cuda.synchronize()
        X = Bd[:, :sc.n].double().cpu().numpy().T
        assert int(desc[0].item()) == len(SIZES)
        assert np.array_equal(X, eager), replay
        assert max_col_rel(X, Xs) <= (1e-10 if prec == "f64" else 1e-4), replay
    assert ct.status(f) == 0
    before = Bd.clone()
    g.launch(g.stream)
    g.stream.synchronize()
    assert torch.equal(Bd, before)
    with pytest.raises(ct.CtError) as e:
        ct.status(f)
    assert e.value.code == -2003


def test_fused_wait_limit_fails_fast_and_recovers(ct):
    """With the wait limit forced to zero from the host, the fused solve's
    grid barriers and flag waits give up at once: the launch ends (no hang)
    and ct_status reports -2006 once; with the default limit restored the
    next fused solve is correct."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 3, 5, 5e4)
    Xs = O.solve(VR, tau, B)
    f, dt = factor(ct, sc, "f32", 8)
    ct.debug_wait_limit(0)
    try:
        Bd = to_dev(B, dt)
        ct.solve_fused(f, Bd)
        with pytest.raises(ct.CtError) as e:
            ct.status(f)
        assert e.value.code == -2006
    finally:
        ct.debug_wait_limit(-1)
    assert ct.status(f) == 0
    Bd = to_dev(B, dt)
    ct.solve_fused(f, Bd)
    assert ct.status(f) == 0
    assert max_col_rel(from_dev(Bd, sc.n), Xs) <= 1e-4


def test_fused_solve_many_quarters_per_workgroup(ct):
    """144 x 144 pixels (n = 20736, 81 row blocks of R, 324 quarters of 64
    rows): more quarters than workgroups, so some workgroups own two in the
    back-substitution of 1..8 columns.  No oracle at this size: the fused solve
    is checked against the multi-kernel solve of the same FP32 factor (itself
    checked against the oracle above), 1e-4 per column, and against A x = b
    through the normal equations of a consistent right-hand side."""
    sc = synth.scanner(144, 100, 300)
    m, n = sc.m, sc.n
    Ad = torch.empty((n, ld16(m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    A64 = Ad[:, :m].double()
    f = ct.qr_factor(Ad, m, n, ct.PREC_F32, max_nrhs=8)
    assert ct.status(f) == 0
    g = torch.Generator(device="cpu").manual_seed(7)
    Xt = torch.rand((8, n), generator=g, dtype=torch.float64).to("cuda")
    Bt = Xt @ A64                                    # rows: A x for 8 images
    for k in (1, 8):
        Bf = torch.zeros((k, ld16(m)), dtype=torch.float32, device="cuda")
        Bf[:, :m] = Bt[:k].float()
        Bm = Bf.clone()
        ct.solve_fused(f, Bf)
        ct.apply_qt(f, Bm)
        ct.trsm_solve(f, Bm)
        assert ct.status(f) == 0
        Xf, Xm = Bf[:, :n].double(), Bm[:, :n].double()
        diff = ((Xf - Xm).norm(dim=1) / Xm.norm(dim=1)).max().item()
        err = ((Xf - Xt[:k]).norm(dim=1) / Xt[:k].norm(dim=1)).max().item()
        print("n", n, "columns", k, "fused vs multi-kernel %.3g, vs the exact images %.3g" % (diff, err))
        assert diff <= 1e-4
        assert err <= 1e-2
