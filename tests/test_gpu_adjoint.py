"""Adjoint of the solve behind torch.autograd: grad_b = Q R^{-T} g, checked
against the oracle's adjoint, the dot-product identity and central finite
differences (the map b -> x is linear, so differences carry rounding only)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import ld16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2412_07631_amd import ctqr
    sc = synth.scanner(48, 40, 84)
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    assert info == 0
    out = {"ct": ctqr, "sc": sc, "A": A, "VR": VR, "tau": tau}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        Ad = torch.empty((sc.n, ld16(sc.m)), dtype=dt, device="cuda")
        ctqr.build_system(sc, Ad)
        out[prec] = ctqr.qr_factor(Ad, sc.m, sc.n, ctqr.PREC_NAMES[prec], max_nrhs=64)
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_autograd_matches_oracle_adjoint(setup, prec, tol):
    ct, sc = setup["ct"], setup["sc"]
    f = setup[prec]
    dt = f.dtype
    g = synth.gradients(sc.n, 8)                       # upstream gradients, FP32 values
    _, P, B = None, None, synth.noisy_sinograms(4, setup["A"] @ synth.phantoms(4, sc.n_pix, range(8)), 5e4, range(8))
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda", dt).requires_grad_(True)
    X = ct.qr_solve(Bt, f)
    X.backward(torch.from_numpy(np.ascontiguousarray(g.T)).to("cuda", dt))
    grad = Bt.grad.double().cpu().numpy().T
    ref = O.adjoint(setup["VR"], setup["tau"], g)
    err = max(np.linalg.norm(grad[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]) for c in range(8))
    assert err <= tol, err


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_dot_product_identity(setup, prec, tol):
    """<x(db), g> = <db, grad_b(g)> on the GPU path itself.  The rounding
    error of either side is bounded relative to ||x|| ||g|| (respectively
    ||db|| ||grad_b||), not to the inner product itself, which can cancel."""
    ct, sc, f = setup["ct"], setup["sc"], setup[prec]
    rng = np.random.default_rng(12)
    db = torch.from_numpy(rng.standard_normal((4, sc.m))).to("cuda", f.dtype).requires_grad_(True)
    g = torch.from_numpy(rng.standard_normal((4, sc.n))).to("cuda", f.dtype)
    x = ct.qr_solve(db, f)
    lhs = (x.double() * g.double()).sum(dim=1)
    x.backward(g)
    rhs = (db.detach().double() * db.grad.double()).sum(dim=1)
    scale = torch.minimum(x.detach().double().norm(dim=1) * g.double().norm(dim=1),
                          db.detach().double().norm(dim=1) * db.grad.double().norm(dim=1))
    rel = torch.max(torch.abs(lhs - rhs) / scale).item()
    print("dot-product identity, error / (||x|| ||g||): %.3g" % rel)
    assert rel <= tol


def test_finite_differences_fp32(setup):
    """Central differences with step 1e-3 along unit directions scaled to ||b||."""
    ct, sc, f = setup["ct"], setup["sc"], setup["f32"]
    A = setup["A"]
    B = synth.noisy_sinograms(4, A @ synth.phantoms(4, sc.n_pix, range(4)), 5e4, range(4))
    D = synth.directions(sc.m, 4) * np.linalg.norm(B, axis=0, keepdims=True)
    g = synth.gradients(sc.n, 4)
    h = 1e-3
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda", torch.float32).requires_grad_(True)
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to("cuda", torch.float32)
    X = ct.qr_solve(Bt, f)
    X.backward(gt)
    an = (Bt.grad.double().cpu().numpy().T * D).sum(axis=0)
    with torch.no_grad():
        Xp = ct.qr_solve(torch.from_numpy(np.ascontiguousarray((B + h * D).T)).to("cuda", torch.float32), f)
        Xm = ct.qr_solve(torch.from_numpy(np.ascontiguousarray((B - h * D).T)).to("cuda", torch.float32), f)
    fd = ((Xp.double() - Xm.double()).cpu().numpy().T * g).sum(axis=0) / (2 * h)
    assert np.max(np.abs(fd - an) / np.abs(an)) <= 1e-2
