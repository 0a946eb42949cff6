"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle on the
same seeded inputs.  Sizes span several panels, several outer blocks and
ragged edges; the oracle finishes each in seconds."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import to_dev, from_dev, rel, max_col_rel, sinograms, ld16

pytestmark = pytest.mark.gpu

# (name, N, views, bins): c1 is the 32^2 workload; the others are ragged in
# every blocking dimension (900 = 7*128 + 4 columns, 1400 rows; 2304 columns).
GEOMS = {
    "c1": (32, 30, 64),
    "ragged": (30, 28, 50),
    "multi": (48, 40, 84),
}


@pytest.fixture(scope="module")
def ct():
    from paper_2412_07631_amd import ctqr
    assert torch.cuda.is_available()
    return ctqr


_cache = {}


def problem(name):
    if name not in _cache:
        sc = synth.scanner(*GEOMS[name])
        A = O.system_dense(sc)
        VR, tau, info = O.householder_qr(A)
        assert info == 0
        _cache[name] = (sc, A, VR, tau)
    return _cache[name]


def gpu_system(ct, sc, dtype):
    A = torch.empty((sc.n, ld16(sc.m)), dtype=dtype, device="cuda")
    ct.build_system(sc, A)
    return A


# ------------------------------------------------------------------- Siddon
@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_siddon_dense_f64(ct, name):
    sc, A, _, _ = problem(name)
    Ag = from_dev(gpu_system(ct, sc, torch.float64), sc.m)
    assert np.max(np.abs(Ag - A)) <= 1e-14
    assert np.array_equal(Ag != 0, np.abs(A) > 0) or np.max(np.abs(Ag - A)) <= 1e-14


def test_siddon_dense_f32_is_rounded_f64(ct):
    sc, A, _, _ = problem("c1")
    Ag = gpu_system(ct, sc, torch.float32)[:, : sc.m].cpu().numpy().T
    ref = A.astype(np.float32)
    # both sides round an FP64 length to nearest; lengths differing in the
    # last FP64 bit may straddle a rounding boundary: allow one FP32 ulp
    assert np.all(np.abs(Ag.astype(np.float64) - ref.astype(np.float64)) <= np.spacing(ref) + 0.0)


def test_csr_matches_oracle(ct):
    sc, A, _, _ = problem("ragged")
    row_ptr, col, val = ct.build_csr(sc)
    rp, c, v = row_ptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    rpo, co, vo = O.system_csr(sc)
    assert np.array_equal(np.diff(rp), np.diff(rpo))
    D = np.zeros_like(A)
    for i in range(sc.m):
        D[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    assert np.max(np.abs(D - A)) <= 1e-14


def test_siddon_rows_axis_aligned(ct):
    N, W = 16, 1.0
    h = W / N
    rays = [(-2.0, -W / 2 + (iy + 0.5) * h, 2.0, -W / 2 + (iy + 0.5) * h) for iy in range(N)]
    rows = ct.siddon_rows(rays, N, W)
    for iy in range(N):
        expect = np.zeros(N * N)
        expect[iy * N:(iy + 1) * N] = h
        assert np.max(np.abs(rows[iy] - expect)) <= 1e-16
    # a diagonal through pixel corners: sqrt(2) W/N on the diagonal pixels only
    row = ct.siddon_rows([(-1.0, -1.0, 1.0, 1.0)], 12, 1.0)[0]
    assert list(np.nonzero(row)[0]) == [i * 12 + i for i in range(12)]


def test_residual_kernel_f64(ct):
    sc, A, _, _ = problem("ragged")
    csr = ct.build_csr(sc)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((sc.n, 11))
    B = rng.standard_normal((sc.m, 11))
    Xd, Bd = to_dev(X, torch.float64), to_dev(B, torch.float64)
    Rd = torch.empty_like(Bd)
    ct.residual(csr, sc.m, Xd, Bd, Rd)
    R = from_dev(Rd, sc.m)
    assert np.max(np.abs(R - (B - A @ X))) <= 1e-12


# ---------------------------------------------------- Joseph's projector
JOSEPH = {"small": (32, 30, 64), "multi": (48, 40, 84)}
_jcache = {}


def joseph_problem(name):
    if name not in _jcache:
        sc = synth.scanner(*JOSEPH[name], projector=1)
        A = O.system_dense(sc)
        _jcache[name] = (sc, A)
    return _jcache[name]


@pytest.mark.parametrize("name", ["small", "multi"])
def test_joseph_dense_and_csr_match_oracle(ct, name):
    sc, A = joseph_problem(name)
    Ag = from_dev(gpu_system(ct, sc, torch.float64), sc.m)
    assert np.max(np.abs(Ag - A)) <= 1e-14
    Af = gpu_system(ct, sc, torch.float32)[:, : sc.m].cpu().numpy().T
    ref = A.astype(np.float32)
    assert np.all(np.abs(Af.astype(np.float64) - ref.astype(np.float64)) <= np.spacing(ref))
    row_ptr, col, val = ct.build_csr(sc)
    rp, c, v = row_ptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    D = np.zeros_like(A)
    for i in range(sc.m):
        D[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    assert np.max(np.abs(D - A)) <= 1e-14


def test_joseph_system_through_the_whole_path(ct):
    """QR, solve and refinement on Joseph's A: R, V, tau and x against the
    oracle (FP64), and the BF16x3 factor refined to the FP64 solution."""
    sc, A = joseph_problem("multi")
    VR, tau, info = O.householder_qr(A)
    assert info == 0
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=8)
    assert ct.status(f) == 0
    VRg = from_dev(Ad, sc.m)
    R, Rg = np.triu(VR[: sc.n]), np.triu(VRg[: sc.n])
    assert np.max(np.abs(Rg - R)) / np.max(np.abs(R)) <= 1e-12
    assert np.max(np.abs(f.tau.cpu().numpy() - tau)) <= 1e-12
    _, P, B = sinograms(sc, A, 1, 4, 1e5)
    Xs = O.solve(VR, tau, B)
    Bd = to_dev(B, torch.float64)
    ct.apply_qt(f, Bd)
    ct.trsm_solve(f, Bd)
    assert max_col_rel(from_dev(Bd, sc.n), Xs) <= 1e-10
    A32 = gpu_system(ct, sc, torch.float32)
    f3 = ct.qr_factor(A32, sc.m, sc.n, ct.PREC_BF16X3, max_nrhs=8)
    sp = ct.SparseA(sc)
    Xd = torch.zeros((4, ld16(sc.n)), dtype=torch.float64, device="cuda")
    ct.solve_refined(f3, sp, to_dev(B, torch.float64), Xd, 4, ct.REFINE_SNE)
    err = max_col_rel(from_dev(Xd, sc.n), Xs)
    print("Joseph A, BF16x3 + 4 SNE: max rel err %.3g" % err)
    assert err <= 1e-10


# ------------------------------------------------------------ factorization
@pytest.fixture(params=["two-reduction", "column-wise"])
def panel_path(request, ct):
    """Panels factored from two Gram reductions (the default) or forced onto
    one reduction per column."""
    ct.debug_panel_cholesky(request.param == "two-reduction")
    yield request.param
    ct.debug_panel_cholesky(True)


@pytest.mark.parametrize("name", ["c1", "ragged", "multi"])
def test_qr_f64_matches_oracle(ct, name, panel_path):
    sc, A, VR, tau = problem(name)
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=8)
    assert ct.status(f) == 0
    VRg = from_dev(Ad, sc.m)
    n = sc.n
    R, Rg = np.triu(VR[:n]), np.triu(VRg[:n])
    scale = np.max(np.abs(R))
    # same sign convention: R, V and tau agree directly
    assert np.max(np.abs(Rg - R)) / scale <= 1e-12
    assert np.max(np.abs(np.tril(VRg, -1) - np.tril(VR, -1))) <= 1e-10
    assert np.max(np.abs(f.tau.cpu().numpy() - tau)) <= 1e-12


@pytest.mark.parametrize("name", ["ragged", "multi"])
def test_qr_f32_matches_oracle(ct, name, panel_path):
    """FP32 storage, FP32 updates, FP64 panels: R against the oracle's within
    the FP32 rounding of the updates.  kappa(A) u32 is about 8e-6 for these
    systems (kappa 134 at 3360 x 2304); measured 3e-7..4e-7."""
    sc, A, VR, tau = problem(name)
    Ad = gpu_system(ct, sc, torch.float32)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F32, max_nrhs=8)
    assert ct.status(f) == 0
    VRg = from_dev(Ad, sc.m)
    n = sc.n
    R, Rg = np.triu(VR[:n]), np.triu(VRg[:n])
    err = np.max(np.abs(Rg - R)) / np.max(np.abs(R))
    etau = float(np.max(np.abs(f.tau.cpu().numpy() - tau)))
    print("FP32 R max error / max |R|: %.3g, tau %.3g" % (err, etau))
    assert err <= 4e-6
    assert etau <= 1e-5


@pytest.mark.parametrize("nb", [64, 96, 512, 768, 1024])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_qr_block_widths_match_oracle(ct, nb, prec):
    """Outer reflector blocks of other widths (ragged last blocks, more join
    levels of the compact-WY factor): R and a solve against the oracle."""
    sc, A, VR, tau = problem("multi")
    ct.debug_block_width(nb)
    try:
        dt = torch.float64 if prec == "f64" else torch.float32
        Ad = gpu_system(ct, sc, dt)
        f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=8)
        assert ct.status(f) == 0
        VRg = from_dev(Ad, sc.m)
        n = sc.n
        R, Rg = np.triu(VR[:n]), np.triu(VRg[:n])
        tol = 1e-12 if prec == "f64" else 1e-4
        assert np.max(np.abs(Rg - R)) / np.max(np.abs(R)) <= tol
        _, P, B = sinograms(sc, A, 1, 3, 1e5)
        Bd = to_dev(B, dt)
        ct.apply_qt(f, Bd)
        ct.trsm_solve(f, Bd)
        err = max_col_rel(from_dev(Bd, n), O.solve(VR, tau, B))
        print("nb %d %s: solve max rel err %.3g" % (nb, prec, err))
        assert err <= (1e-10 if prec == "f64" else 1e-4)
    finally:
        ct.debug_block_width(0)


def test_qr_f64_bitwise_reproducible(ct):
    sc, _, _, _ = problem("multi")
    outs = []
    for _ in range(2):
        Ad = gpu_system(ct, sc, torch.float64)
        f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=1)
        ct.status(f)
        outs.append((Ad.cpu().clone(), f.tau.cpu().clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_rank_deficient_column_reported(ct, panel_path):
    sc = synth.scanner(*GEOMS["ragged"])
    Ad = gpu_system(ct, sc, torch.float64)
    Ad[17].zero_()
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=1)
    assert ct.status(f) == 18


# ------------------------------------------------------------------- solves
@pytest.mark.parametrize("name", ["c1", "ragged", "multi"])
def test_solve_f64_parity(ct, name):
    """x = R^{-1} Q^T b against the oracle's x* on noisy sinograms: <= 1e-10."""
    sc, A, VR, tau = problem(name)
    cfg = 1
    _, P, B = sinograms(sc, A, cfg, 5, 1e5)
    Xs = O.solve(VR, tau, B)
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=8)
    Bd = to_dev(B, torch.float64)
    ct.apply_qt(f, Bd)
    C = from_dev(Bd, sc.m)
    assert np.max(np.abs(C - O.apply_qt(VR, tau, B))) <= 1e-11 * np.max(np.abs(B))
    ct.trsm_solve(f, Bd)
    X = from_dev(Bd, sc.n)
    assert max_col_rel(X, Xs) <= 1e-10


def test_trsm_matches_back_substitution(ct):
    """The blocked triangular solve on the GPU's own R against plain
    back-substitution (oracle) with that same R."""
    sc, _, _, _ = problem("multi")
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=8)
    VRg = from_dev(Ad, sc.m)
    C = np.random.default_rng(8).standard_normal((sc.m, 3))
    Cd = to_dev(C, torch.float64)
    ct.trsm_solve(f, Cd)
    X = from_dev(Cd, sc.n)
    Xo = O.back_substitute(VRg, C)
    assert max_col_rel(X, Xo) <= 1e-12


@pytest.mark.parametrize("nrhs", [1, 17])
def test_solve_f32_parity(ct, nrhs):
    """FP32 path against the FP64 oracle: relative image error <= 1e-4."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 2, nrhs, 5e4)
    Xs = O.solve(VR, tau, B)
    Ad = gpu_system(ct, sc, torch.float32)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F32, max_nrhs=32)
    assert ct.status(f) == 0
    Bd = to_dev(B, torch.float32)
    ct.apply_qt(f, Bd)
    ct.trsm_solve(f, Bd)
    X = from_dev(Bd, sc.n)
    assert max_col_rel(X, Xs) <= 1e-4


def refined(ct, prec, name, nrhs, steps, method, cfg=3):
    sc, A, VR, tau = problem(name)
    _, P, B = sinograms(sc, A, cfg, nrhs, 5e4)
    Xs = O.solve(VR, tau, B)
    Ad = gpu_system(ct, sc, torch.float64 if prec == "f64" else torch.float32)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=max(8, nrhs))
    assert ct.status(f) == 0
    sp = ct.SparseA(sc)
    Bd = to_dev(B, torch.float64)
    Xd = torch.zeros((nrhs, ld16(sc.n)), dtype=torch.float64, device="cuda")
    rn = torch.zeros((steps + 1) * nrhs, dtype=torch.float64, device="cuda")
    gn = torch.zeros((steps + 1) * nrhs, dtype=torch.float64, device="cuda")
    ct.solve_refined(f, sp, Bd, Xd, steps, method, res_norms=rn, grad_norms=gn)
    X = from_dev(Xd, sc.n)
    return max_col_rel(X, Xs), rn.view(steps + 1, nrhs)[:, 0].tolist(), gn.view(steps + 1, nrhs)[:, 0].tolist()


@pytest.mark.parametrize("prec,steps,tol", [("f64", 1, 1e-12), ("f32", 3, 1e-10), ("bf16x3", 4, 1e-10),
                                            ("f16", 6, 1e-8)])
def test_refined_sne_parity(ct, prec, steps, tol):
    """Low-precision factor + FP64-residual refinement (semi-normal
    correction) reproduces the FP64 oracle's least-squares images."""
    err, rn, gn = refined(ct, prec, "multi", 6, steps, ct.REFINE_SNE)
    print("SNE", prec, "steps", steps, "max rel err %.3g" % err, "||A^T r||:", ["%.3g" % v for v in gn])
    assert err <= tol
    assert gn[-1] < gn[0]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("panel_path", ["cholqr2", "columnwise"])
def test_sixteen_column_panels_match_oracle(ct, prec, panel_path):
    """Panels of 16 columns (what the factorization uses when a 32-column
    panel of a very tall matrix does not fit in the LDS of all CUs), in both
    panel forms: R, V and tau against the oracle, and the refined solve."""
    sc, A, VR, tau = problem("multi")
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad = gpu_system(ct, sc, dt)
    ct.debug_panel_width(16)
    ct.debug_panel_cholesky(panel_path == "cholqr2")
    try:
        f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=8)
        assert ct.status(f) == 0
    finally:
        ct.debug_panel_width(0)
        ct.debug_panel_cholesky(True)
    VRd = from_dev(Ad, sc.m)
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-3}[prec]
    assert rel(np.triu(VRd[: sc.n]), np.triu(VR[: sc.n])) <= tol
    assert rel(np.tril(VRd, -1), np.tril(VR, -1)) <= tol * 10
    assert np.max(np.abs(f.tau.cpu().numpy() - tau)) <= tol * 10
    _, P, B = sinograms(sc, A, 3, 6, 5e4)
    Xs = O.solve(VR, tau, B)
    sp = ct.SparseA(sc)
    Xd = torch.zeros((6, ld16(sc.n)), dtype=torch.float64, device="cuda")
    ct.solve_refined(f, sp, to_dev(B, torch.float64), Xd, 6, ct.REFINE_SNE, tol=1e-11)
    assert max_col_rel(from_dev(Xd, sc.n), Xs) <= 1e-9


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_lean_factor_without_solve_copies(ct, prec):
    """CT_QR_NO_SOLVE_COPIES: the same factor in a smaller workspace; its
    solves (which then read V and R in place), the refinement and the
    adjoint give the oracle's results like those of the full factor."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 3, 50, 5e4)
    Xs = O.solve(VR, tau, B)
    dt = torch.float64 if prec == "f64" else torch.float32
    full = ct.qr_workspace(sc.m, sc.n, ct.PREC_NAMES[prec], 64)
    lean = ct.qr_workspace(sc.m, sc.n, ct.PREC_NAMES[prec] | ct.QR_NO_SOLVE_COPIES, 64)
    assert lean < full
    Ad = gpu_system(ct, sc, dt)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=64, solve_copies=False)
    assert ct.status(f) == 0
    assert f.work.numel() == lean
    VRd = from_dev(Ad, sc.m)
    tol_r = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-3}[prec]
    assert rel(np.triu(VRd[: sc.n]), np.triu(VR[: sc.n])) <= tol_r
    sp = ct.SparseA(sc)
    Xd = torch.zeros((50, ld16(sc.n)), dtype=torch.float64, device="cuda")
    k = ct.solve_refined(f, sp, to_dev(B, torch.float64), Xd, 6, ct.REFINE_SNE, tol=1e-10)
    err = max_col_rel(from_dev(Xd, sc.n), Xs)
    print(prec, "lean factor: %d refinement steps, max rel err %.3g" % (k, err))
    assert err <= 1e-9
    Xd.zero_()
    k = ct.solve_refined(f, sp, to_dev(B, torch.float64), Xd, 12, ct.REFINE_PCGLS, tol=1e-10)
    err = max_col_rel(from_dev(Xd, sc.n), Xs)
    print(prec, "lean factor: %d conjugate-gradient steps, max rel err %.3g" % (k, err))
    assert err <= 1e-9
    # the unrefined solve: R's off-diagonal blocks read in place (NN products)
    Bd = to_dev(B, dt)
    ct.apply_qt(f, Bd)
    ct.trsm_solve(f, Bd)
    err = max_col_rel(from_dev(Bd, sc.n), Xs)
    print(prec, "lean factor, unrefined solve: max rel err %.3g" % err)
    assert err <= {"f64": 1e-10, "f32": 1e-4, "bf16x3": 1e-3}[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_refined_stop_rule(ct, prec):
    """Stop rule of the refinement: it ends after the first step whose
    correction is at most tol relative to every slice's image (a huge tol
    stops after one step, tol = 0 runs them all); the images then meet the
    oracle within tol, and the norm rows of steps not taken stay unwritten."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 3, 6, 5e4)
    Xs = O.solve(VR, tau, B)
    Ad = gpu_system(ct, sc, torch.float32)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=8)
    sp = ct.SparseA(sc)
    Bd = to_dev(B, torch.float64)
    steps = 8
    taken = {}
    for tol in (1e300, 1e-7, 1e-12, 0.0):
        Xd = torch.zeros((6, ld16(sc.n)), dtype=torch.float64, device="cuda")
        rn = torch.full(((steps + 1) * 6,), float("nan"), dtype=torch.float64, device="cuda")
        k = ct.solve_refined(f, sp, Bd, Xd, steps, ct.REFINE_SNE, res_norms=rn, tol=tol)
        err = max_col_rel(from_dev(Xd, sc.n), Xs)
        rows = rn.view(steps + 1, 6).cpu().numpy()
        print(prec, "tol %g: %d steps, max rel err %.3g" % (tol, k, err))
        assert np.isfinite(rows[: k + 1]).all() and np.isnan(rows[k + 1:]).all()
        if 0.0 < tol < 1.0:
            assert err <= max(tol, 1e-11)
        taken[tol] = k
    assert taken[1e300] == 1 and taken[0.0] == steps
    assert 1 <= taken[1e-7] <= taken[1e-12] <= steps


@pytest.mark.parametrize("name,nrhs", [("multi", 6), ("ragged", 37)])
def test_refined_bf16x3_block_updates_on_and_off(ct, name, nrhs):
    """The refinement of a BF16x3 factor runs its solves' products in BF16x3
    (by default from 48 slices); with FP32 ones instead it
    reaches the same FP64 oracle images, and both converge step by step
    (ragged: a last diagonal block of 132 rows, 37 slices over three
    workgroups of 16; both forced, whatever the slice count)."""
    was = ct.debug_refine_x3(0)
    try:
        err32, _, g32 = refined(ct, "bf16x3", name, nrhs, 4, ct.REFINE_SNE)
        ct.debug_refine_x3(2)
        err3, _, g3 = refined(ct, "bf16x3", name, nrhs, 4, ct.REFINE_SNE)
    finally:
        ct.debug_refine_x3(was)
    assert was == 1
    print("bf16x3 refine, FP32 updates %.3g, BF16x3 updates %.3g" % (err32, err3), g32, g3)
    assert err3 <= 1e-10 and err32 <= 1e-10
    assert all(b < a for a, b in zip(g3[:3], g3[1:4]))


def test_refined_qr_method_bf16x3_products(ct):
    """The Q~^T-correction refinement of a BF16x3 factor with BF16x3 products
    (every step applies Q~^T in BF16x3) reaches the same fixed point as with
    FP32 products: the two fixed points lie at the same distance, within a
    factor of 3, from the least-squares solution."""
    was = ct.debug_refine_x3(0)
    try:
        e32, _, g32 = refined(ct, "bf16x3", "ragged", 37, 4, ct.REFINE_QR)
        ct.debug_refine_x3(2)
        e3, _, g3 = refined(ct, "bf16x3", "ragged", 37, 4, ct.REFINE_QR)
    finally:
        ct.debug_refine_x3(was)
    print("QR-method refine, FP32 products %.3g, BF16x3 products %.3g" % (e32, e3), g32[-1], g3[-1])
    assert np.isfinite(e3) and e3 <= 3 * e32 + 1e-12 and e32 <= 3 * e3 + 1e-12
    assert g3[-1] < g3[0]


def test_refined_qr_method_stalls_at_its_fixed_point(ct):
    """x += R~^{-1} Q~^T r converges to Q~^T r = 0, not to A^T r = 0: with an
    FP32 factor and noisy data the image error stops far above the SNE one."""
    err_qr, _, g_qr = refined(ct, "f32", "multi", 3, 4, ct.REFINE_QR)
    err_sne, _, g_sne = refined(ct, "f32", "multi", 3, 4, ct.REFINE_SNE)
    print("QR-refine err %.3g  SNE-refine err %.3g" % (err_qr, err_sne))
    assert err_sne < 1e-10 and err_qr > 100 * err_sne
    assert g_qr[-1] > 100 * g_sne[-1]


def test_refinement_error_falls_bf16(ct):
    """Plain bfloat16 updates: the refined error is far below the unrefined one."""
    e0, _, _ = refined(ct, "bf16", "multi", 2, 0, ct.REFINE_SNE)
    e6, _, g6 = refined(ct, "bf16", "multi", 2, 6, ct.REFINE_SNE)
    print("bf16 error: no refinement %.3g, 6 SNE steps %.3g" % (e0, e6))
    assert e6 < 0.1 * e0


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("prec,steps,tol", [("f64", 1, 1e-12), ("f32", 3, 1e-10), ("bf16x3", 4, 1e-10),
                                            ("f16", 6, 1e-10), ("bf16", 10, 1e-8)])
def test_refined_pcgls_parity(ct, prec, steps, tol):
    """Preconditioned conjugate gradients on the normal equations from the
    same start reach the FP64 oracle's least-squares images; the residual
    norms it reports fall, and the last one is ||b - A x|| of the returned
    image (recomputed, not the recurrence)."""
    sc, A, VR, tau = problem("multi")
    err, rn, gn = refined(ct, prec, "multi", 6, steps, ct.REFINE_PCGLS)
    print("PCGLS", prec, "steps", steps, "max rel err %.3g" % err, "||A^T r||:", ["%.3g" % v for v in gn])
    assert err <= tol
    assert gn[-1] < gn[0] and rn[-1] <= rn[0]


def test_pcgls_outpaces_sne_on_a_coarse_factor(ct):
    """With a plain bfloat16 factor (u ~ 4e-3) the stationary SNE step
    contracts by a fixed factor per step; the Krylov iteration with the same
    factor and the same number of steps gets closer to the oracle's images
    (measured: 1.1e-10 against 1.1e-11 after 6 steps)."""
    e_sne, _, _ = refined(ct, "bf16", "multi", 4, 6, ct.REFINE_SNE)
    e_cg, _, _ = refined(ct, "bf16", "multi", 4, 6, ct.REFINE_PCGLS)
    print("bf16 factor, 6 steps: SNE %.3g, PCGLS %.3g" % (e_sne, e_cg))
    assert e_cg < 0.25 * e_sne


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_pcgls_stop_rule_and_true_residual(ct, prec):
    """The stop rule of the Krylov refinement (step c_j p_j against the image)
    ends it early; rows of steps not taken stay unwritten, and the last
    reported residual norm is that of b - A x for the returned x (checked in
    FP64 on the CPU with the oracle's matrix)."""
    sc, A, VR, tau = problem("multi")
    _, P, B = sinograms(sc, A, 3, 6, 5e4)
    Xs = O.solve(VR, tau, B)
    Ad = gpu_system(ct, sc, torch.float32)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=8)
    sp = ct.SparseA(sc)
    Bd = to_dev(B, torch.float64)
    steps = 12
    taken = {}
    for tol in (1e300, 1e-8, 0.0):
        Xd = torch.zeros((6, ld16(sc.n)), dtype=torch.float64, device="cuda")
        rn = torch.full(((steps + 1) * 6,), float("nan"), dtype=torch.float64, device="cuda")
        k = ct.solve_refined(f, sp, Bd, Xd, steps, ct.REFINE_PCGLS, res_norms=rn, tol=tol)
        X = from_dev(Xd, sc.n)
        rows = rn.view(steps + 1, 6).cpu().numpy()
        assert np.isfinite(rows[: k + 1]).all() and np.isnan(rows[k + 1:]).all()
        true_r = np.linalg.norm(B - A @ X, axis=0)
        assert np.max(np.abs(rows[k] - true_r) / true_r) <= 1e-10
        err = max_col_rel(X, Xs)
        print(prec, "PCGLS tol %g: %d steps, max rel err %.3g" % (tol, k, err))
        if 0.0 < tol < 1.0:
            assert err <= 1e-7
        taken[tol] = k
    assert taken[1e300] == 1 and taken[0.0] == steps
    assert 1 <= taken[1e-8] <= steps


def test_adjoint_f64_parity(ct):
    sc, A, VR, tau = problem("ragged")
    G = np.random.default_rng(6).standard_normal((sc.n, 4))
    Ys = O.adjoint(VR, tau, G)
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=8)
    Gd = to_dev(G, torch.float64)
    Yd = torch.empty((4, ld16(sc.m)), dtype=torch.float64, device="cuda")
    ct.solve_backward(f, Gd, Yd)
    Y = from_dev(Yd, sc.m)
    assert max_col_rel(Y, Ys) <= 1e-10


def test_empty_batch_is_a_noop(ct):
    sc, _, _, _ = problem("c1")
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=4)
    Bd = torch.ones((1, ld16(sc.m)), dtype=torch.float64, device="cuda")
    ct.apply_qt(f, Bd, nrhs=0)
    ct.trsm_solve(f, Bd, nrhs=0)
    assert torch.all(Bd == 1)


# --------------------------------------------------------- failure handling
def test_panel_wait_limit_fails_fast_and_recovers(ct):
    """With the wait limit forced to zero from the host, every panel wait gives
    up at once: the factorization ends (no hang) and ct_status reports -2001.
    With the default limit restored the next factorization is correct."""
    sc, A, VR, tau = problem("multi")
    ct.debug_wait_limit(0)
    try:
        Ad = gpu_system(ct, sc, torch.float64)
        f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=1)
        with pytest.raises(ct.CtError) as ei:
            ct.status(f)
        assert ei.value.code == -2001
    finally:
        ct.debug_wait_limit(-1)
    Ad = gpu_system(ct, sc, torch.float64)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_F64, max_nrhs=1)
    assert ct.status(f) == 0
    R, Rg = np.triu(VR[: sc.n]), np.triu(from_dev(Ad, sc.m)[: sc.n])
    assert np.max(np.abs(Rg - R)) / np.max(np.abs(R)) <= 1e-12
