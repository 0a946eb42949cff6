"""Host-pinned streaming (out-of-core) factorization through the C-ABI: the
matrix lives in pinned host memory and passes through the device in column
tiles, with a device buffer forced far below the matrix size so that most
tiles are re-read from the host.  Checked against the FP64 oracle, against
the all-resident run of the same code (bitwise), through every solve call,
and across an injected copy failure followed by a resume."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2412_07631_amd import synth
from gpu_util import to_dev, from_dev, max_col_rel, sinograms, ld16

pytestmark = pytest.mark.gpu

# (name, N, views, bins): "multi" is 3360 x 2304 (18 outer blocks); "ragged"
# is 1400 x 900 (7 blocks + 4 columns), so its last tile is ragged too.
GEOMS = {"multi": (48, 40, 84), "ragged": (30, 28, 50)}


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


def host_system(ct, sc, dtype):
    """The Siddon matrix built on the device, then moved to pinned host memory."""
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=dtype, device="cuda")
    ct.build_system(sc, Ad)
    Ah = torch.empty(Ad.shape, dtype=dtype, pin_memory=True)
    Ah.copy_(Ad)
    return Ah


def budget(ct, sc, prec, tile, resident, max_nrhs=8):
    lo, _ = ct.qr_stream_workspace(sc.m, sc.n, ld16(sc.m), prec, max_nrhs, tile)
    es = 8 if prec == ct.PREC_F64 else 4
    return lo + resident * ((ld16(sc.m) * tile * es + 255) // 256 * 256)


def streamed(ct, name, prec, tile, resident, max_nrhs=8):
    sc, A, VR, tau = problem(name)
    Ah = host_system(ct, sc, torch.float64 if prec == ct.PREC_F64 else torch.float32)
    f = ct.qr_factor_streamed(Ah, sc.m, sc.n, prec, tile_cols=tile,
                              device_bytes=budget(ct, sc, prec, tile, resident, max_nrhs), max_nrhs=max_nrhs)
    assert ct.status(f) == 0
    return sc, A, VR, tau, Ah, f


# (name, tile columns, extra resident tiles asked for, resident tiles expected):
# with no more tiles than staging slots the minimum buffer holds them all.
@pytest.mark.parametrize("name,tile,resident,expect", [("multi", 256, 1, 1), ("ragged", 128, 0, 0),
                                                       ("multi", 512, 0, 0), ("ragged", 384, 0, 3)])
def test_streamed_qr_f64_matches_oracle(ct, name, tile, resident, expect):
    sc, A, VR, tau, Ah, f = streamed(ct, name, ct.PREC_F64, tile, resident)
    tiles, res, nxt = ct.stream_info(f)
    print(name, "tiles", tiles, "resident", res)
    assert tiles == (sc.n + tile - 1) // tile and res == expect and nxt == tiles
    VRg = from_dev(Ah, sc.m)
    n = sc.n
    R, Rg = np.triu(VR[:n]), np.triu(VRg[:n])
    assert np.max(np.abs(Rg - R)) / np.max(np.abs(R)) <= 1e-12
    assert np.max(np.abs(np.tril(VRg, -1) - np.tril(VR, -1))) <= 1e-10
    assert np.max(np.abs(f.tau.cpu().numpy() - tau)) <= 1e-12


def test_streamed_budget_does_not_change_the_result(ct):
    """Minimum buffer (every tile re-read from the host) and all-resident
    buffer run the same kernels on the same data: bitwise equal factors."""
    sc, _, _, _ = problem("multi")
    outs = []
    for dev_bytes in (0, None):
        Ah = host_system(ct, sc, torch.float64)
        f = ct.qr_factor_streamed(Ah, sc.m, sc.n, ct.PREC_F64, tile_cols=256, device_bytes=dev_bytes, max_nrhs=1)
        assert ct.status(f) == 0
        outs.append((Ah.clone(), f.tau.cpu(), ct.stream_info(f)[1]))
    assert outs[0][2] == 0 and outs[1][2] == (sc.n + 255) // 256
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_streamed_solve_and_adjoint_parity(ct):
    """apply_qt, trsm and the adjoint read the factor tile by tile from the host."""
    sc, A, VR, tau, Ah, f = streamed(ct, "multi", ct.PREC_F64, 256, 1)
    _, P, B = sinograms(sc, A, 1, 5, 1e5)
    Xs = O.solve(VR, tau, B)
    Bd = to_dev(B, torch.float64)
    ct.apply_qt(f, Bd)
    assert np.max(np.abs(from_dev(Bd, sc.m) - O.apply_qt(VR, tau, B))) <= 1e-11 * np.max(np.abs(B))
    ct.trsm_solve(f, Bd)
    assert max_col_rel(from_dev(Bd, sc.n), Xs) <= 1e-10
    G = np.random.default_rng(6).standard_normal((sc.n, 3))
    Yd = torch.empty((3, ld16(sc.m)), dtype=torch.float64, device="cuda")
    ct.solve_backward(f, to_dev(G, torch.float64), Yd)
    assert max_col_rel(from_dev(Yd, sc.m), O.adjoint(VR, tau, G)) <= 1e-10


@pytest.mark.parametrize("prec,steps", [("f32", 3), ("bf16x3", 4)])
def test_streamed_low_precision_refined(ct, prec, steps):
    """Low-precision streamed factor + FP64-residual refinement reaches the
    FP64 oracle's least-squares images."""
    sc, A, VR, tau, Ah, f = streamed(ct, "multi", ct.PREC_NAMES[prec], 256, 1)
    _, P, B = sinograms(sc, A, 3, 6, 5e4)
    Xs = O.solve(VR, tau, B)
    sp = ct.SparseA(sc)
    Xd = torch.zeros((6, ld16(sc.n)), dtype=torch.float64, device="cuda")
    ct.solve_refined(f, sp, to_dev(B, torch.float64), Xd, steps, ct.REFINE_SNE)
    err = max_col_rel(from_dev(Xd, sc.n), Xs)
    print("streamed", prec, "refined err %.3g" % err)
    assert err <= 1e-10


def test_streamed_resume_after_injected_failure(ct):
    """A copy failure injected before tile 3 stops the run with -2002; the
    resumed run finishes with exactly the uninterrupted result."""
    sc, _, _, _ = problem("multi")
    dev_bytes = budget(ct, sc, ct.PREC_F64, 256, 1, 1)
    ref = host_system(ct, sc, torch.float64)
    f0 = ct.qr_factor_streamed(ref, sc.m, sc.n, ct.PREC_F64, tile_cols=256, device_bytes=dev_bytes, max_nrhs=1)
    assert ct.status(f0) == 0
    Ah = host_system(ct, sc, torch.float64)
    ct.inject_failure(3)
    with pytest.raises(ct.CtError) as ei:
        ct.qr_factor_streamed(Ah, sc.m, sc.n, ct.PREC_F64, tile_cols=256, device_bytes=dev_bytes, max_nrhs=1)
    assert ei.value.code == -2002
    f = ei.value.factor
    assert ct.stream_info(f)[2] == 3
    ct.qr_resume(f)
    assert ct.status(f) == 0 and ct.stream_info(f)[2] == ct.stream_info(f)[0]
    assert torch.equal(Ah, ref) and torch.equal(f.tau.cpu(), f0.tau.cpu())


@pytest.mark.parametrize("resident,tile,after", [(4, 3, 2), (4, 6, 4), (1, 5, 5), (1, 7, 0)])
def test_streamed_resume_after_failure_inside_a_tile(ct, resident, tile, after):
    """A failure injected after some earlier reflector blocks have been
    applied to a tile -- a resident one (tile < resident) or one held in a
    staging slot -- leaves the tile partly updated on the device; the resume
    redoes it from its untouched host copy and gives bitwise the
    uninterrupted factor."""
    sc, _, _, _ = problem("multi")
    dev_bytes = budget(ct, sc, ct.PREC_F64, 256, resident, 1)
    ref = host_system(ct, sc, torch.float64)
    f0 = ct.qr_factor_streamed(ref, sc.m, sc.n, ct.PREC_F64, tile_cols=256, device_bytes=dev_bytes, max_nrhs=1)
    assert ct.status(f0) == 0 and ct.stream_info(f0)[1] == resident
    Ah = host_system(ct, sc, torch.float64)
    ct.inject_failure(tile, after)
    with pytest.raises(ct.CtError) as ei:
        ct.qr_factor_streamed(Ah, sc.m, sc.n, ct.PREC_F64, tile_cols=256, device_bytes=dev_bytes, max_nrhs=1)
    assert ei.value.code == -2002
    f = ei.value.factor
    assert ct.stream_info(f)[2] == tile
    ct.qr_resume(f)
    assert ct.status(f) == 0 and ct.stream_info(f)[2] == ct.stream_info(f)[0]
    assert torch.equal(Ah, ref) and torch.equal(f.tau.cpu(), f0.tau.cpu())


def test_streamed_rank_deficient_column_reported(ct):
    sc, _, _, _ = problem("ragged")
    Ah = host_system(ct, sc, torch.float64)
    Ah[401].zero_()
    f = ct.qr_factor_streamed(Ah, sc.m, sc.n, ct.PREC_F64, tile_cols=128,
                              device_bytes=budget(ct, sc, ct.PREC_F64, 128, 1, 1), max_nrhs=1)
    assert ct.status(f) == 402


def test_graph_solve_rejects_streamed_factor(ct):
    sc, A, VR, tau, Ah, f = streamed(ct, "ragged", ct.PREC_F64, 128, 0)
    B = torch.zeros((8, ld16(sc.m)), dtype=torch.float64, device="cuda")
    desc = ct.batch_descriptor([3, 5])
    with pytest.raises(ct.CtError):
        ct.SolveGraph(f, B, 8, desc)
