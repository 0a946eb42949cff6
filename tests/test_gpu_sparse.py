"""Grouped sparse copies of A (ct_group_sparse): exact placement of every
stored entry against the oracle's dense matrix, and refinement through the
grouped products against the entry-by-entry products and the oracle."""
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


def ungroup(rows, cols, group, gptr, gidx, gval):
    """Dense rows x cols matrix from a grouped copy (numpy, host)."""
    gptr, gidx, gval = gptr.cpu().numpy(), gidx.cpu().numpy(), gval.cpu().numpy()
    D = np.zeros((rows, cols))
    for g in range(len(gptr) - 1):
        for k in range(gptr[g], gptr[g + 1]):
            for r in range(group):
                i = g * group + r
                if i < rows:
                    assert D[i, gidx[k]] == 0.0
                    D[i, gidx[k]] = gval[k * group + r]
                else:
                    assert gval[k * group + r] == 0.0
    return D


@pytest.mark.parametrize("geom,group", [((32, 30, 64), 8), ((30, 28, 50), 8), ((30, 28, 50), 4), ((17, 13, 22), 1)])
def test_grouped_copies_place_every_entry(ct, geom, group):
    """Both grouped copies hold exactly the oracle's A (rows: rays; the CSC
    copy: pixels), column indices sorted and distinct within a group, for
    ragged row counts (last group partial)."""
    sc = synth.scanner(*geom)
    A = O.system_dense(sc)
    sp = ct.SparseA(sc, group=0)
    g_r, *grp_r = ct.group_sparse(sc.m, sp.row_ptr, sp.col, sp.val, group)
    g_c, *grp_c = ct.group_sparse(sc.n, sp.col_ptr, sp.row, sp.cval, group)
    assert g_r == group and g_c == group
    for gp in (grp_r[0], grp_c[0]):
        gi = (grp_r if gp is grp_r[0] else grp_c)[1].cpu().numpy()
        p = gp.cpu().numpy()
        for g in range(len(p) - 1):
            seg = gi[p[g]:p[g + 1]]
            assert np.all(np.diff(seg) > 0)
    Dr = ungroup(sc.m, sc.n, group, *grp_r)
    Dc = ungroup(sc.n, sc.m, group, *grp_c)
    # exactly the device's own CSR entries (which match the oracle's lengths
    # to 1e-14; the Siddon parity tests pin that)
    rp, cl, vl = (t.cpu().numpy() for t in sp.csr)
    D = np.zeros((sc.m, sc.n))
    for i in range(sc.m):
        D[i, cl[rp[i]:rp[i + 1]]] = vl[rp[i]:rp[i + 1]]
    assert np.array_equal(Dr, D)
    assert np.array_equal(Dc, D.T)
    assert np.abs(D - A).max() <= 1e-14


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_refinement_with_grouped_products(ct, prec):
    """The refinement's FP64 residuals and A^T r through the grouped copies:
    the same oracle images, the same first gradient norm as with the
    entry-by-entry products (to the rounding of a cancelling sum)."""
    sc = synth.scanner(48, 40, 84)
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    _, P, B = sinograms(sc, A, 3, 37, 5e4)
    Xs = O.solve(VR, tau, B)
    Ad = torch.empty((sc.n, ld16(sc.m)), dtype=torch.float32, device="cuda")
    ct.build_system(sc, Ad)
    f = ct.qr_factor(Ad, sc.m, sc.n, ct.PREC_NAMES[prec], max_nrhs=40)
    Bd = to_dev(B, torch.float64)
    res = {}
    for group in (0, 8):
        sp = ct.SparseA(sc, group=group)
        Xd = torch.zeros((37, ld16(sc.n)), dtype=torch.float64, device="cuda")
        gn = torch.zeros(5 * 37, dtype=torch.float64, device="cuda")
        ct.solve_refined(f, sp, Bd, Xd, 4, ct.REFINE_SNE, grad_norms=gn)
        res[group] = (from_dev(Xd, sc.n), gn.view(5, 37).cpu().numpy())
    e0, e8 = max_col_rel(res[0][0], Xs), max_col_rel(res[8][0], Xs)
    print(prec, "oracle rel err: entrywise %.3g, grouped %.3g" % (e0, e8))
    assert e8 <= 1e-10
    # ||A^T r|| is a cancellation (A^T r small against ||A|| ||r||): its
    # rounding, with the sums taken in another order, is relative to that
    assert np.allclose(res[8][1][0], res[0][1][0], rtol=1e-8, atol=0)
    assert max_col_rel(res[8][0], res[0][0]) <= 1e-10
