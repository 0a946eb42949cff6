"""Pins of the oracle's factorization and solve (Eqs. (qr), (solve)) and of
its adjoint, against closed forms, exact rational arithmetic, library special
cases and invariants -- never against the oracle itself."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from paper_2412_07631_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def explicit_q(VR, tau):
    m = VR.shape[0]
    return O.apply_q(VR, tau, np.eye(m))


@pytest.fixture(scope="module")
def c1():
    sc = synth.workload_scanner("c1_32")
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    return sc, A, VR, tau, info


def test_householder_closed_form():
    with open(os.path.join(GOLDEN, "householder_2x1.json")) as f:
        g = json.load(f)
    VR, tau, info = O.householder_qr(np.array(g["x"]).reshape(2, 1))
    assert info == 0
    assert VR[0, 0] == g["beta"]
    assert abs(tau[0] - g["tau"]) <= 1e-16
    assert VR[1, 0] == g["v1"]


def test_orthogonality_and_backward_error():
    sc = synth.scanner(16, 18, 24)            # 432 x 256
    A = O.system_dense(sc)
    VR, tau, info = O.householder_qr(A)
    assert info == 0
    m, n = A.shape
    Q = explicit_q(VR, tau)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12
    R = np.triu(VR[:n])
    assert np.linalg.norm(A - Q[:, :n] @ R) / np.linalg.norm(A) <= 1e-13
    # the reflectors leave zeros below the diagonal of Q^T A
    QtA = O.apply_qt(VR, tau, A)
    assert np.max(np.abs(np.tril(QtA[:n], -1))) <= 1e-14
    assert np.max(np.abs(QtA[n:])) <= 1e-14


def test_r_matches_lapack_up_to_signs(c1):
    """LAPACK dgeqrf (through numpy) is a library special case: R is unique up
    to the signs of its rows for a full-rank A."""
    sc, A, VR, tau, info = c1
    n = A.shape[1]
    R = np.triu(VR[:n])
    Rl = np.linalg.qr(A, mode="r")
    s = np.sign(np.diag(R)) * np.sign(np.diag(Rl))
    assert np.max(np.abs(R - s[:, None] * Rl)) / np.max(np.abs(Rl)) <= 1e-13
    # R^T R = A^T A
    G = A.T @ A
    assert np.linalg.norm(R.T @ R - G) / np.linalg.norm(G) <= 1e-13


def _exact_lstsq(A, b):
    """Normal equations A^T A x = A^T b solved in exact rational arithmetic
    from the binary64 values of A and b (Gauss-Jordan with Fractions)."""
    m, n = A.shape
    Af = [[Fraction(float(v)) for v in row] for row in A]
    bf = [Fraction(float(v)) for v in b]
    G = [[sum((Af[i][p] * Af[i][q] for i in range(m) if Af[i][p] and Af[i][q]), Fraction(0))
          for q in range(n)] for p in range(n)]
    r = [sum((Af[i][p] * bf[i] for i in range(m) if Af[i][p]), Fraction(0)) for p in range(n)]
    M = [G[p] + [r[p]] for p in range(n)]
    for c in range(n):
        piv = next(k for k in range(c, n) if M[k][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for k in range(n):
            if k != c and M[k][c] != 0:
                f = M[k][c]
                M[k] = [a - f * bb for a, bb in zip(M[k], M[c])]
    return np.array([float(M[p][n]) for p in range(n)])


@pytest.mark.slow
def test_exact_rational_normal_equations():
    """Tiny system: 6x6 image, 10 views x 12 bins (m = 120, n = 36)."""
    sc = synth.scanner(6, 10, 12)
    A = O.system_dense(sc)
    b = synth.noisy_sinogram(A @ synth.phantom(6, synth.rng(9, 0, 0)), 1e3, synth.rng(9, 0, 1))
    x_exact = _exact_lstsq(A, b)
    x = O.lstsq(A, b)
    assert np.linalg.norm(x - x_exact) / np.linalg.norm(x_exact) <= 1e-12


def test_square_system_equals_linear_solve():
    """m = n: least squares is the plain solve.  (Square fan-beam systems of
    small images are rank deficient, so a square block of a full-rank system
    matrix plus a diagonal shift is used.)"""
    sc = synth.scanner(8, 12, 16)
    A = O.system_dense(sc)[::3][:64] + 0.05 * np.eye(64)
    b = np.random.default_rng(3).standard_normal(64)
    x = O.lstsq(A, b)
    xr = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-16 * np.linalg.cond(A) * 100


def test_least_squares_optimality_and_recovery(c1):
    sc, A, VR, tau, info = c1
    x_true = synth.phantoms(1, sc.n_pix, range(4))
    p = A @ x_true
    b = synth.noisy_sinograms(1, p, 1e5, range(4))
    X = O.solve(VR, tau, b)
    normA = np.linalg.norm(A, 2)
    for c in range(4):
        r = b[:, c] - A @ X[:, c]
        opt = np.linalg.norm(A.T @ r) / (normA * np.linalg.norm(r))
        assert opt <= 1e-12
    Xc = O.solve(VR, tau, p)
    assert np.linalg.norm(Xc - x_true) / np.linalg.norm(x_true) <= 1e-12
    # Q^T b below row n carries the least-squares residual norm
    C = O.apply_qt(VR, tau, b)
    for c in range(4):
        assert abs(np.linalg.norm(C[sc.n:, c]) - np.linalg.norm(b[:, c] - A @ X[:, c])) <= 1e-12


def test_triangular_solves_match_library(c1):
    sc, A, VR, tau, info = c1
    n = A.shape[1]
    R = np.triu(VR[:n])
    g = np.random.default_rng(5).standard_normal((n, 3))
    assert np.max(np.abs(O.back_substitute(VR, g) - sla.solve_triangular(R, g))) <= 1e-10
    assert np.max(np.abs(O.forward_substitute_rt(VR, g) - sla.solve_triangular(R, g, trans="T"))) <= 1e-10


def test_adjoint_dot_product_identity(c1):
    """<x(db), g> = <db, grad_b(g)> for the linear map b -> x."""
    sc, A, VR, tau, info = c1
    rng = np.random.default_rng(11)
    db = rng.standard_normal((sc.m, 5))
    g = rng.standard_normal((sc.n, 5))
    X = O.solve(VR, tau, db)
    Y = O.adjoint(VR, tau, g)
    for c in range(5):
        lhs, rhs = X[:, c] @ g[:, c], db[:, c] @ Y[:, c]
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-13
    # the adjoint lies in range(A): it equals A (A^T A)^{-1} g
    Z = A @ np.linalg.solve(A.T @ A, g)
    assert np.linalg.norm(Y - Z) / np.linalg.norm(Z) <= 1e-10


def test_adjoint_square_equals_inverse_transpose():
    sc = synth.scanner(8, 12, 16)
    A = O.system_dense(sc)[::3][:64] + 0.05 * np.eye(64)
    VR, tau, info = O.householder_qr(A)
    g = np.random.default_rng(4).standard_normal(64)
    y = O.adjoint(VR, tau, g)
    yr = np.linalg.solve(A.T, g)
    assert np.linalg.norm(y - yr) / np.linalg.norm(yr) <= 1e-16 * np.linalg.cond(A) * 100


def test_rank_deficiency_reported():
    sc = synth.scanner(10, 12, 20)
    A = O.system_dense(sc)
    A[:, 17] = 0.0
    VR, tau, info = O.householder_qr(A)
    assert info == 18 and tau[17] == 0.0
    A2 = O.system_dense(sc)
    A2[:, 30] = A2[:, 4]
    VR2, _, info2 = O.householder_qr(A2)
    assert info2 == 0 and O.rank_report(VR2)["numerically_deficient"]
    assert not O.rank_report(O.householder_qr(O.system_dense(sc))[0])["numerically_deficient"]
