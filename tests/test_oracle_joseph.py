"""Pins of the oracle's Joseph projector (the interpolating projector the
paper builds A with, Sec. 3.1) against closed forms: rays through pixel
centres, a ray between two rows, the diagonal, exactness for images linear in
x and y (linear interpolation and the midpoint rule are both exact there),
the 90-degree rotation symmetry, row sums, second-order convergence to the
exact line integrals of a smooth image, and the CSR form against the dense
one."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2412_07631_amd import synth


def dense_row(pix, w, n):
    row = np.zeros(n)
    np.add.at(row, pix, w)
    return row


@pytest.mark.parametrize("N", [4, 7, 16])
def test_horizontal_ray_through_a_row_of_centres(N):
    h = 1.0 / N
    for iy in (0, N // 2, N - 1):
        yc = -0.5 + (iy + 0.5) * h
        pix, w = O.joseph_ray(-2.0, yc, 2.0, yc, N)
        row = dense_row(pix, w, N * N)
        expect = np.zeros(N * N)
        expect[iy * N:(iy + 1) * N] = h
        assert np.max(np.abs(row - expect)) <= 1e-15


def test_ray_between_two_rows_splits_evenly():
    N = 8
    h = 1.0 / N
    y = -0.5 + 3 * h                                      # between the centres of rows 2 and 3
    row = dense_row(*O.joseph_ray(-2.0, y, 2.0, y, N), N * N)
    expect = np.zeros(N * N)
    expect[2 * N:4 * N] = h / 2
    assert np.max(np.abs(row - expect)) <= 1e-15


def test_vertical_ray_and_diagonal():
    N = 10
    h = 1.0 / N
    xc = -0.5 + (6 + 0.5) * h
    row = dense_row(*O.joseph_ray(xc, -2.0, xc, 2.0, N), N * N)
    expect = np.zeros(N * N)
    expect[6::N] = h
    assert np.max(np.abs(row - expect)) <= 1e-15
    # y = x passes through every diagonal pixel centre: h sqrt(2) each
    row = dense_row(*O.joseph_ray(-1.0, -1.0, 1.0, 1.0, N), N * N)
    expect = np.zeros(N * N)
    expect[[i * N + i for i in range(N)]] = h * math.sqrt(2.0)
    assert np.max(np.abs(row - expect)) <= 1e-14


def test_linear_images_are_integrated_exactly():
    """For f(x, y) = a + b y + c x the sampled, interpolated sum equals the
    line integral over the dominant-axis slab: L W (a + b (y0 - x0 s)) for
    an x-major ray y = y0 + (x - x0) s, L = |p1 - p0| / |dx|, as long as every
    sample falls between pixel centres of the grid."""
    N = 32
    h = 1.0 / N
    c = -0.5 + (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b, cc = rng.uniform(-1, 1, 3)
        img = (a + b * Y + cc * X).ravel()
        s = rng.uniform(-0.6, 0.6)                       # |slope| < 1: x-major
        y0c = rng.uniform(-0.1, 0.1)
        x0, x1 = -2.0, 2.0
        y0, y1 = y0c + (x0 - 0.0) * s, y0c + (x1 - 0.0) * s
        row = dense_row(*O.joseph_ray(x0, y0, x1, y1, N), N * N)
        L = math.hypot(x1 - x0, y1 - y0) / abs(x1 - x0)
        exact = L * 1.0 * (a + b * (y0 - x0 * s))
        assert abs(row @ img - exact) <= 1e-13 * (1 + abs(exact))


def test_rotation_by_ninety_degrees_permutes_pixels():
    N = 12
    rng = np.random.default_rng(8)
    for _ in range(10):
        x0, y0 = 2.0 * np.cos(t := rng.uniform(0, 2 * np.pi)), 2.0 * np.sin(t)
        x1, y1 = rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5)
        r0 = dense_row(*O.joseph_ray(x0, y0, x1, y1, N), N * N).reshape(N, N)       # [iy, ix]
        r1 = dense_row(*O.joseph_ray(-y0, x0, -y1, x1, N), N * N).reshape(N, N)
        # (x, y) -> (-y, x): pixel (ix, iy) -> (N-1-iy, ix)
        expect = np.zeros((N, N))
        for iy in range(N):
            for ix in range(N):
                expect[ix, N - 1 - iy] = r0[iy, ix]
        assert np.max(np.abs(r1 - expect)) <= 1e-13 * max(1.0, np.max(np.abs(r0)))


def gaussian_line_integrals(sc, N, sig, cx, cy):
    """Sampled Gaussian image and the exact line integrals of the continuous
    Gaussian along every ray: sqrt(2 pi) sig exp(-d^2 / (2 sig^2)), d the
    ray's distance from the centre (the tails outside the image are below
    1e-7 of the peak here)."""
    c = -0.5 + (np.arange(N) + 0.5) / N
    X, Y = np.meshgrid(c, c, indexing="xy")
    img = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sig ** 2)).ravel()
    rays = O.rays(sc)
    p0, d = rays[:, :2], rays[:, 2:] - rays[:, :2]
    dn = d / np.linalg.norm(d, axis=1)[:, None]
    v = np.array([cx, cy]) - p0
    dist = np.abs(v[:, 0] * dn[:, 1] - v[:, 1] * dn[:, 0])
    return img, math.sqrt(2 * math.pi) * sig * np.exp(-dist ** 2 / (2 * sig ** 2))


def test_row_sums_and_line_integrals_of_a_smooth_image():
    sc = synth.scanner(48, 30, 64)
    scj = synth.scanner(48, 30, 64, projector=1)
    AJ = O.system_dense(scj)
    # every sample stands for one pixel width along the dominant axis, so a
    # row sum never exceeds the ray's length across the dominant slab
    rays = O.rays(sc)
    d = rays[:, 2:] - rays[:, :2]
    L = np.hypot(d[:, 0], d[:, 1]) / np.maximum(np.abs(d[:, 0]), np.abs(d[:, 1]))
    assert np.all(AJ.sum(axis=1) <= L * 1.0 + 1e-12)
    # a smooth image: the projections approach the exact line integrals of the
    # continuous image at second order in the pixel size
    errs = []
    for N in (24, 48):
        scn = synth.scanner(N, 30, 64, projector=1)
        img, exact = gaussian_line_integrals(scn, N, 0.12, 0.05, -0.02)
        errs.append(np.max(np.abs(O.system_dense(scn) @ img - exact)) / np.max(exact))
    print("Joseph max error / peak at N = 24, 48:", errs)
    assert errs[1] <= 1e-2 and errs[0] / errs[1] >= 3.0
    # Joseph's A of the 3360 x 2304 test system has full column rank too
    scr = synth.scanner(48, 40, 84, projector=1)
    assert np.linalg.matrix_rank(O.system_dense(scr)) == scr.n


def test_csr_equals_dense_joseph():
    scj = synth.scanner(20, 12, 30, projector=1)
    A = O.system_dense(scj)
    row_ptr, col, val = O.system_csr(scj)
    D = np.zeros_like(A)
    for i in range(scj.m):
        D[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    assert np.array_equal(D, A)
    assert all(np.all(np.diff(col[row_ptr[i]:row_ptr[i + 1]]) > 0) for i in range(scj.m))
