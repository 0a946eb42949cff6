"""Seeded synthetic inputs: scanner geometries, ellipse phantoms, Poisson noise.

This module draws random numbers and fixes scanner parameters; it contains
none of the reconstruction arithmetic (no projector, no factorization, no
solve).  Both the HIP path and the CPU oracle consume what it produces, so it
imports neither of them.

The paper's datasets (COVID-CT-MD, the Mayo DICOM-CT-PD scans) are not
available here; seeded random-ellipse phantoms with the shapes of the paper's
fan-beam workloads stand in for them (Sec. 3.1 and 3.2 simulate sinograms by
projecting images with the same projector that builds A, which is what
``noisy_sinogram`` assumes of its ``p`` argument).

Seeds: ``numpy.random.default_rng([config, slice, stream])`` with stream
0 = phantom, 1 = noise, 2 = batch sizes, 3 = gradients / directions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

STREAM_PHANTOM, STREAM_NOISE, STREAM_BATCH, STREAM_GRAD = 0, 1, 2, 3


@dataclass(frozen=True)
class Scanner:
    """Fan-beam scanner parameters (Table 1 / Table 5 list the same fields).

    n_pix: image side N (n = N^2 unknowns); n_angles: views over 360 degrees;
    n_det: detector bins; grid_width: physical side W of the square image;
    sid / sdd: source-to-isocentre / source-to-detector distances;
    det_length: length of the flat detector; angle0: first view angle (rad).
    """

    n_pix: int
    n_angles: int
    n_det: int
    grid_width: float
    sid: float
    sdd: float
    det_length: float
    angle0: float = 0.0
    projector: int = 0          # 0: Siddon's exact lengths, 1: Joseph's interpolation

    @property
    def m(self) -> int:
        return self.n_angles * self.n_det

    @property
    def n(self) -> int:
        return self.n_pix * self.n_pix

    def as_dict(self) -> dict:
        return asdict(self)


def scanner(n_pix: int, n_angles: int, n_det: int, grid_width: float = 1.0,
            angle0: float = 0.0, projector: int = 0) -> Scanner:
    """The scanner reading used for every workload.

    Source-to-isocentre distance 2W; source-to-detector twice that (the 75 cm /
    150 cm ratio of Table 1); a flat detector whose fan just covers the circle
    inscribed in the image, so that every ray crosses the image.  (A fan wide
    enough for the circumscribed circle wastes about a third of the rays on
    empty space and leaves the 120-view x 640-bin system at 256^2 rank
    deficient; the inscribed fan keeps it full rank.)
    """
    W = float(grid_width)
    sid = 2.0 * W
    sdd = 2.0 * sid
    half_fan = math.asin(W / (2.0 * sid))
    det_length = 2.0 * sdd * math.tan(half_fan)
    return Scanner(n_pix, n_angles, n_det, W, sid, sdd, det_length, float(angle0), int(projector))


# Workloads: image side, views, bins, slices, incident photons per bin.
WORKLOADS = {
    "c1_32": dict(cfg=1, n_pix=32, n_angles=30, n_det=64, slices=4, I0=1e5),
    "c2_128": dict(cfg=2, n_pix=128, n_angles=90, n_det=256, slices=64, I0=5e4),
    "c3_256": dict(cfg=3, n_pix=256, n_angles=120, n_det=640, slices=512, I0=5e4),
    "c5_512": dict(cfg=5, n_pix=512, n_angles=180, n_det=1472, slices=1024, I0=5e4),
}


def workload_scanner(name: str) -> Scanner:
    w = WORKLOADS[name]
    return scanner(w["n_pix"], w["n_angles"], w["n_det"])


def rng(cfg: int, slice_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(cfg), int(slice_id), int(stream)])


def phantom(n_pix: int, gen: np.random.Generator, grid_width: float = 1.0) -> np.ndarray:
    """Additive random-ellipse phantom, flattened with column j = iy * N + ix.

    5..10 ellipses; centre at radius U[0, W/4] and angle U[0, 2 pi); semi-axes
    U[0.03 W, 0.2 W]; rotation U[0, pi); density U[0, 1].  A pixel takes the
    sum of the densities of the ellipses containing its centre.
    """
    W = float(grid_width)
    N = int(n_pix)
    c = -0.5 * W + (np.arange(N) + 0.5) * (W / N)
    X, Y = np.meshgrid(c, c, indexing="xy")          # X[iy, ix], Y[iy, ix]
    img = np.zeros((N, N), dtype=np.float64)
    k = int(gen.integers(5, 11))
    for _ in range(k):
        r = gen.uniform(0.0, 0.25 * W)
        phi = gen.uniform(0.0, 2.0 * math.pi)
        cx, cy = r * math.cos(phi), r * math.sin(phi)
        a = gen.uniform(0.03 * W, 0.2 * W)
        b = gen.uniform(0.03 * W, 0.2 * W)
        psi = gen.uniform(0.0, math.pi)
        rho = gen.uniform(0.0, 1.0)
        dx, dy = X - cx, Y - cy
        u = dx * math.cos(psi) + dy * math.sin(psi)
        v = -dx * math.sin(psi) + dy * math.cos(psi)
        img += rho * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img.reshape(-1)


def phantoms(cfg: int, n_pix: int, slice_ids) -> np.ndarray:
    """n x len(slice_ids) column-major stack of phantoms (FP64)."""
    cols = [phantom(n_pix, rng(cfg, s, STREAM_PHANTOM)) for s in slice_ids]
    return np.stack(cols, axis=1)


def noisy_sinogram(p: np.ndarray, I0: float, gen: np.random.Generator) -> np.ndarray:
    """Low-dose measurement of line integrals p: counts ~ Poisson(I0 exp(-p)),
    b = -ln(max(counts, 1) / I0) (zero counts clamped to one)."""
    counts = gen.poisson(I0 * np.exp(-np.asarray(p, dtype=np.float64)))
    return -np.log(np.maximum(counts, 1).astype(np.float64) / I0)


def noisy_sinograms(cfg: int, P: np.ndarray, I0: float, slice_ids) -> np.ndarray:
    """Column s of the result is the noisy version of column s of P."""
    out = np.empty_like(P, dtype=np.float64)
    for c, s in enumerate(slice_ids):
        out[:, c] = noisy_sinogram(P[:, c], I0, rng(cfg, s, STREAM_NOISE))
    return out


def uneven_batches(total: int = 4096, lo: int = 1, hi: int = 512, cfg: int = 4) -> list[int]:
    """Seeded batch sizes in [lo, hi] summing to ``total`` (last one cut)."""
    g = rng(cfg, 0, STREAM_BATCH)
    sizes, acc = [], 0
    while acc < total:
        s = int(g.integers(lo, hi + 1))
        s = min(s, total - acc)
        sizes.append(s)
        acc += s
    return sizes


def gradients(n: int, k: int, cfg: int = 4) -> np.ndarray:
    """k upstream gradients g ~ N(0, 1), FP32 values, n x k column-major."""
    g = rng(cfg, 0, STREAM_GRAD)
    return g.standard_normal((n, k)).astype(np.float32).astype(np.float64)


def directions(m: int, k: int, cfg: int = 4) -> np.ndarray:
    """k unit-norm perturbation directions of length m (for finite differences)."""
    g = rng(cfg, 1, STREAM_GRAD)
    d = g.standard_normal((m, k))
    return d / np.linalg.norm(d, axis=0, keepdims=True)
