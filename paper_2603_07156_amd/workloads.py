"""Seeded synthetic OT instances (inputs only).

This module builds cost matrices and marginals; it holds none of the solver's
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it.  Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in
the order written, builds the squared-Euclidean cost in FP64 and divides it by
its maximum, which is the paper's set-up convention (costs scaled to unit
infinity norm, Section 5 "Setup").

Instances
---------
``uniform_points``   points i.i.d. uniform in [0,1]^d for both sides, uniform
                     weights (the small and the 10^4 workloads).
``gmm_points``       2-D Gaussian mixtures (5 components, std 0.05) per side,
                     weights ~ U(0.1, 1) renormalised.
``cube_vs_gmm``      3-D unit-cube points vs an 8-component 3-D mixture
                     (std 0.08), uniform weights (the 20000 precision form).
``paper_uniform``    C_ij ~ U(0,1), a, b ~ U(0,1) normalised (Section 5.1).
``paper_square``     C_ij = (i-j)^2 / max, a, b ~ U(0,1) normalised (Section 5.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Instance:
    """One OT problem: min <C,X> s.t. X1=a, X^T1=b, X>=0 (eq. (1))."""

    C: np.ndarray          # (m, n) float64, row-major, max entry 1
    a: np.ndarray          # (m,) float64, positive, sums to 1
    b: np.ndarray          # (n,) float64, positive, sums to 1
    eta: float
    name: str
    x: np.ndarray | None = None   # source points, when the cost comes from points
    y: np.ndarray | None = None   # target points

    @property
    def m(self) -> int:
        return self.C.shape[0]

    @property
    def n(self) -> int:
        return self.C.shape[1]


def sqdist_cost(x: np.ndarray, y: np.ndarray, dtype=np.float64, block: int = 2048) -> np.ndarray:
    """C_ij = sum_d (x_id - y_jd)^2 divided by max_ij C_ij, built row-block by row-block.

    The blocked loop gives the same bits as the one-shot expression
    ``((x[:,None]-y[None])**2).sum(-1)`` (each entry is the same left-to-right
    sum over d) without a (m, n, d) temporary.
    """
    m = x.shape[0]
    C = np.empty((m, y.shape[0]), dtype=np.float64)
    for i0 in range(0, m, block):
        i1 = min(m, i0 + block)
        d = x[i0:i1, None, :] - y[None, :, :]
        C[i0:i1] = (d * d).sum(-1)
    C /= C.max()
    if dtype != np.float64:
        C = C.astype(dtype)
    return C


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / v.sum()


def uniform_points(n: int, seed: int, m: int | None = None, d: int = 2, eta: float = 1e-2) -> Instance:
    """Points uniform in [0,1]^d on both sides; a = 1/m, b = 1/n."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.random((m, d))
    y = rng.random((n, d))
    C = sqdist_cost(x, y)
    a = np.full(m, 1.0 / m)
    b = np.full(n, 1.0 / n)
    return Instance(C, a, b, eta, f"uniform_points{d}d_{m}x{n}_s{seed}", x, y)


def _gmm(rng: np.random.Generator, N: int, K: int, d: int, std: float) -> np.ndarray:
    means = rng.random((K, d))
    comp = rng.integers(0, K, N)
    return means[comp] + std * rng.standard_normal((N, d))


def gmm_points(n: int, seed: int, m: int | None = None, eta: float = 1e-2) -> Instance:
    """Source and target each a 5-component 2-D Gaussian mixture (std 0.05, no clipping);
    weights ~ U(0.1, 1) renormalised."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = _gmm(rng, m, 5, 2, 0.05)
    y = _gmm(rng, n, 5, 2, 0.05)
    a = _normalise(rng.uniform(0.1, 1.0, m))
    b = _normalise(rng.uniform(0.1, 1.0, n))
    C = sqdist_cost(x, y)
    return Instance(C, a, b, eta, f"gmm_points_{m}x{n}_s{seed}", x, y)


def cube_vs_gmm(n: int, seed: int, m: int | None = None, eta: float = 1e-2,
                cost_dtype=np.float64) -> Instance:
    """3-D unit-cube points vs an 8-component 3-D mixture (std 0.08); uniform weights."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.random((m, 3))
    y = _gmm(rng, n, 8, 3, 0.08)
    C = sqdist_cost(x, y, dtype=cost_dtype)
    a = np.full(m, 1.0 / m)
    b = np.full(n, 1.0 / n)
    return Instance(C, a, b, eta, f"cube_vs_gmm_{m}x{n}_s{seed}", x, y)


def paper_uniform(n: int, seed: int, m: int | None = None, eta: float = 1e-4) -> Instance:
    """Section 5.1 'Uniform': C_ij ~ U(0,1); a, b ~ U(0,1) normalised."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    a = _normalise(rng.random(m))
    b = _normalise(rng.random(n))
    C = rng.random((m, n))
    C /= C.max()
    return Instance(C, a, b, eta, f"paper_uniform_{m}x{n}_s{seed}")


def paper_square(n: int, seed: int, m: int | None = None, eta: float = 1e-4) -> Instance:
    """Section 5.1 'Square': C_ij = (i-j)^2 normalised; a, b ~ U(0,1) normalised."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    a = _normalise(rng.random(m))
    b = _normalise(rng.random(n))
    i = np.arange(m, dtype=np.float64)[:, None]
    j = np.arange(n, dtype=np.float64)[None, :]
    C = (i - j) ** 2
    C /= C.max()
    return Instance(C, a, b, eta, f"paper_square_{m}x{n}_s{seed}")


def random_dual(n: int, seed: int, scale: float = 1e-2) -> np.ndarray:
    """A centred random dual vector gamma (for evaluating passes away from 0)."""
    rng = np.random.default_rng(seed)
    g = scale * rng.standard_normal(n)
    return g - g.mean()


def _grid_histogram(rng: np.random.Generator, size: int):
    """A histogram on a side x side grid (side = round(sqrt(size))) over [0,1]^2: a sum of
    1-5 Gaussian blobs (centres U[0,1]^2, std U(0.05, 0.2), weights U(0,1)) plus a 1e-6
    floor, normalised; returns (coordinates (side^2, 2), weights)."""
    side = max(2, int(round(np.sqrt(size))))
    u = np.arange(side, dtype=np.float64) / (side - 1)
    pts = np.stack(np.meshgrid(u, u, indexing="ij"), -1).reshape(-1, 2)
    K = int(rng.integers(1, 6))
    centres = rng.random((K, 2))
    stds = rng.uniform(0.05, 0.2, K)
    wts = rng.random(K)
    h = np.full(len(pts), 1e-6)
    for c, s_, w_ in zip(centres, stds, wts):
        h += w_ * np.exp(-((pts - c) ** 2).sum(-1) / (2.0 * s_ * s_))
    return pts, _normalise(h)


def grid_histogram_batch(count: int, seed: int, eta: float = 1e-2, lo: int = 64,
                         hi: int = 2048) -> list:
    """The batched workload: `count` problems whose sizes m, n are drawn uniformly in
    [lo, hi] and rounded to square grids; each side a grid histogram, cost the squared
    coordinate distance divided by its maximum."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        m_req, n_req = (int(v) for v in rng.integers(lo, hi + 1, 2))
        xs, a = _grid_histogram(rng, m_req)
        ys, b = _grid_histogram(rng, n_req)
        C = sqdist_cost(xs, ys)
        out.append(Instance(C, a, b, eta, f"grid_batch_{t}_s{seed}", xs, ys))
    return out


def points_cost(x: np.ndarray, y: np.ndarray, scale: float, block: int = 2048) -> np.ndarray:
    """C_ij = scale * ((x_i1 - y_j1)^2 + (x_i2 - y_j2)^2 [+ (x_i3 - y_j3)^2]): the points cost
    in the library's order of operations (differences, squares, sums left to right, then one
    product with the scale; numpy fuses none of them), so that the oracle sees exactly the
    matrix the kernels form."""
    m = x.shape[0]
    C = np.empty((m, y.shape[0]), dtype=np.float64)
    for i0 in range(0, m, block):
        i1 = min(m, i0 + block)
        d = x[i0:i1, None, :] - y[None, :, :]
        C[i0:i1] = (d * d).sum(-1)
    C *= scale
    return C


def points_scale(x: np.ndarray, y: np.ndarray, block: int = 2048) -> float:
    """1 / max_ij sum_d (x_id - y_jd)^2 (so that the points cost has maximum 1 up to rounding)."""
    mx = 0.0
    for i0 in range(0, x.shape[0], block):
        d = x[i0:i0 + block, None, :] - y[None, :, :]
        mx = max(mx, float((d * d).sum(-1).max()))
    return 1.0 / mx
