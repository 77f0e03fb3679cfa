"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module holds no arithmetic of the method: it only draws landscape
parameters and evaluates the objective f on the mesh, in FP64, so that both
sides of every parity check receive the very same arrays.

Landscape family (it stands in for the paper's 2-D benchmark functions of
App. C.1, which are not reproduced here):

    f(x) = 0.5 * q * ||x - c||^2 + sum_j A_j cos(2 pi k_j . x + theta_j)

with c ~ U[0,1]^d, q ~ U[1,5], A_j ~ U[0.2,1], integer k_j uniform in
[-kmax, kmax]^d (an all-zero draw is redrawn), theta_j ~ U[0, 2 pi).  The
quadratic uses the unwrapped Euclidean distance, mirroring the paper's
truncation of non-periodic test functions to the box (App. C.1).  Draw order
from numpy's PCG64(seed): c, q, then (A_j, k_j, theta_j) per term.

The mesh is the periodic one of App. E.1: x_i = lo + i (hi - lo) / N,
i = 0 .. N-1.  Arrays are C-ordered [..., y, x] (x fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Landscape:
    ndim: int
    c: np.ndarray        # (ndim,)  centre, array-axis order
    q: float
    amp: np.ndarray      # (m,)
    k: np.ndarray        # (m, ndim) integer wave vectors, array-axis order
    theta: np.ndarray    # (m,)


def draw_landscape(seed: int, ndim: int = 2, n_terms: int = 8, kmax: int = 6,
                   rng: np.random.Generator = None) -> Landscape:
    """Draw one landscape (see the module docstring for the distribution)."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.0, 1.0, size=ndim)
    q = float(rng.uniform(1.0, 5.0))
    amp = np.empty(n_terms)
    k = np.empty((n_terms, ndim), dtype=np.int64)
    theta = np.empty(n_terms)
    for j in range(n_terms):
        amp[j] = rng.uniform(0.2, 1.0)
        kj = rng.integers(-kmax, kmax + 1, size=ndim)
        while not np.any(kj):
            kj = rng.integers(-kmax, kmax + 1, size=ndim)
        k[j] = kj
        theta[j] = rng.uniform(0.0, TWO_PI)
    return Landscape(ndim, c, q, amp, k, theta)


def mesh_axes(shape: Sequence[int], box=None) -> List[np.ndarray]:
    nd = len(shape)
    box = box if box is not None else [(0.0, 1.0)] * nd
    return [box[a][0] + np.arange(shape[a], dtype=np.float64) * ((box[a][1] - box[a][0]) / shape[a])
            for a in range(nd)]


def evaluate(ls: Landscape, shape: Sequence[int], box=None) -> np.ndarray:
    """f on the mesh, FP64, C-ordered (array axes as in ``shape``)."""
    nd = len(shape)
    if nd != ls.ndim:
        raise ValueError("landscape dimension does not match the mesh")
    axes = mesh_axes(shape, box)
    f = np.zeros(tuple(shape), dtype=np.float64)
    for a in range(nd):
        sh = [1] * nd
        sh[a] = shape[a]
        f += (0.5 * ls.q) * ((axes[a] - ls.c[a]) ** 2).reshape(sh)
    for j in range(len(ls.amp)):
        # cos(2 pi k.x + theta) = Re( e^{i theta} prod_a e^{2 pi i k_a x_a} )
        term = np.full((1,) * nd, ls.amp[j] * np.exp(1j * ls.theta[j]), dtype=np.complex128)
        for a in range(nd):
            sh = [1] * nd
            sh[a] = shape[a]
            term = term * np.exp(1j * TWO_PI * ls.k[j, a] * axes[a]).reshape(sh)
        f += term.real
    return f


def landscape_grid(seed: int, shape: Sequence[int], n_terms: int = 8, kmax: int = 6,
                   box=None) -> np.ndarray:
    return evaluate(draw_landscape(seed, len(shape), n_terms, kmax), shape, box)


# --------------------------------------------------------------------------------------
# Workload recipes (sizes, schedules and counts of the benchmark configurations)

NESTEROV_EPS = 1e-3  # a(t) = 2/(eps + t^3), b(t) = 2 t^3 (App. C.2.1, eq. nonconvex_QHD_h)


@dataclass
class InstanceSpec:
    seed: int
    shape: Tuple[int, ...]
    nsteps: int
    dt: float
    n_terms: int
    kmax: int

    def grid(self) -> np.ndarray:
        return landscape_grid(self.seed, self.shape, self.n_terms, self.kmax)

    @property
    def points(self) -> int:
        return int(np.prod(self.shape))


def single_2d(n: int, seed: int = 1234, dt: float = 1e-3, T: float = 10.0,
              n_terms: int = 8) -> InstanceSpec:
    """One 2-D instance on [0,1]^2 (the paper's 2-D experiment shape, App. C.2.1)."""
    return InstanceSpec(seed, (n, n), int(round(T / dt)), dt, n_terms, 6)


def batched_2d(count: int = 768, seed_base: int = 20230301, sizes=(128, 256, 512),
               t_range=(5.0, 20.0), dt: float = 1e-3, terms=(8, 24)) -> List[InstanceSpec]:
    """Uneven batch: per instance, from PCG64(seed_base + i), draw the grid size
    uniformly from ``sizes``, T ~ U[t_range], the number of cosine terms
    uniformly in [terms[0], terms[1]]; then the landscape (its own seed)."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        T = float(rng.uniform(t_range[0], t_range[1]))
        m = int(rng.integers(terms[0], terms[1] + 1))
        out.append(InstanceSpec(seed_base + 1_000_000 + i, (n, n), int(round(T / dt)), dt, m, 6))
    return out


def batch_3d(count: int = 16, n: int = 128, seed_base: int = 3030, dt: float = 2e-3,
             T: float = 10.0, n_terms: int = 16) -> List[InstanceSpec]:
    return [InstanceSpec(seed_base + i, (n, n, n), int(round(T / dt)), dt, n_terms, 4)
            for i in range(count)]


def qaa_batch(count: int = 512, seed_base: int = 19820301, sizes=(64, 128), T: float = 10.0,
              dt: float = 1e-3, terms=(8, 24)) -> List[InstanceSpec]:
    """Batch for the baseline-QAA comparison at the paper's QAA resolutions (64 and 128
    points per axis, App. C.2.2) and its evolution time T = 10: per instance, from
    PCG64(seed_base + i), the grid size uniformly from ``sizes`` and the number of
    cosine terms uniformly in [terms[0], terms[1]]; every instance runs T / dt steps."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        m = int(rng.integers(terms[0], terms[1] + 1))
        out.append(InstanceSpec(seed_base + 1_000_000 + i, (n, n), int(round(T / dt)), dt, m, 6))
    return out


def qp_instances(count: int, dim: int = 5, seed_base: int = 5050) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Box-constrained QP instances (App. G.1 recipe for the dense 5-dimensional group):
    the Hessian Q symmetric with entries uniform in [-1, 1] (upper triangle drawn,
    mirrored), the linear term b uniform in [-1, 1]; from PCG64(seed_base + i), draw
    order Q then b."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        U = rng.uniform(-1.0, 1.0, size=(dim, dim))
        Q = np.triu(U) + np.triu(U, 1).T
        b = rng.uniform(-1.0, 1.0, size=dim)
        out.append((Q, b))
    return out
