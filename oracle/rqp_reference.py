"""FP64 CPU reference of the relaxed QHD for box-constrained quadratic programming
(App. F, "A relaxed implementation of QHD for quadratic programming", and
Algorithm 2; simulated classically as in the paper's Sim-QHD).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

Model.  minimise f(x) = 1/2 x^T Q x + b^T x over the box [0, 1]^d.  Each axis is
the lattice x = j / r, j = 0..r (r cells, r + 1 points, not periodic); the state is
a vector over (j_1, ..., j_d) (axis 1 fastest).  The Hamiltonian is

    H(t) = -(a(t) / 2) r^2 A'_d + b(t) F_d,      A'_d = sum_k I x .. x A' x .. x I,

with F_d = diag f on the lattice and A' the relaxed chain adjacency: the symmetric
tridiagonal (r+1) x (r+1) matrix with off-diagonal entries sqrt((j+1)(r-j)/r),
j = 0..r-1 (the Hamming encoding's S_x / sqrt(r) on the symmetric subspace of r
qubits; r^2 = 1/h^2 is the finite-difference scale of the Laplacian).  The initial
state is the discrete Gaussian prod_k sqrt(C(r, j_k) / 2^r), the image of the uniform
superposition of the d r qubits.

Integration: the symmetric split-step product with a, b at the step midpoint,
kinetic factor exp(+i dt a r^2 / 2 A') along every axis (scipy's expm, a library
primitive), each factor exact.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm


def relaxed_adjacency(r: int) -> np.ndarray:
    """A' of one axis, (r+1) x (r+1)."""
    A = np.zeros((r + 1, r + 1))
    for j in range(r):
        v = math.sqrt((j + 1) * (r - j) / r)
        A[j + 1, j] = A[j, j + 1] = v
    return A


def lattice(d: int, r: int):
    """Coordinates x_k = j_k / r of every lattice point, shape (r+1,)*d + (d,), array
    axis order (j_d, ..., j_1) so that axis 1 is the fastest (last) array axis."""
    g = np.arange(r + 1) / r
    mesh = np.meshgrid(*([g] * d), indexing="ij")  # mesh[a] varies along array axis a
    # array axis a holds x_{d-a}
    return np.stack([mesh[d - 1 - k] for k in range(d)], axis=-1)


def objective(Q: np.ndarray, b: np.ndarray, r: int) -> np.ndarray:
    """f on the lattice (FP64), array shape (r+1,)*d with x_1 on the last axis."""
    d = len(b)
    X = lattice(d, r)
    return 0.5 * np.einsum("...i,ij,...j->...", X, Q, X) + X @ b


def initial_state(d: int, r: int) -> np.ndarray:
    amp1 = np.array([math.sqrt(math.comb(r, j) / 2.0 ** r) for j in range(r + 1)])
    psi = np.ones((1,) * 0)
    for _ in range(d):
        psi = np.multiply.outer(psi, amp1)
    return psi.astype(np.complex128)


def nesterov_ab(t: float, eps: float):
    return 2.0 / (eps + t ** 3), 2.0 * t ** 3


def apply_axis(psi: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """Apply M along coordinate axis k (1-based; axis 1 is the last array axis)."""
    ax = psi.ndim - k
    return np.moveaxis(np.tensordot(M, psi, axes=([1], [ax])), 0, ax)


def evolve(f: np.ndarray, psi: np.ndarray, r: int, dt: float, nsteps: int, ab, j0: int = 0) -> np.ndarray:
    """Symmetric split steps j0 .. j0+nsteps-1; ab(t) -> (a, b) at t = (j + 1/2) dt."""
    psi = np.asarray(psi, dtype=np.complex128).copy()
    A = relaxed_adjacency(r)
    d = psi.ndim
    for j in range(j0, j0 + nsteps):
        a, b = ab((j + 0.5) * dt)
        half = np.exp(-0.5j * dt * b * f)
        psi = half * psi
        M = expm(0.5j * dt * a * r * r * A)
        for k in range(1, d + 1):
            psi = apply_axis(psi, M, k)
        psi = half * psi
    return psi


def readout(f: np.ndarray, psi: np.ndarray, tol: float = 1e-9):
    """norm, E[f] (divided by the norm), probability of the lattice minimisers (f within
    tol of the minimum, divided by the norm), per-axis marginals (k = 1..d, each r+1)."""
    rho = np.abs(psi) ** 2
    norm = float(rho.sum())
    fmin = float(f.min())
    d = psi.ndim
    marg = [rho.sum(axis=tuple(a for a in range(d) if a != d - k)) for k in range(1, d + 1)]
    return dict(norm=norm, e_f=float((f * rho).sum()) / norm, p_min=float(rho[f <= fmin + tol].sum()) / norm,
                f_min=fmin, marginals=np.array(marg))


def dense_hamiltonian(Q, b, r, a, bt):
    """H as a dense matrix over the flattened lattice (C order of the array axes)."""
    d = len(b)
    A = relaxed_adjacency(r)
    n = r + 1
    Ad = np.zeros((n ** d, n ** d))
    for k in range(1, d + 1):
        mats = [np.eye(n)] * d
        mats[d - k] = A  # array axis d-k holds coordinate k
        m = np.array([[1.0]])
        for mm in mats:
            m = np.kron(m, mm)
        Ad += m
    F = np.diag(objective(Q, b, r).reshape(-1))
    return -(a / 2.0) * r * r * Ad + bt * F
