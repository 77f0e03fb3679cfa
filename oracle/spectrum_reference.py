"""FP64 CPU reference for the spectrum of the QHD Hamiltonian on the mesh.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

The discrete Hamiltonian at time t is H(t) = a(t) K + b(t) diag(f), with K the
Fourier-diagonal kinetic operator -1/2 Laplacian of the split-operator scheme
(App. C.2.1 eq. prod_qhd_fft; App. E.1): K = F^{-1} diag(|k|^2 / 2) F with
k = 2 pi n / L in FFT order.  The paper studies the low-lying spectrum of H(t)
along the QHD path (App. D, its energy-ratio and probability-spectrum figures);
this module builds H as a dense matrix from that definition and diagonalises it
with numpy's eigh (a library primitive), for meshes small enough to hold H.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def dft_matrix(n: int) -> np.ndarray:
    """F_{jm} = e^{-2 pi i j m / n} (unnormalised forward DFT)."""
    j = np.arange(n)
    return np.exp(-2j * math.pi * np.outer(j, j) / n)


def kinetic_matrix(shape: Sequence[int], box) -> np.ndarray:
    """Dense K = F^{-1} diag(|k|^2/2) F on a C-ordered mesh of the given shape
    (array axes; box[a] = (lo, hi) per array axis)."""
    mats = []
    for a, n in enumerate(shape):
        L = box[a][1] - box[a][0]
        m = np.arange(n)
        kk = 2.0 * math.pi * np.where(m < n // 2, m, m - n) / L
        F = dft_matrix(n)
        Finv = np.conj(F).T / n
        mats.append((F, Finv, 0.5 * kk * kk))
    N = int(np.prod(shape))
    K = np.zeros((N, N), dtype=np.complex128)
    # the Laplacian is a sum over axes of one-axis operators (Kronecker structure)
    for a in range(len(shape)):
        F, Finv, lam = mats[a]
        Ka = Finv @ np.diag(lam) @ F
        op = np.array([[1.0]])
        for b in range(len(shape)):
            op = np.kron(op, Ka if b == a else np.eye(shape[b]))
        K += op
    return K


def hamiltonian(f: np.ndarray, box, a: float, b: float) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    return a * kinetic_matrix(f.shape, box) + b * np.diag(f.reshape(-1)).astype(np.complex128)


def lowest(f: np.ndarray, box, a: float, b: float, nev: int) -> Tuple[np.ndarray, np.ndarray]:
    """The nev lowest eigenvalues and eigenvectors (columns, unit norm)."""
    H = hamiltonian(f, box, a, b)
    w, v = np.linalg.eigh(H)
    return w[:nev], v[:, :nev]


def nesterov_ab(t: float, eps: float = 1e-3) -> Tuple[float, float]:
    """a(t) = 2/(eps + t^3), b(t) = 2 t^3 (App. C.2.1, eq. nonconvex_QHD_h)."""
    return 2.0 / (eps + t ** 3), 2.0 * t ** 3
