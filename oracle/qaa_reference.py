"""FP64 CPU reference of the baseline quantum adiabatic algorithm (QAA) that the
paper compares QHD with (App. C.2, "Quantum Adiabatic Algorithm").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

Model.  Each coordinate of a 2-D mesh point is written in radix 2 (b_x bits for
the x index, b_y for the y index; 7 + 7 bits for the paper's 128 x 128 mesh), so
a mesh point is a computational basis state of b_x + b_y qubits.  The evolution
is i dpsi/dt = [(1 - g(t)) H0 + g(t) H1] psi with H0 = -sum_j sigma_x^(j) over all
qubits, H1 = diag(f) and the linear schedule g(t) = t / T; psi0 is the uniform
superposition, the ground state of H0.

Integration.  The paper integrates with a leapfrog scheme; this reference (and
the GPU path) uses the symmetric split-step product with both coefficients at
the step midpoint, exact for each factor: H0 is diagonal after the Walsh-Hadamard
transform W (W_{ux} = (-1)^{popcount(u & x)} per axis, unnormalised, W W = N I),
with eigenvalue -sum_j (-1)^{u_j} = 2 popcount(u) - bits per axis.

    psi <- e^{-i dt/2 g H1} W^{-1} e^{-i dt (1-g) D0} W e^{-i dt/2 g H1} psi

The Hadamard matrix comes from scipy (a library primitive).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import hadamard


def d0_axis(n: int) -> np.ndarray:
    """Eigenvalues of -sum_j sigma_x^(j) over the log2(n) qubits of one axis, in the
    Walsh-Hadamard basis (natural order): 2 popcount(u) - bits."""
    bits = int(round(math.log2(n)))
    u = np.arange(n)
    pc = np.array([bin(int(k)).count("1") for k in u])
    return 2.0 * pc - bits


def d0(shape) -> np.ndarray:
    ny, nx = shape
    return d0_axis(ny)[:, None] + d0_axis(nx)[None, :]


def wht2(psi: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D Walsh-Hadamard transform (array axes y, x)."""
    ny, nx = psi.shape
    return hadamard(ny) @ psi @ hadamard(nx).T


def linear_g(j: int, dt: float, T: float, left_end: bool = False) -> float:
    t = (j + (0.0 if left_end else 0.5)) * dt
    return t / T


def evolve(f: np.ndarray, psi: np.ndarray, dt: float, nsteps: int, T: float, j0: int = 0) -> np.ndarray:
    """Split-step QAA steps j0 .. j0+nsteps-1 (FP64)."""
    f = np.asarray(f, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.complex128).copy()
    N = psi.size
    D = d0(psi.shape)
    for j in range(j0, j0 + nsteps):
        g = linear_g(j, dt, T)
        half = np.exp(-0.5j * dt * g * f)
        psi = half * psi
        psi = wht2(np.exp(-1j * dt * (1.0 - g) * D) * wht2(psi)) / N
        psi = half * psi
    return psi


def uniform(shape) -> np.ndarray:
    N = int(np.prod(shape))
    return np.full(shape, 1.0 / math.sqrt(N), dtype=np.complex128)


def dense_h0(shape) -> np.ndarray:
    """-sum_j sigma_x^(j) as a dense matrix over the mesh index (y, x) (x fastest,
    bit j of the x index = qubit j of the x register), built from Kronecker products."""
    ny, nx = shape
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])

    def axis_op(n):
        bits = int(round(math.log2(n)))
        op = np.zeros((n, n))
        for j in range(bits):
            # index bit j (value 2^j): Kronecker factor position from the most significant bit
            mats = [np.eye(2)] * bits
            mats[bits - 1 - j] = sx
            m = np.array([[1.0]])
            for mm in mats:
                m = np.kron(m, mm)
            op += m
        return -op

    return np.kron(axis_op(ny), np.eye(nx)) + np.kron(np.eye(ny), axis_op(nx))


# ---- the paper's integrator: leapfrog (App. C.2, "Quantum Adiabatic Algorithm") ------
# With psi = R + i I and H(t) = (1 - g) H0 + g H1 real symmetric, i psi' = H psi reads
# R' = H I, I' = -H R: a separable Hamiltonian system (R as position, I as momentum).
# The kick-drift-kick leapfrog step from t_n to t_{n+1}:
#     I <- I - dt/2 H(t_n) R;   R <- R + dt H(t_{n+1/2}) I;   I <- I - dt/2 H(t_{n+1}) R
# (time-reversible and symplectic, second order; stable for dt |H| < 2).

def apply_h(f: np.ndarray, v: np.ndarray, g: float) -> np.ndarray:
    """H v for a real field v: (1 - g) W^{-1} D0 W v + g f v (W the 2-D Walsh-Hadamard
    transform, W^{-1} = W / N)."""
    N = v.size
    return (1.0 - g) * wht2(d0(v.shape) * wht2(v)) / N + g * f * v


def evolve_leapfrog(f: np.ndarray, psi: np.ndarray, dt: float, nsteps: int, T: float, j0: int = 0) -> np.ndarray:
    """Leapfrog steps j0 .. j0+nsteps-1 (FP64), g(t) = t / T."""
    f = np.asarray(f, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.complex128)
    R, I = psi.real.copy(), psi.imag.copy()
    for j in range(j0, j0 + nsteps):
        t0, th, t1 = j * dt, (j + 0.5) * dt, (j + 1) * dt
        I = I - 0.5 * dt * apply_h(f, R, t0 / T)
        R = R + dt * apply_h(f, I, th / T)
        I = I - 0.5 * dt * apply_h(f, R, t1 / T)
    return R + 1j * I
