"""Pins of the relaxed-QHD box-QP reference (CPU): the spectrum of the relaxed chain
adjacency against the spin representation, the discrete Gaussian as the kinetic
ground state, one step against dense matrix exponentials, second-order convergence
to the exact evolution, the lattice objective and the readouts by brute force, and a
planted mistake."""
import itertools
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import rqp_reference as rq


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8, 12])
def test_relaxed_adjacency_spectrum_is_the_spin_ladder(r):
    # A' is S_x / sqrt(r) on the symmetric subspace of r qubits (a spin r/2), whose
    # eigenvalues are r - 2k, k = 0..r
    w = np.linalg.eigvalsh(rq.relaxed_adjacency(r))
    want = np.sort((r - 2.0 * np.arange(r + 1)) / math.sqrt(r))
    assert np.max(np.abs(w - want)) < 1e-12
    # end entries equal the plain chain's, middle ones are larger
    A = rq.relaxed_adjacency(r)
    assert abs(A[0, 1] - 1.0) < 1e-15 and abs(A[r - 1, r] - 1.0) < 1e-15
    assert all(A[j, j + 1] >= 1.0 for j in range(r))


def test_discrete_gaussian_is_the_kinetic_ground_state():
    d, r = 2, 4
    H = rq.dense_hamiltonian(np.zeros((d, d)), np.zeros(d), r, 1.0, 0.0)
    psi0 = rq.initial_state(d, r).reshape(-1)
    assert abs(np.linalg.norm(psi0) - 1.0) < 1e-14
    E0 = -0.5 * r * r * d * math.sqrt(r)
    assert np.max(np.abs(H @ psi0 - E0 * psi0)) < 1e-12
    assert abs(np.linalg.eigvalsh(H)[0] - E0) < 1e-10
    # stationary under the kinetic evolution (b = 0): only a global phase
    f = np.zeros((r + 1,) * 3)
    out = rq.evolve(f, rq.initial_state(3, r), r, 0.01, 30, lambda t: (0.7, 0.0))
    ph = out.reshape(-1)[0] / rq.initial_state(3, r).reshape(-1)[0]
    assert abs(abs(ph) - 1.0) < 1e-12 and np.max(np.abs(out - ph * rq.initial_state(3, r))) < 1e-12


def _qp(d, seed):
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-1, 1, (d, d))
    return 0.5 * (Q + Q.T) * 4, rng.uniform(-1, 1, d)


def test_objective_on_the_lattice_by_brute_force():
    d, r = 3, 3
    Q, b = _qp(d, 1)
    f = rq.objective(Q, b, r)
    for js in itertools.product(range(r + 1), repeat=d):  # js = (j_1, ..., j_d)
        x = np.array(js) / r
        assert abs(f[tuple(reversed(js))] - (0.5 * x @ Q @ x + b @ x)) < 1e-14


def test_one_step_equals_dense_exponentials():
    d, r, dt = 2, 4, 0.05
    Q, b = _qp(d, 2)
    f = rq.objective(Q, b, r)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape)
    psi /= np.linalg.norm(psi)
    a, bt = rq.nesterov_ab(7.5 * dt, 1e-3)
    K = rq.dense_hamiltonian(Q, b, r, a, 0.0)
    half = np.exp(-0.5j * dt * bt * f.reshape(-1))
    want = half * (expm(-1j * dt * K) @ (half * psi.reshape(-1)))
    got = rq.evolve(f, psi, r, dt, 1, lambda t: rq.nesterov_ab(t, 1e-3), j0=7)
    assert np.max(np.abs(got.reshape(-1) - want)) < 1e-12


def test_second_order_convergence_to_the_exact_evolution():
    d, r, T = 2, 4, 1.0
    Q, b = _qp(d, 4)
    f = rq.objective(Q, b, r)
    psi0 = rq.initial_state(d, r)
    ab = lambda t: rq.nesterov_ab(t, 1.0)

    def rhs(t, y):
        a, bt = ab(t)
        return -1j * (rq.dense_hamiltonian(Q, b, r, a, bt) @ y)

    ref = solve_ivp(rhs, (0.0, T), psi0.reshape(-1), method="DOP853", rtol=1e-12, atol=1e-13).y[:, -1]
    errs = [np.max(np.abs(rq.evolve(f, psi0, r, T / n, n, ab).reshape(-1) - ref)) for n in (32, 64, 128)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_readouts_by_brute_force():
    d, r = 3, 2
    Q, b = _qp(d, 5)
    f = rq.objective(Q, b, r)
    rng = np.random.default_rng(6)
    psi = rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape)
    ro = rq.readout(f, psi)
    rho = np.abs(psi) ** 2
    norm = math.fsum(rho.reshape(-1))
    assert abs(ro["norm"] - norm) < 1e-12
    assert abs(ro["e_f"] - math.fsum((f * rho).reshape(-1)) / norm) < 1e-12
    amin = np.unravel_index(np.argmin(f), f.shape)
    assert abs(ro["p_min"] - rho[amin] / norm) < 1e-12
    for k in range(1, d + 1):
        for j in range(r + 1):
            s = math.fsum(rho[idx] for idx in itertools.product(range(r + 1), repeat=d) if idx[d - k] == j)
            assert abs(ro["marginals"][k - 1, j] - s) < 1e-12


def test_planted_mistake_printed_off_diagonal_is_caught(monkeypatch):
    # the printed formula's (r+1) in place of r couples to a point outside the lattice;
    # truncated to (r+1) x (r+1) it no longer has the spin spectrum
    def wrong(r):
        A = np.zeros((r + 1, r + 1))
        for j in range(r):
            A[j + 1, j] = A[j, j + 1] = math.sqrt((j + 1) * (r + 1 - j) / (r + 1))
        return A
    monkeypatch.setattr(rq, "relaxed_adjacency", wrong)
    r = 8
    w = np.linalg.eigvalsh(rq.relaxed_adjacency(r))
    assert np.max(np.abs(w - np.sort((r - 2.0 * np.arange(r + 1)) / math.sqrt(r)))) > 1e-3
