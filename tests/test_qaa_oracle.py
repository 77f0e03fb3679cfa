"""Pins of the split-step QAA reference (CPU): the Walsh-Hadamard diagonalisation
of -sum sigma_x against dense Kronecker products, one step against dense matrix
exponentials, the stationary uniform state, second-order convergence, time
reversal, and a planted mistake."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import qaa_reference as qa


def test_walsh_hadamard_diagonalises_transverse_field():
    shape = (4, 8)
    H0 = qa.dense_h0(shape)
    N = H0.shape[0]
    # W H0 W^{-1} = diag(D0) with W = W_y (x) W_x acting on the (y, x)-ordered index
    from scipy.linalg import hadamard
    W = np.kron(hadamard(4), hadamard(8))
    D = W @ H0 @ W.T / N
    assert np.max(np.abs(D - np.diag(qa.d0(shape).reshape(-1)))) < 1e-12
    # ground state of H0: the uniform superposition, energy -bits
    w, v = np.linalg.eigh(H0)
    assert abs(w[0] + 5.0) < 1e-12 and abs(abs(v[:, 0].sum()) - math.sqrt(N)) < 1e-10


def _landscape(shape, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 2.0, size=shape)


def test_one_step_equals_product_of_matrix_exponentials():
    shape, dt, T = (4, 4), 0.3, 2.0
    f = _landscape(shape)
    rng = np.random.Generator(np.random.PCG64(4))
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    psi /= np.linalg.norm(psi)
    g = qa.linear_g(2, dt, T)
    H0, H1 = qa.dense_h0(shape), np.diag(f.reshape(-1))
    U = expm(-0.5j * dt * g * H1) @ expm(-1j * dt * (1 - g) * H0) @ expm(-0.5j * dt * g * H1)
    want = (U @ psi.reshape(-1)).reshape(shape)
    got = qa.evolve(f, psi, dt, 1, T, j0=2)
    assert np.max(np.abs(got - want)) < 1e-12


def test_uniform_state_is_stationary_without_problem_term():
    shape = (8, 8)
    psi = qa.uniform(shape)
    # T huge: g ~ 0, H ~ H0 whose ground state is psi0 (only a global phase e^{i bits t})
    out = qa.evolve(_landscape(shape), psi, 0.01, 50, 1e12)
    phase = out.reshape(-1)[0] / psi.reshape(-1)[0]
    assert abs(abs(phase) - 1.0) < 1e-9
    assert np.max(np.abs(out - phase * psi)) < 1e-8
    assert abs(np.angle(phase) - math.remainder(6 * 0.5, 2 * math.pi)) < 1e-6


def _exact(f, psi0, T, t_end):
    H0, H1 = qa.dense_h0(f.shape), np.diag(f.reshape(-1))

    def rhs(t, y):
        g = t / T
        return -1j * (((1 - g) * H0 + g * H1) @ y)

    sol = solve_ivp(rhs, (0.0, t_end), psi0.reshape(-1).astype(complex), method="DOP853", rtol=1e-12, atol=1e-13)
    return sol.y[:, -1].reshape(f.shape)


def test_second_order_convergence_to_the_exact_evolution():
    shape, T = (4, 8), 2.0
    f = _landscape(shape, 7)
    psi0 = qa.uniform(shape)
    ref = _exact(f, psi0, T, T)
    errs = []
    for n in (40, 80, 160):
        errs.append(np.max(np.abs(qa.evolve(f, psi0, T / n, n, T) - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_time_reversal():
    shape, T, dt, n = (8, 4), 1.0, 0.05, 20
    f = _landscape(shape, 9)
    psi0 = qa.uniform(shape)
    fwd = qa.evolve(f, psi0, dt, n, T)
    # reversed: steps n-1 .. 0 with -dt undo the forward steps (g at the same midpoints)
    back = fwd.copy()
    N = back.size
    D = qa.d0(shape)
    for j in reversed(range(n)):
        g = qa.linear_g(j, dt, T)
        half = np.exp(0.5j * dt * g * f)
        back = half * back
        back = qa.wht2(np.exp(1j * dt * (1 - g) * D) * qa.wht2(back)) / N
        back = half * back
    assert np.max(np.abs(back - psi0)) < 1e-12


def test_planted_mistake_sign_of_transverse_field_is_caught(monkeypatch):
    shape, dt, T = (4, 4), 0.3, 2.0
    f = _landscape(shape)
    psi = qa.uniform(shape)
    H0, H1 = qa.dense_h0(shape), np.diag(f.reshape(-1))
    g = qa.linear_g(0, dt, T)
    U = expm(-0.5j * dt * g * H1) @ expm(-1j * dt * (1 - g) * H0) @ expm(-0.5j * dt * g * H1)
    want = (U @ psi.reshape(-1)).reshape(shape)
    monkeypatch.setattr(qa, "d0", lambda s: -qa.d0_axis(s[0])[:, None] - qa.d0_axis(s[1])[None, :])
    assert np.max(np.abs(qa.evolve(f, psi, dt, 1, T) - want)) > 1e-3


# ---- leapfrog (the paper's QAA integrator) ---------------------------------------------

def test_leapfrog_h_application_matches_dense_operator():
    shape, g = (8, 4), 0.3
    f = _landscape(shape, 21)
    rng = np.random.Generator(np.random.PCG64(22))
    v = rng.standard_normal(shape)
    H = (1 - g) * qa.dense_h0(shape) + g * np.diag(f.reshape(-1))
    assert np.max(np.abs(qa.apply_h(f, v, g).reshape(-1) - H @ v.reshape(-1))) < 1e-12


def test_leapfrog_step_is_kick_drift_kick_with_dense_operators():
    shape, dt, T, j = (4, 4), 0.05, 2.0, 3
    f = _landscape(shape, 23)
    rng = np.random.Generator(np.random.PCG64(24))
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = lambda t: (1 - t / T) * qa.dense_h0(shape) + (t / T) * np.diag(f.reshape(-1))
    R, I = psi.real.reshape(-1), psi.imag.reshape(-1)
    I = I - 0.5 * dt * H(j * dt) @ R
    R = R + dt * H((j + 0.5) * dt) @ I
    I = I - 0.5 * dt * H((j + 1) * dt) @ R
    got = qa.evolve_leapfrog(f, psi, dt, 1, T, j0=j).reshape(-1)
    assert np.max(np.abs(got - (R + 1j * I))) < 1e-12


def test_leapfrog_second_order_convergence_and_time_reversal():
    shape, T = (4, 8), 2.0
    f = _landscape(shape, 25)
    psi0 = qa.uniform(shape)
    ref = _exact(f, psi0, T, T)
    errs = [np.max(np.abs(qa.evolve_leapfrog(f, psi0, T / n, n, T) - ref)) for n in (80, 160, 320)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs
    # reversibility: steps n-1 .. 0 with -dt (kicks and drift at the same times) undo the run
    n, dt = 40, 0.05
    fwd = qa.evolve_leapfrog(f, psi0, dt, n, T)
    R, I = fwd.real.copy(), fwd.imag.copy()
    for j in reversed(range(n)):
        I = I + 0.5 * dt * qa.apply_h(f, R, (j + 1) * dt / T)
        R = R - dt * qa.apply_h(f, I, (j + 0.5) * dt / T)
        I = I + 0.5 * dt * qa.apply_h(f, R, j * dt / T)
    assert np.max(np.abs(R + 1j * I - psi0)) < 1e-12


def test_leapfrog_planted_mistake_swapped_schedule_weights_is_caught(monkeypatch):
    # H0 weighted by g and H1 by 1 - g: the convergence check against the exact
    # evolution fails
    shape, T = (4, 8), 2.0
    f = _landscape(shape, 25)
    psi0 = qa.uniform(shape)
    ref = _exact(f, psi0, T, T)
    orig = qa.apply_h
    monkeypatch.setattr(qa, "apply_h", lambda f_, v, g: orig(f_, v, 1.0 - g))
    assert np.max(np.abs(qa.evolve_leapfrog(f, psi0, T / 160, 160, T) - ref)) > 1e-3
