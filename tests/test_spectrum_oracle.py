"""Pins of the dense spectrum reference (CPU): closed forms for the free
particle on the mesh and the anisotropic harmonic oscillator, operator
structure, and a planted mistake the pins catch."""
import math

import numpy as np

from oracle import spectrum_reference as sr


def _ho(N=32, L=12.0, q=(1.0, 2.0)):
    x = -L / 2 + np.arange(N) * (L / N)
    f = 0.5 * (q[0] * x[None, :] ** 2 + q[1] * x[:, None] ** 2)
    return f, [(-L / 2, L / 2)] * 2


def _ho_levels(a, b, q, nev):
    w = [math.sqrt(a * b * qq) for qq in q]
    return np.array(sorted(w[0] * (i + 0.5) + w[1] * (j + 0.5) for i in range(12) for j in range(12))[:nev])


def test_free_particle_is_the_discrete_kinetic_spectrum():
    shape, box, a = (8, 6), [(0.0, 2.0), (-1.0, 2.0)], 0.7
    w, _ = sr.lowest(np.zeros(shape), box, a, 0.0, 48)
    k = []
    for n, (lo, hi) in zip(shape, box):
        m = np.arange(n)
        k.append(2 * math.pi * np.where(m < n // 2, m, m - n) / (hi - lo))
    exact = np.sort((0.5 * a * (k[0][:, None] ** 2 + k[1][None, :] ** 2)).reshape(-1))
    assert np.max(np.abs(w - exact)) < 1e-11 * max(1.0, exact.max())


def test_anisotropic_oscillator_levels():
    # a = b = 1, f = (x^2 + 2 y^2)/2: E = (n1 + 1/2) + sqrt(2) (n2 + 1/2), spectrally exact
    f, box = _ho()
    w, v = sr.lowest(f, box, 1.0, 1.0, 6)
    assert np.max(np.abs(w - _ho_levels(1.0, 1.0, (1.0, 2.0), 6))) < 1e-9
    assert np.allclose(np.linalg.norm(v, axis=0), 1.0)
    # omega = sqrt(a b q): a -> 1.5 a, b -> b / 1.5 keeps the levels (the states widen by
    # 1.5^{1/4}, still resolved on this mesh and box)
    w2, _ = sr.lowest(f, box, 1.5, 1.0 / 1.5, 6)
    assert np.max(np.abs(w2 - w)) < 1e-6


def test_hamiltonian_is_hermitian_and_kinetic_part_is_translation_invariant():
    f, box = _ho(N=12, L=8.0)
    H = sr.hamiltonian(f, box, 0.3, 2.0)
    assert np.max(np.abs(H - H.conj().T)) < 1e-12
    K = sr.kinetic_matrix((12,), [(0.0, 3.0)])
    for s in range(1, 4):
        assert np.max(np.abs(np.roll(np.roll(K, s, 0), s, 1) - K)) < 1e-12


def test_planted_mistake_dropped_half_is_caught(monkeypatch):
    f, box = _ho()
    real = sr.kinetic_matrix

    def wrong(shape, box_):
        return 2.0 * real(shape, box_)  # |k|^2 instead of |k|^2 / 2

    monkeypatch.setattr(sr, "kinetic_matrix", wrong)
    w, _ = sr.lowest(f, box, 1.0, 1.0, 6)
    assert np.max(np.abs(w - _ho_levels(1.0, 1.0, (1.0, 2.0), 6))) > 1e-2


def test_oscillator_virial_theorem():
    # for a harmonic potential every eigenstate splits its energy evenly between the
    # kinetic and the potential term: <a K> = <b V> = E / 2 (the six lowest levels of the
    # anisotropic oscillator are non-degenerate, so each eigenvector is a pure eigenstate)
    f, box = _ho()
    a, b = 0.8, 1.25
    w, v = sr.lowest(f, box, a, b, 6)
    K = sr.kinetic_matrix(f.shape, box)
    for n in range(6):
        psi = v[:, n]
        ek = float(np.real(np.vdot(psi, a * (K @ psi))))
        ev = float(np.real(np.vdot(psi, b * (f.reshape(-1) * psi))))
        assert abs(ek - 0.5 * w[n]) < 1e-8 and abs(ev - 0.5 * w[n]) < 1e-8, (n, ek, ev, w[n])


# App. D, energy ratio E1/E0: the Levy function's quadratic model at its minimiser and the
# two limits of the ratio

def _levy(x1, x2):
    """The 2-D Levy function as the paper prints it, with w_j = 1 + (x_j - 1) / 4."""
    w1, w2 = 1.0 + (x1 - 1.0) / 4.0, 1.0 + (x2 - 1.0) / 4.0
    return (np.sin(np.pi * w1) ** 2 + (w1 - 1.0) ** 2 * (1.0 + 10.0 * np.sin(np.pi * w1 + 1.0) ** 2)
            + (w2 - 1.0) ** 2 * (1.0 + np.sin(2.0 * np.pi * w2) ** 2))


LEVY_OMEGA = (math.sqrt((math.pi ** 2 + 1.0 + 10.0 * math.sin(1.0) ** 2) / 8.0), math.sqrt(1.0 / 8.0))
LEVY_RATIO = (LEVY_OMEGA[0] + 3.0 * LEVY_OMEGA[1]) / (LEVY_OMEGA[0] + LEVY_OMEGA[1])


def test_levy_hessian_and_the_printed_frequencies_and_ratio():
    """The Hessian of the printed Levy function at (1, 1), by central differences, is
    diag((pi^2 + 1 + 10 sin^2 1) / 8, 1/8); its square roots round to the printed 1.4979 and
    0.3536, and the semi-classical ratio (w1 + 3 w2) / (w1 + w2) to the printed 1.3819."""
    h = 1e-4
    H = np.empty((2, 2))
    for i in range(2):
        for j in range(2):
            e = np.eye(2)
            fpp = _levy(*(np.ones(2) + h * e[i] + h * e[j]))
            fpm = _levy(*(np.ones(2) + h * e[i] - h * e[j]))
            fmp = _levy(*(np.ones(2) - h * e[i] + h * e[j]))
            fmm = _levy(*(np.ones(2) - h * e[i] - h * e[j]))
            H[i, j] = (fpp - fpm - fmp + fmm) / (4 * h * h)
    lam = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert abs(_levy(1.0, 1.0)) < 1e-15
    assert abs(lam[0] - LEVY_OMEGA[0] ** 2) < 1e-6 and abs(lam[1] - LEVY_OMEGA[1] ** 2) < 1e-6
    assert round(math.sqrt(lam[0]), 4) == 1.4979 and round(math.sqrt(lam[1]), 4) == 0.3536
    assert round(LEVY_RATIO, 4) == 1.3819


def test_semiclassical_ratio_of_the_levy_model_on_the_mesh():
    """H = a K + b f with f the Levy quadratic model (1/2)(w1^2 x1^2 + w2^2 x2^2) on a periodic
    box wide enough for the lowest states: the dense reference's E1 / E0 equals
    (w1 + 3 w2) / (w1 + w2) = 1.3819 (independent of a, b; the oscillator limit of App. D)."""
    N, L = 40, 20.0
    x = -L / 2 + np.arange(N) * (L / N)
    f = 0.5 * (LEVY_OMEGA[0] ** 2 * x[None, :] ** 2 + LEVY_OMEGA[1] ** 2 * x[:, None] ** 2)
    box = [(-L / 2, L / 2)] * 2
    for a, b in ((1.0, 1.0), (1.5, 1.0 / 1.5)):
        w, _ = sr.lowest(f, box, a, b, 2)
        assert abs(w[1] / w[0] - LEVY_RATIO) < 1e-6, (a, b, w)


def test_kinetic_limit_ratio_with_the_papers_boundary_condition():
    """The kinetic limit E1/E0 = 2.5 holds for the Laplacian on [0, 1]^2 with vanishing
    boundary values (sine modes, E = (n1^2 + n2^2) pi^2 / 2): a second-order finite
    difference of that operator gives 2.5 up to O(h^2).  The split-operator mesh is
    periodic, where the kinetic ground state is the constant (E0 = 0) and the ratio is not
    defined, so this limit is a property of the paper's boundary condition only."""
    for N, tol in ((31, 5e-3), (63, 1.3e-3)):
        h = 1.0 / (N + 1)
        T = (np.diag(np.full(N, 2.0)) - np.diag(np.ones(N - 1), 1) - np.diag(np.ones(N - 1), -1)) / (h * h)
        K = 0.5 * (np.kron(T, np.eye(N)) + np.kron(np.eye(N), T))
        w = np.linalg.eigvalsh(K)[:3]
        assert abs(w[0] - math.pi ** 2) < 0.01 * math.pi ** 2
        assert abs(w[1] - w[2]) < 1e-9 * w[1]  # (1, 2) and (2, 1) degenerate
        assert abs(w[1] / w[0] - 2.5) < tol
    wp, _ = sr.lowest(np.zeros((8, 8)), [(0.0, 1.0)] * 2, 1.0, 0.0, 2)
    assert abs(wp[0]) < 1e-12 and wp[1] > 1.0
