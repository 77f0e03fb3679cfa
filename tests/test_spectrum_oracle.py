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
