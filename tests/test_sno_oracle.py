"""Pins of the FP64 surrogate reference (CPU): the spectral operator against its
term-by-term definition and a band-limited closed form, the backward pass
against central finite differences, and planted mistakes that these pins catch."""
import math

import numpy as np
import pytest

from oracle import sno_reference as ref


def _h(B, S, C, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((B, S, S, C))


@pytest.mark.parametrize("S,M", [(8, 1), (8, 2), (8, 4), (6, 3)])
def test_spec_matches_term_by_term_definition(S, M):
    C = 3
    rng = np.random.Generator(np.random.PCG64(7))
    Rr = rng.standard_normal((2 * M, M, C, C))
    Ri = rng.standard_normal((2 * M, M, C, C))
    h = _h(2, S, C, 3)
    fast = ref.spec_apply(h, Rr, Ri)
    slow = ref.spec_direct(h, Rr, Ri)
    assert np.max(np.abs(fast - slow)) < 1e-12 * max(1.0, np.max(np.abs(slow)))


def test_spec_identity_reproduces_band_limited_field():
    # with R = identity at every retained mode and M = S/2, Spec reproduces any
    # real field whose spectrum has no kx = S/2 (Nyquist) component
    S, C, M = 16, 2, 8
    y, x = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    h = np.zeros((1, S, S, C))
    h[0, :, :, 0] = 0.3 + np.cos(2 * math.pi * (3 * x - 5 * y) / S) + 0.5 * np.sin(2 * math.pi * (7 * x + 8 * y) / S)
    h[0, :, :, 1] = np.cos(2 * math.pi * (0 * x + 8 * y) / S) - 2 * np.sin(2 * math.pi * (6 * x - 2 * y) / S)
    Rr = np.broadcast_to(np.eye(C), (2 * M, M, C, C)).copy()
    Ri = np.zeros_like(Rr)
    assert np.max(np.abs(ref.spec_apply(h, Rr, Ri) - h)) < 1e-13


def test_spec_drops_modes_outside_the_band():
    S, C, M = 16, 1, 3
    y, x = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    h = np.zeros((1, S, S, C))
    inside = np.cos(2 * math.pi * (2 * x - 3 * y) / S)       # kx=2, ky=-3: retained
    outside = np.cos(2 * math.pi * (3 * x + 1 * y) / S)      # kx=3: dropped
    h[0, :, :, 0] = inside + outside
    Rr = np.ones((2 * M, M, C, C))
    Ri = np.zeros_like(Rr)
    assert np.max(np.abs(ref.spec_apply(h, Rr, Ri)[0, :, :, 0] - inside)) < 1e-13


def test_softmax_density_and_zero_loss():
    cfg = ref.Config(S=8, C=4, M=2, L=1)
    p = ref.random_params(cfg, 1)
    f = np.random.Generator(np.random.PCG64(2)).standard_normal((3, 8, 8))
    rho = ref.forward(p, f, cfg)
    assert np.allclose(rho.reshape(3, -1).sum(axis=1), 1.0, atol=1e-14)
    assert np.all(rho > 0)
    assert ref.loss(rho, rho) == 0.0


def test_features_standardise_each_sample():
    f = np.random.Generator(np.random.PCG64(4)).uniform(2.0, 9.0, (2, 8, 8))
    x0 = ref.features(f)
    assert np.allclose(x0[..., 0].mean(axis=(1, 2)), 0.0, atol=1e-14)
    assert np.allclose(x0[..., 0].std(axis=(1, 2)), 1.0, atol=1e-14)
    assert x0[0, 2, 5, 1] == 5 / 8 and x0[0, 2, 5, 2] == 2 / 8


def _fd_check(cfg, seed, n_coords=4, step=1e-5, backward=ref.backward):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = ref.random_params(cfg, seed, spectral_scale=0.5 / cfg.C)
    B = 2
    f = rng.standard_normal((B, cfg.S, cfg.S))
    rho = rng.dirichlet(np.ones(cfg.S * cfg.S), size=B).reshape(B, cfg.S, cfg.S)
    L, g = backward(p, f, rho, cfg)
    assert abs(L - ref.loss_of_params(p, f, rho, cfg)) < 1e-14
    # relative error against the larger of the two values, floored at 1% of the
    # largest gradient entry (central differences leave ~1e-12 absolute error)
    floor = 1e-2 * np.max(np.abs(g))
    worst = 0.0
    o = 0
    for name, shape in ref.param_layout(cfg):
        n = int(np.prod(shape))
        for k in rng.choice(n, size=min(n, n_coords), replace=False):
            e = np.zeros_like(p)
            e[o + k] = step
            fd = (ref.loss_of_params(p + e, f, rho, cfg) - ref.loss_of_params(p - e, f, rho, cfg)) / (2 * step)
            scale = max(abs(fd), abs(g[o + k]), floor)
            worst = max(worst, abs(fd - g[o + k]) / scale)
        o += n
    return worst


@pytest.mark.parametrize("cfg", [ref.Config(S=8, C=4, M=2, L=2), ref.Config(S=8, C=3, M=4, L=1),
                                 ref.Config(S=16, C=2, M=3, L=3)])
def test_backward_matches_finite_differences(cfg):
    assert _fd_check(cfg, seed=11) < 1e-6


def test_finite_difference_pin_catches_planted_adjoint_mistakes(monkeypatch):
    cfg = ref.Config(S=8, C=4, M=2, L=2)
    # planted mistake 1: forget the complex conjugates in dR and dH
    def bad_conj(p, f, rho, cfg_):
        monkeypatch.setattr(ref.np, "conj", lambda a: a)
        try:
            return ref.backward(p, f, rho, cfg_)
        finally:
            monkeypatch.undo()

    assert _fd_check(cfg, 11, backward=bad_conj) > 1e-3

    # planted mistake 2: drop the w(kx) weights of the adjoint synthesis
    def bad_weights(p, f, rho, cfg_):
        monkeypatch.setattr(ref, "weights", lambda M: np.ones(M))
        try:
            return ref.backward(p, f, rho, cfg_)
        finally:
            monkeypatch.undo()

    assert _fd_check(cfg, 11, backward=bad_weights) > 1e-3
