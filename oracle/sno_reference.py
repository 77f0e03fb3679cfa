"""FP64 CPU reference of the spectral neural-operator surrogate (forward, loss,
backward).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

The surrogate is not part of the paper's method: it maps a potential f to the
final position density |psi_T|^2 of the QHD evolution (the measurement
distribution of Algorithm 1, App. E.1).  The network is the one the surrogate's
C header defines; this module writes it out in plain numpy, FP64:

    x0        = ((f - mean f) / std f, x / S, y / S)          (population std)
    h0        = x0 Wl^T + bl
    h_{l+1}   = GELU(Spec_l(h_l) + h_l W_l^T + b_l)          GELU(z) = z (1 + erf(z / sqrt 2)) / 2
    Spec(h)   = (1/S^2) sum_{ky in [-M, M), kx in [0, M)} w(kx) Re(R(ky,kx) H(ky,kx) e^{i theta})
                H(ky,kx) = sum_{y,x} h(y,x) e^{-i theta},  theta = 2 pi (ky y + kx x) / S,
                w(0) = 1, w(kx > 0) = 2
    q         = h_L Wp + bp ;  rho_hat = softmax of q over the S^2 points of a sample
    loss      = (1/B) sum_b sum_p |rho_hat - rho|

Spec uses numpy's real FFTs as a library primitive: the truncated forward sum
is a slice of rfft2, and (1/S^2) sum w Re(G e^{i theta}) is irfft2 of G placed
in an otherwise zero half spectrum (irfft drops the imaginary part of the
kx = 0 column, which is the Re() of the definition).  ``spec_direct`` is the
definition summed term by term, for tiny meshes.

The backward pass is written from the chain rule by hand (adjoints below); the
tests pin it to central finite differences of ``loss``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np
from scipy.special import erf


@dataclass(frozen=True)
class Config:
    S: int      # mesh points per axis
    C: int      # channels
    M: int      # retained modes per axis
    L: int      # spectral layers


def param_layout(cfg: Config) -> List[Tuple[str, Tuple[int, ...]]]:
    """Names and shapes of the flat parameter vector, in order."""
    C, M = cfg.C, cfg.M
    out = [("Wl", (C, 3)), ("bl", (C,))]
    for l in range(cfg.L):
        out += [(f"Rr{l}", (2 * M, M, C, C)), (f"Ri{l}", (2 * M, M, C, C)), (f"W{l}", (C, C)), (f"b{l}", (C,))]
    out += [("Wp", (C,)), ("bp", (1,))]
    return out


def param_count(cfg: Config) -> int:
    return sum(int(np.prod(s)) for _, s in param_layout(cfg))


def unpack(p: np.ndarray, cfg: Config) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    assert o == p.size
    return out


def pack(d: Dict[str, np.ndarray], cfg: Config) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in param_layout(cfg)])


def random_params(cfg: Config, seed: int, spectral_scale: float = None) -> np.ndarray:
    """Seeded parameters of the initialisation's shape and scale (test inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = cfg.C
    sc = spectral_scale if spectral_scale is not None else 1.0 / (C * C)
    d = {}
    for name, shape in param_layout(cfg):
        if name.startswith("R"):
            d[name] = rng.uniform(0.0, sc, size=shape)
        else:
            fan = 3 if name in ("Wl", "bl") else C
            d[name] = rng.uniform(-1.0, 1.0, size=shape) / math.sqrt(fan)
    return pack(d, cfg)


# ----------------------------------------------------------------------------------
# building blocks


def features(f: np.ndarray) -> np.ndarray:
    """f [B, S, S] -> x0 [B, S, S, 3] = (standardised f, x / S, y / S)."""
    B, S, _ = f.shape
    mean = f.mean(axis=(1, 2), keepdims=True)
    std = np.sqrt(((f - mean) ** 2).mean(axis=(1, 2), keepdims=True))
    x0 = np.empty((B, S, S, 3))
    x0[..., 0] = (f - mean) / std
    x0[..., 1] = (np.arange(S) / S)[None, None, :]
    x0[..., 2] = (np.arange(S) / S)[None, :, None]
    return x0


def ky_rows(S: int, M: int) -> np.ndarray:
    """Row index in an S-point FFT of ky = j (j < M) and ky = j - 2M (j >= M)."""
    j = np.arange(2 * M)
    return np.where(j < M, j, S + j - 2 * M)


def weights(M: int) -> np.ndarray:
    w = np.full(M, 2.0)
    w[0] = 1.0
    return w


def spec_forward_modes(h: np.ndarray, M: int) -> np.ndarray:
    """H(ky, kx) = sum h e^{-i theta} at the retained modes: [B, 2M, M, C] complex."""
    S = h.shape[1]
    full = np.fft.rfft2(h, axes=(1, 2))              # [B, S, S/2+1, C]
    return full[:, ky_rows(S, M), :M, :]


def spec_synthesis(G: np.ndarray, S: int) -> np.ndarray:
    """(1/S^2) sum w(kx) Re(G e^{i theta}) on the mesh: [B, S, S, C]."""
    B, twoM, M, C = G.shape
    X = np.zeros((B, S, S // 2 + 1, C), dtype=np.complex128)
    X[:, ky_rows(S, M), :M, :] = G
    return np.fft.irfft2(X, s=(S, S), axes=(1, 2))


def mix(R: np.ndarray, H: np.ndarray) -> np.ndarray:
    """G[b, j, k, o] = sum_i R[j, k, o, i] H[b, j, k, i]."""
    return np.einsum("jkoi,bjki->bjko", R, H)


def spec_apply(h: np.ndarray, Rr: np.ndarray, Ri: np.ndarray) -> np.ndarray:
    M = Rr.shape[1]
    return spec_synthesis(mix(Rr + 1j * Ri, spec_forward_modes(h, M)), h.shape[1])


def spec_direct(h: np.ndarray, Rr: np.ndarray, Ri: np.ndarray) -> np.ndarray:
    """The definition of Spec summed term by term (tiny meshes only)."""
    B, S, _, C = h.shape
    M = Rr.shape[1]
    out = np.zeros_like(h)
    ys, xs = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    for j in range(2 * M):
        ky = j if j < M else j - 2 * M
        for kx in range(M):
            theta = 2.0 * math.pi * (ky * ys + kx * xs) / S
            e_minus = np.exp(-1j * theta)
            R = Rr[j, kx] + 1j * Ri[j, kx]
            w = 1.0 if kx == 0 else 2.0
            for b in range(B):
                H = np.array([(h[b, :, :, i] * e_minus).sum() for i in range(C)])
                G = R @ H
                for o in range(C):
                    out[b, :, :, o] += w * (G[o] * np.exp(1j * theta)).real / (S * S)
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def softmax_grid(q: np.ndarray) -> np.ndarray:
    B = q.shape[0]
    flat = q.reshape(B, -1)
    e = np.exp(flat - flat.max(axis=1, keepdims=True))
    return (e / e.sum(axis=1, keepdims=True)).reshape(q.shape)


# ----------------------------------------------------------------------------------
# network


def forward(p: np.ndarray, f: np.ndarray, cfg: Config, keep: bool = False):
    """rho_hat [B, S, S] (and the activations when ``keep``)."""
    P = unpack(p, cfg)
    x0 = features(np.asarray(f, dtype=np.float64).reshape(-1, cfg.S, cfg.S))
    h = x0 @ P["Wl"].T + P["bl"]
    hs, zs, Hs = [h], [], []
    for l in range(cfg.L):
        Rr, Ri = P[f"Rr{l}"], P[f"Ri{l}"]
        H = spec_forward_modes(h, cfg.M)
        z = spec_synthesis(mix(Rr + 1j * Ri, H), cfg.S) + h @ P[f"W{l}"].T + P[f"b{l}"]
        h = gelu(z)
        hs.append(h)
        zs.append(z)
        Hs.append(H)
    q = h @ P["Wp"] + P["bp"][0]
    rho = softmax_grid(q)
    if keep:
        return rho, dict(x0=x0, hs=hs, zs=zs, Hs=Hs, P=P)
    return rho


def loss(rho_hat: np.ndarray, rho: np.ndarray) -> float:
    B = rho_hat.shape[0]
    return float(np.abs(rho_hat - rho.reshape(rho_hat.shape)).sum() / B)


def loss_of_params(p, f, rho, cfg) -> float:
    return loss(forward(p, f, cfg), rho)


def backward(p: np.ndarray, f: np.ndarray, rho: np.ndarray, cfg: Config) -> Tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the flat parameter vector (FP64)."""
    rho_hat, c = forward(p, f, cfg, keep=True)
    P, hs, zs, Hs, x0 = c["P"], c["hs"], c["zs"], c["Hs"], c["x0"]
    B, S, M = rho_hat.shape[0], cfg.S, cfg.M
    rho = rho.reshape(rho_hat.shape)
    L = loss(rho_hat, rho)
    g = {}
    # L1 then softmax: dq = rho_hat (s - <rho_hat, s>) per sample, s = sign(rho_hat - rho) / B
    s = np.sign(rho_hat - rho) / B
    inner = (rho_hat * s).reshape(B, -1).sum(axis=1)[:, None, None]
    dq = rho_hat * (s - inner)
    hL = hs[-1]
    g["Wp"] = np.einsum("byx,byxc->c", dq, hL)
    g["bp"] = np.array([dq.sum()])
    dh = dq[..., None] * P["Wp"]
    w = weights(M)[None, None, :, None]
    for l in reversed(range(cfg.L)):
        Rr, Ri = P[f"Rr{l}"], P[f"Ri{l}"]
        R = Rr + 1j * Ri
        dz = dh * gelu_grad(zs[l])
        g[f"b{l}"] = dz.sum(axis=(0, 1, 2))
        g[f"W{l}"] = np.einsum("byxo,byxi->oi", dz, hs[l])
        # Spec: s = (1/S^2) sum w Re(G e^{i theta})  =>  dL/dG = (w/S^2) sum dz e^{-i theta}
        dG = spec_forward_modes(dz, M) * w / (S * S)
        # G = R H  =>  dR = sum_b dG conj(H)^T,  dH = R^H dG
        dR = np.einsum("bjko,bjki->jkoi", dG, np.conj(Hs[l]))
        g[f"Rr{l}"] = dR.real
        g[f"Ri{l}"] = dR.imag
        dH = np.einsum("jkoi,bjko->bjki", np.conj(R), dG)
        # H = sum h e^{-i theta}  =>  dh = Re(sum dH e^{i theta}) = S^2 * synthesis(dH / w)
        dh = spec_synthesis(dH / w, S) * (S * S) + dz @ P[f"W{l}"]
    g["bl"] = dh.sum(axis=(0, 1, 2))
    g["Wl"] = np.einsum("byxo,byxi->oi", dh, x0)
    return L, pack(g, cfg)
