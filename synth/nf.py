"""Seeded inputs of the neural-field workload: the fixed Fourier frequencies and an initial parameter
vector.  Random numbers only; the network itself is not evaluated here.

Sizes: 128 frequencies drawn N(0, sigma^2) in cycles per mm with sigma = 2, four hidden layers of width
128, a scalar head; the SOS is v0 + amp tanh(head) inside the mask disc.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class NfConfig:
    n_freq: int = 128
    sigma: float = 2.0          # cycles per mm
    width: int = 128
    depth: int = 4
    amp: float = 0.15           # mm/us: the SOS spans v0 +- amp
    seed: int = 0

    @property
    def n_params(self) -> int:
        H, K = self.width, 2 * self.n_freq
        return H * K + H + 3 * (H * H + H) + H + 1


NF = NfConfig()


def frequencies(cfg: NfConfig = NF, seed: int | None = None) -> np.ndarray:
    """B [n_freq][2], float32, cycles per mm."""
    rng = np.random.default_rng(cfg.seed if seed is None else seed)
    return rng.normal(0.0, cfg.sigma, (cfg.n_freq, 2)).astype(np.float32)


def init_params(cfg: NfConfig = NF, seed: int | None = None, head_scale: float = 0.1) -> np.ndarray:
    """Parameter vector (float32) in the order W1 [H][2F], b1, W2 [H][H], b2, W3, b3, W4, b4, w5 [H], b5:
    weights uniform in +-sqrt(6 / fan_in), biases uniform in +-0.05, the head scaled by head_scale."""
    rng = np.random.default_rng(1000 + (cfg.seed if seed is None else seed))
    H, K = cfg.width, 2 * cfg.n_freq
    parts = []
    for fan_in in (K, H, H, H):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, H * fan_in))
        parts.append(rng.uniform(-0.05, 0.05, H))
    parts.append(head_scale * rng.uniform(-math.sqrt(6.0 / H), math.sqrt(6.0 / H), H))
    parts.append(np.zeros(1))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == cfg.n_params
    return p


def siren_params(hidden: int = 256, omega0: float = 30.0, seed: int = 0, s0: float = 0.05) -> np.ndarray:
    """Initial parameters of the paper's sinusoidal network (float32), layout W1 [hidden][2], b1, w2, b2, s, o:
    first layer uniform in +-1/fan_in (fan_in = 2), output layer uniform in +-sqrt(6 / hidden) / omega0 (the
    usual initialisation of sinusoidal networks), b2 = o = 0 and output scale s0 (mm/us)."""
    rng = np.random.default_rng(2000 + seed)
    lim2 = math.sqrt(6.0 / hidden) / omega0
    p = np.concatenate([rng.uniform(-0.5, 0.5, 2 * hidden), rng.uniform(-0.5, 0.5, hidden),
                        rng.uniform(-lim2, lim2, hidden), [0.0, s0, 0.0]]).astype(np.float32)
    assert p.size == 4 * hidden + 3
    return p
