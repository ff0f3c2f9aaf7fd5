"""Adam (Sec. 3.3 trains the SOS parameters with Adam; the settings beyond the
learning rate are not stated, so the usual defaults beta = (0.9, 0.999),
eps = 1e-8 with bias correction are taken).  Only free nodes move.
"""
from __future__ import annotations

import math

import torch


class Adam:
    def __init__(self, params: torch.Tensor, mask, lr: float, b1: float = 0.9, b2: float = 0.999,
                 eps: float = 1e-8):
        self.p = params.detach().clone().to(torch.float64)
        self.mask = torch.as_tensor(mask).bool()
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, grad: torch.Tensor) -> torch.Tensor:
        g = torch.where(self.mask, grad.to(torch.float64), torch.zeros_like(self.p))
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        m_hat = self.m / (1.0 - self.b1 ** self.t)
        v_hat = self.v / (1.0 - self.b2 ** self.t)
        upd = self.lr * m_hat / (torch.sqrt(v_hat) + self.eps)
        self.p = torch.where(self.mask, self.p - upd, self.p)
        return self.p

    def state(self):
        return dict(p=self.p.clone(), m=self.m.clone(), v=self.v.clone(), t=self.t)


def bias_corrections(b1: float, b2: float, t: int):
    return 1.0 - b1 ** t, math.sqrt(1.0 - b2 ** t)
