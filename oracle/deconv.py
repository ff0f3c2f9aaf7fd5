"""Eq. fm_fourier and Eq. multi-deconv (Sec. 3.2): multichannel deconvolution.

The stack over the M delays is overdetermined: Y_i = H_i X_i per frequency.
The paper's pseudo-inverse writes H^T Y / (H^T H).  Reading taken: for a
complex column the least-squares pseudo-inverse uses the conjugate
transpose, and a Tikhonov term eps keeps the denominator away from zero
where every channel's transfer function vanishes (the paper does not say
what it does there):
    X_hat_i(k) = sum_j conj(H_ij(k)) Y_ij(k) / (sum_j |H_ij(k)|^2 + eps).
"""
from __future__ import annotations

import torch


def multichannel_deconv(Y: torch.Tensor, H: torch.Tensor, eps: float) -> torch.Tensor:
    """Y, H [N][M][P][P] -> X_hat [N][P][P]."""
    num = (torch.conj(H) * Y).sum(1)
    den = (H.real ** 2 + H.imag ** 2).sum(1) + eps
    return num / den


def single_channel_deconv(Y: torch.Tensor, H: torch.Tensor, eps: float) -> torch.Tensor:
    """The M = 1 case written as the textbook Tikhonov (Wiener-like) division."""
    return torch.conj(H) * Y / (torch.abs(H) ** 2 + eps)


def patch_images(X: torch.Tensor) -> torch.Tensor:
    """x_hat = Re(IFFT2(X_hat))."""
    return torch.fft.ifft2(X).real
