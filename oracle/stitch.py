"""Gaussian-weighted stitching of deconvolved patches (Supp. S1.4).

Patches are placed back at their positions and summed; the result is
divided by the sum of the window weights wherever that sum is positive.
The deconvolved patch x_hat_i estimates the windowed clean patch, so the
window appears once in the sum of weights.
"""
from __future__ import annotations

import torch

from .geometry import F64, gaussian_window, patch_counts


def stitch(patches: torch.Tensor, ny: int, nx: int, P: int, stride: int, px: float, fwhm: float,
           floor: float = 1e-12) -> torch.Tensor:
    """patches [N][P][P] (windowed patch images) -> image [ny][nx]."""
    g = gaussian_window(P, px, fwhm)
    npy, npx = patch_counts(ny, nx, P, stride)
    acc = torch.zeros(ny, nx, dtype=F64)
    wsum = torch.zeros(ny, nx, dtype=F64)
    for a in range(npy):
        for b in range(npx):
            acc[a * stride:a * stride + P, b * stride:b * stride + P] += patches[a * npx + b]
            wsum[a * stride:a * stride + P, b * stride:b * stride + P] += g
    return torch.where(wsum > floor, acc / wsum.clamp_min(floor), torch.zeros_like(acc))
