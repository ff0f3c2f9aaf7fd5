"""Isoplanatic patches and their spectra (Eq. conv, Sec. 3.3, Supp. S1.4).

Each image of the DAS stack is cut into P x P patches on a Cartesian grid
of patch origins (stride s), multiplied by a Gaussian window centred on the
patch, and Fourier transformed: Y_ij = FFT2(g * y_j[patch i]) with the
unnormalised e^{-j k.r} forward transform (numpy / torch convention).
"""
from __future__ import annotations

import numpy as np
import torch

from .geometry import gaussian_window, patch_counts, F64


def extract_patches(stack, P: int, stride: int) -> torch.Tensor:
    """[M][ny][nx] -> [N][M][P][P], patch i = a * npx + b."""
    stack = torch.as_tensor(np.asarray(stack), dtype=F64)
    M, ny, nx = stack.shape
    npy, npx = patch_counts(ny, nx, P, stride)
    out = torch.empty(npy * npx, M, P, P, dtype=F64)
    for a in range(npy):
        for b in range(npx):
            out[a * npx + b] = stack[:, a * stride:a * stride + P, b * stride:b * stride + P]
    return out


def patch_spectra(stack, P: int, stride: int, px: float, fwhm: float) -> torch.Tensor:
    """Y [N][M][P][P] complex128."""
    g = gaussian_window(P, px, fwhm)
    return torch.fft.fft2(extract_patches(stack, P, stride) * g)


def half_spectrum(Y: torch.Tensor) -> torch.Tensor:
    """Columns 0 .. P // 2 of the last axis (the stored half of a real patch's spectrum)."""
    P = Y.shape[-1]
    return Y[..., : P // 2 + 1]
