"""Geometry of the ring array, image grid, patches and frequency grid (FP64).

Conventions (shared by every oracle function):
* lengths in mm, times in us, SOS in mm/us;
* an image of ny x nx pixels of size px is centred on the origin; pixel
  (r, c) has centre x = (c - (nx - 1) / 2) px, y = (r - (ny - 1) / 2) px;
  array axis 0 is y, axis 1 is x; angles are atan2(y, x);
* element n of an N-element ring of radius R sits at angle
  phi_n = phi0 + 2 pi n / N (counter-clockwise), Sec. 3.1 and Supp. S1.1.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64


def ring_positions(n_elem: int, radius: float, phi0: float = 0.0) -> torch.Tensor:
    """Element positions r_n [n_elem][2] as (x, y)."""
    n = torch.arange(n_elem, dtype=F64)
    phi = phi0 + 2.0 * math.pi * n / n_elem
    return torch.stack([radius * torch.cos(phi), radius * torch.sin(phi)], dim=-1)


def cell_centres(n: int, spacing: float) -> torch.Tensor:
    return (torch.arange(n, dtype=F64) - (n - 1) / 2.0) * spacing


def patch_counts(ny: int, nx: int, P: int, stride: int):
    return (ny - P) // stride + 1, (nx - P) // stride + 1


def patch_centres(ny: int, nx: int, px: float, P: int, stride: int) -> torch.Tensor:
    """Centre of each patch as the mean of its pixel centres, [N][2] (x, y).

    Patch i = a * npx + b covers rows a*stride .. a*stride+P-1 and columns
    b*stride .. b*stride+P-1 (Supp. S1.4: patch centres on a Cartesian grid).
    """
    npy, npx = patch_counts(ny, nx, P, stride)
    ys = cell_centres(ny, px)
    xs = cell_centres(nx, px)
    out = torch.empty(npy * npx, 2, dtype=F64)
    for a in range(npy):
        for b in range(npx):
            out[a * npx + b, 0] = xs[b * stride: b * stride + P].mean()
            out[a * npx + b, 1] = ys[a * stride: a * stride + P].mean()
    return out


def gaussian_window(P: int, px: float, fwhm: float) -> torch.Tensor:
    """Window g[u][v] = exp(-r^2 / (2 sigma^2)) about the patch centre, sigma = FWHM / (2 sqrt(2 ln 2))."""
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    u = (torch.arange(P, dtype=F64) - (P - 1) / 2.0) * px
    r2 = u[:, None] ** 2 + u[None, :] ** 2
    return torch.exp(-r2 / (2.0 * sigma * sigma))


def wavenumbers(P: int, px: float):
    """Angular wavenumbers (rad/mm) of the P x P FFT grid: ky [P][1], kx [1][P], |k| [P][P], angle [P][P]."""
    f = torch.fft.fftfreq(P, d=px, dtype=F64) * 2.0 * math.pi
    ky = f[:, None]
    kx = f[None, :]
    kabs = torch.sqrt(ky * ky + kx * kx)
    theta = torch.atan2(ky.expand(P, P), kx.expand(P, P))
    return ky, kx, kabs, theta


def sos_box_half_extent(Gy: int, Gx: int, spacing: float):
    """Half-widths of the box outside which the bilinear SOS equals v0 everywhere.

    With node centres at (b - (G - 1) / 2) * spacing and every node outside
    the grid at v0, the field differs from v0 only inside
    |x| < (Gx + 1) spacing / 2, |y| < (Gy + 1) spacing / 2.
    """
    return (Gx + 1) * spacing / 2.0, (Gy + 1) * spacing / 2.0


def as_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()
