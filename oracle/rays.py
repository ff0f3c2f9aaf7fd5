"""Eq. TOF / Eq. wf (Sec. 3.1): straight-ray wavefront error per element.

w(theta; r', v) = |r' - r(theta)| - v0 t(r', r(theta), v) = integral from r' to
the element of (1 - v0 / v(l)) dl.

Reading taken (the paper does not state its quadrature): the integrand is
exactly zero where the SOS equals v0, i.e. outside the SOS box, so the ray
from the patch centre r'_i towards element n is clipped at the distance L
where it leaves the box (or at the element, if that comes first), and the
integral over [0, L] is taken with the midpoint rule on n_samples equal
steps: w[i][n] = sum_s (L / N_s) (1 - v0 / v(r'_i + (s + 1/2)(L / N_s) u)).
"""
from __future__ import annotations

import math

import torch

from .geometry import F64, ring_positions, sos_box_half_extent
from .sos import field


def exit_distance(px: torch.Tensor, py: torch.Tensor, ux: torch.Tensor, uy: torch.Tensor,
                  hx: float, hy: float) -> torch.Tensor:
    """Distance along unit direction u from a point inside [-hx, hx] x [-hy, hy] to the box edge."""
    inf = torch.full_like(ux, math.inf)
    tx = torch.where(ux > 0, (hx - px) / ux, torch.where(ux < 0, (-hx - px) / ux, inf))
    ty = torch.where(uy > 0, (hy - py) / uy, torch.where(uy < 0, (-hy - py) / uy, inf))
    return torch.minimum(tx, ty)


def ray_lengths(centres: torch.Tensor, ring: torch.Tensor, hx: float, hy: float):
    """Clipped lengths L[i][n] and unit directions for every (patch, element) ray."""
    dx = ring[None, :, 0] - centres[:, None, 0]
    dy = ring[None, :, 1] - centres[:, None, 1]
    dist = torch.sqrt(dx * dx + dy * dy)
    ux, uy = dx / dist, dy / dist
    L = torch.minimum(exit_distance(centres[:, None, 0], centres[:, None, 1], ux, uy, hx, hy), dist)
    return L.clamp_min(0.0), ux, uy


def sos_to_delays(v: torch.Tensor, spacing: float, v0: float, centres, n_elem: int, radius: float,
                  phi0: float, n_samples: int, chunk: int = 8) -> torch.Tensor:
    """w [N][n_elem] (mm) for the node field v [Gy][Gx]; differentiable with respect to v."""
    centres = torch.as_tensor(centres, dtype=F64)
    ring = ring_positions(n_elem, radius, phi0)
    Gy, Gx = v.shape
    hx, hy = sos_box_half_extent(Gy, Gx, spacing)
    s = (torch.arange(n_samples, dtype=F64) + 0.5) / n_samples
    out = []
    for i0 in range(0, centres.shape[0], chunk):
        c = centres[i0:i0 + chunk]
        L, ux, uy = ray_lengths(c, ring, hx, hy)
        t = L[..., None] * s                                  # [n][e][Ns]
        x = c[:, None, None, 0] + t * ux[..., None]
        y = c[:, None, None, 1] + t * uy[..., None]
        f = 1.0 - v0 / field(v, spacing, v0, x, y)
        out.append(f.sum(-1) * (L / n_samples))
    return torch.cat(out, 0)
