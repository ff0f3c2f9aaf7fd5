"""Interpolated pixel-grid SOS representation (Sec. 3.3, "PG").

The SOS is a grid of nodes v[a][b] (Gy x Gx, spacing ds, node centres placed
like pixel centres).  Between nodes it is bilinear in node coordinates.  The
background is fixed: every node outside the grid has the value v0, and so
does every node outside the user's circular mask (those nodes are simply
not optimised).  The field is therefore v0 everywhere outside the box of
half-width (G + 1) ds / 2.
"""
from __future__ import annotations

import torch

from .geometry import F64


def node_value(v: torch.Tensor, v0: float, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    Gy, Gx = v.shape
    inside = (a >= 0) & (a < Gy) & (b >= 0) & (b < Gx)
    val = v[a.clamp(0, Gy - 1), b.clamp(0, Gx - 1)]
    return torch.where(inside, val, torch.as_tensor(v0, dtype=v.dtype))


def field(v: torch.Tensor, spacing: float, v0: float, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Bilinear SOS at points (x, y); differentiable with respect to v."""
    Gy, Gx = v.shape
    gx = x / spacing + (Gx - 1) / 2.0
    gy = y / spacing + (Gy - 1) / 2.0
    b0 = torch.floor(gx)
    a0 = torch.floor(gy)
    fx = gx - b0
    fy = gy - a0
    b0 = b0.long()
    a0 = a0.long()
    v00 = node_value(v, v0, a0, b0)
    v01 = node_value(v, v0, a0, b0 + 1)
    v10 = node_value(v, v0, a0 + 1, b0)
    v11 = node_value(v, v0, a0 + 1, b0 + 1)
    return (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11)


def full_field(params: torch.Tensor, mask: torch.Tensor, v0: float) -> torch.Tensor:
    """Node values: the parameters on free (masked-in) nodes, v0 on fixed ones."""
    return torch.where(torch.as_tensor(mask).bool(), params, torch.as_tensor(v0, dtype=F64))
