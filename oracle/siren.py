"""The paper's neural-field SOS: a SIREN on the SOS-grid node coordinates (Sec. 3.3), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's network has one hidden layer of 256 sinusoidal features mapping a coordinate to the SOS,
restricted to the circular mask with the background fixed, and 1027 parameters in all; Eq. jr uses no TV
for it.  It is evaluated at the node centres of the SOS grid, which the straight-ray model then
interpolates bilinearly like the pixel grid (Eq. TOF, Eq. wf).

Readings taken (the paper does not give these):

* Hidden features h_k = sin(omega0 (W1[k] . x + b1[k])) with omega0 = 30 (the usual first-layer
  frequency of a sinusoidal network), x = node centre / mask radius (the mask maps to the unit disc).
* Output f = w2 . h + b2, and SOS v = v0 + s f + o on the free nodes, v0 on the fixed ones.  The two
  scalars s and o are the parameters beyond 2 -> 256 -> 1 (1025): 512 + 256 + 256 + 1 + 2 = 1027.
* Parameter vector layout: W1 [256][2] (x, y), b1 [256], w2 [256], b2 [1], s [1], o [1].
"""
from __future__ import annotations

import torch

from .geometry import cell_centres

F64 = torch.float64


def layout(hidden: int = 256):
    return [("W1", (hidden, 2)), ("b1", (hidden,)), ("w2", (hidden,)), ("b2", (1,)), ("s", (1,)), ("o", (1,))]


def n_params(hidden: int = 256) -> int:
    return 4 * hidden + 3


def unpack(params: torch.Tensor, hidden: int = 256) -> dict:
    out, o = {}, 0
    for name, shape in layout(hidden):
        k = 1
        for d in shape:
            k *= d
        out[name] = params[o:o + k].reshape(shape)
        o += k
    assert o == params.numel()
    return out


def node_coordinates(Gy: int, Gx: int, spacing: float, mask_radius: float) -> torch.Tensor:
    """Node centres of the SOS grid (placed like pixel centres) over the mask radius, [Gy][Gx][2] (x, y)."""
    y = cell_centres(Gy, spacing) / mask_radius
    x = cell_centres(Gx, spacing) / mask_radius
    return torch.stack(torch.meshgrid(x, y, indexing="xy"), dim=-1)


def sos_grid(params: torch.Tensor, Gy: int, Gx: int, spacing: float, mask_radius: float, mask, v0: float,
             omega0: float = 30.0) -> torch.Tensor:
    """SOS on the node grid [Gy][Gx]: v0 + s f + o on the free nodes, v0 elsewhere."""
    hidden = (params.numel() - 3) // 4
    net = unpack(params, hidden)
    xy = node_coordinates(Gy, Gx, spacing, mask_radius)
    h = torch.sin(omega0 * (xy @ net["W1"].T + net["b1"]))
    f = h @ net["w2"] + net["b2"]
    m = torch.as_tensor(mask).bool()
    return torch.where(m, v0 + net["s"] * f + net["o"], torch.full_like(f, v0))
