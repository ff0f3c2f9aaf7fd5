"""Seeded phantoms of the learned warm start's training and evaluation sets.

Inputs only: SOS maps on the SOS node grid and initial-pressure blobs.  The scans themselves (arrival
times, channel data, delay-and-sum stacks) are made from these by the reconstruction library's own
forward model.

Each phantom is drawn from its own generator, seeded by (set seed, phantom index), so a phantom does
not depend on how the set is split into batches.  Training phantoms have indices 0 .. n_train - 1, the
held-out ones n_train .. n_train + n_eval - 1.

* SOS: background v0 plus six ellipses as in the paper-shaped workload (centres within 16 mm,
  semi-axes U(3, 8) mm, random rotation, smooth edges of width 1 mm through erfc), with signed offsets
  U(-0.05, +0.12) mm/us, clipped to [1.450, 1.620] mm/us, and v0 on every node outside the mask disc.
* Initial pressure: n_blobs Gaussian blobs, centres uniform over the blob disc, sigma U(0.3, 1.5) mm,
  amplitude U(0.2, 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .configs import Scan
from .phantoms import axis


@dataclass(frozen=True)
class WarmSet:
    n_train: int = 20000
    n_eval: int = 100
    vmin: float = 1.450
    vmax: float = 1.620
    n_ellipses: int = 6
    seed: int = 5


WARM = WarmSet()


def _draw(scan: Scan, ws: WarmSet, index: int):
    rng = np.random.default_rng([ws.seed, index])
    ell = np.empty((ws.n_ellipses, 6))
    for e in range(ws.n_ellipses):
        rr = 16.0 * np.sqrt(rng.uniform())
        aa = rng.uniform(0, 2 * np.pi)
        ell[e] = (rr * np.cos(aa), rr * np.sin(aa), rng.uniform(3.0, 8.0), rng.uniform(3.0, 8.0),
                  rng.uniform(0, np.pi), rng.uniform(ws.vmin - scan.v0, ws.vmax - scan.v0))
    n = scan.n_blobs
    r = scan.blob_radius * np.sqrt(rng.uniform(size=n))
    a = rng.uniform(0, 2 * np.pi, size=n)
    blobs = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(0.3, 1.5, size=n), rng.uniform(0.2, 1.0, size=n)],
                     axis=-1)
    return ell, blobs


def phantom_batch(scan: Scan, indices, ws: WarmSet = WARM, sigma_edge: float = 1.0):
    """SOS node grids [B][G][G] (float32) and blobs [B][n_blobs][4] (x, y, sigma, amp; float32) of the
    phantoms with the given indices."""
    draws = [_draw(scan, ws, int(i)) for i in indices]
    ell = torch.tensor(np.stack([d[0] for d in draws]), dtype=torch.float64)        # [B][E][6]
    blobs = np.stack([d[1] for d in draws]).astype(np.float32)
    g = torch.tensor(axis(scan.sos_n, scan.sos_spacing), dtype=torch.float64)
    X = g[None, None, None, :]
    Y = g[None, None, :, None]
    cx, cy, a, b, rot, dv = (ell[..., k][..., None, None] for k in range(6))
    c, s = torch.cos(rot), torch.sin(rot)
    xr = c * (X - cx) + s * (Y - cy)
    yr = -s * (X - cx) + c * (Y - cy)
    dist = (torch.sqrt((xr / a) ** 2 + (yr / b) ** 2) - 1.0) * torch.sqrt(a * b)
    v = scan.v0 + (dv * 0.5 * torch.special.erfc(dist / (np.sqrt(2.0) * sigma_edge))).sum(dim=1)
    v = v.clamp(ws.vmin, ws.vmax)
    inside = (X[0, 0] ** 2 + Y[0, 0] ** 2) <= scan.mask_radius ** 2
    v = torch.where(inside, v, torch.full_like(v, scan.v0))
    return v.to(torch.float32).numpy(), blobs
