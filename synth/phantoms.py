"""Seeded synthetic phantoms: speed of sound (SOS) maps and initial pressure.

These are inputs only.  They stand in for the paper's numerical phantoms
(Supp. S1.1: SOS between 1490 and 1650 m/s, water background), which are
not available.  Nothing here implements the reconstruction method.

* ``disc``: background v0 plus one faster disc (1.560 mm/us, radius 8 mm)
  whose centre is uniform within 3 mm of the origin.
* ``ellipses``: background plus six ellipses (centres within 16 mm,
  semi-axes U(3, 8) mm, random rotation, signed SOS offsets) with smooth
  edges: each ellipse enters through 0.5 * erfc(s / (sqrt(2) sigma)) with
  sigma = 1 mm and s an approximate signed distance to its boundary.  The
  sum is clipped to [1.480, 1.600] mm/us.

Initial pressure: Gaussian blobs, sigma ~ U(0.3, 1.5) mm, amplitude
~ U(0.2, 1), centres uniform over a disc.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erfc

from .configs import Scan


@dataclass
class SosPhantom:
    kind: str
    v0: float
    params: dict

    def __call__(self, x, y):
        """SOS (mm/us) at points (x, y) in mm; numpy broadcasting."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if self.kind == "uniform":
            return np.full(np.broadcast(x, y).shape, self.v0)
        if self.kind == "disc":
            cx, cy, r, v1 = (self.params[k] for k in ("cx", "cy", "r", "v1"))
            inside = (x - cx) ** 2 + (y - cy) ** 2 < r * r
            return np.where(inside, v1, self.v0)
        if self.kind == "ellipses":
            v = np.full(np.broadcast(x, y).shape, self.v0)
            sig = self.params["sigma"]
            for (cx, cy, a, b, rot, dv) in self.params["ellipses"]:
                c, s = np.cos(rot), np.sin(rot)
                xr = c * (x - cx) + s * (y - cy)
                yr = -s * (x - cx) + c * (y - cy)
                rho = np.sqrt((xr / a) ** 2 + (yr / b) ** 2)
                dist = (rho - 1.0) * np.sqrt(a * b)
                v = v + dv * 0.5 * erfc(dist / (np.sqrt(2.0) * sig))
            return np.clip(v, self.params["vmin"], self.params["vmax"])
        raise ValueError(self.kind)

    @property
    def support_radius(self) -> float:
        """Radius outside which the SOS equals v0 (to double precision)."""
        if self.kind == "uniform":
            return 0.0
        if self.kind == "disc":
            return float(np.hypot(self.params["cx"], self.params["cy"]) + self.params["r"])
        if self.kind == "ellipses":
            sig = self.params["sigma"]
            return float(max(np.hypot(e[0], e[1]) + max(e[2], e[3]) * (1 + 12 * sig / np.sqrt(e[2] * e[3]))
                             for e in self.params["ellipses"]))
        raise ValueError(self.kind)


@dataclass
class Blobs:
    cx: np.ndarray
    cy: np.ndarray
    sigma: np.ndarray
    amp: np.ndarray

    def __len__(self):
        return len(self.cx)


def make_sos_phantom(scan: Scan, rng: np.random.Generator) -> SosPhantom:
    if scan.phantom == "uniform":
        return SosPhantom("uniform", scan.v0, {})
    if scan.phantom == "disc":
        r0 = 3.0 * np.sqrt(rng.uniform())
        a0 = rng.uniform(0, 2 * np.pi)
        return SosPhantom("disc", scan.v0, dict(cx=r0 * np.cos(a0), cy=r0 * np.sin(a0), r=8.0, v1=1.560))
    if scan.phantom == "ellipses":
        ell = []
        for _ in range(6):
            rr = 16.0 * np.sqrt(rng.uniform())
            aa = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(3.0, 8.0)
            b = rng.uniform(3.0, 8.0)
            rot = rng.uniform(0, np.pi)
            dv = rng.uniform(-0.020, 0.100) if rng.uniform() < 0.8 else rng.uniform(-0.020, 0.0)
            ell.append((rr * np.cos(aa), rr * np.sin(aa), a, b, rot, dv))
        return SosPhantom("ellipses", scan.v0,
                          dict(ellipses=ell, sigma=1.0, vmin=1.480, vmax=1.600))
    raise ValueError(scan.phantom)


def make_blobs(scan: Scan, rng: np.random.Generator) -> Blobs:
    n = scan.n_blobs
    r = scan.blob_radius * np.sqrt(rng.uniform(size=n))
    a = rng.uniform(0, 2 * np.pi, size=n)
    return Blobs(cx=r * np.cos(a), cy=r * np.sin(a),
                 sigma=rng.uniform(0.3, 1.5, size=n), amp=rng.uniform(0.2, 1.0, size=n))


def axis(n: int, spacing: float) -> np.ndarray:
    """Centres of n cells of the given spacing, symmetric about 0."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * spacing


def render_ip(scan: Scan, blobs: Blobs) -> np.ndarray:
    """Clean initial-pressure image [ny][nx] (row = y, column = x)."""
    ys = axis(scan.ny, scan.px)[:, None]
    xs = axis(scan.nx, scan.px)[None, :]
    img = np.zeros((scan.ny, scan.nx))
    for cx, cy, s, A in zip(blobs.cx, blobs.cy, blobs.sigma, blobs.amp):
        img += A * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * s * s))
    return img


def sos_grid_truth(scan: Scan, ph: SosPhantom) -> np.ndarray:
    """The phantom sampled at the SOS grid node centres [G][G]."""
    g = axis(scan.sos_n, scan.sos_spacing)
    return ph(g[None, :], g[:, None])


def free_node_mask(scan: Scan) -> np.ndarray:
    """Nodes whose centre lies within the user's circular mask are free."""
    g = axis(scan.sos_n, scan.sos_spacing)
    return (g[None, :] ** 2 + g[:, None] ** 2 <= scan.mask_radius ** 2).astype(np.uint8)


def ring_xy(scan: Scan) -> np.ndarray:
    """Element positions [n_elem][2] as (x, y): evenly spaced, counter-clockwise from phi0."""
    phi = scan.phi0 + 2 * np.pi * np.arange(scan.n_elem) / scan.n_elem
    return np.stack([scan.radius * np.cos(phi), scan.radius * np.sin(phi)], -1)
