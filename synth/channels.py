"""Ring-array channel data S[n][t], standing in for the paper's k-Wave data.

The paper simulated full-wave data and took S = -2 dp/dt at each transducer
(Supp. S1.1).  k-Wave is not available, so each Gaussian initial-pressure
blob b is propagated along a straight acoustic ray (the ray model of Eq. TOF):
its arrival time at element n is the slowness integral T_bn from the blob
centre to the element through the analytic SOS phantom, evaluated here by
a fine midpoint rule over the part of the segment where the SOS differs from
v0 (plus the exact v0 part).  The recorded trace is a sum of even Ricker
pulses psi(u) = (1 - u^2) exp(-u^2 / 2), u = v0 (t - T_bn) / sigma_b: the
negated time derivative of a Gaussian's projection, so that delay-and-sum
back-projection gives a positive peak at the source.  Optional seeded
Gaussian noise at a given SNR.

This is input generation: it evaluates the phantom directly and shares no
code with the reconstruction library or with the oracle.
"""
from __future__ import annotations

import numpy as np

from .configs import Scan
from .phantoms import Blobs, SosPhantom, ring_xy


def travel_times(scan: Scan, ph: SosPhantom, bx, by, n_quad: int = 1024) -> np.ndarray:
    """Straight-ray slowness integrals T[b][n] (us) from points (bx, by) to every element."""
    bx = np.asarray(bx, dtype=np.float64)
    by = np.asarray(by, dtype=np.float64)
    ring = ring_xy(scan)
    T = np.empty((bx.size, scan.n_elem))
    Rs = ph.support_radius
    for b in range(bx.size):
        dx = ring[:, 0] - bx[b]
        dy = ring[:, 1] - by[b]
        dist = np.hypot(dx, dy)
        ux, uy = dx / dist, dy / dist
        if Rs <= 0.0:
            T[b] = dist / scan.v0
            continue
        # part of the segment [0, dist] inside the support disc of radius Rs
        pb = bx[b] * ux + by[b] * uy
        disc = pb * pb - (bx[b] ** 2 + by[b] ** 2 - Rs * Rs)
        root = np.sqrt(np.maximum(disc, 0.0))
        t_lo = np.clip(-pb - root, 0.0, dist)
        t_hi = np.clip(-pb + root, 0.0, dist)
        seg = t_hi - t_lo
        s = (np.arange(n_quad) + 0.5) / n_quad
        tt = t_lo[:, None] + s[None, :] * seg[:, None]
        v = ph(bx[b] + tt * ux[:, None], by[b] + tt * uy[:, None])
        T[b] = (dist - seg) / scan.v0 + seg * np.mean(1.0 / v, axis=1)
    return T


def channel_data(scan: Scan, ph: SosPhantom, blobs: Blobs, rng: np.random.Generator | None = None,
                 snr_db: float | None = None, n_quad: int = 1024) -> np.ndarray:
    """S[n_elem][n_t] float32."""
    T = travel_times(scan, ph, blobs.cx, blobs.cy, n_quad=n_quad)
    S = np.zeros((scan.n_elem, scan.n_t))
    t = scan.t0 + np.arange(scan.n_t) / scan.fs
    for b in range(len(blobs)):
        half = 8.0 * blobs.sigma[b] / scan.v0             # pulse support (us)
        lo = np.maximum(((T[b] - half - scan.t0) * scan.fs).astype(np.int64), 0)
        width = int(np.ceil(2 * half * scan.fs)) + 2
        idx = lo[:, None] + np.arange(width)[None, :]
        ok = idx < scan.n_t
        idx = np.minimum(idx, scan.n_t - 1)
        u = scan.v0 * (t[idx] - T[b][:, None]) / blobs.sigma[b]
        pulse = blobs.amp[b] * (1.0 - u * u) * np.exp(-0.5 * u * u) * ok
        np.add.at(S, (np.repeat(np.arange(scan.n_elem), width).reshape(scan.n_elem, width), idx), pulse)
    if snr_db is not None:
        rng = rng if rng is not None else np.random.default_rng(1234)
        p = np.mean(S ** 2)
        S = S + rng.normal(0.0, np.sqrt(p / 10 ** (snr_db / 10.0)), size=S.shape)
    return S.astype(np.float32)


def point_source_data(scan: Scan, ph: SosPhantom, x: float, y: float, sigma: float = 0.15) -> np.ndarray:
    """Channel data of a single narrow source at (x, y)."""
    blobs = Blobs(cx=np.array([x]), cy=np.array([y]), sigma=np.array([sigma]), amp=np.array([1.0]))
    return channel_data(scan, ph, blobs)
