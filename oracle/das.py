"""Eq. DAS (Sec. 3.1): delay-and-sum image for an extra delay d.

y(r'; d) = sum_n S(t = (|r' - r_n| - d) / v0, n).  The channel is a sampled
record S[n][m] at times t0 + m / fs; S(t, n) is its linear interpolation,
zero outside the record.  The sum is plain (no apodisation, no weights), as
the equation writes it.  FP64 numpy, one element at a time.
"""
from __future__ import annotations

import math

import numpy as np


def _ring(n_elem: int, radius: float, phi0: float) -> np.ndarray:
    phi = phi0 + 2.0 * math.pi * np.arange(n_elem) / n_elem
    return np.stack([radius * np.cos(phi), radius * np.sin(phi)], -1)


def _lerp_record(rec: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Linear interpolation of rec at fractional sample positions, 0 outside [0, len-1]."""
    n = rec.shape[0]
    i0 = np.floor(pos)
    a = pos - i0
    i0 = i0.astype(np.int64)
    i1 = i0 + 1
    s0 = np.where((i0 >= 0) & (i0 < n), rec[np.clip(i0, 0, n - 1)], 0.0)
    s1 = np.where((i1 >= 0) & (i1 < n), rec[np.clip(i1, 0, n - 1)], 0.0)
    return (1.0 - a) * s0 + a * s1


def das_points(S: np.ndarray, fs: float, t0: float, n_elem: int, radius: float, phi0: float,
               v0: float, delays, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """DAS values at arbitrary points: returns [M][*x.shape]."""
    S = np.asarray(S, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ring = _ring(n_elem, radius, phi0)
    delays = np.asarray(delays, dtype=np.float64)
    out = np.zeros((delays.size,) + x.shape)
    for n in range(n_elem):
        dist = np.hypot(x - ring[n, 0], y - ring[n, 1])
        for j, d in enumerate(delays):
            t = (dist - d) / v0
            out[j] += _lerp_record(S[n], (t - t0) * fs)
    return out


def das_stack(S: np.ndarray, fs: float, t0: float, n_elem: int, radius: float, phi0: float,
              v0: float, delays, ny: int, nx: int, px: float) -> np.ndarray:
    """The DAS stack y[j][r][c] over the image grid (Sec. 3.2: one image per delay)."""
    ys = (np.arange(ny) - (ny - 1) / 2.0) * px
    xs = (np.arange(nx) - (nx - 1) / 2.0) * px
    X, Y = np.meshgrid(xs, ys)
    return das_points(S, fs, t0, n_elem, radius, phi0, v0, delays, X, Y)
