"""Pins of the oracle's delay-and-sum stack (Eq. DAS)."""
import math

import numpy as np

import synth
from oracle import das


def _ring(n, R, phi0=0.0):
    a = phi0 + 2 * np.pi * np.arange(n) / n
    return R * np.cos(a), R * np.sin(a)


def test_affine_records_give_closed_form():
    """Linear interpolation is exact on affine records, so for S[n][m] = alpha_n m + beta_n the DAS
    value is sum_n alpha_n fs ((|r'-r_n| - d)/v0 - t0) + beta_n (all lookups inside the record)."""
    rng = np.random.default_rng(3)
    n_elem, R, n_t, fs, t0, v0 = 12, 20.0, 1600, 20.0, 1.5, 1.47
    alpha = rng.uniform(0.5, 2.0, n_elem)
    beta = rng.uniform(-1, 1, n_elem)
    S = alpha[:, None] * np.arange(n_t)[None, :] + beta[:, None]
    d = np.array([-0.7, 0.0, 0.45])
    x = rng.uniform(-5, 5, 7)
    y = rng.uniform(-5, 5, 7)
    got = das.das_points(S, fs, t0, n_elem, R, 0.3, v0, d, x, y)
    rx, ry = _ring(n_elem, R, 0.3)
    for j in range(3):
        dist = np.hypot(x[:, None] - rx[None], y[:, None] - ry[None])
        want = (alpha * fs * ((dist - d[j]) / v0 - t0) + beta).sum(1)
        np.testing.assert_allclose(got[j], want, rtol=1e-12)


def test_outside_record_is_zero():
    S = np.ones((4, 10))
    got = das.das_points(S, 1.0, 0.0, 4, 100.0, 0.0, 1.0, [0.0], np.array([0.0]), np.array([0.0]))
    assert got[0, 0] == 0.0          # every lookup time 100 us is far beyond the 10-sample record


def test_point_source_focus_and_ring():
    """Uniform SOS: a point source refocuses at d = 0 (Sec. 3.1, one velocity and d = 0 give a sharp
    image) and spreads into a ring of radius |d| for a wrong delay (Fig. 2 caption: rings)."""
    scan = synth.TINY.with_(phantom="uniform")
    ph = synth.make_sos_phantom(scan, np.random.default_rng(0))
    xs, ys = 1.0, -0.6
    S = synth.point_source_data(scan, ph, xs, ys, sigma=0.12)
    n = 81
    g = (np.arange(n) - (n - 1) / 2) * 0.05
    X, Y = np.meshgrid(xs + g, ys + g)
    img = das.das_points(S, scan.fs, scan.t0, scan.n_elem, scan.radius, scan.phi0, scan.v0,
                         [0.0, 0.8], X, Y)
    r, c = np.unravel_index(np.argmax(img[0]), img[0].shape)
    assert abs(X[r, c] - xs) < 0.051 and abs(Y[r, c] - ys) < 0.051
    # with d = 0.8 mm the energy sits on a ring of radius 0.8 mm about the source
    rad = np.hypot(X - xs, Y - ys)
    bins = np.round(rad / 0.05).astype(int)
    prof = np.bincount(bins.ravel(), weights=img[1].ravel()) / np.maximum(np.bincount(bins.ravel()), 1)
    peak_r = np.argmax(prof[:30]) * 0.05
    assert abs(peak_r - 0.8) <= 0.1
    assert img[1][r, c] < 0.2 * img[0][r, c]


def test_stack_layout_matches_points():
    scan = synth.TINY
    rng = np.random.default_rng(0)
    S = rng.normal(size=(scan.n_elem, scan.n_t))
    st = das.das_stack(S, scan.fs, scan.t0, scan.n_elem, scan.radius, 0.0, scan.v0, [0.2], 6, 5, 0.3)
    r, c = 4, 1
    x = (c - 2) * 0.3
    y = (r - 2.5) * 0.3
    p = das.das_points(S, scan.fs, scan.t0, scan.n_elem, scan.radius, 0.0, scan.v0, [0.2], np.array([x]),
                       np.array([y]))
    np.testing.assert_allclose(st[0, r, c], p[0, 0], rtol=1e-13)
