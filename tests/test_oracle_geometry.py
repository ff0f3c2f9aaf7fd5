"""Pins of the oracle's geometry (ring, patches, window, frequency grid)."""
import json
import math
import os

import numpy as np
import torch

from oracle import geometry as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_ring_counter_clockwise_from_phi0():
    r = G.ring_positions(8, 10.0, 0.0).numpy()
    np.testing.assert_allclose(r[0], [10.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(r[2], [0.0, 10.0], atol=1e-12)       # a quarter turn later: +y
    np.testing.assert_allclose(np.hypot(r[:, 0], r[:, 1]), 10.0, rtol=1e-15)
    r2 = G.ring_positions(8, 10.0, math.pi / 8).numpy()
    np.testing.assert_allclose(np.arctan2(r2[0, 1], r2[0, 0]), math.pi / 8, atol=1e-15)


def test_patch_centres_are_centroids_of_pixel_blocks():
    ny, nx, px, P, s = 24, 20, 0.3, 8, 4
    c = G.patch_centres(ny, nx, px, P, s).numpy()
    npy, npx = G.patch_counts(ny, nx, P, s)
    assert c.shape == (npy * npx, 2) and (npy, npx) == (5, 4)
    # centroid of an indicator image of the block, an independent computation
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    X = (xx - (nx - 1) / 2) * px
    Y = (yy - (ny - 1) / 2) * px
    for a in range(npy):
        for b in range(npx):
            ind = np.zeros((ny, nx))
            ind[a * s:a * s + P, b * s:b * s + P] = 1
            np.testing.assert_allclose(c[a * npx + b], [np.average(X, weights=ind), np.average(Y, weights=ind)],
                                       atol=1e-12)


def test_tiny_workload_patch_count():
    assert G.patch_counts(128, 128, 32, 16) == (7, 7)      # 49 patches
    assert G.patch_counts(560, 560, 80, 40) == (13, 13)    # 169 patches


def test_window_half_maximum_at_half_fwhm():
    # P odd so that a pixel sits exactly on the centre; FWHM chosen as a whole number of pixels
    P, px = 31, 0.1
    fwhm = 1.0
    g = G.gaussian_window(P, px, fwhm).numpy()
    c = P // 2
    assert g[c, c] == 1.0
    np.testing.assert_allclose(g[c, c + 5], 0.5, rtol=1e-12)     # 5 px = 0.5 mm = FWHM / 2
    np.testing.assert_allclose(g[c + 5, c], 0.5, rtol=1e-12)


def test_wavenumbers_match_fftfreq():
    P, px = 10, 0.2
    ky, kx, kabs, th = G.wavenumbers(P, px)
    f = 2 * np.pi * np.fft.fftfreq(P, px)
    np.testing.assert_allclose(kx.numpy()[0], f, rtol=1e-15)
    np.testing.assert_allclose(ky.numpy()[:, 0], f, rtol=1e-15)
    assert kx[0, P // 2] < 0                                # Nyquist index carries the negative frequency
    np.testing.assert_allclose(kabs[0, P // 2].item(), np.pi / px, rtol=1e-15)
    assert th[0, 0].item() == 0.0


def test_paper_constants_fixture():
    """Constants the paper prints (tests/golden/paper_constants.json, each with its citation)."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        c = json.load(f)
    import synth
    d = synth.uniform_delays(c["delay_range_mm"][0], c["delay_range_mm"][1], c["default_delays"])
    assert len(d) == 16 and d[0] == -0.8 and abs(d[-1] - 0.8) < 1e-15
    # 75 % overlap of 3.2 mm patches -> stride 0.8 mm; the synthetic workloads keep the FWHM/patch ratio
    assert abs(c["patch_mm"] * (1 - c["patch_overlap"]) - 0.8) < 1e-12
    assert abs(synth.configs.fwhm_for_patch(32, 0.1) - c["window_fwhm_mm"]) < 1e-12
