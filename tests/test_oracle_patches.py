"""Pins of the oracle's patch extraction and windowed patch spectra (Eq. conv, Sec. 3.3, Supp. S1.4).

An impulse at a known pixel of a non-square image (npy != npx) must land, in every patch that covers it,
at the local position fixed by the patch's origin, and nowhere else; its windowed spectrum must equal the
closed form g[u, v] exp(-j (k_y u + k_x v) px) written out from exponentials (no FFT).  The pixel's
physical position relative to the centre the geometry gives for that patch ties the extraction order to
the patch centres (pinned separately as centroids of pixel blocks).  The same checks run on two planted
mistakes (patch order transposed, stride applied on the wrong axis) and must reject both.
"""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as G
from oracle import patches as Opatch

NY, NX, P, S, PX, FWHM = 28, 20, 8, 4, 0.25, 0.9      # npy = 6, npx = 4


def _window_value(u, v):
    """Gaussian of the stated FWHM at local pixel (u, v), from its definition."""
    sigma = FWHM / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    r2 = ((u - (P - 1) / 2.0) ** 2 + (v - (P - 1) / 2.0) ** 2) * PX * PX
    return math.exp(-r2 / (2.0 * sigma * sigma))


def _impulse_stack(row, col, amp=1.7, M=3, j=1):
    stack = np.zeros((M, NY, NX))
    stack[j, row, col] = amp
    return stack


def _check_impulse(extract, row, col, amp=1.7, M=3, j=1):
    """Raises AssertionError unless `extract` places the impulse where the patch geometry says."""
    npy, npx = G.patch_counts(NY, NX, P, S)
    assert npy != npx
    out = extract(_impulse_stack(row, col, amp, M, j), P, S).numpy()
    assert out.shape == (npy * npx, M, P, P)
    centres = G.patch_centres(NY, NX, PX, P, S).numpy()
    x_imp, y_imp = (col - (NX - 1) / 2) * PX, (row - (NY - 1) / 2) * PX
    hits = 0
    for a in range(npy):
        for b in range(npx):
            i = a * npx + b
            u, v = row - a * S, col - b * S
            expect = np.zeros((M, P, P))
            if 0 <= u < P and 0 <= v < P:
                expect[j, u, v] = amp
                hits += 1
                # the local pixel sits at the impulse's position relative to this patch's centre
                np.testing.assert_allclose([(v - (P - 1) / 2) * PX, (u - (P - 1) / 2) * PX],
                                           [x_imp - centres[i, 0], y_imp - centres[i, 1]], atol=1e-12)
            np.testing.assert_array_equal(out[i], expect)
    return hits


@pytest.mark.parametrize("row,col", [(13, 6), (0, 19), (27, 0), (9, 13)])
def test_impulse_lands_at_local_offset(row, col):
    hits = _check_impulse(Opatch.extract_patches, row, col)
    # rows covered by ceil-many patches: an interior pixel at stride 4, P 8 is in 2 x 2 patches
    n_rows = sum(1 for a in range(G.patch_counts(NY, NX, P, S)[0]) if 0 <= row - a * S < P)
    n_cols = sum(1 for b in range(G.patch_counts(NY, NX, P, S)[1]) if 0 <= col - b * S < P)
    assert hits == n_rows * n_cols > 0


def test_impulse_spectrum_closed_form():
    row, col, amp, j = 13, 6, 1.7, 1
    npy, npx = G.patch_counts(NY, NX, P, S)
    Y = Opatch.patch_spectra(_impulse_stack(row, col, amp, 3, j), P, S, PX, FWHM).numpy()
    k = 2.0 * np.pi * np.fft.fftfreq(P, d=PX)             # rad/mm along rows (k_y) and columns (k_x)
    for a in range(npy):
        for b in range(npx):
            i = a * npx + b
            u, v = row - a * S, col - b * S
            if not (0 <= u < P and 0 <= v < P):
                assert np.abs(Y[i]).max() == 0.0
                continue
            phase = np.exp(-1j * (k[:, None] * u * PX + k[None, :] * v * PX))
            np.testing.assert_allclose(Y[i, j], amp * _window_value(u, v) * phase, rtol=1e-12, atol=1e-14)
            assert np.abs(Y[i, [0, 2]]).max() == 0.0
    # the stored half keeps columns 0 .. P/2 of the same spectra
    Yh = Opatch.half_spectrum(torch.tensor(Y)).numpy()
    np.testing.assert_array_equal(Yh, Y[..., : P // 2 + 1])


def _transposed_order(stack, P, stride):
    """Planted mistake: patch (a, b) stored at index b * npy + a."""
    stack = torch.as_tensor(np.asarray(stack), dtype=torch.float64)
    M, ny, nx = stack.shape
    npy, npx = G.patch_counts(ny, nx, P, stride)
    out = torch.empty(npy * npx, M, P, P, dtype=torch.float64)
    for a in range(npy):
        for b in range(npx):
            out[b * npy + a] = stack[:, a * stride:a * stride + P, b * stride:b * stride + P]
    return out


def _stride_on_wrong_axis(stack, P, stride):
    """Planted mistake: the row origin advances with the column index and vice versa (clamped in range)."""
    stack = torch.as_tensor(np.asarray(stack), dtype=torch.float64)
    M, ny, nx = stack.shape
    npy, npx = G.patch_counts(ny, nx, P, stride)
    out = torch.empty(npy * npx, M, P, P, dtype=torch.float64)
    for a in range(npy):
        for b in range(npx):
            r0, c0 = min(b * stride, ny - P), min(a * stride, nx - P)
            out[a * npx + b] = stack[:, r0:r0 + P, c0:c0 + P]
    return out


@pytest.mark.parametrize("mutant", [_transposed_order, _stride_on_wrong_axis])
def test_checks_reject_planted_mistakes(mutant):
    with pytest.raises(AssertionError):
        for row, col in [(13, 6), (0, 19), (27, 0), (9, 13)]:
            _check_impulse(mutant, row, col)
