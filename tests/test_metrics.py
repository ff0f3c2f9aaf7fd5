"""The image-quality figures against their definitions: PSNR from a known mean-squared error, SSIM = 1 for
identical images and its closed form for images that differ by a constant offset."""
import math

import numpy as np
import torch

from paper_2409_10876_amd import metrics


def test_psnr_closed_form():
    rng = np.random.default_rng(0)
    ref = torch.tensor(rng.random((64, 64)))
    noise = torch.full_like(ref, 0.01)
    noise[::2] *= -1
    assert abs(metrics.psnr(ref + noise, ref) - 40.0) < 1e-9          # MSE 1e-4 -> 40 dB
    assert metrics.psnr(ref, ref) == math.inf


def test_ssim_identity_and_offset():
    rng = np.random.default_rng(1)
    ref = torch.tensor(rng.random((48, 48)))
    assert abs(metrics.ssim(ref, ref) - 1.0) < 1e-12
    # a constant offset d changes only the luminance term: (2 mu (mu + d) + c1) / (mu^2 + (mu + d)^2 + c1)
    flat = torch.full((32, 32), 0.4, dtype=torch.float64)
    d = 0.1
    c1 = 0.01 ** 2
    want = (2 * 0.4 * 0.5 + c1) / (0.4 ** 2 + 0.5 ** 2 + c1)
    assert abs(metrics.ssim(flat + d, flat) - want) < 1e-12


def test_normalise_removes_scale():
    rng = np.random.default_rng(2)
    ref = torch.tensor(rng.random((20, 20))) * 3 + 1
    a, b = metrics.normalise(7.5 * ref, ref)
    assert torch.allclose(a, b, atol=1e-12) and abs(b.min().item()) < 1e-12 and abs(b.max().item() - 1) < 1e-12
