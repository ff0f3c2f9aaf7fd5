"""Image-quality figures used to report a reconstruction (the paper's Table 1 reports PSNR and SSIM of the
initial-pressure and SOS images).  Evaluation only: these run on whatever device the images are on and
are not part of the optimisation step.

Reading: both images are scaled to [0, 1] by the reference's range before comparison, since the
delay-and-sum image carries an arbitrary overall scale.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F


def normalise(img: torch.Tensor, ref: torch.Tensor):
    """Scale img by least squares onto ref, then both by ref's range to [0, 1]."""
    img = img.to(torch.float64)
    ref = ref.to(torch.float64)
    a = (img * ref).sum() / (img * img).sum().clamp_min(1e-300)
    lo, hi = ref.min(), ref.max()
    span = (hi - lo).clamp_min(1e-300)
    return (a * img - lo) / span, (ref - lo) / span


def psnr(img: torch.Tensor, ref: torch.Tensor, data_range: float = 1.0) -> float:
    """Peak signal-to-noise ratio in dB, 10 log10(range^2 / MSE)."""
    mse = ((img.to(torch.float64) - ref.to(torch.float64)) ** 2).mean().item()
    return math.inf if mse == 0 else 10.0 * math.log10(data_range ** 2 / mse)


def ssim(img: torch.Tensor, ref: torch.Tensor, data_range: float = 1.0, sigma: float = 1.5, size: int = 11) -> float:
    """Mean structural similarity (Wang, Bovik, Sheikh, Simoncelli 2004): Gaussian window (size 11,
    sigma 1.5), K1 = 0.01, K2 = 0.03, over the valid region."""
    x = img.to(torch.float64)[None, None]
    y = ref.to(torch.float64)[None, None]
    r = torch.arange(size, dtype=torch.float64, device=x.device) - (size - 1) / 2
    g1 = torch.exp(-r * r / (2 * sigma * sigma))
    g1 = g1 / g1.sum()
    w = (g1[:, None] * g1[None, :])[None, None]
    mu_x, mu_y = F.conv2d(x, w), F.conv2d(y, w)
    sxx = F.conv2d(x * x, w) - mu_x ** 2
    syy = F.conv2d(y * y, w) - mu_y ** 2
    sxy = F.conv2d(x * y, w) - mu_x * mu_y
    c1, c2 = (0.01 * data_range) ** 2, (0.03 * data_range) ** 2
    s = ((2 * mu_x * mu_y + c1) * (2 * sxy + c2)) / ((mu_x ** 2 + mu_y ** 2 + c1) * (sxx + syy + c2))
    return s.mean().item()
