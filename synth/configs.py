"""Workload definitions: plain numbers only (sizes, physical constants, seeds).

Units everywhere: millimetres, microseconds, mm/us (1 mm/us = 1000 m/s),
sampling rate in samples per microsecond (40 MHz = 40 /us).

Two scan workloads, both seeded and synthetic:

* ``tiny``  -- 128^2 pixels at 0.2 mm, 256-element ring of radius 50 mm,
  2048 samples at 40 MHz, a single faster disc, 5 delays, 32^2 patches at
  stride 16 (49 patches), 32^2 SOS grid.  Small enough for the FP64 oracle
  to run end to end in seconds.
* ``paper`` -- 560^2 pixels at 0.1 mm, 512-element ring of radius 110 mm,
  4096 samples, six blurred ellipses spanning 1.48-1.60 mm/us, 11 delays
  uniform in [-0.8, 0.8] mm (the paper's delay range, Supp. ablation on the
  number of delays), 80^2 patches at stride 40 (169 patches), 140^2 SOS grid.

Choices the paper leaves open are fields here (window FWHM, Tikhonov eps,
samples per ray, mask radius, learning rate); the readings are listed in the
design notes of the repository.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict, replace
from typing import Tuple


def fwhm_for_patch(P: int, px: float) -> float:
    """Keep the paper's window-to-patch ratio (1.5 mm FWHM on 3.2 mm patches)."""
    return 1.5 / 3.2 * P * px


def delays_from_sos_offsets(radius: float, v0: float, offsets) -> Tuple[float, ...]:
    """Delay (mm) that refocuses a ring of radius ``radius`` for a uniform
    SOS of v0 + offset: the path-length change R (1 - v0 / (v0 + dv))."""
    return tuple(radius * (1.0 - v0 / (v0 + dv)) for dv in offsets)


def uniform_delays(lo: float, hi: float, M: int) -> Tuple[float, ...]:
    if M == 1:
        return (0.5 * (lo + hi),)
    return tuple(lo + (hi - lo) * j / (M - 1) for j in range(M))


@dataclass(frozen=True)
class Scan:
    name: str
    # image grid (pixels centred on the origin)
    ny: int
    nx: int
    px: float
    # ring array
    n_elem: int
    radius: float
    phi0: float
    # channel data
    fs: float          # samples per microsecond
    n_t: int
    t0: float          # time of sample 0 (us)
    v0: float          # background / assumed SOS (mm/us)
    # DAS stack delays (mm)
    delays: Tuple[float, ...]
    # patches
    P: int
    stride: int
    fwhm: float
    # SOS pixel grid
    sos_n: int
    sos_spacing: float
    mask_radius: float
    # ray sampling and solver
    n_samples: int
    eps: float
    lam_tv: float
    lr: float
    steps: int
    # phantom recipe
    phantom: str
    n_blobs: int
    blob_radius: float
    seed: int = 0

    @property
    def M(self) -> int:
        return len(self.delays)

    @property
    def n_patch_y(self) -> int:
        return (self.ny - self.P) // self.stride + 1

    @property
    def n_patch_x(self) -> int:
        return (self.nx - self.P) // self.stride + 1

    @property
    def n_patches(self) -> int:
        return self.n_patch_y * self.n_patch_x

    def with_(self, **kw) -> "Scan":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


TINY = Scan(
    name="tiny", ny=128, nx=128, px=0.2,
    n_elem=256, radius=50.0, phi0=0.0,
    fs=40.0, n_t=2048, t0=0.0, v0=1.5,
    delays=delays_from_sos_offsets(50.0, 1.5, (-0.020, -0.010, 0.0, 0.010, 0.020)),
    P=32, stride=16, fwhm=fwhm_for_patch(32, 0.2),
    sos_n=32, sos_spacing=0.8, mask_radius=12.0,
    n_samples=256, eps=1e-6, lam_tv=1e7, lr=2e-3, steps=10,
    phantom="disc", n_blobs=20, blob_radius=11.0,
)

# TV weights.  The loss here is an unnormalised sum (about 4e12 at v = v0 for the paper-shaped scan, 1e10
# for the small one), so the paper's lambda = 1e-4, which belongs to its own normalisation, would leave TV
# without effect.  lambda = 3e9 with lr = 1e-3 mm/us gave the lowest SOS error over 500 steps in a sweep
# of lr in {3e-4, 1e-3} x lambda in {1e9, 3e9, 1e10, 3e10} on the paper-shaped scan (9.8 -> 5.6 m/s); the
# small scan takes the same ratio to its loss.
PAPER = Scan(
    name="paper", ny=560, nx=560, px=0.1,
    n_elem=512, radius=110.0, phi0=0.0,
    fs=40.0, n_t=4096, t0=0.0, v0=1.5,
    delays=uniform_delays(-0.8, 0.8, 11),
    P=80, stride=40, fwhm=fwhm_for_patch(80, 0.1),
    sos_n=140, sos_spacing=0.4, mask_radius=26.0,
    n_samples=256, eps=1e-6, lam_tv=3e9, lr=1e-3, steps=500,
    phantom="ellipses", n_blobs=100, blob_radius=25.0,
)

WORKLOADS = {"tiny": TINY, "paper": PAPER}


def describe(s: Scan) -> str:
    return (f"{s.name}: {s.ny}x{s.nx} px @ {s.px} mm, ring {s.n_elem} el R={s.radius} mm, "
            f"{s.n_t} samples @ {s.fs} /us, M={s.M}, patches {s.n_patches} of {s.P}^2 "
            f"(stride {s.stride}), SOS {s.sos_n}^2 @ {s.sos_spacing} mm, N_s={s.n_samples}")


def batch_scans(n: int = 32, seed: int = 0, n_blobs: int = 10) -> list:
    """Independent scans of uneven sizes for batched solves: square images of 256^2 to 768^2 pixels at
    0.1 mm, 256 to 1024 ring elements (radius 110 mm), 7 to 15 delays uniform in [-0.8, 0.8] mm, patches of
    64^2 or 80^2 at half-patch stride, SOS node grid at 0.4 mm over the image, mask radius 0.45 of the
    image side, records long enough for the farthest pixel."""
    import math
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        side = int(rng.integers(16, 49)) * 16                      # 256 .. 768 pixels
        P = int(rng.choice([64, 80]))
        n_elem = int(rng.choice([256, 384, 512, 768, 1024]))
        M = int(rng.integers(7, 16))
        field = side * 0.1
        G = int(round(field / 0.4))
        reach = 110.0 + field * math.sqrt(2) / 2 + 2.0             # farthest pixel, mm
        n_t = int(math.ceil(reach / 1.5 * 40.0 / 512.0)) * 512
        out.append(PAPER.with_(name=f"batch{k}", ny=side, nx=side, n_elem=n_elem, n_t=n_t,
                               delays=uniform_delays(-0.8, 0.8, M), P=P, stride=P // 2,
                               fwhm=fwhm_for_patch(P, 0.1), sos_n=G, sos_spacing=0.4,
                               mask_radius=0.45 * field, n_blobs=n_blobs, blob_radius=0.4 * field,
                               seed=seed * 1000 + k))
    return out
