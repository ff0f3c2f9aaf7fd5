"""Shared set-up of the GPU parity tests: workloads, the oracle's view of the same geometry, tolerances.

Every scalar handed to the library is a float32; the oracle receives the same float32-rounded values (in
float64), so that both sides compute the same mathematical quantity.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import synth
from oracle import geometry as OG

# Tolerances (relative L2 error against the FP64 oracle).  Delays and PSFs / transfer functions 1e-5,
# deconvolved patches 1e-4, gradients 1e-3, all in FP32.  Quantities with no stated tolerance take one
# derived from their FP32 arithmetic: DAS stack and patch spectra 1e-5 (sums of a few hundred FP32 terms
# with FP64 positions), loss values 1e-4 (sums of ~1e6 positive FP32 terms, each correct to ~1e-6).
TOL_DELAYS = 1e-5
TOL_PSF = 1e-5
TOL_DECONV = 1e-4
TOL_GRAD = 1e-3
TOL_DAS = 1e-5
TOL_SPECTRA = 1e-5
TOL_LOSS = 1e-4


def f32(x):
    return float(np.float32(x))


def rel_l2(a, b) -> float:
    a = torch.as_tensor(a).detach().cpu().to(torch.complex128 if torch.is_complex(torch.as_tensor(a)) or
                                            torch.is_complex(torch.as_tensor(b)) else torch.float64)
    b = torch.as_tensor(b).detach().cpu().to(a.dtype)
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


def announce(what: str):
    print(f"\n[gpu case] {what}", flush=True)
    sys.stdout.flush()


# A deliberately ragged workload: image not a multiple of the DAS tile, odd SOS grid, odd delay count,
# non-power-of-two even patch, samples per ray not a multiple of the lanes per ray.
RAGGED = synth.TINY.with_(name="ragged", ny=100, nx=90, px=0.25, n_elem=200, radius=40.0, phi0=0.3, n_t=2048,
                          delays=tuple(synth.uniform_delays(-0.7, 0.6, 7)), P=24, stride=12,
                          fwhm=synth.configs.fwhm_for_patch(24, 0.25), sos_n=23, sos_spacing=1.0, n_samples=100,
                          mask_radius=9.0, n_blobs=12, blob_radius=9.0)

# An SOS grid too large for one CU's LDS as a whole (the ray adjoint then works tile by tile).
FINEGRID = RAGGED.with_(name="finegrid", sos_n=150, sos_spacing=0.16, n_samples=120)


class OracleView:
    """The oracle's arguments for a workload, with every scalar rounded to float32."""

    def __init__(self, scan):
        self.scan = scan
        self.px = f32(scan.px)
        self.R = f32(scan.radius)
        self.phi0 = f32(scan.phi0)
        self.fs = f32(scan.fs)
        self.t0 = f32(scan.t0)
        self.v0 = f32(scan.v0)
        self.ds = f32(scan.sos_spacing)
        self.fwhm = f32(scan.fwhm)
        self.delays = np.asarray(scan.delays, dtype=np.float32).astype(np.float64)
        self.centres = torch.tensor(np.asarray(
            OG.patch_centres(scan.ny, scan.nx, self.px, scan.P, scan.stride).numpy(), dtype=np.float32),
            dtype=torch.float64)

    def geom(self, n_samples=None, eps=None):
        s = self.scan
        return dict(sos_spacing=self.ds, v0=self.v0, centres=self.centres, n_elem=s.n_elem, radius=self.R,
                    phi0=self.phi0, n_samples=n_samples or s.n_samples, delays=self.delays, px=self.px,
                    eps=f32(s.eps if eps is None else eps))


def dev32(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.float32).cuda().contiguous()


def devc64(x):
    return torch.as_tensor(x).to(torch.complex64).cuda().contiguous()


def random_real_patches_spectra(N, M, P, rng):
    """Spectra of real patches (so that a half spectrum determines them)."""
    x = torch.tensor(rng.normal(size=(N, M, P, P)) * 50.0)
    return torch.fft.fft2(x)
