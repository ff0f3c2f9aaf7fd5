"""Eq. TF (Sec. 3.1): wavefront-based transfer function and PSF of a patch.

H_i(k; d, v) = 1/2 (e^{-j|k|(d - w(angle k))} + e^{+j|k|(d - w(angle k + pi))}) as
printed.  Readings taken:

* Sign convention.  Back-projection puts element theta's contribution to a
  point source at signed offset w(theta) - d along the unit vector u(theta)
  (Eq. DAS with Eq. wf); the transform of that line under the forward
  transform used for the data, e^{-j k.r}, is e^{+j|k|(d - w)} at k along u
  and e^{-j|k|(d - w(theta + pi))} at k opposite.  So with numpy's FFT the
  printed expression appears conjugated:
      H_ij(k) = 1/2 (e^{+j|k|(d_j - W_i(th))} + e^{-j|k|(d_j - W_i(th + pi))}),
  th = atan2(k_y, k_x) (th = 0 at k = 0).  A wavefront w = a . u(theta)
  then shifts the PSF to +a.  The loss of Eq. jr is the same under either
  sign; only the position of the deconvolved patch differs.
* k is the angular wavenumber 2 pi fftfreq(P, px) in rad/mm, so |k| d is a
  phase.
* w is known at the ring elements only.  W_i(th) takes the element where
  the ray from r'_i at angle th meets the ring: tau = -(r'.u) +
  sqrt((r'.u)^2 - |r'|^2 + R^2), q = r' + tau u, fractional element index
  f = ((atan2(q_y, q_x) - phi0) mod 2 pi) N / (2 pi), and interpolates
  linearly between elements floor(f) and floor(f) + 1 (cyclically).
* The PSF is h = Re(IFFT2(H)), a circular kernel with its origin at index 0.
"""
from __future__ import annotations

import math

import torch

from .geometry import F64, wavenumbers


def ring_index(centre: torch.Tensor, theta: torch.Tensor, radius: float, phi0: float, n_elem: int) -> torch.Tensor:
    """Fractional element index f where the ray from ``centre`` at angle theta meets the ring."""
    ux, uy = torch.cos(theta), torch.sin(theta)
    cx, cy = centre[0], centre[1]
    b = cx * ux + cy * uy
    tau = -b + torch.sqrt(b * b - (cx * cx + cy * cy) + radius * radius)
    qx = cx + tau * ux
    qy = cy + tau * uy
    return torch.remainder(torch.atan2(qy, qx) - phi0, 2.0 * math.pi) * n_elem / (2.0 * math.pi)


def wavefront_at(w_i: torch.Tensor, centre: torch.Tensor, theta: torch.Tensor, radius: float,
                 phi0: float) -> torch.Tensor:
    """W_i(theta): the element-sampled wavefront of patch i at arbitrary angles (differentiable in w_i)."""
    n_elem = w_i.shape[0]
    f = ring_index(centre, theta, radius, phi0, n_elem)
    n0 = torch.floor(f)
    a = f - n0
    n0 = n0.long()
    return (1.0 - a) * w_i[torch.remainder(n0, n_elem)] + a * w_i[torch.remainder(n0 + 1, n_elem)]


def transfer_functions(w: torch.Tensor, centres, radius: float, phi0: float, delays, P: int,
                       px: float) -> torch.Tensor:
    """H [N][M][P][P] complex128 from the wavefront table w [N][n_elem]."""
    centres = torch.as_tensor(centres, dtype=F64)
    d = torch.as_tensor(delays, dtype=F64)
    _, _, kabs, theta = wavenumbers(P, px)
    out = []
    for i in range(w.shape[0]):
        W1 = wavefront_at(w[i], centres[i], theta, radius, phi0)
        W2 = wavefront_at(w[i], centres[i], theta + math.pi, radius, phi0)
        ph1 = kabs * (d[:, None, None] - W1)                  # [M][P][P]
        ph2 = kabs * (d[:, None, None] - W2)
        out.append(0.5 * (torch.complex(torch.cos(ph1), torch.sin(ph1)) + torch.complex(torch.cos(ph2), -torch.sin(ph2))))
    return torch.stack(out, 0)


def psf(H: torch.Tensor) -> torch.Tensor:
    """h = Re(IFFT2(H)), same leading shape as H."""
    return torch.fft.ifft2(H).real
