"""Eq. jr (Sec. 3.3): the self-supervised aberrated-image-matching loss.

L(v) = sum_i sum_k |k| sum_j |Y_ij(k) - H_ij(k; v) X_hat_i(k)|^2 + lambda TV(v),

summed over all P x P frequency bins of every patch and delay with the
unnormalised FFT (the paper gives no normalisation; it only rescales lambda
and the learning rate), X_hat from Eq. multi-deconv with the same H.

TV (reading: the paper names total variation without a formula): the
anisotropic sum of |forward differences| between neighbouring SOS nodes,
over every pair with at least one free node; the subgradient of |0| is 0.

The gradient is obtained by reverse-mode differentiation of these plain
definitions in float64 (the paper backpropagates through its model), so it
is independent of any hand-derived adjoint.
"""
from __future__ import annotations

import torch

from .geometry import F64, wavenumbers
from .rays import sos_to_delays
from .psf import transfer_functions
from .deconv import multichannel_deconv
from .sos import full_field


def data_loss(Y: torch.Tensor, H: torch.Tensor, X: torch.Tensor, px: float) -> torch.Tensor:
    P = Y.shape[-1]
    _, _, kabs, _ = wavenumbers(P, px)
    R = Y - H * X[:, None]
    return (kabs * (R.real ** 2 + R.imag ** 2)).sum()


def tv(v: torch.Tensor, mask) -> torch.Tensor:
    m = torch.as_tensor(mask).bool()
    dy = v[1:, :] - v[:-1, :]
    dx = v[:, 1:] - v[:, :-1]
    my = m[1:, :] | m[:-1, :]
    mx = m[:, 1:] | m[:, :-1]
    return (torch.abs(dy) * my).sum() + (torch.abs(dx) * mx).sum()


def loss_from_delays(w: torch.Tensor, Y: torch.Tensor, centres, radius: float, phi0: float, delays,
                     px: float, eps: float) -> torch.Tensor:
    """Data term of Eq. jr as a function of the wavefront table w [N][n_elem]."""
    P = Y.shape[-1]
    H = transfer_functions(w, centres, radius, phi0, delays, P, px)
    X = multichannel_deconv(Y, H, eps)
    return data_loss(Y, H, X, px)


def total_loss(v: torch.Tensor, Y, scan_geom: dict, mask, lam: float) -> torch.Tensor:
    """Eq. jr for the full node field v [G][G] (fixed nodes already at v0)."""
    g = scan_geom
    w = sos_to_delays(v, g["sos_spacing"], g["v0"], g["centres"], g["n_elem"], g["radius"], g["phi0"],
                      g["n_samples"])
    L = loss_from_delays(w, Y, g["centres"], g["radius"], g["phi0"], g["delays"], g["px"], g["eps"])
    return L + lam * tv(v, mask)


def loss_and_grad(params: torch.Tensor, mask, Y, scan_geom: dict, lam: float):
    """(L, dL/dv over all nodes, dL/dw, w) at node parameters ``params``; fixed nodes are set to v0 first."""
    v = full_field(torch.as_tensor(params, dtype=F64), mask, scan_geom["v0"]).detach().requires_grad_(True)
    g = scan_geom
    w = sos_to_delays(v, g["sos_spacing"], g["v0"], g["centres"], g["n_elem"], g["radius"], g["phi0"],
                      g["n_samples"])
    w_leaf = w.detach().requires_grad_(True)
    Ld = loss_from_delays(w_leaf, Y, g["centres"], g["radius"], g["phi0"], g["delays"], g["px"], g["eps"])
    (gw,) = torch.autograd.grad(Ld, w_leaf)
    (gv,) = torch.autograd.grad(w, v, grad_outputs=gw)
    vt = v.detach().requires_grad_(True)
    Lt = lam * tv(vt, mask)
    (gt,) = torch.autograd.grad(Lt, vt)
    return (Ld + Lt).detach(), (gv + gt).detach(), gw.detach(), w.detach()


def vjp(fn, inputs, grad_out):
    """Vector-Jacobian product of fn at inputs (a tuple of tensors) with grad_out."""
    inputs = tuple(x.detach().requires_grad_(True) for x in inputs)
    out = fn(*inputs)
    return torch.autograd.grad(out, inputs, grad_outputs=grad_out, allow_unused=True)
