"""Neural-field SOS queried at every ray sample, and its wavefront errors (Sec. 3.3, Eq. wf).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's second SOS representation is a coordinate-based neural field: a network maps a position to
the SOS, with the background fixed (Sec. 3.3).  The network built here is the neural-field workload's
one: random Fourier features of the position, four hidden ReLU layers of width 128, and a scalar head.
The wavefront error of a ray is Eq. wf, the integral of 1 - v0 / v along the straight ray, with v read
from the network at every midpoint sample.

Readings taken (the paper does not give these for this network):

* Features: gamma(p) = [cos(2 pi B p), sin(2 pi B p)], with B a fixed F x 2 matrix of frequencies in
  cycles per mm (random Fourier features; p in mm).
* Network: h_0 = gamma, h_l = relu(W_l h_{l-1} + b_l) for l = 1..4, f = w_5 . h_4 + b_5.
* SOS: v = v0 + a tanh(f) inside the disc |p| <= rho (the mask), v0 outside it.  Because v = v0 outside,
  the ray is clipped to the disc and the N_s midpoint samples are taken on the chord inside it:
  w = sum_s dl (1 - v0 / v(p_s)), dl = chord / N_s; w = 0 when the ray misses the disc.
* Precision: the workload runs weights and activations in BF16 with FP32 accumulation.  The weights
  passed here are BF16-representable values.  With ``bf16=True`` the oracle also rounds, to the
  nearest bfloat16 (ties to even), every value that the workload feeds to a BF16 product: the
  features, each hidden activation, and, in the backward pass, each layer's pre-activation gradient.
  All arithmetic is float64 otherwise.
* Parameter vector layout (float64 here, float32 on the device), row-major:
  W1 [H][2F], b1 [H], W2 [H][H], b2 [H], W3 [H][H], b3 [H], W4 [H][H], b4 [H], w5 [H], b5 [1].
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64


def layout(n_freq: int = 128, width: int = 128):
    """(name, shape) of the parameter blocks, in order."""
    H, K = width, 2 * n_freq
    return [("W1", (H, K)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
            ("W4", (H, H)), ("b4", (H,)), ("w5", (H,)), ("b5", (1,))]


def n_params(n_freq: int = 128, width: int = 128) -> int:
    return sum(math.prod(s) for _, s in layout(n_freq, width))


def unpack(params: torch.Tensor, n_freq: int = 128, width: int = 128) -> dict:
    out, o = {}, 0
    for name, shape in layout(n_freq, width):
        k = math.prod(shape)
        out[name] = params[o:o + k].reshape(shape)
        o += k
    assert o == params.numel()
    return out


def pack(blocks: dict, n_freq: int = 128, width: int = 128) -> torch.Tensor:
    return torch.cat([blocks[name].reshape(-1) for name, _ in layout(n_freq, width)])


def round_bf16(x: torch.Tensor) -> torch.Tensor:
    """Nearest bfloat16 (ties to even), returned as float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(F64)


def features(p: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """Random Fourier features of positions p [..., 2] (mm) for frequencies B [F, 2] (cycles/mm)."""
    phase = p @ B.T
    return torch.cat([torch.cos(2 * math.pi * phase), torch.sin(2 * math.pi * phase)], dim=-1)


def forward(params: torch.Tensor, B: torch.Tensor, p: torch.Tensor, bf16: bool = False, keep: bool = False):
    """Head output f at positions p [P, 2]; with keep=True also the list of BF16-fed activations
    [h_0 .. h_4] (each [P, width]) for the backward pass."""
    n_freq = B.shape[0]
    net = unpack(params, n_freq, _width(params, n_freq))
    r = round_bf16 if bf16 else (lambda t: t)
    h = r(features(p, B))
    hs = [h]
    for l in (1, 2, 3, 4):
        h = r(torch.relu(h @ net[f"W{l}"].T + net[f"b{l}"]))
        hs.append(h)
    f = h @ net["w5"] + net["b5"]
    return (f, hs) if keep else f


def _width(params: torch.Tensor, n_freq: int) -> int:
    # solve n_params(n_freq, H) = numel for H (3 H^2 + (2F + 5) H + 1 = numel)
    n = params.numel()
    a, b, c = 3.0, 2.0 * n_freq + 5.0, 1.0 - n
    H = int(round((-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)))
    assert n_params(n_freq, H) == n, "parameter vector does not match the layout"
    return H


def disc_chord(c: torch.Tensor, u: torch.Tensor, L: torch.Tensor, rho: float):
    """Part [t_a, t_b] of the segment c + t u, 0 <= t <= L (|u| = 1), inside the disc |p| <= rho;
    t_b <= t_a when the segment misses the disc."""
    cu = (c * u).sum(-1)
    disc = cu * cu - (c * c).sum(-1) + rho * rho
    root = torch.sqrt(torch.clamp(disc, min=0.0))
    ta = torch.clamp(-cu - root, min=0.0)
    tb = torch.minimum(-cu + root, L)
    miss = disc <= 0
    return torch.where(miss, torch.zeros_like(ta), ta), torch.where(miss, torch.zeros_like(tb), tb)


def sample_points(centres, ring: torch.Tensor, rho: float, n_samples: int):
    """Midpoint sample positions [N, n_elem, n_samples, 2] and step lengths dl [N, n_elem] of every
    (patch, element) ray, clipped to the disc."""
    c = torch.as_tensor(centres, dtype=F64)[:, None, :]
    d = ring[None, :, :] - c
    L = torch.linalg.norm(d, dim=-1)
    u = d / L[..., None]
    ta, tb = disc_chord(c.expand_as(d), u, L, rho)
    dl = torch.clamp(tb - ta, min=0.0) / n_samples
    s = torch.arange(n_samples, dtype=F64) + 0.5
    t = ta[..., None] + s * dl[..., None]
    p = c[..., None, :] + t[..., None] * u[..., None, :]
    return p, dl


def sos_to_delays(params, B, centres, ring, rho: float, v0: float, amp: float, n_samples: int,
                  bf16: bool = False) -> torch.Tensor:
    """w[i, n] = sum_s dl (1 - v0 / v(p_s)), v = v0 + amp tanh(f(p_s)) (Eq. wf on the neural field)."""
    p, dl = sample_points(centres, ring, rho, n_samples)
    f = forward(params, B, p.reshape(-1, 2), bf16=bf16).reshape(p.shape[:-1])
    v = v0 + amp * torch.tanh(f)
    return dl * (1.0 - v0 / v).sum(-1)


def sos_to_delays_vjp(params, B, centres, ring, rho: float, v0: float, amp: float, n_samples: int,
                      gw: torch.Tensor, bf16: bool = False) -> torch.Tensor:
    """sum_{i,n} gw[i,n] dw[i,n]/dparams, by backpropagation written out layer by layer.

    Per sample, dw/df = dl v0 / v^2 * amp (1 - tanh(f)^2).  Then, with delta_l = dL/dz_l:
      dL/dw5 = sum df h_4,  dL/db5 = sum df,
      delta_4 = (df w5) * [h_4 > 0],  delta_{l-1} = (W_l^T delta_l) * [h_{l-1} > 0],
      dL/dW_l = sum delta_l h_{l-1}^T,  dL/db_l = sum delta_l,
    where [h > 0] is the ReLU derivative (h = relu(z)) and delta_l is rounded to bfloat16 when bf16."""
    r = round_bf16 if bf16 else (lambda t: t)
    p, dl = sample_points(centres, ring, rho, n_samples)
    P = p.reshape(-1, 2)
    f, hs = forward(params, B, P, bf16=bf16, keep=True)
    n_freq = B.shape[0]
    net = unpack(params, n_freq, _width(params, n_freq))
    th = torch.tanh(f)
    v = v0 + amp * th
    df = (gw[..., None] * dl[..., None]).expand(p.shape[:-1]).reshape(-1) * v0 / (v * v) * amp * (1.0 - th * th)
    grads = {"w5": hs[4].T @ df, "b5": df.sum().reshape(1)}
    delta = r(df[:, None] * net["w5"][None, :] * (hs[4] > 0))
    for l in (4, 3, 2, 1):
        grads[f"W{l}"] = delta.T @ hs[l - 1]
        grads[f"b{l}"] = delta.sum(0)
        if l > 1:
            delta = r((delta @ net[f"W{l}"]) * (hs[l - 1] > 0))
    return pack(grads, n_freq, _width(params, n_freq))
