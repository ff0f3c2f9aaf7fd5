"""Pins of the neural-field oracle (oracle/nf.py) against closed forms, textbook identities, reverse-mode
differentiation and finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import nf as Onf
from oracle.geometry import ring_positions

F64 = torch.float64


def _random_params(n_freq, width, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    blocks = {}
    for name, shape in Onf.layout(n_freq, width):
        fan = shape[-1] if len(shape) == 2 else width
        blocks[name] = (torch.rand(shape, generator=g, dtype=F64) * 2 - 1) * scale * math.sqrt(6.0 / fan)
    return Onf.pack(blocks, n_freq, width)


def test_parameter_count():
    # 128 x 256 + 3 (128 x 128) weights, 4 x 128 biases, a 128-vector head and its bias
    assert Onf.n_params(128, 128) == 128 * 256 + 3 * 128 * 128 + 4 * 128 + 128 + 1 == 82561
    p = torch.arange(Onf.n_params(8, 16), dtype=F64)
    assert torch.equal(Onf.pack(Onf.unpack(p, 8, 16), 8, 16), p)
    assert Onf._width(p, 8) == 16


def test_features_closed_forms():
    rng = np.random.default_rng(0)
    B = torch.tensor(rng.normal(0, 2, (16, 2)))
    p = torch.tensor(rng.uniform(-20, 20, (50, 2)))
    g = Onf.features(p, B)
    assert g.shape == (50, 32)
    # cos^2 + sin^2 = 1 for every frequency
    assert torch.allclose(g[:, :16] ** 2 + g[:, 16:] ** 2, torch.ones(50, 16, dtype=F64), atol=1e-14)
    # zero frequency: cos = 1, sin = 0
    g0 = Onf.features(p, torch.zeros(3, 2, dtype=F64))
    assert torch.equal(g0, torch.cat([torch.ones(50, 3), torch.zeros(50, 3)], 1).to(F64))
    # integer numbers of cycles per shift leave the features unchanged
    Bi = torch.tensor([[1.0, 0.0], [0.5, 2.0], [-3.0, 1.5]], dtype=F64)
    shift = torch.tensor([2.0, 4.0], dtype=F64)          # B shift = (2, 9, 0): whole cycles
    assert torch.allclose(Onf.features(p + shift, Bi), Onf.features(p, Bi), atol=1e-9)
    # a single frequency along x: cos(2 pi b x)
    b = torch.tensor([[0.25, 0.0]], dtype=F64)
    assert torch.allclose(Onf.features(p, b)[:, 0], torch.cos(2 * math.pi * 0.25 * p[:, 0]), atol=1e-14)


def test_network_composes_layers_in_order():
    """A ReLU network built to compute sum_k c_k cos(2 pi B_k . p) exactly: layer 1 passes +cos and -cos
    (relu splits them), layers 2-4 are identities on non-negative inputs, the head recombines.  A
    transposed weight or a layer applied out of order breaks it."""
    F, H = 64, 128
    rng = np.random.default_rng(1)
    B = torch.tensor(rng.normal(0, 0.3, (F, 2)))
    c = torch.tensor(rng.normal(0, 1, F))
    W1 = torch.zeros(H, 2 * F, dtype=F64)
    W1[:F, :F] = torch.eye(F, dtype=F64)                 # +cos_k (the sin half is ignored)
    W1[F:, :F] = -torch.eye(F, dtype=F64)                # -cos_k
    eye = torch.eye(H, dtype=F64)
    blocks = {"W1": W1, "b1": torch.zeros(H, dtype=F64), "W2": eye, "b2": torch.zeros(H, dtype=F64),
              "W3": eye, "b3": torch.zeros(H, dtype=F64), "W4": eye, "b4": torch.zeros(H, dtype=F64),
              "w5": torch.cat([c, -c]), "b5": torch.tensor([0.7], dtype=F64)}
    params = Onf.pack(blocks, F, H)
    p = torch.tensor(rng.uniform(-10, 10, (40, 2)))
    want = torch.cos(2 * math.pi * p @ B.T) @ c + 0.7
    assert torch.allclose(Onf.forward(params, B, p), want, atol=1e-12)
    # a permutation of layer 2's rows with the inverse permutation of layer 3's columns changes nothing
    perm = torch.tensor(rng.permutation(H))
    blocks2 = dict(blocks, W2=eye[perm], W3=eye[:, perm])
    assert torch.allclose(Onf.forward(Onf.pack(blocks2, F, H), B, p), want, atol=1e-12)
    # but an unmatched permutation does change it
    blocks3 = dict(blocks, W2=eye[perm])
    assert not torch.allclose(Onf.forward(Onf.pack(blocks3, F, H), B, p), want, atol=1e-3)


def test_relu_positive_homogeneity():
    F, H = 8, 16
    params = _random_params(F, H, 2)
    B = torch.tensor(np.random.default_rng(2).normal(0, 1, (F, 2)))
    p = torch.tensor(np.random.default_rng(3).uniform(-5, 5, (30, 2)))
    net = Onf.unpack(params.clone(), F, H)
    net = {k: v.clone() for k, v in net.items()}
    net["W4"] *= 3.0
    net["b4"] *= 3.0
    net["w5"] /= 3.0
    assert torch.allclose(Onf.forward(Onf.pack(net, F, H), B, p), Onf.forward(params, B, p), atol=1e-12)


def test_disc_chord():
    rho = 10.0
    c = torch.tensor([[0.0, 0.0], [3.0, 0.0], [30.0, 0.0], [-4.0, 0.0], [0.0, 0.0]], dtype=F64)
    u = torch.tensor([[1.0, 0.0], [0.0, 1.0], [0.0, 1.0], [1.0, 0.0], [0.6, 0.8]], dtype=F64)
    L = torch.tensor([100.0, 100.0, 100.0, 100.0, 5.0], dtype=F64)
    ta, tb = Onf.disc_chord(c, u, L, rho)
    assert torch.allclose(ta, torch.tensor([0.0, 0.0, 0.0, 0.0, 0.0], dtype=F64))
    assert torch.allclose(tb, torch.tensor([10.0, math.sqrt(91.0), 0.0, 14.0, 5.0], dtype=F64))
    # a centre outside the disc looking at it: enters at 20, leaves at 40
    ta, tb = Onf.disc_chord(torch.tensor([[-30.0, 0.0]], dtype=F64), torch.tensor([[1.0, 0.0]], dtype=F64),
                            torch.tensor([100.0], dtype=F64), rho)
    assert torch.allclose(ta, torch.tensor([20.0], dtype=F64)) and torch.allclose(tb, torch.tensor([40.0],
                                                                                                  dtype=F64))


def test_constant_field_closed_form():
    """All weights zero: f = b5 everywhere, so w = chord (1 - v0 / (v0 + a tanh b5)) exactly, with the
    chord inside the mask disc; rays that miss the disc give 0."""
    F, H = 8, 16
    blocks = {name: torch.zeros(shape, dtype=F64) for name, shape in Onf.layout(F, H)}
    blocks["b5"] = torch.tensor([0.4], dtype=F64)
    params = Onf.pack(blocks, F, H)
    B = torch.tensor(np.random.default_rng(4).normal(0, 2, (F, 2)))
    ring = ring_positions(64, 60.0, 0.1)
    centres = torch.tensor([[0.0, 0.0], [5.0, -3.0], [25.0, 25.0]], dtype=F64)
    rho, v0, amp = 20.0, 1.5, 0.15
    w = Onf.sos_to_delays(params, B, centres, ring, rho, v0, amp, 7)
    d = ring[None] - centres[:, None]
    L = d.norm(dim=-1)
    u = d / L[..., None]
    cu = (centres[:, None] * u).sum(-1)
    disc = cu ** 2 - (centres ** 2).sum(-1)[:, None] + rho ** 2
    t_out = -cu + torch.sqrt(disc.clamp(min=0))
    t_in = (-cu - torch.sqrt(disc.clamp(min=0))).clamp(min=0)
    chord = torch.where(disc > 0, (t_out - t_in).clamp(min=0), torch.zeros_like(disc))
    want = chord * (1 - v0 / (v0 + amp * math.tanh(0.4)))
    assert torch.allclose(w, want, atol=1e-12)
    assert (w[2] == 0).sum() > 0 and (w[2] != 0).sum() > 0      # the far corner sees the disc only sideways


def _small_case(seed=5):
    F, H = 8, 16
    params = _random_params(F, H, seed)
    rng = np.random.default_rng(seed)
    B = torch.tensor(rng.normal(0, 0.5, (F, 2)))
    ring = ring_positions(12, 30.0, 0.2)
    centres = torch.tensor([[0.0, 1.0], [-4.0, 2.5], [6.0, -3.0]], dtype=F64)
    gw = torch.tensor(rng.normal(size=(3, 12)))
    return F, H, params, B, ring, centres, gw


def test_backward_matches_reverse_mode():
    F, H, params, B, ring, centres, gw = _small_case()
    args = (B, centres, ring, 9.0, 1.5, 0.15, 10)
    got = Onf.sos_to_delays_vjp(params, *args, gw)
    p = params.clone().requires_grad_(True)
    (Onf.sos_to_delays(p, *args) * gw).sum().backward()
    assert torch.allclose(got, p.grad, rtol=1e-11, atol=1e-13)


def test_backward_matches_finite_differences():
    F, H, params, B, ring, centres, gw = _small_case(6)
    args = (B, centres, ring, 9.0, 1.5, 0.15, 10)
    got = Onf.sos_to_delays_vjp(params, *args, gw)
    L = lambda q: (Onf.sos_to_delays(q, *args) * gw).sum()
    rng = np.random.default_rng(7)
    idx = rng.choice(params.numel(), 25, replace=False)
    for i in idx:
        h = 1e-6
        e = torch.zeros_like(params)
        e[i] = h
        fd = (L(params + e) - L(params - e)) / (2 * h)
        assert abs(fd.item() - got[i].item()) <= 1e-6 * (1 + abs(fd.item())), (i, fd.item(), got[i].item())


def test_bf16_rounding_points():
    """With bf16=True the forward pass equals a literal evaluation that rounds the features and each hidden
    activation to bfloat16; with bfloat16-exact inputs nothing changes."""
    F, H, params, B, ring, centres, gw = _small_case(8)
    p = torch.tensor(np.random.default_rng(9).uniform(-8, 8, (20, 2)))
    net = Onf.unpack(params, F, H)
    r = lambda t: t.to(torch.float32).to(torch.bfloat16).to(F64)
    h = r(Onf.features(p, B))
    for l in (1, 2, 3, 4):
        h = r(torch.relu(h @ net[f"W{l}"].T + net[f"b{l}"]))
    assert torch.equal(Onf.forward(params, B, p, bf16=True), h @ net["w5"] + net["b5"])
    # zero frequencies give exact features (1 and 0); a network whose weights and activations are all
    # bfloat16-exact is unchanged by the rounding
    blocks = {name: torch.zeros(shape, dtype=F64) for name, shape in Onf.layout(F, H)}
    blocks["W1"][:, :F] = 0.5
    for l in (2, 3, 4):
        blocks[f"W{l}"] = torch.eye(H, dtype=F64)
    blocks["w5"][:] = 0.25
    q = Onf.pack(blocks, F, H)
    B0 = torch.zeros(F, 2, dtype=F64)
    assert torch.equal(Onf.forward(q, B0, p, bf16=True), Onf.forward(q, B0, p))
    assert torch.allclose(Onf.forward(q, B0, p), torch.full((20,), 0.25 * H * 0.5 * F, dtype=F64))
