"""Pins of the paper's neural-field oracle (oracle/siren.py): the paper's parameter count, closed forms of
the sinusoidal network, the fixed background, and reverse mode against central differences."""
import math

import numpy as np
import torch

from oracle import siren as Os
from oracle.loss import vjp

F64 = torch.float64


def test_parameter_count_is_the_papers():
    # one hidden layer of 256 sinusoidal features, 2 -> 256 -> 1 plus the output scale and offset
    assert Os.n_params(256) == 1027


def test_node_coordinates():
    xy = Os.node_coordinates(5, 4, 0.5, 2.0)
    assert xy.shape == (5, 4, 2)
    assert torch.allclose(xy[2, :, 1], torch.zeros(4, dtype=F64))            # middle row y = 0
    assert torch.allclose(xy[:, 0, 0], torch.full((5,), -0.75 / 2.0, dtype=F64))   # x of column 0: -1.5 * 0.5 / 2
    assert torch.allclose(xy[0, 0, 1], torch.tensor(-1.0 / 2.0, dtype=F64))        # y of row 0: -2 * 0.5 / 2


def _mask(G):
    m = np.zeros((G, G), dtype=np.uint8)
    m[1:-1, 2:-1] = 1
    return m


def test_constant_features_closed_form():
    G, H = 7, 16
    rng = np.random.default_rng(0)
    blocks = {"W1": torch.zeros(H, 2, dtype=F64), "b1": torch.tensor(rng.normal(size=H)),
              "w2": torch.tensor(rng.normal(size=H)), "b2": torch.tensor([0.3], dtype=F64),
              "s": torch.tensor([0.05], dtype=F64), "o": torch.tensor([-0.01], dtype=F64)}
    p = torch.cat([blocks[n].reshape(-1) for n, _ in Os.layout(H)])
    v = Os.sos_grid(p, G, G, 0.4, 1.2, _mask(G), 1.5)
    f = (torch.sin(30.0 * blocks["b1"]) * blocks["w2"]).sum() + 0.3
    want = torch.full((G, G), 1.5, dtype=F64)
    want[torch.tensor(_mask(G)).bool()] = 1.5 + 0.05 * f - 0.01
    assert torch.allclose(v, want, atol=1e-14)


def test_single_feature_is_a_sinusoid_in_x():
    G, H = 9, 4
    blocks = {"W1": torch.zeros(H, 2, dtype=F64), "b1": torch.zeros(H, dtype=F64), "w2": torch.zeros(H, dtype=F64),
              "b2": torch.zeros(1, dtype=F64), "s": torch.ones(1, dtype=F64), "o": torch.zeros(1, dtype=F64)}
    blocks["W1"][1, 0] = 0.07
    blocks["w2"][1] = 2.0
    p = torch.cat([blocks[n].reshape(-1) for n, _ in Os.layout(H)])
    m = np.ones((G, G), dtype=np.uint8)
    v = Os.sos_grid(p, G, G, 0.5, 2.0, m, 1.5)
    x = (torch.arange(G, dtype=F64) - (G - 1) / 2) * 0.5 / 2.0
    want = 1.5 + 2.0 * torch.sin(30.0 * 0.07 * x)
    assert torch.allclose(v, want[None, :].expand(G, G), atol=1e-14)       # varies along x only


def test_reverse_mode_matches_central_differences():
    G, H = 6, 8
    rng = np.random.default_rng(1)
    p = torch.tensor(rng.normal(scale=0.3, size=Os.n_params(H)))
    m = _mask(G)
    gv = torch.tensor(rng.normal(size=(G, G)))
    (got,) = vjp(lambda q: Os.sos_grid(q, G, G, 0.4, 1.0, m, 1.5), (p,), gv)
    L = lambda q: (Os.sos_grid(q, G, G, 0.4, 1.0, m, 1.5) * gv).sum()
    for i in range(p.numel()):
        e = torch.zeros_like(p)
        e[i] = 1e-6
        fd = (L(p + e) - L(p - e)) / 2e-6
        assert abs(fd.item() - got[i].item()) <= 1e-6 * (1 + abs(fd.item())), i
