"""Pins of the learned warm start's oracle (oracle/warmstart.py): the convolution against scalar sums and
shifted identities, the resolution schedule and skips in closed form, reverse mode against central
differences, adjoint identities, the input average, and the channel model against the independent
synthetic-data generator."""
import numpy as np
import torch

import synth
from oracle import warmstart as Ow

F64 = torch.float64


def _rand(*shape, seed=0):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(*shape, generator=g, dtype=F64)


def test_parameter_count():
    # 16 -> 64, six 64 -> 64, 64 -> 16 (3 x 3 weights and biases)
    assert Ow.n_params() == (64 * 9 * 16 + 64) + 6 * (64 * 9 * 64 + 64) + (16 * 9 * 64 + 16)


def test_conv_against_scalar_sums():
    x, W, b = _rand(2, 5, 7, 3, seed=1), _rand(4, 3, 3, 3, seed=2), _rand(4, seed=3)
    y = Ow.conv3x3(x, W, b)
    for (n, r, c, o) in [(0, 0, 0, 0), (1, 4, 6, 3), (0, 2, 3, 1), (1, 0, 5, 2), (0, 4, 0, 3)]:
        s = float(b[o])
        for ky in range(3):
            for kx in range(3):
                rr, cc = r + ky - 1, c + kx - 1
                if 0 <= rr < 5 and 0 <= cc < 7:
                    for i in range(3):
                        s += float(W[o, ky, kx, i] * x[n, rr, cc, i])
        assert abs(float(y[n, r, c, o]) - s) < 1e-12
    assert torch.allclose(y, Ow.conv3x3_loops(x, W, b), atol=1e-12)


def test_conv_shifted_identity():
    # a single tap (ky, kx) = identity moves the image by (ky - 1, kx - 1) with zeros shifted in
    x = _rand(1, 6, 5, 2, seed=4)
    for ky in range(3):
        for kx in range(3):
            W = torch.zeros(2, 3, 3, 2, dtype=F64)
            W[:, ky, kx, :] = torch.eye(2, dtype=F64)
            y = Ow.conv3x3(x, W, None)
            ref = torch.zeros_like(x)
            dy, dx = ky - 1, kx - 1
            for r in range(6):
                for c in range(5):
                    if 0 <= r + dy < 6 and 0 <= c + dx < 5:
                        ref[0, r, c] = x[0, r + dy, c + dx]
            assert torch.equal(y, ref)


def test_pool_and_up():
    a = _rand(1, 4, 6, 3, seed=5)
    p = Ow.pool2(a)
    assert p.shape == (1, 2, 3, 3)
    assert torch.allclose(p[0, 1, 2], a[0, 2:4, 4:6].mean(dim=(0, 1)))
    u = Ow.up2(p)
    assert u.shape == a.shape and torch.equal(u[0, 3, 5], p[0, 1, 2]) and torch.equal(u[0, 2, 4], p[0, 1, 2])
    assert torch.allclose(Ow.pool2(Ow.up2(p)), p)


def _zero_net():
    return {name: torch.zeros(shape, dtype=F64) for name, shape in Ow.layout()}


def _pack(blocks):
    return torch.cat([blocks[name].reshape(-1) for name, _ in Ow.layout()])


def test_constant_maps_closed_form():
    # with W1..W7 = 0 every hidden map is relu(b_l); the skips give u5 = relu(b5) + relu(b4) and
    # u6 = relu(b6) + relu(b2); z = conv8 of the constant relu(b7) with zero padding
    blocks = _zero_net()
    for l in range(1, 9):
        blocks[f"b{l}"] = _rand(blocks[f"b{l}"].numel(), seed=10 + l)
    blocks["W8"] = _rand(16, 3, 3, 64, seed=30)
    x = _rand(1, 8, 12, 16, seed=31)
    z, act = Ow.forward(_pack(blocks), x, keep=True)
    r = {l: torch.relu(blocks[f"b{l}"]) for l in range(1, 8)}
    assert torch.allclose(act["u5"], (r[5] + r[4]).expand_as(act["u5"]))
    assert torch.allclose(act["u6"], (r[6] + r[2]).expand_as(act["u6"]))
    assert torch.allclose(act["p4"], r[4].expand_as(act["p4"]))
    per_tap = torch.einsum("okti,i->okt", blocks["W8"], r[7])          # [16][3][3]
    interior = blocks["b8"] + per_tap.sum(dim=(1, 2))
    corner = blocks["b8"] + per_tap[:, 1:, 1:].sum(dim=(1, 2))            # top-left pixel: taps ky, kx >= 1
    edge = blocks["b8"] + per_tap[:, 1:, :].sum(dim=(1, 2))               # top row, interior column
    assert torch.allclose(z[0, 3, 5], interior)
    assert torch.allclose(z[0, 0, 0], corner)
    assert torch.allclose(z[0, 0, 5], edge)


def test_skip_path_reaches_the_output():
    # layer 6 switched off (a6 = 0) and layer 7 the centre-tap identity: a7 = u6 = a2, so z = c8(a2)
    blocks = _zero_net()
    for k, name in enumerate(("W1", "W2", "b1", "b2", "W8", "b8")):
        blocks[name] = _rand(*blocks[name].shape, seed=100 + k)
    blocks["W7"][:, 1, 1, :] = torch.eye(64, dtype=F64)
    x = _rand(2, 8, 8, 16, seed=40)
    z, act = Ow.forward(_pack(blocks), x, keep=True)
    assert torch.equal(act["a6"], torch.zeros_like(act["a6"]))
    assert torch.allclose(act["a7"], act["a2"])
    assert torch.allclose(z, Ow.conv3x3(act["a2"], blocks["W8"], blocks["b8"]))


def test_positive_homogeneity_without_biases():
    # relu, averaging, doubling, skips and bias-free convolutions are positively homogeneous
    blocks = _zero_net()
    for l in range(1, 9):
        blocks[f"W{l}"] = 0.1 * _rand(*blocks[f"W{l}"].shape, seed=50 + l)
    p = _pack(blocks)
    x = _rand(1, 8, 8, 16, seed=60)
    assert torch.allclose(Ow.forward(p, 2.5 * x), 2.5 * Ow.forward(p, x), rtol=1e-12, atol=1e-12)


def _small_problem(seed=0):
    g = torch.Generator().manual_seed(seed)
    # He-scaled weights keep the activations O(1) through the eight layers
    p = torch.cat([(np.sqrt(2.0 / (9 * s[3])) if len(s) == 4 else 0.1) *
                   torch.randn(int(np.prod(s)), generator=g, dtype=F64) for _, s in Ow.layout()])
    x = torch.randn(2, 8, 8, 16, generator=g, dtype=F64)
    t = torch.randn(2, 8, 8, generator=g, dtype=F64)
    mask = torch.zeros(8, 8, dtype=torch.uint8)
    mask[1:7, 2:8] = 1
    return p, x, t, mask


def test_gradient_against_central_differences():
    p, x, t, mask = _small_problem()
    L, g = Ow.loss_and_grad(p, x, t, mask)
    rng = np.random.default_rng(0)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in Ow.layout()])
    # one coordinate in every weight and bias block (the unused output rows of W8 / b8 excluded)
    idx = []
    for k, (name, shape) in enumerate(Ow.layout()):
        n = int(np.prod(shape))
        if name in ("W8", "b8"):
            n = n // 16
        idx.append(int(offs[k] + rng.integers(n)))
    # a ReLU kink within +-h of a pre-activation would spoil a difference; at h = 1e-6 none is hit here
    h = 1e-6
    for i in idx:
        e = torch.zeros_like(p)
        e[i] = h
        fd = (Ow.loss(Ow.forward(p + e, x), t, mask) - Ow.loss(Ow.forward(p - e, x), t, mask)) / (2 * h)
        assert abs(float(fd) - float(g[i])) <= 1e-6 * (abs(float(fd)) + 1e-3), (i, float(fd), float(g[i]))


def test_unused_output_channels_get_zero_gradient():
    p, x, t, mask = _small_problem(1)
    _, g = Ow.loss_and_grad(p, x, t, mask)
    blk = dict(zip([n for n, _ in Ow.layout()], torch.split(g, [int(np.prod(s)) for _, s in Ow.layout()])))
    assert torch.count_nonzero(blk["W8"].reshape(16, -1)[1:]) == 0
    assert torch.count_nonzero(blk["b8"][1:]) == 0


def test_conv_adjoint_identities():
    x, W, g = _rand(2, 6, 5, 4, seed=70), _rand(3, 3, 3, 4, seed=71), _rand(2, 6, 5, 3, seed=72)
    dx, dW, db = Ow.conv_adjoints(x, W, g)
    y = Ow.conv3x3(x, W, None)
    inner = float((y * g).sum())
    assert abs(inner - float((x * dx).sum())) < 1e-9 * abs(inner)
    assert abs(inner - float((W * dW).sum())) < 1e-9 * abs(inner)
    assert torch.allclose(db, g.sum(dim=(0, 1, 2)))


def test_prepare_input():
    st = _rand(3, 8, 12, seed=80)
    x = Ow.prepare_input(st, 4, 2.0, 16)
    assert x.shape == (2, 3, 16)
    assert abs(float(x[1, 2, 1]) - 2.0 * float(st[1, 4:8, 8:12].mean())) < 1e-12
    assert torch.count_nonzero(x[..., 3:]) == 0
    c = Ow.prepare_input(torch.full((2, 8, 8), 0.7, dtype=F64), 4, 1.0, 8)
    assert torch.allclose(c[..., :2], torch.full((2, 2, 2), 0.7, dtype=F64))


def test_channel_model_against_the_synthetic_generator():
    # uniform SOS: w = 0, T = |r_n - c_b| / v0, and the trace must equal the independent generator's
    scan = synth.TINY.with_(n_elem=16, n_t=1024, phantom="uniform")
    ph = synth.make_sos_phantom(scan, np.random.default_rng(0))
    rng = np.random.default_rng(1)
    blobs = synth.Blobs(cx=rng.uniform(-5, 5, 4), cy=rng.uniform(-5, 5, 4), sigma=rng.uniform(0.3, 1.5, 4),
                        amp=rng.uniform(0.2, 1.0, 4))
    S_ref = synth.channel_data(scan, ph, blobs).astype(np.float64)
    phi = 2 * np.pi * np.arange(16) / 16
    el = torch.tensor(np.stack([50.0 * np.cos(phi), 50.0 * np.sin(phi)], -1))
    src = torch.tensor(np.stack([blobs.cx, blobs.cy], -1))
    T = Ow.arrival_times(torch.zeros(4, 16, dtype=F64), src, el, scan.v0)
    assert torch.allclose(T, torch.linalg.norm(el[None] - src[:, None], dim=-1) / 1.5)
    S = Ow.ricker_channels(T, torch.tensor(blobs.amp), torch.tensor(blobs.sigma), scan.v0, scan.n_t, scan.fs)
    assert float((S - torch.tensor(S_ref)).abs().max()) < 1e-6 * float(torch.tensor(S_ref).abs().max())


def test_arrival_time_uses_the_wavefront_error():
    # Eq. TOF through Eq. wf: a ray with w = 0.3 mm of "1 - v0 / v" arrives 0.3 / v0 us early
    src = torch.tensor([[1.0, 2.0]], dtype=F64)
    el = torch.tensor([[40.0, 0.0], [0.0, -40.0]], dtype=F64)
    T0 = Ow.arrival_times(torch.zeros(1, 2, dtype=F64), src, el, 1.5)
    T1 = Ow.arrival_times(torch.full((1, 2), 0.3, dtype=F64), src, el, 1.5)
    assert torch.allclose(T0 - T1, torch.full((1, 2), 0.2, dtype=F64))
