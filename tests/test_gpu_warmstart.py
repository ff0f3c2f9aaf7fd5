"""GPU parity of the learned warm start's kernels against the FP64 oracle of oracle/warmstart.py.

Bounds.  A BF16 result of an FP32 sum s of K products of BF16 values: with the FP64 reference ref and
S = sum |terms|, |s - ref| <= K 2^-24 S (FP32 accumulation) and the final rounding adds at most half a
BF16 unit, 2^-8 |s|; so |gpu - ref| <= 2^-8 |ref| + 1.01 K 2^-24 S.  FP32 results (weight gradients,
loss) are held to K_chain 2^-24 S with K_chain the length of the longest FP32 summation chain (bounded
here by the number of terms).  The whole network is compared by relative L2 error with tolerances derived
in the comments of those tests."""
import numpy as np
import pytest
import torch

from oracle import warmstart as Ow

from gpu_common import announce, rel_l2

pytestmark = pytest.mark.gpu

F64 = torch.float64
BF = torch.bfloat16
PAIRS = [(16, 64), (64, 64), (64, 16)]


@pytest.fixture(scope="module")
def lib():
    import paper_2409_10876_amd as P
    return P


def _bf(t):
    """A float tensor rounded to BF16 on the device."""
    return torch.as_tensor(t).to(torch.float32).to(BF).cuda().contiguous()


def _f64(t):
    return t.detach().float().cpu().to(F64)


def _check_bf16(got, ref, S, K, what):
    got, ref, S = _f64(got), ref.to(F64), S.to(F64)
    bound = 2.0 ** -8 * ref.abs() + 1.01 * K * 2.0 ** -24 * S + 1e-30
    err = (got - ref).abs()
    worst = float((err / bound).max())
    assert worst <= 1.0, f"{what}: error / bound = {worst:.3g}"


def _rand(shape, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return scale * torch.randn(*shape, generator=g, dtype=F64)


@pytest.mark.parametrize("ci,co", PAIRS)
@pytest.mark.parametrize("shape", [(2, 20, 28), (1, 9, 37), (3, 35, 35)], ids=lambda s: "x".join(map(str, s)))
def test_conv_forward(lib, ci, co, shape):
    n, H, W = shape
    announce(f"conv3x3 ci={ci} co={co} {shape}")
    x = _bf(_rand((n, H, W, ci), 1))
    Wt = _rand((co, 3, 3, ci), 2, 1.0 / np.sqrt(9 * ci)).to(torch.float32)
    b = _rand((co,), 3, 0.1).to(torch.float32)
    pk, _ = lib.pact.conv3x3_pack(Wt.cuda().contiguous(), ci, co)
    y = lib.pact.conv3x3(x, pk, co, bias=b.cuda(), relu=True)
    Wb = Wt.to(BF).to(F64)
    xr = _f64(x)
    ref = torch.relu(Ow.conv3x3(xr, Wb, b.to(F64)))
    S = Ow.conv3x3(xr.abs(), Wb.abs(), b.to(F64).abs())
    _check_bf16(y, ref, S, 9 * ci, "conv forward")
    # mask: zero wherever the mask tensor is <= 0
    m = _bf(_rand((n, H, W, co), 4))
    y2 = lib.pact.conv3x3(x, pk, co, bias=b.cuda(), relu=False, mask=m)
    ref2 = torch.where(_f64(m) > 0, Ow.conv3x3(xr, Wb, b.to(F64)), torch.zeros((), dtype=F64))
    _check_bf16(y2, ref2, S, 9 * ci, "conv forward, masked")


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv_input_gradient(lib, ci, co):
    n, H, W = 2, 20, 28
    announce(f"conv3x3 input gradient ci={ci} co={co}")
    Wt = _rand((co, 3, 3, ci), 5, 1.0 / np.sqrt(9 * ci)).to(torch.float32)
    _, adj = lib.pact.conv3x3_pack(Wt.cuda().contiguous(), ci, co)
    g = _bf(_rand((n, H, W, co), 6))
    mask = _bf(torch.relu(_rand((n, H, W, ci), 7)))
    dx = lib.pact.conv3x3(g, adj, ci, mask=mask)
    Wb = Wt.to(BF).to(F64)
    x0 = torch.zeros(n, H, W, ci, dtype=F64)
    ref, _, _ = Ow.conv_adjoints(x0, Wb, _f64(g))
    S, _, _ = Ow.conv_adjoints(x0, Wb.abs(), _f64(g).abs())
    ref = torch.where(_f64(mask) > 0, ref, torch.zeros((), dtype=F64))
    _check_bf16(dx, ref, S, 9 * co, "conv input gradient")


@pytest.mark.parametrize("ci,co", PAIRS)
@pytest.mark.parametrize("shape", [(2, 20, 28), (3, 35, 35)], ids=lambda s: "x".join(map(str, s)))
def test_conv_weight_gradient(lib, ci, co, shape):
    n, H, W = shape
    announce(f"conv3x3 weight gradient ci={ci} co={co} {shape}")
    x = _bf(_rand((n, H, W, ci), 8))
    g = _bf(_rand((n, H, W, co), 9))
    got = lib.pact.conv3x3_wgrad(x, g).cpu().to(F64)
    W0 = torch.zeros(co, 3, 3, ci, dtype=F64)
    _, dW, db = Ow.conv_adjoints(_f64(x), W0, _f64(g))
    _, SW, Sb = Ow.conv_adjoints(_f64(x).abs(), W0, _f64(g).abs())
    ref = torch.cat([dW.reshape(-1), db])
    S = torch.cat([SW.reshape(-1), Sb])
    K = n * H * W
    err = (got - ref).abs()
    worst = float((err / (K * 2.0 ** -24 * S + 1e-30)).max())
    assert worst <= 1.0, f"weight gradient: error / bound = {worst:.3g}"
    assert rel_l2(got, ref) < 1e-5


def test_resampling(lib):
    n, H, W, C = 2, 14, 10, 64
    announce("pool2 / up2_add / adjoints")
    a = _bf(_rand((n, H, W, C), 10))
    lo = _bf(_rand((n, H // 2, W // 2, C), 11))
    sk = _bf(_rand((n, H, W, C), 12))
    mh = _bf(_rand((n, H, W, C), 13))
    ml = _bf(_rand((n, H // 2, W // 2, C), 14))
    ar, lor, skr, mhr, mlr = (_f64(t) for t in (a, lo, sk, mh, ml))
    z = torch.zeros((), dtype=F64)
    _check_bf16(lib.pact.pool2(a), Ow.pool2(ar), Ow.pool2(ar.abs()), 4, "pool2")
    _check_bf16(lib.pact.up2_add(lo, sk), Ow.up2(lor) + skr, Ow.up2(lor.abs()) + skr.abs(), 2, "up2_add")
    ref = torch.where(mlr > 0, 4 * Ow.pool2(ar), z)
    _check_bf16(lib.pact.up2_add_adjoint(a, mask_low=ml), ref, 4 * Ow.pool2(ar.abs()), 4, "up2_add adjoint")
    _check_bf16(lib.pact.up2_add_adjoint(a), 4 * Ow.pool2(ar), 4 * Ow.pool2(ar.abs()), 4, "up2_add adjoint, no mask")
    ref = torch.where(mhr > 0, Ow.up2(lor) / 4 + skr, z)
    _check_bf16(lib.pact.pool2_adjoint(lo, skip=sk, mask=mh), ref, Ow.up2(lor.abs()) / 4 + skr.abs(), 2,
                "pool2 adjoint")
    _check_bf16(lib.pact.pool2_adjoint(lo), Ow.up2(lor) / 4, Ow.up2(lor.abs()) / 4, 1, "pool2 adjoint, no skip")


def test_input_loss_and_sos(lib):
    announce("warm input / loss / sos")
    M, H, W = 11, 56, 44
    st = _rand((M, H, W), 20).to(torch.float32)
    x = lib.pact.warm_input(st.cuda().contiguous(), 4, 0.37, 16)
    ref = Ow.prepare_input(st.to(F64), 4, float(np.float32(0.37)), 16)
    _check_bf16(x, ref, Ow.prepare_input(st.to(F64).abs(), 4, float(np.float32(0.37)), 16), 16, "input")
    n, h, w = 3, 14, 11
    z = _bf(_rand((n, h, w, 16), 21))
    t = _rand((n, h, w), 22).to(torch.float32)
    mask = (torch.rand(h, w, generator=torch.Generator().manual_seed(23)) > 0.3).to(torch.uint8)
    nf = int(mask.sum())
    norm = float(np.float32(1.0 / (n * nf)))
    loss, g = lib.pact.warm_loss(z, t.cuda().contiguous(), mask.cuda(), norm)
    zr = _f64(z)
    L_ref = Ow.loss(zr, t.to(F64), mask)
    assert abs(float(loss) - float(L_ref)) <= 1e-5 * float(L_ref)
    d = (zr[..., 0] - t.to(F64)) * mask.to(F64)
    gref = torch.zeros(n, h, w, 16, dtype=F64)
    gref[..., 0] = 2 * norm * d
    _check_bf16(g, gref, gref.abs(), 2, "loss gradient")
    sos = lib.pact.warm_sos(z, mask.cuda(), 1.5, Ow.OUT_SCALE).cpu().to(F64)
    sref = torch.where(mask.bool(), 1.5 + float(np.float32(Ow.OUT_SCALE)) * zr[..., 0], torch.full((), 1.5, dtype=F64))
    assert float((sos - sref).abs().max()) < 4e-7


def test_ricker_channels(lib):
    announce("ricker channels")
    import synth
    from oracle import geometry as OG
    scan = synth.TINY.with_(n_elem=64, phi0=0.2)
    g = lib.geometry_from(scan)
    rng = np.random.default_rng(30)
    nb = 300                                              # more sources than one staging pass (256)
    r = 10 * np.sqrt(rng.uniform(size=nb))
    a = rng.uniform(0, 2 * np.pi, nb)
    src = np.stack([r * np.cos(a), r * np.sin(a)], -1).astype(np.float32)
    amp = rng.uniform(0.2, 1.0, nb).astype(np.float32)
    sig = rng.uniform(0.3, 1.5, nb).astype(np.float32)
    w = rng.uniform(-0.3, 0.3, (nb, 64)).astype(np.float32)
    S = lib.pact.ricker_channels(torch.tensor(w).cuda(), torch.tensor(src).cuda(), torch.tensor(amp).cuda(),
                                 torch.tensor(sig).cuda(), g, 1.5, scan.n_t, scan.fs).cpu().to(F64)
    el = OG.ring_positions(64, scan.radius, float(np.float32(0.2)))
    T = Ow.arrival_times(torch.tensor(w, dtype=F64), torch.tensor(src, dtype=F64), el, 1.5)
    ref = Ow.ricker_channels(T, torch.tensor(amp, dtype=F64), torch.tensor(sig, dtype=F64), 1.5, scan.n_t, scan.fs)
    # FP32 arrival times near 70 us carry ~1e-5 us of rounding, times v0 / sigma <= 5 per us in u
    assert rel_l2(S, ref) < 3e-4
    assert float((S - ref).abs().max()) < 1e-3 * float(ref.abs().max())


def _net_case(lib, seed, n=2, H=20, W=28):
    Pw = lib.warmstart
    p = Pw.init_params(11, seed)
    # nonzero biases so that every bias path is exercised
    rng = np.random.default_rng(seed)
    for (ow, ob, ci, co) in Pw.LAYOUT[:-1]:
        p[ob:ob + co] = rng.uniform(-0.05, 0.05, co)
    p[Pw.LAYOUT[-1][1]] = 0.1
    x = np.zeros((n, H, W, 16), dtype=np.float32)
    x[..., :11] = rng.normal(size=(n, H, W, 11))
    t = rng.normal(size=(n, H, W)).astype(np.float32)
    mask = np.zeros((H, W), dtype=np.uint8)
    mask[2:-2, 3:-1] = 1
    return p, x, t, mask


def _oracle_params(lib, p):
    """The oracle's parameters: the weights as the BF16 values the kernels use, biases in FP32."""
    q = torch.tensor(p, dtype=F64)
    for (ow, ob, ci, co) in lib.warmstart.LAYOUT:
        q[ow:ob] = torch.tensor(p[ow:ob]).to(BF).to(F64)
    return q


def test_network_forward_and_gradient(lib):
    announce("warm-start network forward + backward (2 x 20 x 28)")
    p, x, t, mask = _net_case(lib, 1)
    net = lib.warmstart.WarmStartNet(2, 20, 28, params=p)
    xd = _bf(torch.tensor(x))
    n_free = int(mask.sum())
    loss = net.loss_grad(xd, torch.tensor(t).cuda(), torch.tensor(mask).cuda(), n_free)
    z = _f64(net.z[:2])
    q = _oracle_params(lib, p)
    xr = _f64(xd)
    # Forward: against the oracle with the same BF16 rounding points, the remaining differences are FP32
    # sums and rounding flips they cause (half a BF16 unit, 2^-9 relative, each), carried through eight
    # layers: a few 1e-3 of relative L2.  Against the unrounded FP64 network: the roundings themselves,
    # about 2^-9 per stored tensor over ~12 tensors, summed in quadrature.
    z_bf = Ow.forward(q, xr, bf16=True)
    z_64 = Ow.forward(q, xr, bf16=False)
    assert rel_l2(z[..., 0], z_bf[..., 0]) < 1e-2
    assert rel_l2(z[..., 0], z_64[..., 0]) < 2e-2
    assert torch.count_nonzero(z[..., 1:]) == 0          # unused output channels stay zero
    L_ref, g_ref = Ow.loss_and_grad(q, xr, torch.tensor(t, dtype=F64), torch.tensor(mask), bf16=True)
    assert abs(float(loss) - float(L_ref)) < 2e-2 * float(L_ref)
    # Gradient: the backward pass also rounds every pre-activation gradient to BF16 (2^-9 relative each,
    # about 14 tensors on the longest path) and the weight gradients sum ~10^3 products per pixel row;
    # per-layer relative L2 within 3e-2.
    got = net.grad.cpu().to(F64)
    for l, (ow, ob, ci, co) in enumerate(lib.warmstart.LAYOUT):
        e_w = rel_l2(got[ow:ob], g_ref[ow:ob])
        e_b = rel_l2(got[ob:ob + co], g_ref[ob:ob + co]) if l < 7 else abs(float(got[ob] - g_ref[ob])) / abs(float(g_ref[ob]))
        assert e_w < 3e-2 and e_b < 3e-2, (l, e_w, e_b)
    Wl = got[lib.warmstart.LAYOUT[-1][0]:lib.warmstart.LAYOUT[-1][1]].reshape(16, -1)
    assert torch.count_nonzero(Wl[1:]) == 0 and torch.count_nonzero(got[lib.warmstart.LAYOUT[-1][1] + 1:]) == 0


def test_network_full_size_sampled(lib):
    # the training shape (140 x 140 nodes, the bench's batch): one layer's output at sampled pixels
    # against scalar sums, and the determinism of the whole forward pass
    announce("warm-start network at 8 x 140 x 140, sampled")
    p, _, _, _ = _net_case(lib, 2, n=1, H=4, W=4)
    net = lib.warmstart.WarmStartNet(8, 140, 140, params=p)
    rng = np.random.default_rng(3)
    x = np.zeros((8, 140, 140, 16), dtype=np.float32)
    x[..., :11] = rng.normal(size=(8, 140, 140, 11))
    xd = _bf(torch.tensor(x))
    z1 = net.forward(xd).clone()
    z2 = net.forward(xd).clone()
    assert torch.equal(z1, z2)
    # layer 2 (64 -> 64) output a2 at sampled pixels from the device's own a1
    a1 = _f64(net.a1)
    a2 = _f64(net.a2)
    ow, ob, ci, co = lib.warmstart.LAYOUT[1]
    Wb = torch.tensor(p[ow:ob]).to(BF).to(F64).reshape(co, 3, 3, ci)
    b = torch.tensor(p[ob:ob + co], dtype=F64)
    for (n, r, c) in [(0, 0, 0), (7, 139, 139), (3, 70, 1), (5, 138, 77), (1, 64, 139)]:
        acc = b.clone()
        s = b.abs().clone()
        for ky in range(3):
            for kx in range(3):
                rr, cc = r + ky - 1, c + kx - 1
                if 0 <= rr < 140 and 0 <= cc < 140:
                    acc += Wb[:, ky, kx, :] @ a1[n, rr, cc]
                    s += Wb[:, ky, kx, :].abs() @ a1[n, rr, cc].abs()
        _check_bf16(a2[n, r, c], torch.relu(acc), s, 9 * ci, f"a2 at {(n, r, c)}")


def test_training_steps_reduce_the_loss(lib):
    announce("warm-start training steps")
    Pw = lib.warmstart
    rng = np.random.default_rng(4)
    n, H, W = 4, 28, 28
    x = np.zeros((n, H, W, 16), dtype=np.float32)
    x[..., :11] = rng.normal(size=(n, H, W, 11))
    # a target the network can fit: a smooth function of the input
    t = (0.5 * x[..., 0] - 0.25 * x[..., 3]).astype(np.float32)
    mask = np.ones((H, W), dtype=np.uint8)
    net = Pw.WarmStartNet(n, H, W, params=Pw.init_params(11, 0))
    xd, td, md = _bf(torch.tensor(x)), torch.tensor(t).cuda(), torch.tensor(mask).cuda()
    losses = [float(net.train_step(xd, td, md, H * W, 1e-3)) for _ in range(60)]
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_trained_network_gain(lib):
    # the committed trained initialiser on two held-out scans of the paper-shaped geometry: its SOS is much
    # closer to the truth than the uniform v0, and at least as close as 500 plain optimisation steps
    import os
    import synth
    from synth.warm import WARM, phantom_batch
    from paper_2409_10876_amd import train_warm_start as T, warmstart as W
    path = os.path.join(os.path.dirname(lib.__file__), "weights", "warm_start.safetensors")
    assert os.path.exists(path), "trained weights missing"
    announce("trained warm start on 2 held-out scans")
    params, scale, _ = W.load_params(path)
    scan = synth.PAPER
    sim = T.make_sim(scan, "cuda")
    net = W.WarmStartNet(1, scan.sos_n, scan.sos_n, params=params, n_inputs=scan.M)
    rows = []
    for i in (WARM.n_train, WARM.n_train + 1):
        sos, blobs = phantom_batch(scan, [i])
        rows.append(T.evaluate_scan(net, sim, scan, sos[0], blobs[0], scale))
    for r in rows:
        assert r["rmse_net"] < 0.6 * r["rmse_v0"], r
        assert r["t_warm_to_rmse_s"] is not None, r          # reaches the plain run's final SOS error
    assert np.mean([r["rmse_net"] for r in rows]) <= np.mean([r["rmse_plain"] for r in rows])
