"""GPU parity of the neural-field path (MFMA kernels) against the FP64 oracle of oracle/nf.py.

The workload runs the network's dense layers with BF16 operands and FP32 accumulation.  Every value
rounded to BF16 (the features, each hidden activation, each pre-activation gradient) moves by up to half
a BF16 step, 2^-9 relative (u = 3.9e-3 is the step 2^-8).  Two comparisons:

* against the oracle with the same BF16 rounding points: the logic of the kernels (point order, layer
  order, transposes, biases, ReLU masks, ray sums).  What remains is the FP32-vs-FP64 difference in the
  values being rounded, which flips a share of the rounding decisions, each by one BF16 step; at the
  workload's 2 cycles/mm the phases reach ~80 cycles, so FP32 positions alone change w by ~7e-4.  Bound:
  about one BF16 step, TOL_NF_W = 5e-3 on delays, and TOL_NF_GRAD = 1.5e-2 on parameter gradients,
  whose two or three extra rounding stages (delta_l) add in quadrature.
* against the plain FP64 network (no rounding): the BF16 error of the workload itself, stated (printed)
  and bounded by five rounding stages in quadrature, sqrt(5) u ~ 9e-3: TOL_NF_W_FP64 = 1e-2; gradients
  3e-2.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nf as Onf
from oracle.geometry import ring_positions

from gpu_common import RAGGED, OracleView, announce, dev32, f32, rel_l2

pytestmark = pytest.mark.gpu

TOL_NF_W = 5e-3
TOL_NF_GRAD = 1.5e-2
TOL_NF_W_FP64 = 1e-2
TOL_NF_GRAD_FP64 = 3e-2

F64 = torch.float64


@pytest.fixture(scope="module")
def lib():
    import paper_2409_10876_amd as P
    return P


def _oracle_params(params32: np.ndarray, cfg) -> torch.Tensor:
    """The parameters the kernels use: weights rounded to bfloat16, biases as given."""
    p = torch.tensor(params32, dtype=F64)
    blocks = Onf.unpack(p, cfg.n_freq, cfg.width)
    for name in ("W1", "W2", "W3", "W4", "w5"):
        blocks[name] = Onf.round_bf16(blocks[name])
    return Onf.pack(blocks, cfg.n_freq, cfg.width)


class NfCase:
    def __init__(self, lib, scan, n_samples, rho, seed, freq_scale=1.0):
        cfg = synth.nf.NF
        self.cfg, self.scan, self.n_samples = cfg, scan, n_samples
        self.ov = OracleView(scan)
        self.B32 = (synth.nf.frequencies(cfg, seed) * np.float32(freq_scale)).astype(np.float32)
        self.params32 = synth.nf.init_params(cfg, seed, head_scale=1.0)
        self.net = lib.pact.NfNet(cfg.n_freq, cfg.width, cfg.amp, rho)
        self.g = lib.geometry_from(scan)
        self.rho, self.amp, self.v0 = f32(rho), f32(cfg.amp), self.ov.v0
        self.B = dev32(self.B32)
        self.params = dev32(self.params32)
        self.packed = lib.pact.nf_pack(self.params, self.net)
        self.centres = dev32(self.ov.centres.numpy())
        self.ring = ring_positions(scan.n_elem, self.ov.R, self.ov.phi0)
        self.oparams = _oracle_params(self.params32, cfg)
        self.oB = torch.tensor(self.B32, dtype=F64)

    def oracle_w(self, centres, ring, bf16):
        return Onf.sos_to_delays(self.oparams, self.oB, centres, ring, self.rho, self.v0, self.amp, self.n_samples,
                                 bf16=bf16)

    def oracle_vjp(self, centres, ring, gw, bf16):
        return Onf.sos_to_delays_vjp(self.oparams, self.oB, centres, ring, self.rho, self.v0, self.amp,
                                     self.n_samples, gw, bf16=bf16)


SMALL = RAGGED.with_(name="nf-small", n_elem=64)


def test_nf_pack_is_round_to_nearest_even(lib):
    announce("nf_pack")
    cfg = synth.nf.NF
    p32 = synth.nf.init_params(cfg, 3)
    p32[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0e38]     # ties and a large value
    net = lib.pact.NfNet()
    packed = lib.pact.nf_pack(dev32(p32), net).cpu()
    b = Onf.unpack(torch.tensor(p32, dtype=torch.float32), cfg.n_freq, cfg.width)
    want = torch.cat([b["W1"].reshape(-1), b["W2"].reshape(-1), b["W3"].reshape(-1), b["W4"].reshape(-1),
                      b["W2"].T.reshape(-1), b["W3"].T.reshape(-1), b["W4"].T.reshape(-1), b["w5"]]).to(torch.bfloat16)
    assert torch.equal(packed.view(torch.int16), want.view(torch.int16))


@pytest.mark.parametrize("n_samples", [40, 64])
def test_nf_sos_to_delays(lib, n_samples):
    announce(f"nf_sos_to_delays small N_s={n_samples}")
    c = NfCase(lib, SMALL, n_samples, rho=9.0, seed=1)
    got = lib.pact.nf_sos_to_delays(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, n_samples)
    torch.cuda.synchronize()
    want = c.oracle_w(c.ov.centres, c.ring, bf16=True)
    plain = c.oracle_w(c.ov.centres, c.ring, bf16=False)
    e, e64 = rel_l2(got, want), rel_l2(got, plain)
    print(f"nf delays rel L2: vs BF16-rounding oracle {e:.2e}, vs FP64 network {e64:.2e}")
    assert ((got.cpu() == 0) & (want == 0)).any() and (want != 0).any()     # some rays miss the disc
    assert e < TOL_NF_W
    assert e64 < TOL_NF_W_FP64


def test_nf_adjoint(lib):
    announce("nf_sos_to_delays_adjoint small")
    c = NfCase(lib, SMALL, 40, rho=9.0, seed=2)
    rng = np.random.default_rng(5)
    gw = rng.normal(size=(c.ov.centres.shape[0], SMALL.n_elem)).astype(np.float32)
    gw[rng.random(gw.shape) < 0.3] = 0.0                      # skipped rays
    got = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, c.n_samples,
                                           dev32(gw))
    two = torch.full((1,), 2.0, device="cuda")
    got2 = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, c.n_samples,
                                            dev32(gw), scale=two)
    torch.cuda.synchronize()
    gwt = torch.tensor(gw, dtype=F64)
    want = c.oracle_vjp(c.ov.centres, c.ring, gwt, bf16=True)
    plain = c.oracle_vjp(c.ov.centres, c.ring, gwt, bf16=False)
    e, e64 = rel_l2(got, want), rel_l2(got, plain)
    blocks_got = Onf.unpack(got.cpu().to(F64))
    blocks_want = Onf.unpack(want)
    per = {k: rel_l2(blocks_got[k], blocks_want[k]) for k in blocks_want}
    print(f"nf adjoint rel L2: vs BF16-rounding oracle {e:.2e}, vs FP64 network {e64:.2e}; per block " +
          ", ".join(f"{k} {v:.1e}" for k, v in per.items()))
    assert e < TOL_NF_GRAD
    assert max(per.values()) < 3 * TOL_NF_GRAD
    assert e64 < TOL_NF_GRAD_FP64
    assert rel_l2(got2, 2.0 * got) < 1e-6


@pytest.mark.parametrize("n_samples", [40, 64])
def test_nf_stored_activations_match_recompute(lib, n_samples):
    """The forward pass with activation storage gives the same delays, and the two-pass adjoint from the
    stored activations the same gradient as the four-pass recomputing adjoint (same operations on the
    same BF16 values)."""
    announce(f"nf stored activations N_s={n_samples}")
    c = NfCase(lib, SMALL, n_samples, rho=9.0, seed=9)
    N = c.ov.centres.shape[0]
    act = torch.empty(lib.pact.nf_activation_bytes(N, c.g, n_samples), dtype=torch.uint8, device="cuda")
    w0 = lib.pact.nf_sos_to_delays(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, n_samples)
    w1 = lib.pact.nf_sos_to_delays(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, n_samples, act=act)
    rng = np.random.default_rng(10)
    gw = dev32(rng.normal(size=(N, SMALL.n_elem)).astype(np.float32))
    g0 = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, n_samples, gw)
    g1 = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, n_samples, gw,
                                          act=act)
    torch.cuda.synchronize()
    print(f"stored vs recompute: delays equal {torch.equal(w0, w1)}, gradient rel L2 {rel_l2(g1, g0):.2e}")
    assert torch.equal(w0, w1)
    assert rel_l2(g1, g0) < 1e-6
    want = c.oracle_vjp(c.ov.centres, c.ring, gw.cpu().double(), bf16=True)
    assert rel_l2(g1, want) < TOL_NF_GRAD


def test_nf_adjoint_smooth_features(lib):
    """Low frequencies (0.05 cycles/mm): smooth features, little cancellation in the weight-gradient sums and
    few flipped roundings, so the kernels' backward logic is held to the delay bound."""
    announce("nf_sos_to_delays_adjoint smooth features")
    c = NfCase(lib, SMALL, 40, rho=9.0, seed=6, freq_scale=0.025)
    rng = np.random.default_rng(8)
    gw = rng.normal(size=(c.ov.centres.shape[0], SMALL.n_elem)).astype(np.float32)
    got = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, c.n_samples,
                                           dev32(gw))
    w = lib.pact.nf_sos_to_delays(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, c.n_samples)
    torch.cuda.synchronize()
    want = c.oracle_vjp(c.ov.centres, c.ring, torch.tensor(gw, dtype=F64), bf16=True)
    e = rel_l2(got, want)
    ew = rel_l2(w, c.oracle_w(c.ov.centres, c.ring, bf16=True))
    per = {k: rel_l2(v, Onf.unpack(want)[k]) for k, v in Onf.unpack(got.cpu().to(F64)).items()}
    print(f"nf smooth: delays rel L2 {ew:.2e}, adjoint rel L2 {e:.2e}; per block " +
          ", ".join(f"{k} {v:.1e}" for k, v in per.items()))
    assert ew < TOL_NF_W and e < TOL_NF_W and max(per.values()) < TOL_NF_GRAD


def test_nf_paper_scale_sampled_rays(lib):
    """The launch configuration of the neural-field workload (169 patches x 512 elements x 256 samples):
    all delays from one launch, checked on sampled rays; the adjoint with dL/dw nonzero on 64 rays (8 patches x 8
    elements, some of them missing the disc), against the oracle's backward over those rays."""
    announce("nf paper scale, sampled rays")
    scan = synth.PAPER
    c = NfCase(lib, scan, scan.n_samples, rho=scan.mask_radius, seed=3)
    got = lib.pact.nf_sos_to_delays(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, scan.n_samples)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    flat = rng.choice(scan.n_patches * scan.n_elem, 24, replace=False)
    rays = [(int(f) // scan.n_elem, int(f) % scan.n_elem) for f in flat]
    want = torch.stack([c.oracle_w(c.ov.centres[i:i + 1], c.ring[n:n + 1], bf16=True)[0, 0] for i, n in rays])
    sel = torch.stack([got[i, n].cpu() for i, n in rays]).to(F64)
    e = rel_l2(sel, want)
    print(f"nf paper-scale sampled delays rel L2 {e:.2e}")
    assert e < TOL_NF_W
    # adjoint: dL/dw nonzero on 64 rays, 8 patches x 8 elements, two of the patches in the corners (their centres
    # lie outside the disc, so some of their rays miss it: w = 0 and no gradient)
    pats = [0, scan.n_patches - 1] + [int(x) for x in rng.choice(np.arange(1, scan.n_patches - 1), 6, replace=False)]
    els = sorted(int(x) for x in (rng.integers(0, scan.n_elem // 8) + np.arange(8) * (scan.n_elem // 8)))
    cen = c.ov.centres.numpy()[pats]
    ring = c.ring.numpy()[els]
    misses = 0
    for a in range(len(pats)):
        for b in range(len(els)):
            d = ring[b] - cen[a]
            u = d / np.linalg.norm(d)
            t = float(cen[a] @ u)
            disc = t * t - (float(cen[a] @ cen[a]) - float(c.rho) ** 2)
            clear_miss = disc < -1e-3 or (-t + np.sqrt(max(disc, 0.0))) < -1e-3     # no tangent cases
            if clear_miss:
                misses += 1
                assert got[pats[a], els[b]].item() == 0.0, "a ray that misses the disc has w = 0"
    print(f"nf paper-scale adjoint: {len(pats) * len(els)} rays, {misses} miss the disc")
    assert misses >= 2
    # positive weights: with random signs the 64 ray gradients cancel to 3 % of the sum of their norms, and any
    # rounding difference is then measured against that small remainder
    gsel = torch.tensor(np.abs(rng.normal(size=(len(pats), len(els)))) + 0.1, dtype=F64)
    gw = torch.zeros(scan.n_patches, scan.n_elem, dtype=torch.float32)
    gw[np.ix_(pats, els)] = gsel.to(torch.float32)
    vjp = c.oracle_vjp(c.ov.centres[pats], c.ring[els], gw[np.ix_(pats, els)].to(F64), bf16=True)
    got_g = lib.pact.nf_sos_to_delays_adjoint(c.B, c.params, c.packed, c.net, c.v0, c.centres, c.g, scan.n_samples,
                                             gw.cuda())
    torch.cuda.synchronize()
    e = rel_l2(got_g, vjp)
    print(f"nf paper-scale sampled adjoint (64 rays) rel L2 {e:.2e}")
    assert e < TOL_NF_GRAD


def test_nf_step_gradient_matches_oracle_chain(lib):
    """One neural-field optimisation step's gradient (delays through the network -> fused deconvolution loss
    and dL/dw -> network adjoint) against the oracle's chain on the same spectra: loss of Eq. jr from the
    oracle's delays, dL/dw by reverse mode, then the network backward."""
    from oracle import loss as Oloss, patches as Opatch
    from gpu_common import devc64, random_real_patches_spectra
    announce("nf step gradient, small")
    c = NfCase(lib, SMALL, 40, rho=9.0, seed=4)
    N = c.ov.centres.shape[0]
    rng = np.random.default_rng(15)
    Y = random_real_patches_spectra(N, SMALL.M, SMALL.P, rng).to(torch.complex64).to(torch.complex128)
    eps = f32(1e-3)
    w_o = c.oracle_w(c.ov.centres, c.ring, bf16=True).requires_grad_(True)
    L = Oloss.loss_from_delays(w_o, Y, c.ov.centres, c.ov.R, c.ov.phi0, c.ov.delays, c.ov.px, eps)
    (gw_o,) = torch.autograd.grad(L, w_o)
    want = c.oracle_vjp(c.ov.centres, c.ring, gw_o, bf16=True)

    sd = lib.ScanData(c.g, torch.zeros(1, device="cuda"), dev32(c.ov.delays), 1.0, 0.0, c.v0)
    sd.use_spectra(devc64(Opatch.half_spectrum(Y)))
    solver = lib.NeuralFieldSolver(sd, c.B32, c.params32, c.net, lr=1e-3, eps=eps, n_samples=40)
    solver.pack()
    solver.delays()
    solver.loss_grad()
    solver.adjoint()
    torch.cuda.synchronize()
    el = abs(solver.loss.item() - L.item()) / L.item()
    eg = rel_l2(solver.grad, want)
    print(f"nf step: loss rel {el:.2e}, dL/dparams rel L2 {eg:.2e}")
    assert el < 1e-4 and eg < TOL_NF_GRAD
    # the Adam step moves every parameter against its gradient's sign
    p0 = solver.params.clone()
    solver.update()
    torch.cuda.synchronize()
    moved = (solver.params - p0).cpu()
    gsign = torch.sign(solver.grad.cpu())
    assert torch.all((moved * gsign)[gsign != 0] < 0)
