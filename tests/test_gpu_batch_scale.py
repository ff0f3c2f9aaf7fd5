"""The batched workload at its real sizes (independent scans of 256^2 to 768^2 pixels, 256 to 1024 elements, 7 to
15 delays, 64^2 or 80^2 patches, SOS grids up to 188^2).  Three of its 32 seeded scans: the largest image (752^2,
484 patches, a 188^2 grid on the banded adjoint), 1024 elements with 15 delays (496^2), and a 144^2 grid that
takes two bands (576^2, 15 delays).  For each, one optimisation step at a random SOS is held to the oracle on
sampled patches, in the launch configuration of the batched solver (support disc, staged contrast, autotuned ray
tiling): the patch spectra from the channel data, the wavefront errors, dL/dw of the fused loss, and the ray
adjoint of those patches' dL/dw.  Then the three scans solved together (graphs on their own streams, or one
launch per stage over all three) reach, bit for bit, the states they reach alone."""
import numpy as np
import pytest
import torch

import synth
from oracle import das as Odas, patches as Opatch, rays as Orays, loss as Oloss

from gpu_common import (OracleView, TOL_DELAYS, TOL_GRAD, TOL_SPECTRA, announce, dev32, f32, rel_l2)

pytestmark = pytest.mark.gpu

ALL = synth.configs.batch_scans(32, seed=0)
PICKS = [31, 13, 4]


@pytest.fixture(scope="module")
def lib():
    import paper_2409_10876_amd as P
    return P


def _setup(P, k):
    scan = ALL[k]
    inp = synth.make_inputs(scan, seed=100 + k)
    sd = P.prepare_scan(scan, inp.S, np.asarray(scan.delays, dtype=np.float32))
    solver = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples,
                               support_radius=scan.mask_radius)
    return scan, inp, sd, solver


@pytest.mark.parametrize("k", PICKS, ids=lambda k: f"scan{k}")
def test_batch_scan_step_matches_oracle(lib, k):
    P = lib
    scan, inp, sd, solver = _setup(P, k)
    announce(f"batched workload scan {k}: {synth.describe(scan)}")
    ov = OracleView(scan)
    rng = np.random.default_rng(50 + k)
    free = np.asarray(inp.mask, bool)
    v = np.asarray(synth.random_sos((scan.sos_n, scan.sos_n), scan.v0, rng, amp=0.03, smooth=4), dtype=np.float32)
    v = np.where(free, v, np.float32(scan.v0)).astype(np.float32)
    solver.autotune()
    solver.set_sos(torch.tensor(v))
    solver.delays()
    solver.loss_grad()
    torch.cuda.synchronize()
    N = scan.n_patches
    npx = scan.n_patch_x
    pats = sorted({0, N - 1, N // 2, int(rng.integers(0, N))})
    idx = torch.tensor(pats)

    # patch spectra of one patch from the channel data: the oracle's delay-and-sum over its pixels
    i = pats[2]
    a, b = divmod(i, npx)
    rows = (np.arange(a * scan.stride, a * scan.stride + scan.P) - (scan.ny - 1) / 2.0) * ov.px
    cols = (np.arange(b * scan.stride, b * scan.stride + scan.P) - (scan.nx - 1) / 2.0) * ov.px
    X, Yg = np.meshgrid(cols, rows)
    sub = Odas.das_points(inp.S, ov.fs, ov.t0, scan.n_elem, ov.R, ov.phi0, ov.v0, ov.delays, X, Yg)
    want_y = Opatch.half_spectrum(Opatch.patch_spectra(sub, scan.P, scan.stride, ov.px, ov.fwhm)[0])
    ey = rel_l2(sd.Y[i].cpu(), want_y)

    # wavefront errors of the sampled patches (all elements)
    w_want = Orays.sos_to_delays(torch.tensor(v, dtype=torch.float64), ov.ds, ov.v0, ov.centres[idx], scan.n_elem,
                                 ov.R, ov.phi0, scan.n_samples)
    ew = rel_l2(solver.w.cpu()[idx], w_want)

    # dL/dw of the sampled patches from the GPU's spectra (each patch's share of Eq. jr alone)
    Yh = sd.Y.cpu()[idx].to(torch.complex128)
    full = torch.fft.fft2(torch.fft.irfft2(Yh, s=(scan.P, scan.P)))          # the real patches' full spectra
    wl = solver.w.cpu()[idx].double().requires_grad_(True)
    L = Oloss.loss_from_delays(wl, full, ov.centres[idx], ov.R, ov.phi0, ov.delays, ov.px, f32(scan.eps))
    (gw_want,) = torch.autograd.grad(L, wl)
    eg = rel_l2(solver.gw.cpu()[idx], gw_want)

    # the ray adjoint of those patches' dL/dw, on the free nodes
    gw = torch.zeros_like(solver.gw)
    gw[idx.cuda()] = solver.gw[idx.cuda()]
    got_a = P.pact.sos_to_delays_adjoint(solver.sos, sd.geom, scan.v0, sd.centres, scan.n_samples, gw,
                                         support=scan.mask_radius, staged=solver._staged[solver._cur])
    fn = lambda vv: Orays.sos_to_delays(vv, ov.ds, ov.v0, ov.centres[idx], scan.n_elem, ov.R, ov.phi0,  # noqa: E731
                                        scan.n_samples)
    (a_want,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), gw.cpu()[idx].double())
    torch.cuda.synchronize()
    fr = torch.tensor(free)
    ea = rel_l2(got_a.cpu()[fr], a_want[fr])
    print(f"scan {k}: Y rel L2 {ey:.2e}, w {ew:.2e}, dL/dw {eg:.2e}, adjoint {ea:.2e} (patches {pats})")
    assert ey < 10 * TOL_SPECTRA          # DAS and transform errors compound, as in the small workload's test
    assert ew < TOL_DELAYS and eg < TOL_GRAD and ea < TOL_GRAD


@pytest.mark.parametrize("form", ["streams", "grouped", "grouped_2",
                                  pytest.param("persistent", marks=pytest.mark.skip(
                                      reason="the persistent step is switched off: an earlier form did not finish on the GPU and the rewritten kernel is untested there"))])
def test_batch_of_real_size_scans_matches_solo(lib, form):
    """The three scans solved together (their step graphs on their own streams, one launch per stage over all
    three, one per stage over each of two groups on their own streams, or one persistent launch per step) reach
    the states they reach alone, bit for bit."""
    P = lib
    announce(f"batched workload: three real-size scans together ({form}) vs alone")
    solvers = [_setup(P, k)[3] for k in PICKS]
    if form == "streams":
        batch = P.BatchedSolver(solvers, graph_steps=2, autotune=True)
    else:
        batch = P.GroupedBatchSolver(solvers, graph_steps=2, autotune=True, groups=2 if form == "grouped_2" else 1,
                                     persistent=form == "persistent")
        assert len(batch.groups) == (2 if form == "grouped_2" else 1)
    solo = [_setup(P, k)[3] for k in PICKS]
    for s in solo:
        s.step()                                  # the batch ran one eager step before capturing
    batch.run(4)
    torch.cuda.synchronize()
    for s in solo:
        s.run(4)
    torch.cuda.synchronize()
    for a, b in zip(batch.solvers, solo):
        assert a.t.tolist() == b.t.tolist() == [5, 0]
        assert torch.equal(a.sos, b.sos) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
