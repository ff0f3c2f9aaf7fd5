"""End-to-end behaviour of the oracle on the tiny workload (Sec. 3.3): the loss prefers the true SOS, and
a few Adam steps from the background lower both the loss and the SOS error.  Which SOS the iteration
reaches is not unique (the loss sees the SOS only through path integrals), so nothing here compares
trajectories; only the direction of travel is checked."""
import numpy as np
import pytest
import torch

import synth
from oracle import das, patches, loss, psf, adam, sos
from oracle.geometry import F64, patch_centres, gaussian_window


def _geom(scan, centres, delays):
    return dict(sos_spacing=scan.sos_spacing, v0=scan.v0, centres=centres, n_elem=scan.n_elem,
                radius=scan.radius, phi0=scan.phi0, n_samples=scan.n_samples, delays=delays, px=scan.px,
                eps=scan.eps)


@pytest.mark.slow
def test_ray_synthesised_data_prefers_true_sos():
    scan = synth.TINY
    inp = synth.make_inputs(scan, seed=1)
    st = das.das_stack(inp.S, scan.fs, scan.t0, scan.n_elem, scan.radius, scan.phi0, scan.v0, inp.delays,
                       scan.ny, scan.nx, scan.px)
    Y = patches.patch_spectra(st, scan.P, scan.stride, scan.px, scan.fwhm)
    geom = _geom(scan, patch_centres(scan.ny, scan.nx, scan.px, scan.P, scan.stride), inp.delays)
    v0f = torch.full((scan.sos_n, scan.sos_n), scan.v0, dtype=F64)
    vt = sos.full_field(torch.tensor(inp.sos_true), inp.mask, scan.v0)
    L0 = loss.total_loss(v0f, Y, geom, inp.mask, 0.0).item()
    Lt = loss.total_loss(vt, Y, geom, inp.mask, 0.0).item()
    assert Lt < 0.8 * L0


@pytest.mark.slow
def test_adam_on_exact_model_data_lowers_loss_and_sos_error():
    scan = synth.TINY.with_(n_samples=64)
    inp = synth.make_inputs(scan, seed=2, with_channels=False)
    cen = patch_centres(scan.ny, scan.nx, scan.px, scan.P, scan.stride)
    geom = _geom(scan, cen, inp.delays)
    vt = sos.full_field(torch.tensor(inp.sos_true), inp.mask, scan.v0)
    from oracle import rays
    wt = rays.sos_to_delays(vt, scan.sos_spacing, scan.v0, cen, scan.n_elem, scan.radius, scan.phi0,
                            scan.n_samples)
    Ht = psf.transfer_functions(wt, cen, scan.radius, scan.phi0, inp.delays, scan.P, scan.px)
    x = patches.extract_patches(inp.ip_true[None], scan.P, scan.stride)[:, 0] * gaussian_window(scan.P, scan.px,
                                                                                                   scan.fwhm)
    Y = Ht * torch.fft.fft2(x)[:, None]
    opt = adam.Adam(torch.full_like(vt, scan.v0), inp.mask, lr=scan.lr)
    m = torch.tensor(inp.mask).bool()
    rmse = lambda p: torch.sqrt(((p - vt)[m] ** 2).mean()).item()
    losses, errs = [], [rmse(opt.p)]
    for _ in range(scan.steps):
        L, gv, _, _ = loss.loss_and_grad(opt.p, inp.mask, Y, geom, 0.0)    # data term only: its minimum is the truth
        losses.append(L.item())
        opt.step(gv)
        errs.append(rmse(opt.p))
    assert losses[-1] < 0.7 * losses[0]
    assert errs[-1] < errs[0]
    L_true = loss.total_loss(vt, Y, geom, inp.mask, 0.0).item()
    assert L_true < 1e-3 * losses[0]
