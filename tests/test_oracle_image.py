"""The image figures of the reconstruction (Table 1, Supp. S1.4) discriminate when measured against a
band-limited reference.  On seeded small scans, entirely with the FP64 oracle: the aberration-free image (the
same blobs in a uniform medium, through the same DAS, windowed patch spectra, deconvolution and stitching) is
matched better by the deconvolution with the true SOS than by the deconvolution that assumes v0 everywhere, by
several dB and in SSIM; against the unfiltered synthetic initial pressure the two differ by a fraction of a dB
(which is why the bench reports both)."""
import numpy as np
import pytest
import torch

import synth
from synth.phantoms import SosPhantom
from oracle import das as Odas, patches as Opatch, rays as Orays, psf as Opsf, deconv as Odec, stitch as Ostitch
from oracle.geometry import patch_centres
from paper_2409_10876_amd import metrics

SCAN = synth.TINY


def _image(S, w, cen):
    st = Odas.das_stack(S, SCAN.fs, SCAN.t0, SCAN.n_elem, SCAN.radius, SCAN.phi0, SCAN.v0, np.asarray(SCAN.delays),
                        SCAN.ny, SCAN.nx, SCAN.px)
    Y = Opatch.patch_spectra(st, SCAN.P, SCAN.stride, SCAN.px, SCAN.fwhm)
    H = Opsf.transfer_functions(w, cen, SCAN.radius, SCAN.phi0, np.asarray(SCAN.delays), SCAN.P, SCAN.px)
    X = Odec.multichannel_deconv(Y, H, 1e-3)
    return Ostitch.stitch(Odec.patch_images(X), SCAN.ny, SCAN.nx, SCAN.P, SCAN.stride, SCAN.px, SCAN.fwhm)


def _scores(img, ref):
    a, b = metrics.normalise(img, ref)
    return metrics.psnr(a, b), metrics.ssim(a, b)


@pytest.mark.parametrize("seed", [1, 2])
def test_true_sos_deconvolution_beats_uniform_against_aberration_free_image(seed):
    rng = np.random.default_rng(seed)
    ph = synth.make_sos_phantom(SCAN, rng)
    blobs = synth.make_blobs(SCAN, rng)
    S = synth.channel_data(SCAN, ph, blobs, rng=rng)
    S_free = synth.channel_data(SCAN, SosPhantom("uniform", SCAN.v0, {}), blobs, rng=np.random.default_rng(seed))
    cen = patch_centres(SCAN.ny, SCAN.nx, SCAN.px, SCAN.P, SCAN.stride)
    mask = torch.tensor(synth.free_node_mask(SCAN)).bool()
    vt = torch.tensor(synth.sos_grid_truth(SCAN, ph))
    vt = torch.where(mask, vt, torch.full_like(vt, SCAN.v0))
    w = Orays.sos_to_delays(vt, SCAN.sos_spacing, SCAN.v0, cen, SCAN.n_elem, SCAN.radius, SCAN.phi0, SCAN.n_samples)
    ref = _image(S_free, torch.zeros_like(w), cen)
    p_true, s_true = _scores(_image(S, w, cen), ref)
    p_uni, s_uni = _scores(_image(S, torch.zeros_like(w), cen), ref)
    truth = torch.tensor(synth.render_ip(SCAN, blobs))
    pt_true, _ = _scores(_image(S, w, cen), truth)
    pt_uni, _ = _scores(_image(S, torch.zeros_like(w), cen), truth)
    print(f"seed {seed}: vs aberration-free {p_true:.2f} / {p_uni:.2f} dB, SSIM {s_true:.3f} / {s_uni:.3f}; "
          f"vs synthetic truth {pt_true:.2f} / {pt_uni:.2f} dB")
    assert p_true > p_uni + 1.5 and s_true > s_uni + 0.01
    assert abs(pt_true - pt_uni) < 1.0
