"""The allocation-free loss entry point against pact_loss_and_grad (the same kernels: bit-identical results),
called through the C ABI twice in a row, the second time with fewer patches."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import patches as Opatch

from gpu_common import OracleView, announce, dev32, devc64, f32, random_real_patches_spectra

pytestmark = pytest.mark.gpu


def _case(P, scan, N, seed):
    ov = OracleView(scan)
    rng = np.random.default_rng(seed)
    w = rng.normal(scale=0.05, size=(N, scan.n_elem)).astype(np.float32)
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng)
    return devc64(Opatch.half_spectrum(Y)), dev32(w), dev32(ov.centres[:N]), dev32(ov.delays)


def test_noalloc_matches_workspace_form():
    import paper_2409_10876_amd as P
    lib = P.pact.load()
    for scan, N, seed in ((synth.TINY, 49, 31), (synth.TINY.with_(P=24, stride=12), 20, 32)):
        announce(f"loss_and_grad_noalloc N={N} P={scan.P}")
        g = P.geometry_from(scan)
        Yh, w, c, d = _case(P, scan, N, seed)
        eps = f32(1e-3)
        loss_a, gw_a = P.pact.loss_and_grad(Yh, w, c, g, d, eps)
        loss_b = torch.full((1,), -1.0, device="cuda")
        gw_b = torch.full_like(gw_a, -1.0)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        st = lib.pact_loss_and_grad_noalloc(ctypes.c_void_p(Yh.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                            ctypes.c_void_p(c.data_ptr()), N, g.ring, ctypes.c_void_p(d.data_ptr()),
                                            scan.M, scan.P, g.px, eps, ctypes.c_void_p(loss_b.data_ptr()),
                                            ctypes.c_void_p(gw_b.data_ptr()), None, stream)
        assert st == 0, lib.pact_last_error()
        torch.cuda.synchronize()
        assert torch.equal(loss_a, loss_b) and torch.equal(gw_a, gw_b)


def test_noalloc_refuses_too_many_patches():
    import paper_2409_10876_amd as P
    lib = P.pact.load()
    g = P.geometry_from(synth.TINY)
    fake = ctypes.c_void_p(0x1000)
    st = lib.pact_loss_and_grad_noalloc(fake, fake, fake, 16385, g.ring, fake, 5, 32, g.px, 1e-3, fake, fake, None,
                                        None)
    assert st == -4 and b"16384" in lib.pact_last_error()
