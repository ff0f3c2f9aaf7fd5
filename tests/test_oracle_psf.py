"""Pins of the wavefront-at-angle interpolation and the transfer function / PSF (Eq. TF)."""
import math

import numpy as np
import torch
from scipy.optimize import brentq

import synth
from oracle import psf, das, patches, deconv, rays
from oracle.geometry import F64, wavenumbers, ring_positions


def test_ring_index_matches_root_finding():
    rng = np.random.default_rng(2)
    R, N, phi0 = 30.0, 64, 0.2
    for _ in range(20):
        c = rng.uniform(-8, 8, 2)
        th = rng.uniform(-np.pi, np.pi)
        u = np.array([np.cos(th), np.sin(th)])
        tau = brentq(lambda t: np.hypot(*(c + t * u)) - R, 0.0, 2 * R)
        q = c + tau * u
        want = ((np.arctan2(q[1], q[0]) - phi0) % (2 * np.pi)) * N / (2 * np.pi)
        got = psf.ring_index(torch.tensor(c), torch.tensor(th, dtype=F64), R, phi0, N).item()
        assert abs(got - want) < 1e-9 or abs(abs(got - want) - N) < 1e-9


def test_wavefront_exact_at_elements_and_linear_between():
    R, N = 25.0, 32
    c = torch.tensor([1.3, -2.1], dtype=F64)
    ring = ring_positions(N, R)
    w = torch.tensor(np.random.default_rng(0).normal(size=N))
    th = torch.atan2(ring[:, 1] - c[1], ring[:, 0] - c[0])
    np.testing.assert_allclose(psf.wavefront_at(w, c, th, R, 0.0).numpy(), w.numpy(), atol=1e-12)
    # w linear in the element index inside one cell -> W linear in the fractional index
    w2 = torch.arange(N, dtype=F64) * 0.01
    t = torch.linspace(-3.0, -2.0, 11, dtype=F64)
    f = psf.ring_index(c, t, R, 0.0, N)
    ok = (torch.floor(f) < N - 1)
    np.testing.assert_allclose(psf.wavefront_at(w2, c, t, R, 0.0).numpy()[ok], (0.01 * f).numpy()[ok], atol=1e-12)


def _tf(w, centres, R, d, P, px):
    return psf.transfer_functions(torch.as_tensor(w, dtype=F64), centres, R, 0.0, d, P, px)


def test_uniform_sos_gives_real_even_centred_psf():
    """w = 0: H = cos(|k| d) -- real and even, so h is real, symmetric and centred (zero shift)."""
    P, px, R, N = 16, 0.1, 20.0, 64
    d = [-0.3, 0.0, 0.25]
    H = _tf(np.zeros((1, N)), torch.tensor([[0.4, -0.2]], dtype=F64), R, d, P, px)
    _, _, kabs, _ = wavenumbers(P, px)
    for j, dj in enumerate(d):
        np.testing.assert_allclose(H[0, j].real.numpy(), np.cos(kabs.numpy() * dj), atol=1e-14)
        np.testing.assert_allclose(H[0, j].imag.numpy(), 0.0, atol=1e-14)
        h = psf.psf(H[0, j]).numpy()
        np.testing.assert_allclose(h, np.roll(np.flip(h, (0, 1)), (1, 1), (0, 1)), atol=1e-14)   # h[-u] = h[u]
    h0 = psf.psf(H[0, 1]).numpy()
    assert abs(h0[0, 0] - 1.0) < 1e-12 and np.abs(h0).sum() - 1.0 < 1e-12       # d = 0: a delta


def test_constant_wavefront_most_compact_psf_at_matching_delay():
    """w = c for every direction: H = cos(|k|(d - c)); the delay closest to c gives the most compact PSF
    (Sec. 3.1: the most concentrated PSF marks the best delay at each location)."""
    P, px, R, N = 32, 0.1, 20.0, 64
    cval = 0.33
    d = np.linspace(-0.8, 0.8, 9)
    H = _tf(np.full((1, N), cval), torch.tensor([[0.0, 0.0]], dtype=F64), R, d, P, px)
    u = np.minimum(np.arange(P), P - np.arange(P)) * px
    r2 = u[:, None] ** 2 + u[None, :] ** 2
    spread = [(np.abs(psf.psf(H[0, j]).numpy()) * r2).sum() / np.abs(psf.psf(H[0, j]).numpy()).sum()
              for j in range(len(d))]
    assert int(np.argmin(spread)) == int(np.argmin(np.abs(d - cval)))


def test_first_order_wavefront_is_a_shift_to_plus_a():
    """W(theta) = a . u(theta): H = e^{-j k.a} at d = 0, a pure shift of the PSF to +a (reading of the
    sign convention; Supp. S2: first-order terms shift the PSF)."""
    P, px, R, N = 16, 0.1, 40.0, 2048
    c = torch.tensor([[0.7, 0.3]], dtype=F64)
    a = np.array([2 * px, 1 * px])                      # two pixels in x, one in y
    ring = ring_positions(N, R).numpy()
    th = np.arctan2(ring[:, 1] - 0.3, ring[:, 0] - 0.7)
    w = (a[0] * np.cos(th) + a[1] * np.sin(th))[None]
    H = _tf(w, c, R, [0.0], P, px)[0, 0]
    h = psf.psf(H).numpy()
    assert np.unravel_index(np.argmax(h), h.shape) == (1, 2)
    assert abs(h[1, 2] - 1.0) < 1e-3
    assert (np.abs(H.numpy()) <= 1 + 1e-12).all()


def test_transfer_function_magnitude_bounded():
    rng = np.random.default_rng(4)
    H = _tf(rng.normal(scale=0.3, size=(3, 40)), torch.tensor(rng.uniform(-2, 2, (3, 2))), 20.0,
            [-0.5, 0.1, 0.6], 12, 0.15)
    assert (torch.abs(H) <= 1 + 1e-12).all()


def test_sign_convention_against_das_of_a_point_source():
    """The A3 sign reading tied to Eq. DAS itself: a point source seen through a faster disc is shifted
    in the DAS stack; deconvolving with H built from the true SOS puts it back at its true position,
    while the printed (conjugated) expression would move it further away."""
    scan = synth.TINY.with_(phantom="disc")
    ph = synth.SosPhantom("disc", scan.v0, dict(cx=-4.0, cy=0.0, r=6.0, v1=1.65))
    xs, ys = 1.6, 0.0
    S = synth.point_source_data(scan, ph, xs, ys, sigma=0.15)
    P, px = 32, scan.px
    # one patch centred on the source's pixel neighbourhood
    n = P
    c0x = round(xs / px) * px + px / 2
    c0y = round(ys / px) * px + px / 2
    g = (np.arange(n) - (n - 1) / 2) * px
    X, Y = np.meshgrid(c0x + g, c0y + g)
    d = np.linspace(-0.8, 1.2, 11)
    st = das.das_points(S, scan.fs, scan.t0, scan.n_elem, scan.radius, scan.phi0, scan.v0, d, X, Y)
    Yk = torch.fft.fft2(torch.tensor(st)[None] * torch.tensor(
        np.exp(-(g[:, None] ** 2 + g[None, :] ** 2) / (2 * (1.2) ** 2))))
    v = torch.tensor(synth.sos_grid_truth(scan.with_(sos_n=64, sos_spacing=0.4), ph))
    cen = torch.tensor([[c0x, c0y]], dtype=F64)
    w = rays.sos_to_delays(v, 0.4, scan.v0, cen, scan.n_elem, scan.radius, scan.phi0, 512)
    H = psf.transfer_functions(w, cen, scan.radius, scan.phi0, d, P, px)
    for conj, expect_close in ((False, True), (True, False)):
        Hc = torch.conj(H) if conj else H
        x = deconv.patch_images(deconv.multichannel_deconv(Yk, Hc, 1e-2))[0].numpy()
        r, cidx = np.unravel_index(np.argmax(x), x.shape)
        err = math.hypot(X[r, cidx] - xs, Y[r, cidx] - ys)
        if expect_close:
            assert err <= 1.5 * px, err
        else:
            assert err > 2.5 * px, err
    # and the sharpest DAS image itself is shifted towards the fast disc (so the test has teeth):
    # the first-order wavefront term (w(0) - w(pi)) / 2 is about -0.5 mm here
    j = int(np.argmax(st.reshape(d.size, -1).max(1)))
    r, cidx = np.unravel_index(np.argmax(st[j]), X.shape)
    assert X[r, cidx] - xs < -1.5 * px
