"""Pins of the multichannel deconvolution (Eq. multi-deconv), the loss (Eq. jr) and TV."""
import math

import numpy as np
import torch

from oracle import deconv, loss, psf
from oracle.geometry import F64, wavenumbers


def _rand_H(rng, N, M, P, R=20.0, n_elem=48, px=0.1):
    w = torch.tensor(rng.normal(scale=0.4, size=(N, n_elem)))
    c = torch.tensor(rng.uniform(-2, 2, (N, 2)))
    d = np.linspace(-0.8, 0.8, M)
    return psf.transfer_functions(w, c, R, 0.0, d, P, px), w, c, d


def _crand(rng, shape):
    return torch.tensor(rng.normal(size=shape) + 1j * rng.normal(size=shape))


def test_noiseless_model_data_recovered_exactly():
    """Y_j = H_j X  =>  X_hat = X D / (D + eps); eps = 0 gives X back ("exact recovery with the true PSF")."""
    rng = np.random.default_rng(0)
    H, *_ = _rand_H(rng, 3, 5, 12)
    X = _crand(rng, (3, 12, 12))
    Y = H * X[:, None]
    D = (torch.abs(H) ** 2).sum(1)
    for eps in (0.0, 1e-3):
        Xh = deconv.multichannel_deconv(Y, H, eps)
        ok = D > 1e-3
        np.testing.assert_allclose(Xh[ok].numpy(), (X * D / (D + eps))[ok].numpy(), rtol=1e-12)


def test_single_channel_is_tikhonov_division():
    rng = np.random.default_rng(1)
    H, *_ = _rand_H(rng, 2, 1, 10)
    Y = _crand(rng, (2, 1, 10, 10))
    a = deconv.multichannel_deconv(Y, H, 0.05)
    b = deconv.single_channel_deconv(Y[:, 0], H[:, 0], 0.05)
    np.testing.assert_allclose(a.numpy(), b.numpy(), rtol=1e-13)


def test_least_squares_optimality():
    """With eps = 0 the pseudo-inverse is the least-squares solution: the residual is orthogonal to H
    (sum_j conj(H_j) r_j = 0) -- the conjugate-transpose reading of H^T."""
    rng = np.random.default_rng(2)
    H, *_ = _rand_H(rng, 2, 4, 8)
    Y = _crand(rng, (2, 4, 8, 8))
    X = deconv.multichannel_deconv(Y, H, 0.0)
    r = Y - H * X[:, None]
    D = (torch.abs(H) ** 2).sum(1)
    ok = D > 1e-3
    np.testing.assert_allclose((torch.conj(H) * r).sum(1)[ok].abs().numpy(), 0.0, atol=1e-10)


def test_loss_zero_at_truth_and_nonnegative():
    rng = np.random.default_rng(3)
    H, w, c, d = _rand_H(rng, 2, 4, 10)
    X = _crand(rng, (2, 10, 10))
    Y = H * X[:, None]
    L0 = loss.loss_from_delays(w, Y, c, 20.0, 0.0, d, 0.1, 0.0)
    assert abs(L0.item()) < 1e-18 * (torch.abs(Y) ** 2).sum().item() + 1e-20
    Y2 = Y + 0.1 * _crand(rng, Y.shape)
    assert loss.loss_from_delays(w, Y2, c, 20.0, 0.0, d, 0.1, 1e-6).item() > 0


def test_closed_form_of_the_residual():
    """Per bin, with H_j = e^{j psi} c_j (c_j real), N = sum c_j Y_j and D = sum c_j^2:
    sum_j |Y_j - H_j X_hat|^2 = sum |Y_j|^2 - |N|^2 (D + 2 eps) / (D + eps)^2 -- independent algebra."""
    rng = np.random.default_rng(4)
    N_, M, P, eps = 2, 5, 8, 1e-2
    H, w, c, d = _rand_H(rng, N_, M, P)
    Y = _crand(rng, (N_, M, P, P))
    _, _, kabs, _ = wavenumbers(P, 0.1)
    L = loss.loss_from_delays(w, Y, c, 20.0, 0.0, d, 0.1, eps).item()
    # split H into a common phase and real amplitudes: c_j = Re(H_j e^{-j psi}) with psi from channel 0
    ph = torch.angle(H[:, :1])
    cj = (H * torch.exp(-1j * ph)).real
    # (the imaginary remainder must vanish: every channel shares the phase)
    assert torch.abs((H * torch.exp(-1j * ph)).imag).max() < 1e-12
    Nn = (cj * Y).sum(1)
    D = (cj ** 2).sum(1)
    per_bin = (torch.abs(Y) ** 2).sum(1) - torch.abs(Nn) ** 2 * (D + 2 * eps) / (D + eps) ** 2
    np.testing.assert_allclose(L, (kabs * per_bin).sum().item(), rtol=1e-11)


def test_loss_invariant_to_common_phase():
    rng = np.random.default_rng(5)
    H, *_ = _rand_H(rng, 2, 3, 8)
    Y = _crand(rng, (2, 3, 8, 8))
    phase = torch.exp(1j * torch.tensor(rng.uniform(-3, 3, (2, 1, 8, 8))))
    L1 = loss.data_loss(Y, H, deconv.multichannel_deconv(Y, H, 1e-3), 0.1)
    H2 = H * phase
    L2 = loss.data_loss(Y, H2, deconv.multichannel_deconv(Y, H2, 1e-3), 0.1)
    np.testing.assert_allclose(L1.item(), L2.item(), rtol=1e-12)


def test_single_channel_degeneracy():
    """M = 1, eps = 0: a single channel is always fit exactly, so L = 0 whatever the SOS (the reason the
    method needs several delays, Sec. 3.2)."""
    rng = np.random.default_rng(6)
    H, w, c, d = _rand_H(rng, 2, 1, 8)
    Y = _crand(rng, (2, 1, 8, 8))
    L = loss.loss_from_delays(w, Y, c, 20.0, 0.0, d, 0.1, 0.0).item()
    assert abs(L) < 1e-20 * (torch.abs(Y) ** 2).sum().item() + 1e-12


def test_tv_brute_force():
    rng = np.random.default_rng(7)
    v = rng.normal(size=(5, 6))
    m = rng.uniform(size=(5, 6)) < 0.4
    want = 0.0
    for a in range(5):
        for b in range(6):
            if a + 1 < 5 and (m[a, b] or m[a + 1, b]):
                want += abs(v[a + 1, b] - v[a, b])
            if b + 1 < 6 and (m[a, b] or m[a, b + 1]):
                want += abs(v[a, b + 1] - v[a, b])
    np.testing.assert_allclose(loss.tv(torch.tensor(v), m).item(), want, rtol=1e-14)
