"""Pins of the oracle's gradient: central finite differences on tiny problems, stage by stage and end to
end, and the Adam step against torch.optim.Adam."""
import numpy as np
import torch

from oracle import loss, rays, psf, deconv, sos, adam, stitch
from oracle.geometry import F64, patch_centres, gaussian_window


def _tiny_problem(seed=0, G=7, n_elem=12, P=8, M=3, lam=0.0):
    rng = np.random.default_rng(seed)
    ds, v0, R, px = 0.5, 1.5, 8.0, 0.25
    ny = nx = 16
    cent = patch_centres(ny, nx, px, P, 8)                       # 4 patches
    Y = torch.tensor(rng.normal(size=(4, M, P, P)) + 1j * rng.normal(size=(4, M, P, P)))
    geom = dict(sos_spacing=ds, v0=v0, centres=cent, n_elem=n_elem, radius=R, phi0=0.1, n_samples=48,
                delays=np.linspace(-0.6, 0.6, M), px=px, eps=1e-3)
    v = torch.tensor(v0 + 0.05 * rng.uniform(-1, 1, (G, G)))
    mask = np.ones((G, G), dtype=bool)
    mask[0, :] = False
    return v, mask, Y, geom, lam


def test_end_to_end_gradient_matches_central_differences():
    v, mask, Y, geom, lam = _tiny_problem(lam=0.3)
    v = sos.full_field(v, mask, geom["v0"])          # fixed nodes at the background, as the solver keeps them
    L, gv, gw, w = loss.loss_and_grad(v, mask, Y, geom, lam)
    np.testing.assert_allclose(L.item(), loss.total_loss(v, Y, geom, mask, lam).item(), rtol=1e-13)
    f = lambda vv: loss.total_loss(vv, Y, geom, mask, lam).item()
    rng = np.random.default_rng(1)
    idx = [tuple(rng.integers(0, 7, 2)) for _ in range(10)] + [(3, 3), (0, 2)]
    for (a, b) in idx:
        h = 1e-6 * v[a, b].item()
        vp = v.clone(); vp[a, b] += h
        vm = v.clone(); vm[a, b] -= h
        fd = (f(vp) - f(vm)) / (2 * h)
        assert abs(fd - gv[a, b].item()) <= 1e-6 * gv.abs().max().item(), (a, b, fd, gv[a, b].item())


def test_gradient_wrt_wavefront_matches_central_differences():
    v, mask, Y, geom, _ = _tiny_problem(seed=2)
    w = rays.sos_to_delays(v, geom["sos_spacing"], geom["v0"], geom["centres"], geom["n_elem"], geom["radius"],
                           geom["phi0"], geom["n_samples"])
    w = w + 0.2 * torch.tensor(np.random.default_rng(3).normal(size=w.shape))
    fn = lambda ww: loss.loss_from_delays(ww, Y, geom["centres"], geom["radius"], geom["phi0"], geom["delays"],
                                          geom["px"], geom["eps"])
    (g,) = loss.vjp(fn, (w,), torch.tensor(1.0, dtype=F64))
    rng = np.random.default_rng(4)
    for _ in range(12):
        i, n = int(rng.integers(0, 4)), int(rng.integers(0, geom["n_elem"]))
        h = 1e-7
        wp = w.clone(); wp[i, n] += h
        wm = w.clone(); wm[i, n] -= h
        fd = (fn(wp) - fn(wm)).item() / (2 * h)
        assert abs(fd - g[i, n].item()) <= 1e-6 * g.abs().max().item()


def test_ray_adjoint_dot_product():
    """<J dv, g> = <dv, J^T g> for the ray stage, J dv by central differences (the stage is linear in
    1/v, so the directional derivative is exact to O(h^2))."""
    v, mask, Y, geom, _ = _tiny_problem(seed=5)
    fn = lambda vv: rays.sos_to_delays(vv, geom["sos_spacing"], geom["v0"], geom["centres"], geom["n_elem"],
                                       geom["radius"], geom["phi0"], geom["n_samples"])
    rng = np.random.default_rng(6)
    g = torch.tensor(rng.normal(size=(4, geom["n_elem"])))
    dv = torch.tensor(rng.normal(size=v.shape))
    (jt,) = loss.vjp(fn, (v,), g)
    h = 1e-6
    jd = (fn(v + h * dv) - fn(v - h * dv)) / (2 * h)
    np.testing.assert_allclose((jd * g).sum().item(), (jt * dv).sum().item(), rtol=1e-8)


def test_tv_gradient_away_from_kinks():
    rng = np.random.default_rng(8)
    v = torch.tensor(rng.normal(size=(5, 5)))
    m = rng.uniform(size=(5, 5)) < 0.5
    (g,) = loss.vjp(lambda vv: loss.tv(vv, m), (v,), torch.tensor(1.0, dtype=F64))
    for a in range(5):
        for b in range(5):
            h = 1e-7
            vp = v.clone(); vp[a, b] += h
            vm = v.clone(); vm[a, b] -= h
            fd = (loss.tv(vp, m) - loss.tv(vm, m)).item() / (2 * h)
            assert abs(fd - g[a, b].item()) < 1e-6


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(9)
    p0 = torch.tensor(rng.normal(size=(4, 5)))
    mask = rng.uniform(size=(4, 5)) < 0.7
    ours = adam.Adam(p0, mask, lr=0.05)
    ref = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=0.05)
    for _ in range(6):
        g = torch.tensor(rng.normal(size=(4, 5)))
        ours.step(g)
        opt.zero_grad()
        ref.grad = torch.where(torch.tensor(mask), g, torch.zeros_like(g))
        opt.step()
    np.testing.assert_allclose(ours.p.numpy(), ref.detach().numpy(), rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(ours.p.numpy()[~mask], p0.numpy()[~mask])


def test_stitching_partition_of_unity():
    """Stitching the windowed (not deconvolved) patches of an image gives the image back wherever the
    summed window weight is positive (Supp. S1.4)."""
    rng = np.random.default_rng(10)
    ny, nx, P, s, px, fwhm = 40, 48, 16, 8, 0.1, 0.7
    img = torch.tensor(rng.normal(size=(ny, nx)))
    g = gaussian_window(P, px, fwhm)
    npx = (nx - P) // s + 1
    npy = (ny - P) // s + 1
    pts = torch.stack([img[a * s:a * s + P, b * s:b * s + P] * g for a in range(npy) for b in range(npx)])
    out = stitch.stitch(pts, ny, nx, P, s, px, fwhm)
    np.testing.assert_allclose(out.numpy(), img.numpy(), rtol=1e-12, atol=1e-12)
