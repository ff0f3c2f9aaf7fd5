"""Pins of the SOS field (bilinear pixel grid) and the ray wavefront (Eq. TOF, Eq. wf)."""
import math

import numpy as np
import pytest
import torch
from scipy.integrate import quad
from scipy.interpolate import RegularGridInterpolator

from oracle import rays, sos
from oracle.geometry import F64


def _padded_interpolator(v, spacing, v0):
    """scipy's linear grid interpolator on the node grid with a ring of v0 nodes around it."""
    Gy, Gx = v.shape
    vp = np.full((Gy + 2, Gx + 2), v0)
    vp[1:-1, 1:-1] = v
    ya = (np.arange(-1, Gy + 1) - (Gy - 1) / 2) * spacing
    xa = (np.arange(-1, Gx + 1) - (Gx - 1) / 2) * spacing
    f = RegularGridInterpolator((ya, xa), vp, method="linear", bounds_error=False, fill_value=v0)
    return lambda x, y: f(np.stack([np.broadcast_to(y, np.broadcast(x, y).shape),
                                    np.broadcast_to(x, np.broadcast(x, y).shape)], -1))


def test_bilinear_matches_scipy_and_background():
    rng = np.random.default_rng(1)
    v = 1.5 + 0.05 * rng.normal(size=(7, 9))
    sp, v0 = 0.6, 1.5
    f = _padded_interpolator(v, sp, v0)
    x = rng.uniform(-4, 4, 500)
    y = rng.uniform(-3.5, 3.5, 500)
    got = sos.field(torch.tensor(v), sp, v0, torch.tensor(x), torch.tensor(y)).numpy()
    np.testing.assert_allclose(got, f(x, y), rtol=1e-14, atol=1e-14)
    far = sos.field(torch.tensor(v), sp, v0, torch.tensor([10.0, -3.0]), torch.tensor([0.0, 9.0])).numpy()
    np.testing.assert_array_equal(far, [v0, v0])


def test_uniform_background_gives_zero_wavefront():
    v = torch.full((8, 8), 1.5, dtype=F64)
    c = torch.tensor([[0.3, -0.2], [1.0, 1.0]], dtype=F64)
    w = rays.sos_to_delays(v, 0.5, 1.5, c, 16, 30.0, 0.0, 32)
    assert torch.all(w == 0)


def test_axis_ray_through_uniform_grid_closed_form():
    """v = v1 on every node, v0 outside: along +x from the grid centre the field is v1 up to the last
    node centre and linear from v1 to v0 over the one-node padding band, so
    w = L_in (1 - v0/v1) + ds (1 - v0 ln(v0/v1) / (v0 - v1))."""
    G, ds, v0, v1 = 9, 0.5, 1.5, 1.6
    v = torch.full((G, G), v1, dtype=F64)
    c = torch.tensor([[0.0, 0.0]], dtype=F64)           # centre node (G odd)
    L_in = (G - 1) / 2 * ds
    exact = L_in * (1 - v0 / v1) + ds * (1 - v0 * math.log(v0 / v1) / (v0 - v1))
    errs = []
    # Ns a multiple of 5 puts the kink at the last node centre (x = 0.8 L) on a step boundary,
    # so that the error falls by 4 per halving of the step
    for Ns in (80, 160, 320):
        w = rays.sos_to_delays(v, ds, v0, c, 4, 40.0, 0.0, Ns)   # element 0 at (40, 0): ray along +x
        errs.append(abs(w[0, 0].item() - exact))
        # element 1 at (0, 40): the +y ray sees the same profile by symmetry
        assert abs(w[0, 1].item() - w[0, 0].item()) < 1e-13
    assert errs[-1] < 5e-6 * abs(exact)
    assert 3.0 < errs[0] / errs[1] < 5.0                  # midpoint rule: O(step^2)


def test_piecewise_linear_profile_along_row():
    """Nodes on the ray's row carry an arbitrary profile; the bilinear field along the row is piecewise
    linear between node centres (and the v0 padding node), so the exact integral is a sum of
    closed-form segment integrals  h (1 - v0 ln(vb/va) / (vb - va))."""
    rng = np.random.default_rng(5)
    G, ds, v0 = 11, 0.4, 1.5
    v = np.full((G, G), v0) + 0.08 * rng.uniform(-1, 1, (G, G))
    row = (G - 1) // 2
    start_col = 3
    cx = (start_col - (G - 1) / 2) * ds
    # exact: from x = cx (a node centre) through nodes start_col .. G-1 then to the padding node at v0
    prof = list(v[row, start_col:]) + [v0]
    exact = 0.0
    for va, vb in zip(prof[:-1], prof[1:]):
        exact += ds * (1 - v0 / va) if abs(vb - va) < 1e-15 else ds * (1 - v0 * math.log(vb / va) / (vb - va))
    w = rays.sos_to_delays(torch.tensor(v), ds, v0, torch.tensor([[cx, 0.0]]), 4, 25.0, 0.0, 8192)
    assert abs(w[0, 0].item() - exact) < 1e-7


def test_oblique_rays_converge_to_quadrature_of_scipy_field():
    """Generic directions: the midpoint sums converge (O(step^2)) to an adaptive quadrature of
    (1 - v0 / v) along the full segment to the element, v from scipy's interpolator.  This also pins
    the clipping reading: the integrand vanishes outside the SOS box."""
    rng = np.random.default_rng(7)
    G, ds, v0, R, ne = 10, 0.5, 1.5, 12.0, 7
    v = v0 + 0.06 * rng.uniform(-1, 1, (G, G))
    f = _padded_interpolator(v, ds, v0)
    c = np.array([[0.37, -0.81], [-1.6, 1.1]])
    ring = R * np.stack([np.cos(2 * np.pi * np.arange(ne) / ne), np.sin(2 * np.pi * np.arange(ne) / ne)], -1)
    ws = {Ns: rays.sos_to_delays(torch.tensor(v), ds, v0, torch.tensor(c), ne, R, 0.0, Ns).numpy()
          for Ns in (200, 400, 3200)}
    e1 = e2 = 0.0
    for i in range(2):
        for n in range(ne):
            d = ring[n] - c[i]
            dist = np.hypot(*d)
            u = d / dist
            g = lambda t: 1.0 - v0 / f(c[i, 0] + t * u[0], c[i, 1] + t * u[1])
            exact = quad(lambda t: float(g(t)), 0.0, dist, limit=400, epsabs=1e-13, epsrel=1e-12, points=np.linspace(0, 4, 40))[0]
            e1 += abs(ws[200][i, n] - exact)
            e2 += abs(ws[400][i, n] - exact)
            assert abs(ws[3200][i, n] - exact) < 2e-5 * max(abs(exact), 1e-3)
    assert e2 < 0.4 * e1


def test_wavefront_equals_path_difference_definition():
    """Eq. wf, first line: w = |r' - r| - v0 t with t the slowness integral to the element."""
    rng = np.random.default_rng(11)
    G, ds, v0, R, ne = 8, 0.5, 1.5, 9.0, 5
    v = v0 + 0.05 * rng.uniform(-1, 1, (G, G))
    f = _padded_interpolator(v, ds, v0)
    c = np.array([[0.2, 0.4]])
    w = rays.sos_to_delays(torch.tensor(v), ds, v0, torch.tensor(c), ne, R, 0.0, 4096).numpy()
    for n in range(ne):
        e = R * np.array([np.cos(2 * np.pi * n / ne), np.sin(2 * np.pi * n / ne)])
        d = e - c[0]
        dist = np.hypot(*d)
        u = d / dist
        t = quad(lambda s: float(1.0 / f(c[0, 0] + s * u[0], c[0, 1] + s * u[1])), 0, dist, limit=400,
                 epsabs=1e-14, epsrel=1e-13, points=np.linspace(0, 3, 30))[0]
        assert abs(w[0, n] - (dist - v0 * t)) < 1e-6


def test_exit_distance_box_edges():
    hx, hy = 2.0, 1.0
    px_ = torch.tensor([0.0, 0.5, 0.0], dtype=F64)
    py_ = torch.tensor([0.0, 0.0, 0.0], dtype=F64)
    ux = torch.tensor([1.0, -1.0, 1 / math.sqrt(2)], dtype=F64)
    uy = torch.tensor([0.0, 0.0, 1 / math.sqrt(2)], dtype=F64)
    L = rays.exit_distance(px_, py_, ux, uy, hx, hy).numpy()
    np.testing.assert_allclose(L, [2.0, 2.5, math.sqrt(2)], rtol=1e-12)
