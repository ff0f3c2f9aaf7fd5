"""GPU parity: every libpact entry point against the FP64 oracle on the same seeded inputs.

Sizes: the tiny workload (128^2 image, 256 elements, 49 patches of 32^2, M = 5) and a ragged one
(100 x 90 image, 200 elements, 42 patches of 24^2, M = 7, 23^2 SOS grid, 100 samples per ray), so that
every kernel sees several tiles and a partial last tile.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import das as Odas, patches as Opatch, rays as Orays, psf as Opsf, deconv as Odec, loss as Oloss
from oracle import adam as Oadam, sos as Osos

from gpu_common import (FINEGRID, RAGGED, OracleView, TOL_DAS, TOL_DECONV, TOL_DELAYS, TOL_GRAD, TOL_LOSS, TOL_PSF,
                        TOL_SPECTRA, announce, dev32, devc64, f32, rel_l2, random_real_patches_spectra)

pytestmark = pytest.mark.gpu

WORKLOADS = [synth.TINY, RAGGED]


@pytest.fixture(scope="module")
def lib():
    import paper_2409_10876_amd as P
    return P


def _geom(P, scan):
    return P.geometry_from(scan)


# coarse pixels (0.5 mm): a 16 x 16 tile's distances to one element span about 280 samples
DAS_CASES = WORKLOADS + [RAGGED.with_(name="ragged_coarse", ny=90, nx=80, px=0.5)]


@pytest.mark.parametrize("scan", DAS_CASES, ids=lambda s: s.name)
def test_das_stack(lib, scan):
    announce(f"das_stack {scan.name}")
    inp = synth.make_inputs(scan, seed=1)
    ov = OracleView(scan)
    want = Odas.das_stack(inp.S, ov.fs, ov.t0, scan.n_elem, ov.R, ov.phi0, ov.v0, ov.delays, scan.ny, scan.nx, ov.px)
    got = lib.pact.das_stack(dev32(inp.S), scan.fs, scan.t0, _geom(lib, scan), scan.v0, dev32(ov.delays))
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print(f"das_stack rel L2 {err:.2e}")
    assert err < TOL_DAS


# patch sides for the transform paths: 32 = 4 4 2 and 24 = 4 2 3 (FFT), 45 = 3 3 5 (FFT, odd), 28 = 4 7 (DFT)
PATCH_CASES = WORKLOADS + [
    RAGGED.with_(name="ragged_p45", P=45, stride=22, fwhm=synth.configs.fwhm_for_patch(45, 0.25)),
    RAGGED.with_(name="ragged_p28", P=28, stride=14, fwhm=synth.configs.fwhm_for_patch(28, 0.25)),
]


@pytest.mark.parametrize("scan", PATCH_CASES, ids=lambda s: s.name)
def test_patch_fft_half_and_full(lib, scan):
    announce(f"patch_fft {scan.name}")
    rng = np.random.default_rng(2)
    stack = rng.normal(size=(scan.M, scan.ny, scan.nx)).astype(np.float32)
    ov = OracleView(scan)
    want = Opatch.patch_spectra(stack.astype(np.float64), scan.P, scan.stride, ov.px, ov.fwhm)
    g = _geom(lib, scan)
    half = lib.pact.patch_fft(dev32(stack), g, half=True)
    full = lib.pact.patch_fft(dev32(stack), g, half=False)
    torch.cuda.synchronize()
    e1, e2 = rel_l2(half, Opatch.half_spectrum(want)), rel_l2(full, want)
    print(f"patch_fft rel L2 half {e1:.2e} full {e2:.2e}")
    assert e1 < TOL_SPECTRA and e2 < TOL_SPECTRA


@pytest.mark.parametrize("P_", [24, 25, 28, 45, 80, 96])
def test_ifft2_real(lib, P_):
    announce(f"ifft2_real P={P_}")
    rng = np.random.default_rng(3)
    X = torch.tensor(rng.normal(size=(5, P_, P_)) + 1j * rng.normal(size=(5, P_, P_)))
    got = lib.pact.ifft2_real(devc64(X))
    torch.cuda.synchronize()
    want = Odec.patch_images(X.to(torch.complex64).to(torch.complex128))
    assert rel_l2(got, want) < TOL_SPECTRA


def _random_sos(scan, seed):
    rng = np.random.default_rng(seed)
    v = synth.random_sos((scan.sos_n, scan.sos_n), scan.v0, rng, amp=0.06)
    return np.asarray(v, dtype=np.float32)


@pytest.mark.parametrize("scan", WORKLOADS + [FINEGRID], ids=lambda s: s.name)
def test_sos_to_delays(lib, scan):
    announce(f"sos_to_delays {scan.name}")
    ov = OracleView(scan)
    v = _random_sos(scan, 4)
    want = Orays.sos_to_delays(torch.tensor(v, dtype=torch.float64), ov.ds, ov.v0, ov.centres, scan.n_elem, ov.R,
                               ov.phi0, scan.n_samples)
    got = lib.pact.sos_to_delays(dev32(v), _geom(lib, scan), scan.v0, dev32(ov.centres), scan.n_samples)
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print(f"sos_to_delays rel L2 {err:.2e}")
    assert err < TOL_DELAYS


@pytest.mark.parametrize("scan", WORKLOADS + [FINEGRID], ids=lambda s: s.name)
def test_sos_to_delays_adjoint(lib, scan):
    announce(f"sos_to_delays_adjoint {scan.name}")
    ov = OracleView(scan)
    v = _random_sos(scan, 5)
    rng = np.random.default_rng(6)
    gw = rng.normal(size=(ov.centres.shape[0], scan.n_elem)).astype(np.float32)
    fn = lambda vv: Orays.sos_to_delays(vv, ov.ds, ov.v0, ov.centres, scan.n_elem, ov.R, ov.phi0, scan.n_samples)
    (want,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), torch.tensor(gw, dtype=torch.float64))
    g = _geom(lib, scan)
    got = lib.pact.sos_to_delays_adjoint(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw))
    again = lib.pact.sos_to_delays_adjoint(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw))
    # accumulate and device-side scale
    acc = torch.ones_like(got)
    two = torch.full((1,), 2.0, device="cuda")
    lib.pact.sos_to_delays_adjoint(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw), out=acc,
                                   scale=two, accumulate=True)
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print(f"sos_to_delays_adjoint rel L2 {err:.2e}")
    assert err < TOL_GRAD
    assert torch.equal(got, again), "the adjoint is deterministic"
    assert rel_l2(acc - 1.0, 2.0 * want) < TOL_GRAD


@pytest.mark.parametrize("Gx", [300, 190, 191])
def test_rays_on_a_wide_grid(lib, Gx):
    """Forward and adjoint on 6-row grids whose padded rows are staged in passes of the kernels' 64-column
    chunks: 302 nodes take several passes, 192 exactly one full pass, and 193 a second pass of one column."""
    announce(f"rays on a 6 x {Gx} node grid")
    Gy, ds, v0, n_elem, R, phi0, Ns = 6, 0.5, 1.5, 64, 90.0, 0.1, 64
    g = lib.pact.Geometry(n_elem=n_elem, radius=R, phi0=phi0, ny=64, nx=64, px=0.1, P=16, stride=8, fwhm=1.0,
                          sos_ny=Gy, sos_nx=Gx, sos_spacing=ds)
    rng = np.random.default_rng(21)
    # smoother than the other cases' fields: FP32 rounds positions at node coordinates up to 301, twice
    # those of the 140-node grids, and the delay error scales with the field's slope between nodes
    v = np.asarray(synth.random_sos((Gy, Gx), v0, rng, amp=0.06, smooth=8), dtype=np.float32)
    hx = 70.0 * Gx / 300.0
    centres = np.stack([np.linspace(-hx, hx, 7), np.linspace(-1.5, 1.5, 7)], axis=1).astype(np.float32)
    c64 = torch.tensor(centres, dtype=torch.float64)
    fn = lambda vv: Orays.sos_to_delays(vv, f32(ds), f32(v0), c64, n_elem, f32(R), f32(phi0), Ns)
    want = fn(torch.tensor(v, dtype=torch.float64))
    got = lib.pact.sos_to_delays(dev32(v), g, v0, dev32(centres), Ns)
    gw = rng.standard_normal((centres.shape[0], n_elem)).astype(np.float32)
    (want_adj,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), torch.tensor(gw, dtype=torch.float64))
    got_adj = lib.pact.sos_to_delays_adjoint(dev32(v), g, v0, dev32(centres), Ns, dev32(gw))
    torch.cuda.synchronize()
    e, ea = rel_l2(got, want), rel_l2(got_adj, want_adj)
    print(f"6 x {Gx} grid: delays rel L2 {e:.2e}, adjoint rel L2 {ea:.2e}")
    assert e < TOL_DELAYS
    assert ea < TOL_GRAD


@pytest.mark.parametrize("shape", [(300, 300), (8, 2300)], ids=["banded_300x300", "tiled_8x2300"])
def test_rays_adjoint_beyond_one_cu(lib, shape):
    """The ray adjoint on grids whose contrast and accumulator do not fit one CU's LDS together: 300 x 300
    nodes run in bands of rows (5 bands, each workgroup holding its band), 8 x 2300 in the tiled form (a
    band of 8 rows does not fit either).  Against the oracle's reverse mode, deterministic."""
    Gy, Gx = shape
    announce(f"ray adjoint on a {Gy} x {Gx} grid")
    ds, v0, n_elem, R, phi0, Ns = (0.2, 1.5, 64, 90.0, 0.1, 64) if Gy > 8 else (0.05, 1.5, 64, 90.0, 0.1, 64)
    g = lib.pact.Geometry(n_elem=n_elem, radius=R, phi0=phi0, ny=64, nx=64, px=0.1, P=16, stride=8, fwhm=1.0,
                          sos_ny=Gy, sos_nx=Gx, sos_spacing=ds)
    rng = np.random.default_rng(22)
    v = np.asarray(synth.random_sos((Gy, Gx), v0, rng, amp=0.06, smooth=8), dtype=np.float32)
    hy = 0.4 * (Gy + 1) * ds
    centres = np.stack([np.linspace(-25.0, 25.0, 7), np.linspace(-hy, hy, 7)], axis=1).astype(np.float32)
    c64 = torch.tensor(centres, dtype=torch.float64)
    fn = lambda vv: Orays.sos_to_delays(vv, f32(ds), f32(v0), c64, n_elem, f32(R), f32(phi0), Ns)
    gw = rng.standard_normal((centres.shape[0], n_elem)).astype(np.float32)
    (want,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), torch.tensor(gw, dtype=torch.float64))
    got = lib.pact.sos_to_delays_adjoint(dev32(v), g, v0, dev32(centres), Ns, dev32(gw))
    again = lib.pact.sos_to_delays_adjoint(dev32(v), g, v0, dev32(centres), Ns, dev32(gw))
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print(f"adjoint on {Gy} x {Gx}: rel L2 {err:.2e}")
    assert err < TOL_GRAD
    assert torch.equal(got, again), "the adjoint is deterministic"


SUPPORT_CASES = [
    # (name, Gy, Gx, spacing, support radius, centres half-extent, delay tolerance): the whole-grid, banded and
    # tiled adjoints.  At node coordinates near 2300, FP32 rounds sample positions 16 times as coarsely as at
    # 140 (2^-13 of a node spacing), and the delays of the tiled case carry the 3e-5 that rounding gives with
    # or without a support (the two agree to 1e-6).
    ("whole_23x23", 23, 23, 1.0, 9.0, 8.0, TOL_DELAYS),
    ("banded_150x150", 150, 150, 0.16, 9.0, 9.0, TOL_DELAYS),
    ("tiled_8x2300", 8, 2300, 0.05, 30.0, 25.0, 1e-4),
]


@pytest.mark.parametrize("case", SUPPORT_CASES, ids=lambda c: c[0])
def test_rays_with_support(lib, case):
    """The ray maps with a support disc (the mask radius): with every node outside the disc at v0, the delays
    equal the oracle's and those computed without the support (only samples that add zero are skipped); nodes
    outside the disc are ignored whatever they hold (bit-identical delays); the adjoint equals the oracle's
    gradient on the nodes inside and is exactly zero beyond the radius."""
    name, Gy, Gx, ds, rho, hc, tol_w = case
    announce(f"rays with support {name}")
    v0, n_elem, R, phi0, Ns = 1.5, 64, 90.0, 0.1, 64
    g = lib.pact.Geometry(n_elem=n_elem, radius=R, phi0=phi0, ny=64, nx=64, px=0.1, P=16, stride=8, fwhm=1.0,
                          sos_ny=Gy, sos_nx=Gx, sos_spacing=ds)
    rng = np.random.default_rng(23)
    ax = lambda n: (np.arange(n) - (n - 1) / 2.0) * f32(ds)  # noqa: E731
    dist = np.sqrt(ax(Gx)[None, :] ** 2 + ax(Gy)[:, None] ** 2)
    inside = dist <= f32(rho)
    v = np.asarray(synth.random_sos((Gy, Gx), v0, rng, amp=0.06, smooth=8), dtype=np.float32)
    v = np.where(inside, v, np.float32(v0)).astype(np.float32)
    hy = min(hc, 0.4 * (Gy + 1) * ds)
    centres = np.stack([np.linspace(-hc, hc, 7), np.linspace(-hy, hy, 7)], axis=1).astype(np.float32)
    c64 = torch.tensor(centres, dtype=torch.float64)
    fn = lambda vv: Orays.sos_to_delays(vv, f32(ds), f32(v0), c64, n_elem, f32(R), f32(phi0), Ns)  # noqa: E731
    want = fn(torch.tensor(v, dtype=torch.float64))
    c = dev32(centres)
    got = lib.pact.sos_to_delays(dev32(v), g, v0, c, Ns, support=rho)
    full = lib.pact.sos_to_delays(dev32(v), g, v0, c, Ns)
    junk = np.where(inside, v, v + np.float32(0.07)).astype(np.float32)
    got_junk = lib.pact.sos_to_delays(dev32(junk), g, v0, c, Ns, support=rho)
    gw = rng.standard_normal((centres.shape[0], n_elem)).astype(np.float32)
    (want_adj,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), torch.tensor(gw, dtype=torch.float64))
    got_adj = lib.pact.sos_to_delays_adjoint(dev32(v), g, v0, c, Ns, dev32(gw), support=rho)
    junk_adj = lib.pact.sos_to_delays_adjoint(dev32(junk), g, v0, c, Ns, dev32(gw), support=rho)
    torch.cuda.synchronize()
    e, ef = rel_l2(got, want), rel_l2(got, full)
    ins = torch.tensor(inside)
    ea = rel_l2(got_adj.cpu()[ins], want_adj[ins])
    print(f"support {name}: delays rel L2 {e:.2e} (vs no support {ef:.2e}), adjoint inside rel L2 {ea:.2e}")
    assert e < tol_w and ef < 1e-6
    assert torch.equal(got, got_junk), "nodes outside the support are ignored"
    assert ea < TOL_GRAD
    beyond = torch.tensor(dist > f32(rho) * (1 + 1e-5))
    assert (got_adj.cpu()[beyond] == 0).all(), "no gradient beyond the support"
    assert torch.equal(got_adj, junk_adj)


STAGED_CASES = [
    # (name, Gy, Gx, spacing, support radius): whole grid with and without a support, a ragged grid, the banded
    # adjoint (bands start on rows whose offset is not a multiple of four floats) and the tiled one (which does
    # not take the staged grid)
    ("whole_23x23_support", 23, 23, 1.0, 9.0),
    ("whole_23x23_none", 23, 23, 1.0, 0.0),
    ("ragged_31x17", 31, 17, 0.9, 7.5),
    ("banded_150x150", 150, 150, 0.16, 9.0),
    ("tiled_8x2300", 8, 2300, 0.05, 30.0),
]


@pytest.mark.parametrize("case", STAGED_CASES, ids=lambda c: c[0])
def test_staged_contrast(lib, case):
    """pact_stage_contrast forms the padded contrast grid exactly (sos - v0 inside the grid and the support,
    zero elsewhere), and the ray maps given it return what they return when they form it themselves, bit for
    bit."""
    name, Gy, Gx, ds, rho = case
    announce(f"staged contrast {name}")
    v0, n_elem, R, phi0, Ns = 1.5, 64, 90.0, 0.1, 64
    g = lib.pact.Geometry(n_elem=n_elem, radius=R, phi0=phi0, ny=64, nx=64, px=0.1, P=16, stride=8, fwhm=1.0,
                          sos_ny=Gy, sos_nx=Gx, sos_spacing=ds)
    rng = np.random.default_rng(29)
    v = np.asarray(synth.random_sos((Gy, Gx), v0, rng, amp=0.06, smooth=8), dtype=np.float32)
    ax = lambda n: (np.arange(n) - (n - 1) / 2.0) * f32(ds)  # noqa: E731
    dist = np.sqrt(ax(Gx)[None, :] ** 2 + ax(Gy)[:, None] ** 2)
    inside = dist <= f32(rho) * (1 + 1e-6) if rho > 0 else np.ones((Gy, Gx), bool)
    want = np.zeros((Gy + 2, Gx + 2), np.float32)
    want[1:-1, 1:-1] = np.where(inside, v - np.float32(v0), np.float32(0.0))
    sos = dev32(v)
    st = lib.pact.stage_contrast(sos, g, v0, support=rho)
    hc = min(0.4 * (Gx + 1) * ds, 8.0)
    hy = min(hc, 0.4 * (Gy + 1) * ds)
    c = dev32(np.stack([np.linspace(-hc, hc, 7), np.linspace(-hy, hy, 7)], axis=1).astype(np.float32))
    gw = dev32(rng.standard_normal((7, n_elem)).astype(np.float32))
    w_a = lib.pact.sos_to_delays(sos, g, v0, c, Ns, support=rho)
    w_b = lib.pact.sos_to_delays(sos, g, v0, c, Ns, support=rho, staged=st)
    a_a = lib.pact.sos_to_delays_adjoint(sos, g, v0, c, Ns, gw, support=rho)
    a_b = lib.pact.sos_to_delays_adjoint(sos, g, v0, c, Ns, gw, support=rho, staged=st)
    torch.cuda.synchronize()
    got = st.cpu().numpy().reshape(Gy + 2, Gx + 2)
    # the kernel tests the support with its FP32 node coordinates: at most nodes on the rim may differ
    rim = np.zeros((Gy + 2, Gx + 2), bool)
    rim[1:-1, 1:-1] = np.abs(dist - f32(rho)) < 1e-4 * max(rho, 1.0)
    assert np.array_equal(got[~rim], want[~rim])
    assert torch.equal(w_a, w_b) and torch.equal(a_a, a_b)


def test_fused_adjoint_tv_adam_step(lib):
    """The fused end of a step (ray adjoint, partial sums, TV, Adam) against the separate calls on the paper's
    SOS grid size: the same SOS, moments and gradient on the free nodes, bit for bit; the staged grid it writes
    for the updated SOS equals pact_stage_contrast's, and a step given the staged grid of its input equals one
    without."""
    announce("fused adjoint + TV + Adam")
    scan = synth.PAPER.with_(ny=240, nx=240, n_elem=128)
    g = lib.geometry_from(scan)
    rng = np.random.default_rng(31)
    G = scan.sos_n
    free = np.asarray(synth.free_node_mask(scan), bool)
    v = np.asarray(synth.random_sos((G, G), scan.v0, rng, amp=0.03), dtype=np.float32)
    v = np.where(free, v, np.float32(scan.v0)).astype(np.float32)
    from oracle.geometry import patch_centres
    cent = patch_centres(scan.ny, scan.nx, f32(scan.px), scan.P, scan.stride).numpy().astype(np.float32)
    N = cent.shape[0]
    c = dev32(cent)
    gw = dev32(rng.standard_normal((N, scan.n_elem)).astype(np.float32) * 1e3)
    mask = torch.tensor(free.astype(np.uint8), device="cuda")
    rho, lam, lr = scan.mask_radius, f32(3e9), f32(1e-3)
    m0 = dev32(rng.standard_normal((G, G)).astype(np.float32) * 1e-3)
    s0 = dev32(np.abs(rng.standard_normal((G, G))).astype(np.float32) * 1e-6)
    t0 = torch.tensor([7, 0], dtype=torch.int32, device="cuda")
    sos = dev32(v)
    # separate calls
    grad = lib.pact.sos_to_delays_adjoint(sos, g, scan.v0, c, scan.n_samples, gw, support=rho)
    a_out, a_m, a_v, a_t = torch.empty_like(sos), m0.clone(), s0.clone(), t0.clone()
    lib.pact.tv_adam_step(sos, a_out, a_m, a_v, a_t, mask, g, grad, lam, None, lr)
    # fused, without and with the staged grid
    outs = []
    for staged in (None, lib.pact.stage_contrast(sos, g, scan.v0, support=rho)):
        b_out, b_m, b_v, b_t = torch.empty_like(sos), m0.clone(), s0.clone(), t0.clone()
        b_grad = torch.empty_like(sos)
        st_out = torch.full((lib.pact.staged_contrast_floats(g),), float("nan"), device="cuda")
        lib.pact.sos_adjoint_tv_adam_step(sos, b_out, b_m, b_v, b_t, mask, g, scan.v0, c, scan.n_samples, gw, lam,
                                          None, lr, support=rho, grad=b_grad, staged_in=staged, staged_out=st_out)
        outs.append((b_out, b_m, b_v, b_t, b_grad, st_out))
    torch.cuda.synchronize()
    fr = mask.bool()
    for b_out, b_m, b_v, b_t, b_grad, st_out in outs:
        assert torch.equal(b_out, a_out) and torch.equal(b_m[fr], a_m[fr]) and torch.equal(b_v[fr], a_v[fr])
        assert torch.equal(b_grad[fr], grad[fr]) and b_t.tolist() == a_t.tolist()
        assert torch.equal(st_out, lib.pact.stage_contrast(b_out, g, scan.v0, support=rho))


def _wavefronts(scan, seed):
    """A plausible float32 wavefront table (oracle rays through a random SOS)."""
    ov = OracleView(scan)
    v = _random_sos(scan, seed)
    w = Orays.sos_to_delays(torch.tensor(v, dtype=torch.float64), ov.ds, ov.v0, ov.centres, scan.n_elem, ov.R,
                            ov.phi0, scan.n_samples)
    return w.to(torch.float32).to(torch.float64), ov


@pytest.mark.parametrize("scan", WORKLOADS, ids=lambda s: s.name)
def test_delays_to_psf(lib, scan):
    announce(f"delays_to_psf {scan.name}")
    w, ov = _wavefronts(scan, 7)
    H_want = Opsf.transfer_functions(w, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px)
    h_want = Opsf.psf(H_want)
    H, h = lib.pact.delays_to_psf(dev32(w), dev32(ov.centres), _geom(lib, scan), dev32(ov.delays), with_psf=True)
    torch.cuda.synchronize()
    e1, e2 = rel_l2(H, H_want), rel_l2(h, h_want)
    print(f"delays_to_psf rel L2 H {e1:.2e} h {e2:.2e}")
    assert e1 < TOL_PSF and e2 < TOL_PSF
    assert torch.abs(H).max().item() <= 1.0 + 1e-6


@pytest.mark.parametrize("scan", WORKLOADS, ids=lambda s: s.name)
def test_delays_to_psf_adjoint(lib, scan):
    announce(f"delays_to_psf_adjoint {scan.name}")
    w, ov = _wavefronts(scan, 8)
    rng = np.random.default_rng(9)
    N = w.shape[0]
    gH = torch.tensor(rng.normal(size=(N, scan.M, scan.P, scan.P)) + 1j * rng.normal(size=(N, scan.M, scan.P, scan.P)))
    gH = gH.to(torch.complex64).to(torch.complex128)
    fn = lambda ww: Opsf.transfer_functions(ww, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px)
    (want,) = Oloss.vjp(fn, (w,), gH)
    got = lib.pact.delays_to_psf_adjoint(dev32(w), dev32(ov.centres), _geom(lib, scan), dev32(ov.delays), devc64(gH))
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print(f"delays_to_psf_adjoint rel L2 {err:.2e}")
    assert err < TOL_GRAD


def _Y_H(scan, seed):
    w, ov = _wavefronts(scan, seed)
    rng = np.random.default_rng(seed + 100)
    N = w.shape[0]
    H = Opsf.transfer_functions(w, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px).to(torch.complex64)
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng).to(torch.complex64)
    return Y.to(torch.complex128), H.to(torch.complex128), w, ov


@pytest.mark.parametrize("scan", WORKLOADS, ids=lambda s: s.name)
def test_multichannel_deconv_and_adjoint(lib, scan):
    announce(f"multichannel_deconv {scan.name}")
    Y, H, w, ov = _Y_H(scan, 10)
    eps = f32(1e-3)
    X_want = Odec.multichannel_deconv(Y, H, eps)
    X = lib.pact.multichannel_deconv(devc64(Y), devc64(H), eps)
    rng = np.random.default_rng(11)
    gX = torch.tensor(rng.normal(size=X_want.shape) + 1j * rng.normal(size=X_want.shape)).to(torch.complex64)
    (gH_want,) = Oloss.vjp(lambda HH: Odec.multichannel_deconv(Y, HH, eps), (H,), gX.to(torch.complex128))
    gH = lib.pact.multichannel_deconv_adjoint(devc64(Y), devc64(H), eps, devc64(gX))
    torch.cuda.synchronize()
    e1, e2 = rel_l2(X, X_want), rel_l2(gH, gH_want)
    print(f"deconv rel L2 X {e1:.2e} adjoint {e2:.2e}")
    assert e1 < TOL_DECONV and e2 < TOL_GRAD


@pytest.mark.parametrize("scan", WORKLOADS, ids=lambda s: s.name)
def test_residual_loss(lib, scan):
    announce(f"residual_loss {scan.name}")
    Y, H, w, ov = _Y_H(scan, 12)
    X = Odec.multichannel_deconv(Y, H, 1e-3).to(torch.complex64).to(torch.complex128)
    Hl, Xl = H.clone().requires_grad_(True), X.clone().requires_grad_(True)
    L = Oloss.data_loss(Y, Hl, Xl, ov.px)
    gH_want, gX_want = torch.autograd.grad(L, (Hl, Xl))
    loss, gH, gX = lib.pact.residual_loss(devc64(Y), devc64(H), devc64(X), scan.px)
    torch.cuda.synchronize()
    print(f"residual loss rel {abs(loss.item() - L.item()) / L.item():.2e}")
    assert abs(loss.item() - L.item()) <= TOL_LOSS * L.item()
    assert rel_l2(gH, gH_want) < TOL_GRAD and rel_l2(gX, gX_want) < TOL_GRAD


@pytest.mark.parametrize("scan,P_", [(synth.TINY, None), (RAGGED, None), (RAGGED, 25)],
                         ids=["tiny", "ragged-even", "ragged-odd-P"])
def test_loss_and_grad_fused(lib, scan, P_):
    """The fused kernel over half spectra equals the oracle's full-spectrum definition (loss, dL/dw, X_hat);
    P odd and even exercise the Nyquist-row handling."""
    if P_ is not None:
        scan = scan.with_(P=P_, fwhm=synth.configs.fwhm_for_patch(P_, scan.px))
    announce(f"loss_and_grad {scan.name} P={scan.P}")
    w, ov = _wavefronts(scan, 13)
    rng = np.random.default_rng(14)
    N = w.shape[0]
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng).to(torch.complex64).to(torch.complex128)
    eps = f32(1e-3)
    fn = lambda ww: Oloss.loss_from_delays(ww, Y, ov.centres, ov.R, ov.phi0, ov.delays, ov.px, eps)
    wl = w.clone().requires_grad_(True)
    L = fn(wl)
    (gw_want,) = torch.autograd.grad(L, wl)
    H = Opsf.transfer_functions(w, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px)
    X_want = Odec.multichannel_deconv(Y, H, eps)
    g = lib.geometry_from(scan)
    Yh = devc64(Opatch.half_spectrum(Y))
    X = torch.empty(N, scan.P, scan.P, dtype=torch.complex64, device="cuda")
    loss, gw = lib.pact.loss_and_grad(Yh, dev32(w), dev32(ov.centres), g, dev32(ov.delays), eps, X=X)
    torch.cuda.synchronize()
    el = abs(loss.item() - L.item()) / L.item()
    eg, ex = rel_l2(gw, gw_want), rel_l2(X, X_want)
    print(f"loss_and_grad: loss rel {el:.2e}, dL/dw rel L2 {eg:.2e}, X rel L2 {ex:.2e}")
    assert el < TOL_LOSS and eg < TOL_GRAD and ex < TOL_DECONV


@pytest.mark.parametrize("scan,P_,M_", [(synth.TINY, None, None), (RAGGED, None, None), (RAGGED, 25, None),
                                         (RAGGED, None, 1)], ids=["tiny", "ragged-even", "ragged-odd-P", "M1"])
def test_loss_and_grad_projected(lib, scan, P_, M_):
    """The fused step from projected spectra equals the oracle's full-spectrum definition (loss, dL/dw, X_hat)
    and the direct form on the same spectra.  The small workload's delays are not uniformly spaced, the ragged
    one's are not symmetric about zero (so the sine sums of the projection are not zero)."""
    if P_ is not None:
        scan = scan.with_(P=P_, fwhm=synth.configs.fwhm_for_patch(P_, scan.px))
    if M_ is not None:
        scan = scan.with_(delays=(0.31,))
    announce(f"loss_and_grad_projected {scan.name} P={scan.P} M={scan.M}")
    w, ov = _wavefronts(scan, 13)
    rng = np.random.default_rng(14)
    N = w.shape[0]
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng).to(torch.complex64).to(torch.complex128)
    eps = f32(1e-3)
    fn = lambda ww: Oloss.loss_from_delays(ww, Y, ov.centres, ov.R, ov.phi0, ov.delays, ov.px, eps)  # noqa: E731
    wl = w.clone().requires_grad_(True)
    L = fn(wl)
    (gw_want,) = torch.autograd.grad(L, wl)
    H = Opsf.transfer_functions(w, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px)
    X_want = Odec.multichannel_deconv(Y, H, eps)
    g = lib.geometry_from(scan)
    Yh = devc64(Opatch.half_spectrum(Y))
    d = dev32(ov.delays)
    T = lib.pact.project_spectra(Yh, g, d, dev32(ov.centres))
    X = torch.empty(N, scan.P, scan.P, dtype=torch.complex64, device="cuda")
    loss, gw = lib.pact.loss_and_grad_projected(T, scan.M, dev32(w), dev32(ov.centres), g, eps, X=X)
    loss_d, gw_d = lib.pact.loss_and_grad(Yh, dev32(w), dev32(ov.centres), g, d, eps)
    torch.cuda.synchronize()
    el = abs(loss.item() - L.item()) / L.item()
    eg, ex = rel_l2(gw, gw_want), rel_l2(X, X_want)
    print(f"loss_and_grad_projected: loss rel {el:.2e}, dL/dw rel L2 {eg:.2e}, X rel L2 {ex:.2e}")
    assert el < TOL_LOSS and eg < TOL_GRAD and ex < TOL_DECONV
    assert abs(loss.item() - loss_d.item()) <= TOL_LOSS * abs(loss_d.item()) and rel_l2(gw, gw_d) < TOL_GRAD


def test_modular_chain_matches_fused(lib):
    """sos -> w -> H -> X -> loss with the standalone calls and their adjoints gives the fused result."""
    scan = RAGGED
    announce("modular chain vs fused")
    ov = OracleView(scan)
    v = dev32(_random_sos(scan, 15))
    g = lib.geometry_from(scan)
    rng = np.random.default_rng(16)
    N = ov.centres.shape[0]
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng)
    Yf = devc64(Y)
    Yh = devc64(Opatch.half_spectrum(Y))
    c, d = dev32(ov.centres), dev32(ov.delays)
    eps = f32(1e-3)
    w = lib.pact.sos_to_delays(v, g, scan.v0, c, scan.n_samples)
    H = lib.pact.delays_to_psf(w, c, g, d)
    X = lib.pact.multichannel_deconv(Yf, H, eps)
    loss_m, gH, gX = lib.pact.residual_loss(Yf, H, X, scan.px)
    gH = gH + lib.pact.multichannel_deconv_adjoint(Yf, H, eps, gX)
    gw_m = lib.pact.delays_to_psf_adjoint(w, c, g, d, gH)
    loss_f, gw_f = lib.pact.loss_and_grad(Yh, w, c, g, d, eps)
    gs_m = lib.pact.sos_to_delays_adjoint(v, g, scan.v0, c, scan.n_samples, gw_m)
    gs_f = lib.pact.sos_to_delays_adjoint(v, g, scan.v0, c, scan.n_samples, gw_f)
    torch.cuda.synchronize()
    assert abs(loss_m.item() - loss_f.item()) <= TOL_LOSS * loss_f.item()
    assert rel_l2(gw_m, gw_f) < TOL_GRAD
    assert rel_l2(gs_m, gs_f) < TOL_GRAD


def test_tv_and_adam(lib):
    announce("tv_grad + adam_step")
    scan = RAGGED
    rng = np.random.default_rng(17)
    v = _random_sos(scan, 18)
    mask = synth.free_node_mask(scan)
    lam = f32(0.37)
    (tv_g,) = Oloss.vjp(lambda vv: Oloss.tv(vv, mask), (torch.tensor(v, dtype=torch.float64),),
                        torch.tensor(1.0, dtype=torch.float64))
    tv_v = Oloss.tv(torch.tensor(v, dtype=torch.float64), mask).item()
    g = lib.geometry_from(scan)
    base = rng.normal(size=v.shape).astype(np.float32)
    grad = dev32(base)
    loss = torch.full((1,), 5.0, device="cuda")
    lib.pact.tv_grad(dev32(v), dev32(mask).to(torch.uint8), g, lam, grad, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - (5.0 + lam * tv_v)) <= 1e-5 * (5.0 + lam * tv_v)
    assert rel_l2(grad.cpu().double() - torch.tensor(base, dtype=torch.float64), lam * tv_g) < 1e-5
    # Adam: a few steps with fixed gradients against the oracle's FP64 Adam
    p = dev32(v)
    m = torch.zeros_like(p)
    s2 = torch.zeros_like(p)
    t = torch.zeros(2, dtype=torch.int32, device="cuda")
    mk = dev32(mask).to(torch.uint8)
    ref = Oadam.Adam(torch.tensor(v, dtype=torch.float64), mask, lr=f32(1e-3))
    for k in range(4):
        gk = rng.normal(size=v.shape).astype(np.float32)
        lib.pact.adam_step(p, m, s2, t, mk, dev32(gk), f32(1e-3))
        ref.step(torch.tensor(gk, dtype=torch.float64))
    torch.cuda.synchronize()
    assert t.tolist() == [4, 0]
    dp = p.cpu().double() - torch.tensor(v, dtype=torch.float64)
    dref = ref.p - torch.tensor(v, dtype=torch.float64)
    assert rel_l2(dp, dref) < 1e-4
    assert torch.equal(p.cpu()[torch.tensor(mask == 0)], torch.tensor(v)[torch.tensor(mask == 0)])


def test_tv_adam_fused_matches_oracle(lib):
    """The fused TV + Adam update (reads one SOS buffer, writes the other) against the oracle: TV subgradient
    at the old SOS added to the data gradient, then the FP64 Adam step; loss gains lambda TV."""
    announce("tv_adam_step")
    scan = RAGGED
    rng = np.random.default_rng(19)
    v = _random_sos(scan, 20)
    mask = synth.free_node_mask(scan)
    lam = f32(0.37)
    g = lib.geometry_from(scan)
    mk = dev32(mask).to(torch.uint8)
    a, b = dev32(v), torch.empty(v.shape, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(a)
    s2 = torch.zeros_like(a)
    t = torch.zeros(2, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ref = Oadam.Adam(torch.tensor(v, dtype=torch.float64), mask, lr=f32(1e-3))
    tv_sum = 0.0
    for k in range(4):
        gk = rng.normal(size=v.shape).astype(np.float32)
        cur = ref.p.clone()
        (tv_g,) = Oloss.vjp(lambda vv: Oloss.tv(vv, mask), (cur,), torch.tensor(1.0, dtype=torch.float64))
        tv_sum += lam * Oloss.tv(cur, mask).item()
        ref.step(torch.tensor(gk, dtype=torch.float64) + lam * tv_g)
        lib.pact.tv_adam_step(a, b, m, s2, t, mk, g, dev32(gk), lam, loss, f32(1e-3))
        a, b = b, a
    torch.cuda.synchronize()
    assert t.tolist() == [4, 0]
    dp = a.cpu().double() - torch.tensor(v, dtype=torch.float64)
    dref = ref.p - torch.tensor(v, dtype=torch.float64)
    print(f"tv_adam_step rel L2 {rel_l2(dp, dref):.2e}")
    assert rel_l2(dp, dref) < 1e-4
    assert abs(loss.item() - tv_sum) <= 1e-5 * tv_sum
    assert torch.equal(a.cpu()[torch.tensor(mask == 0)], torch.tensor(v)[torch.tensor(mask == 0)])


@pytest.mark.parametrize("scan", WORKLOADS, ids=lambda s: s.name)
def test_stitch(lib, scan):
    """Gaussian-weighted stitching of patch images against the oracle's, on random patches and on the
    deconvolved patches of a real stack (X_hat from the fused kernel, then the inverse transform)."""
    from oracle import stitch as Ostitch
    announce(f"stitch {scan.name}")
    ov = OracleView(scan)
    g = lib.geometry_from(scan)
    N = ov.centres.shape[0]
    rng = np.random.default_rng(21)
    x = rng.normal(size=(N, scan.P, scan.P)).astype(np.float32)
    got = lib.pact.stitch(dev32(x), g)
    torch.cuda.synchronize()
    want = Ostitch.stitch(torch.tensor(x, dtype=torch.float64), scan.ny, scan.nx, scan.P, scan.stride, ov.px, ov.fwhm)
    err = rel_l2(got, want)
    print(f"stitch rel L2 {err:.2e}")
    assert err < TOL_SPECTRA
    # the reconstruction's last step: X_hat -> patches -> image
    w, _ = _wavefronts(scan, 22)
    Y = random_real_patches_spectra(N, scan.M, scan.P, rng).to(torch.complex64).to(torch.complex128)
    eps = f32(1e-3)
    H = Opsf.transfer_functions(w, ov.centres, ov.R, ov.phi0, ov.delays, scan.P, ov.px)
    img_want = Ostitch.stitch(Odec.patch_images(Odec.multichannel_deconv(Y, H, eps)), scan.ny, scan.nx, scan.P,
                              scan.stride, ov.px, ov.fwhm)
    X = torch.empty(N, scan.P, scan.P, dtype=torch.complex64, device="cuda")
    lib.pact.loss_and_grad(devc64(Opatch.half_spectrum(Y)), dev32(w), dev32(ov.centres), g, dev32(ov.delays), eps,
                           X=X)
    img = lib.pact.stitch(lib.pact.ifft2_real(X), g)
    torch.cuda.synchronize()
    e2 = rel_l2(img, img_want)
    print(f"X_hat -> image rel L2 {e2:.2e}")
    assert e2 < TOL_DECONV


def test_rays_autotune(lib):
    # a geometry no other test uses (the tuned tilings are kept per geometry for the process)
    scan = RAGGED.with_(n_samples=90)
    announce(f"rays autotune {scan.name} N_s={scan.n_samples}")
    ov = OracleView(scan)
    v = _random_sos(scan, 7)
    rng = np.random.default_rng(8)
    N = ov.centres.shape[0]
    gw = rng.normal(size=(N, scan.n_elem)).astype(np.float32)
    g = _geom(lib, scan)
    w = torch.empty(N, scan.n_elem, device="cuda")
    gs = torch.empty(scan.sos_n, scan.sos_n, device="cuda")
    ws = torch.empty(max(1, lib.pact.sos_to_delays_adjoint_workspace_size(g, N)), dtype=torch.uint8, device="cuda")
    kf, ka = lib.pact.rays_autotune(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw), w, gs, ws)
    assert kf in (1, 2, 4, 8) and ka == 0, (kf, ka)      # the adjoint's work items need no tuning
    # the calls now run with the tuned tilings and still match the oracle
    want = Orays.sos_to_delays(torch.tensor(v, dtype=torch.float64), ov.ds, ov.v0, ov.centres, scan.n_elem, ov.R,
                               ov.phi0, scan.n_samples)
    got = lib.pact.sos_to_delays(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples)
    fn = lambda vv: Orays.sos_to_delays(vv, ov.ds, ov.v0, ov.centres, scan.n_elem, ov.R, ov.phi0, scan.n_samples)
    (gwant,) = Oloss.vjp(fn, (torch.tensor(v, dtype=torch.float64),), torch.tensor(gw, dtype=torch.float64))
    ggot = lib.pact.sos_to_delays_adjoint(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw))
    again = lib.pact.sos_to_delays_adjoint(dev32(v), g, scan.v0, dev32(ov.centres), scan.n_samples, dev32(gw))
    torch.cuda.synchronize()
    assert rel_l2(got, want) < TOL_DELAYS
    assert rel_l2(ggot, gwant) < TOL_GRAD
    assert torch.equal(ggot, again)
