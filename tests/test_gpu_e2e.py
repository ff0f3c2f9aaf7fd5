"""GPU end to end on the tiny workload: scan preparation, whole-step gradients at matched states, a short
optimisation, HIP-graph replay and the autograd wrapper."""
import numpy as np
import pytest
import torch

import synth
from oracle import das as Odas, patches as Opatch, loss as Oloss, sos as Osos

from gpu_common import OracleView, TOL_GRAD, TOL_LOSS, TOL_SPECTRA, announce, dev32, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2409_10876_amd as P
    scan = synth.TINY
    inp = synth.make_inputs(scan, seed=1)
    ov = OracleView(scan)
    st = Odas.das_stack(inp.S, ov.fs, ov.t0, scan.n_elem, ov.R, ov.phi0, ov.v0, ov.delays, scan.ny, scan.nx, ov.px)
    Y_or = Opatch.patch_spectra(st, scan.P, scan.stride, ov.px, ov.fwhm)
    sd = P.prepare_scan(scan, inp.S, np.asarray(scan.delays, dtype=np.float32))
    torch.cuda.synchronize()
    return P, scan, inp, ov, Y_or, sd


def test_scan_preparation_matches_oracle(setup):
    P, scan, inp, ov, Y_or, sd = setup
    announce("prepare_scan tiny")
    err = rel_l2(sd.Y, Opatch.half_spectrum(Y_or))
    print(f"Y rel L2 {err:.2e}")
    assert err < 10 * TOL_SPECTRA       # DAS and FFT errors compound


def _oracle_grad(ov, scan, mask, Y_or, sos, lam):
    return Oloss.loss_and_grad(torch.tensor(sos, dtype=torch.float64), mask, Y_or, ov.geom(), lam)


@pytest.mark.parametrize("support", [False, True], ids=["full_grid", "mask_support"])
def test_step_gradient_matches_oracle_at_matched_states(setup, support):
    """Teacher forcing: at each GPU state along a short run, the GPU's loss and dL/dsos (data + TV) equal the
    oracle's at that same state.  With the mask radius as the rays' support, the gradient is compared on the
    free nodes (the only ones Adam updates; the data gradient of the fixed ones is then not computed)."""
    P, scan, inp, ov, Y_or, sd = setup
    announce(f"steps with per-step oracle gradients (support {support})")
    lam = 1e8                          # large enough for the TV subgradient to show next to the data term
    solver = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=lam, lr=scan.lr, n_samples=scan.n_samples,
                               support_radius=scan.mask_radius if support else 0.0)
    free = torch.tensor(inp.mask).bool()
    for k in range(4):
        state = solver.sos.cpu().numpy().copy()
        solver.delays(); solver.loss_grad(); solver.adjoint(); solver.regularise()
        torch.cuda.synchronize()
        L, gv, _, _ = _oracle_grad(ov, scan, inp.mask, Y_or, state, f32(lam))
        eg = rel_l2(solver.grad.cpu()[free], gv[free]) if support else rel_l2(solver.grad, gv)
        el = abs(solver.loss.item() - L.item()) / L.item()
        print(f"step {k}: loss {solver.loss.item():.6e} (rel {el:.1e})  grad rel L2 {eg:.1e}")
        assert el < TOL_LOSS and eg < TOL_GRAD
        solver.update()


def test_short_run_lowers_loss_and_sos_error(setup):
    P, scan, inp, ov, Y_or, sd = setup
    announce(f"{scan.steps} Adam steps")
    solver = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples)
    m = torch.tensor(inp.mask).bool()
    vt = torch.tensor(inp.sos_true)
    rmse = lambda p: torch.sqrt(((p.cpu().double() - vt)[m] ** 2).mean()).item()
    e0 = rmse(solver.sos)
    losses = []
    for k in range(scan.steps):
        solver.step()
        losses.append(solver.loss.item())
    e1 = rmse(solver.sos)
    print(f"loss {losses[0]:.4e} -> {losses[-1]:.4e}; SOS RMSE {e0 * 1e3:.2f} -> {e1 * 1e3:.2f} m/s")
    assert losses[-1] < losses[0]
    assert e1 < e0


def f32(x):
    return float(np.float32(x))


def test_graph_replay_matches_eager(setup):
    P, scan, inp, ov, Y_or, sd = setup
    announce("graph capture and replay")
    rho = scan.mask_radius
    a = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples,
                          support_radius=rho)
    b = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples,
                          support_radius=rho)
    a.step(); b.step()
    a.capture(4)                       # capturing does not run the steps
    torch.cuda.synchronize()
    assert torch.equal(a.sos, b.sos)
    for _ in range(3):
        a.run(4)
        torch.cuda.synchronize()       # eager work and syncs between replays
        b.run(4)
        torch.cuda.synchronize()
        assert a.t.tolist() == b.t.tolist()
        # every kernel of the step is deterministic: the replayed state is the eager state, bit for bit
        assert torch.equal(a.sos, b.sos) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
        assert abs(a.loss.item() - b.loss.item()) <= 1e-6 * abs(b.loss.item())


def test_autograd_function(setup):
    P, scan, inp, ov, Y_or, sd = setup
    announce("SosLoss autograd")
    sos = torch.tensor(synth.random_sos((scan.sos_n, scan.sos_n), scan.v0, np.random.default_rng(3), amp=0.03),
                       dtype=torch.float32, device="cuda", requires_grad=True)
    L = P.SosLoss.apply(sos, sd, f32(scan.eps), scan.n_samples)
    (2.5 * L).backward()
    Lo, gv, _, _ = Oloss.loss_and_grad(sos.detach().cpu().double(), np.ones((scan.sos_n, scan.sos_n), bool), Y_or,
                                       ov.geom(), 0.0)
    torch.cuda.synchronize()
    assert abs(L.item() - Lo.item()) <= TOL_LOSS * Lo.item()
    assert rel_l2(sos.grad, 2.5 * gv) < TOL_GRAD
