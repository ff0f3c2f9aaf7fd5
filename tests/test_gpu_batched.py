"""Batched solves of independent, unevenly sized scans: each scan's state after concurrent graph replays on
separate streams equals, bit for bit, the state it reaches when solved alone (deterministic kernels, no
shared buffers).  The kernels themselves are held to the oracle by the parity tests."""
import numpy as np
import pytest
import torch

import synth

from gpu_common import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2409_10876_amd as P
    return P


def _scans():
    base = synth.TINY
    return [base.with_(name="b0", ny=96, nx=96, n_elem=128, delays=tuple(synth.uniform_delays(-0.6, 0.6, 5)), P=24,
                       stride=12, fwhm=synth.configs.fwhm_for_patch(24, 0.2), sos_n=24, mask_radius=9.0,
                       n_blobs=6, blob_radius=8.0),
            base.with_(name="b1", ny=128, nx=128, n_elem=192, delays=tuple(synth.uniform_delays(-0.7, 0.7, 7)),
                       n_blobs=8),
            base.with_(name="b2", ny=160, nx=160, n_elem=256, delays=tuple(synth.uniform_delays(-0.8, 0.8, 9)),
                       P=32, stride=16, sos_n=40, mask_radius=15.0, n_blobs=8, blob_radius=14.0)]


def _solvers(P, scans):
    out = []
    for k, sc in enumerate(scans):
        inp = synth.make_inputs(sc, seed=10 + k)
        sd = P.prepare_scan(sc, inp.S, np.asarray(sc.delays, dtype=np.float32))
        out.append(P.PixelGridSolver(sd, inp.mask, eps=sc.eps, lam=sc.lam_tv, lr=sc.lr, n_samples=sc.n_samples))
    return out


def test_batched_matches_solo(lib):
    announce("batched solves vs solo")
    scans = _scans()
    batch = lib.BatchedSolver(_solvers(lib, scans), graph_steps=4)
    solo = _solvers(lib, scans)
    for s in solo:
        s.step()                                  # the batch ran one eager step before capturing
    batch.run(8)
    torch.cuda.synchronize()
    for s in solo:
        s.run(8)
    torch.cuda.synchronize()
    for a, b in zip(batch.solvers, solo):
        assert a.t.tolist() == b.t.tolist() == [9, 0]
        assert torch.equal(a.sos, b.sos)


PERSISTENT_OFF = pytest.mark.skip(reason="the persistent step is switched off: an earlier form did not finish on the GPU and the rewritten kernel is untested there")


@pytest.mark.parametrize("groups,persistent", [(1, False), (2, False),
                                               pytest.param(1, True, marks=PERSISTENT_OFF),
                                               pytest.param(2, True, marks=PERSISTENT_OFF)],
                         ids=["stages_1", "stages_2", "persistent_1", "persistent_2"])
def test_grouped_launches_match_solo(lib, groups, persistent):
    """One launch per stage over all scans (pact_batch_step), or over each of two groups of scans on their own
    streams, or the whole step in one persistent launch per group (pact_batch_step_persistent), reaches each
    scan's solo state, bit for bit; the scalar loss of the last step too."""
    announce(f"grouped batched step ({groups} groups, persistent={persistent}) vs solo")
    scans = _scans()
    grouped = lib.GroupedBatchSolver(_solvers(lib, scans), graph_steps=4, groups=groups, persistent=persistent)
    solo = _solvers(lib, scans)
    for s in solo:
        s.step()                                  # the grouped solver ran one eager step before capturing
    grouped.run(8)
    torch.cuda.synchronize()
    for s in solo:
        s.run(8)
    torch.cuda.synchronize()
    for a, b in zip(grouped.solvers, solo):
        assert a.t.tolist() == b.t.tolist() == [9, 0]
        assert torch.equal(a.sos, b.sos) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
        assert torch.equal(a.w, b.w) and torch.equal(a.gw, b.gw)
        assert abs(a.loss.item() - b.loss.item()) <= 1e-6 * abs(b.loss.item())   # TV's float atomics aside


def test_persistent_step_refuses_a_real_plan(lib):
    """The switched-off persistent step refuses a valid plan with PACT_EUNSUPPORTED before launching anything, and
    the plan still drives the per-stage step, whose states then match solo runs bit for bit."""
    announce("persistent batched step refuses a real plan")
    P = lib
    scans = _scans()[:2]
    solvers = _solvers(P, scans)
    desc = (P.pact.BatchScan * len(solvers))()
    for q, s in enumerate(solvers):
        desc[q] = P.GroupedBatchSolver._describe(s)
    plan, table = P.pact.batch_plan(desc)
    with pytest.raises(P.pact.PactError, match="status -4.*switched off"):
        P.pact.batch_step_persistent(plan, 0, True)
    solo = _solvers(P, scans)
    P.pact.batch_step(plan, 0, True)
    for s in solvers:
        s._cur = 1
    for s in solo:
        s.step()
    torch.cuda.synchronize()
    for a, b in zip(solvers, solo):
        assert torch.equal(a.sos, b.sos) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
