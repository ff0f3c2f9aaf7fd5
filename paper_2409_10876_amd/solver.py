"""Optimisation of the pixel-grid and neural-field SOS (Sec. 3.3) on top of the libpact calls.

* ``prepare_scan``: channel data -> DAS stack -> windowed half spectra Y, once
  per scan (Eq. DAS, Eq. conv), resident in HBM for every step.
* ``PixelGridSolver``: one step = sos_to_delays -> loss_and_grad (fused
  Eq. TF + Eq. multi-deconv + Eq. jr and dL/dw) -> sos_to_delays_adjoint ->
  tv_adam_step, all on torch's current stream with preallocated
  buffers, so that a run of steps can be captured once into a HIP graph and
  replayed.
* ``SosLoss``: the data term of Eq. jr as a torch.autograd.Function whose
  backward is the library's hand-written adjoint (dL/dw is produced by the
  forward pass, which recomputes the transfer functions instead of storing
  them).
"""
from __future__ import annotations

import torch

from . import pact
from .pact import Geometry, F32


def geometry_from(cfg) -> Geometry:
    """Geometry from any object with the workload attributes (n_elem, radius, phi0, ny, nx, px, P, stride,
    fwhm, sos_n, sos_spacing)."""
    return Geometry(n_elem=cfg.n_elem, radius=float(cfg.radius), phi0=float(cfg.phi0), ny=cfg.ny, nx=cfg.nx,
                    px=float(cfg.px), P=cfg.P, stride=cfg.stride, fwhm=float(cfg.fwhm), sos_ny=cfg.sos_n,
                    sos_nx=cfg.sos_n, sos_spacing=float(cfg.sos_spacing))


class ScanData:
    """Device-resident data of one scan."""

    def __init__(self, geom: Geometry, S: torch.Tensor, delays: torch.Tensor, fs: float, t0: float, v0: float):
        self.geom = geom
        self.S = S
        self.d = delays
        self.fs, self.t0, self.v0 = fs, t0, v0
        self.centres = pact.patch_centres(geom, device=S.device)
        self.stack = None
        self.Y = None
        self.T = None

    @property
    def M(self) -> int:
        return self.d.numel()

    def prepare(self):
        """DAS stack, windowed half spectra and their step-invariant projections (once per scan)."""
        self.stack = pact.das_stack(self.S, self.fs, self.t0, self.geom, self.v0, self.d, out=self.stack)
        self.Y = pact.patch_fft(self.stack, self.geom, half=True, out=self.Y)
        self.T = pact.project_spectra(self.Y, self.geom, self.d, self.centres, out=self.T)
        return self.Y

    def use_spectra(self, Y):
        """Take given half spectra [N][M][P][P/2+1] (instead of the DAS stack's) and project them."""
        self.Y = Y
        self.T = pact.project_spectra(Y, self.geom, self.d, self.centres)
        return self

    def loss_and_grad(self, w, eps, **kw):
        """The fused data term and dL/dw at wavefront table w, from the projected spectra."""
        return pact.loss_and_grad_projected(self.T, self.M, w, self.centres, self.geom, eps, **kw)


def prepare_scan(cfg, S, delays, device="cuda") -> ScanData:
    g = geometry_from(cfg)
    S = torch.as_tensor(S, dtype=F32).to(device).contiguous()
    d = torch.as_tensor(delays, dtype=F32).to(device).contiguous()
    sd = ScanData(g, S, d, float(cfg.fs), float(cfg.t0), float(cfg.v0))
    sd.prepare()
    return sd


class PixelGridSolver:
    """Adam on the free nodes of the SOS grid; all state on the device."""

    def __init__(self, scan: ScanData, mask, eps: float, lam: float, lr: float, n_samples: int, sos_init=None,
                 b1=0.9, b2=0.999, adam_eps=1e-8, support_radius: float = 0.0):
        """support_radius: when the mask is the disc of free nodes within this radius (mm) of the origin, the
        ray kernels skip the samples that touch only fixed nodes (0: no such skipping)."""
        g = scan.geom
        dev = scan.S.device
        self.scan, self.g = scan, g
        self.eps, self.lam, self.lr, self.n_samples = float(eps), float(lam), float(lr), int(n_samples)
        self.support = float(support_radius)
        self.b1, self.b2, self.adam_eps = b1, b2, adam_eps
        self.mask = torch.as_tensor(mask, dtype=torch.uint8).to(dev).contiguous()
        v0 = scan.v0
        if sos_init is None:
            sos = torch.full((g.sos_ny, g.sos_nx), v0, dtype=F32, device=dev)
        else:
            sos = torch.as_tensor(sos_init, dtype=F32).to(dev).clone()
        sos = torch.where(self.mask.bool(), sos, torch.full_like(sos, v0))
        # two SOS buffers: the fused TV + Adam update reads one and writes the other; beside each, the staged
        # contrast grid of its SOS that the ray kernels copy (the fused update writes the next one)
        self._bufs = [sos.contiguous(), torch.empty_like(sos)]
        ns = pact.staged_contrast_floats(g)
        self._staged = [torch.empty(ns, dtype=F32, device=dev), torch.empty(ns, dtype=F32, device=dev)]
        self._cur = 0
        self._restage()
        self._graph_cur0 = 0
        self.m = torch.zeros_like(self.sos)
        self.v = torch.zeros_like(self.sos)
        self.t = torch.zeros(2, dtype=torch.int32, device=dev)
        N = scan.centres.shape[0]
        M = scan.d.numel()
        self.w = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.gw = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.grad = torch.empty_like(self.sos)
        self.loss = torch.zeros(1, dtype=F32, device=dev)
        self.ws_loss = torch.zeros(max(1, pact.loss_and_grad_workspace_size(N, M, g.P, g.n_elem)),
                                   dtype=torch.uint8, device=dev)
        self.ws_adj_bytes = pact.sos_to_delays_adjoint_workspace_size(g, N)
        self.ws_adj = torch.empty(max(1, self.ws_adj_bytes), dtype=torch.uint8, device=dev)
        self.graph = None
        self.graph_steps = 0

    @property
    def sos(self) -> torch.Tensor:
        """The current SOS node grid (read only: set it with set_sos)."""
        return self._bufs[self._cur]

    def set_sos(self, sos):
        """Replace the current SOS node grid (fixed nodes keep v0)."""
        v0 = self.scan.v0
        sos = torch.as_tensor(sos, dtype=F32).to(self.sos.device)
        self.sos.copy_(torch.where(self.mask.bool(), sos, torch.full_like(sos, v0)))
        self._restage()

    def _restage(self):
        pact.stage_contrast(self.sos, self.g, self.scan.v0, self.support, out=self._staged[self._cur])

    # one optimisation step (a2 -> a8), enqueued on the current stream
    def delays(self):
        pact.sos_to_delays(self.sos, self.g, self.scan.v0, self.scan.centres, self.n_samples, out=self.w,
                           support=self.support, staged=self._staged[self._cur])

    def loss_grad(self, with_loss=True):
        """with_loss False: only dL/dw (the scalar loss is formed on the steps whose loss is read)."""
        self.scan.loss_and_grad(self.w, self.eps, loss=self.loss, dL_dw=self.gw, ws=self.ws_loss, want_loss=with_loss)

    def adjoint(self):
        pact.sos_to_delays_adjoint(self.sos, self.g, self.scan.v0, self.scan.centres, self.n_samples, self.gw,
                                   out=self.grad, ws=self.ws_adj, support=self.support,
                                   staged=self._staged[self._cur])

    def regularise(self):
        """TV value and subgradient added to loss and grad (the separate form of the fused update)."""
        if self.lam != 0.0:
            pact.tv_grad(self.sos, self.mask, self.g, self.lam, self.grad, self.loss)

    def update(self):
        """Adam in place with grad as it stands (the separate form of the fused update)."""
        pact.adam_step(self.sos, self.m, self.v, self.t, self.mask, self.grad, self.lr, self.b1, self.b2,
                       self.adam_eps)
        self._restage()

    def tv_update(self, with_loss=True):
        """TV and Adam in one kernel, from the current buffer into the other one."""
        pact.tv_adam_step(self._bufs[self._cur], self._bufs[1 - self._cur], self.m, self.v, self.t, self.mask,
                          self.g, self.grad, self.lam, self.loss if with_loss else None, self.lr, self.b1, self.b2,
                          self.adam_eps)
        self._cur = 1 - self._cur
        self._restage()

    def adjoint_update(self, with_loss=True):
        """Ray adjoint, TV and Adam: two launches where the grid takes the whole-grid or banded adjoint (the
        partial grids' sum fused with TV and Adam), else the adjoint and the fused TV + Adam."""
        if self.ws_adj_bytes > 0:
            pact.sos_adjoint_tv_adam_step(self._bufs[self._cur], self._bufs[1 - self._cur], self.m, self.v, self.t,
                                          self.mask, self.g, self.scan.v0, self.scan.centres, self.n_samples, self.gw,
                                          self.lam, self.loss if with_loss else None, self.lr, self.b1, self.b2,
                                          self.adam_eps, support=self.support, grad=self.grad, ws=self.ws_adj,
                                          staged_in=self._staged[self._cur], staged_out=self._staged[1 - self._cur])
            self._cur = 1 - self._cur
        else:
            self.adjoint()
            self.tv_update(with_loss)

    def step(self, with_loss=True):
        """One step; with_loss False leaves `loss` as it was (the gradient and the update are the same)."""
        self.delays()
        self.loss_grad(with_loss)
        self.adjoint_update(with_loss)

    def autotune(self):
        """Time the ray tilings on this scan's geometry (at the current SOS and its loss gradient) and keep
        the fastest for every later step of scans of the same shape; call before capture()."""
        self.delays()
        self.loss_grad()
        return pact.rays_autotune(self.sos, self.g, self.scan.v0, self.scan.centres, self.n_samples, self.gw,
                                  self.w, self.grad, self.ws_adj, support=self.support)

    def capture(self, steps: int):
        """Capture `steps` (even) consecutive steps into one HIP graph (run one eager step first).  The
        steps alternate the two SOS buffers, so a replay starts and ends on the same one."""
        if steps % 2:
            raise ValueError("capture an even number of steps (the SOS buffers alternate)")
        self._graph_cur0 = self._cur
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for k in range(steps):
                    # the loss is formed on the last step of the graph only: a replay leaves the loss of its last
                    # step, the value a caller reads
                    self.step(with_loss=k == steps - 1)
        torch.cuda.current_stream().wait_stream(s)
        self.graph, self.graph_steps = g, steps
        return g

    def run(self, steps: int):
        """Advance `steps` steps, by graph replays where a captured graph divides the count."""
        if self.graph is not None and steps % self.graph_steps == 0:
            if self._cur != self._graph_cur0:         # an odd number of eager steps since the capture
                self._bufs[self._graph_cur0].copy_(self.sos)
                self._staged[self._graph_cur0].copy_(self._staged[self._cur])
                self._cur = self._graph_cur0
            for _ in range(steps // self.graph_steps):
                self.graph.replay()
        else:
            for _ in range(steps):
                self.step()


class SosLoss(torch.autograd.Function):
    """Data term of Eq. jr as a function of the SOS node grid; backward by the library's adjoint."""

    @staticmethod
    def forward(ctx, sos, scan: ScanData, eps: float, n_samples: int):
        g = scan.geom
        sos = sos.contiguous()
        w = pact.sos_to_delays(sos, g, scan.v0, scan.centres, n_samples)
        loss, gw = scan.loss_and_grad(w, eps)
        ctx.save_for_backward(sos, gw)
        ctx.scan, ctx.n_samples = scan, n_samples
        return loss.view(())

    @staticmethod
    def backward(ctx, gout):
        sos, gw = ctx.saved_tensors
        scan = ctx.scan
        scale = gout.reshape(1).to(F32).contiguous()
        grad = pact.sos_to_delays_adjoint(sos, scan.geom, scan.v0, scan.centres, ctx.n_samples, gw, scale=scale)
        return grad, None, None, None


class NeuralFieldSolver:
    """Adam on the parameters of the neural-field SOS (coordinate network of Sec. 3.3); all state on the
    device.  One step = pack the BF16 weights -> delays through the network at every ray sample -> fused
    deconvolution loss and dL/dw -> network adjoint -> Adam."""

    def __init__(self, scan: ScanData, B, params, net: "pact.NfNet", lr: float, eps: float, n_samples: int,
                 b1=0.9, b2=0.999, adam_eps=1e-8, store_activations: bool = True):
        g = scan.geom
        dev = scan.S.device
        self.scan, self.g, self.net = scan, g, net
        self.lr, self.eps, self.n_samples = float(lr), float(eps), int(n_samples)
        self.b1, self.b2, self.adam_eps = b1, b2, adam_eps
        self.B = torch.as_tensor(B, dtype=F32).to(dev).contiguous()
        self.params = torch.as_tensor(params, dtype=F32).to(dev).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = torch.zeros(2, dtype=torch.int32, device=dev)
        self.packed = pact.nf_pack(self.params, net)
        N = scan.centres.shape[0]
        M = scan.d.numel()
        self.w = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.gw = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.grad = torch.empty_like(self.params)
        self.loss = torch.zeros(1, dtype=F32, device=dev)
        self.ws_loss = torch.zeros(max(1, pact.loss_and_grad_workspace_size(N, M, g.P, g.n_elem)),
                                   dtype=torch.uint8, device=dev)
        self.ws_nf = torch.empty(max(1, pact.nf_sos_to_delays_adjoint_workspace_size(net)), dtype=torch.uint8,
                                 device=dev)
        # every sample's activations from the forward pass, read back by the adjoint (else it recomputes them)
        self.act = (torch.empty(pact.nf_activation_bytes(N, g, self.n_samples), dtype=torch.uint8, device=dev)
                    if store_activations else None)

    def pack(self):
        pact.nf_pack(self.params, self.net, out=self.packed)

    def delays(self):
        pact.nf_sos_to_delays(self.B, self.params, self.packed, self.net, self.scan.v0, self.scan.centres, self.g,
                              self.n_samples, out=self.w, act=self.act)

    def loss_grad(self):
        self.scan.loss_and_grad(self.w, self.eps, loss=self.loss, dL_dw=self.gw, ws=self.ws_loss)

    def adjoint(self):
        pact.nf_sos_to_delays_adjoint(self.B, self.params, self.packed, self.net, self.scan.v0, self.scan.centres,
                                      self.g, self.n_samples, self.gw, out=self.grad, ws=self.ws_nf, act=self.act)

    def update(self):
        pact.adam_step(self.params, self.m, self.v, self.t, None, self.grad, self.lr, self.b1, self.b2,
                       self.adam_eps)

    def step(self):
        self.pack()
        self.delays()
        self.loss_grad()
        self.adjoint()
        self.update()


class SirenSolver:
    """The paper's neural-field form (Sec. 3.3): Adam on the 1027 parameters of a sinusoidal network on the
    SOS-grid nodes; each step evaluates the network on the nodes, then runs the pixel-grid path (rays, fused
    loss, ray adjoint) and the network's adjoint.  No TV (the paper sets lambda = 0 for the neural field)."""

    def __init__(self, scan: ScanData, mask, params, hidden: int, omega0: float, mask_radius: float, lr: float,
                 eps: float, n_samples: int, b1=0.9, b2=0.999, adam_eps=1e-8, support_radius: float = 0.0):
        g = scan.geom
        dev = scan.S.device
        self.scan, self.g = scan, g
        self.hidden, self.omega0, self.rho = int(hidden), float(omega0), float(mask_radius)
        self.support = float(support_radius)
        self.lr, self.eps, self.n_samples = float(lr), float(eps), int(n_samples)
        self.b1, self.b2, self.adam_eps = b1, b2, adam_eps
        self.mask = torch.as_tensor(mask, dtype=torch.uint8).to(dev).contiguous()
        self.params = torch.as_tensor(params, dtype=F32).to(dev).contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = torch.zeros(2, dtype=torch.int32, device=dev)
        self.sos = torch.empty(g.sos_ny, g.sos_nx, dtype=F32, device=dev)
        self.staged = torch.empty(pact.staged_contrast_floats(g), dtype=F32, device=dev)
        N = scan.centres.shape[0]
        M = scan.d.numel()
        self.w = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.gw = torch.empty(N, g.n_elem, dtype=F32, device=dev)
        self.grad_sos = torch.empty_like(self.sos)
        self.grad = torch.empty_like(self.params)
        self.loss = torch.zeros(1, dtype=F32, device=dev)
        self.ws_loss = torch.zeros(max(1, pact.loss_and_grad_workspace_size(N, M, g.P, g.n_elem)),
                                   dtype=torch.uint8, device=dev)
        self.ws_adj = torch.empty(max(1, pact.sos_to_delays_adjoint_workspace_size(g, N)), dtype=torch.uint8,
                                  device=dev)
        self.ws_net = torch.empty(max(1, int(pact.load().pact_siren_sos_adjoint_workspace_size(g.sosg,
                                                                                               self.hidden))),
                                  dtype=torch.uint8, device=dev)
        self.graph = None
        self.graph_steps = 0

    def sos_grid(self):
        """The node SOS from the network, and its staged contrast (formed once for both ray kernels)."""
        pact.siren_sos(self.params, self.hidden, self.omega0, self.mask, self.g, self.rho, self.scan.v0,
                       out=self.sos)
        pact.stage_contrast(self.sos, self.g, self.scan.v0, support=self.support, out=self.staged)

    def delays(self):
        pact.sos_to_delays(self.sos, self.g, self.scan.v0, self.scan.centres, self.n_samples, out=self.w,
                           support=self.support, staged=self.staged)

    def loss_grad(self):
        self.scan.loss_and_grad(self.w, self.eps, loss=self.loss, dL_dw=self.gw, ws=self.ws_loss)

    def adjoint(self):
        pact.sos_to_delays_adjoint(self.sos, self.g, self.scan.v0, self.scan.centres, self.n_samples, self.gw,
                                   out=self.grad_sos, ws=self.ws_adj, support=self.support, staged=self.staged)
        pact.siren_sos_adjoint(self.params, self.hidden, self.omega0, self.mask, self.g, self.rho, self.grad_sos,
                               out=self.grad, ws=self.ws_net)

    def update(self):
        pact.adam_step(self.params, self.m, self.v, self.t, None, self.grad, self.lr, self.b1, self.b2,
                       self.adam_eps)

    def step(self):
        self.sos_grid()
        self.delays()
        self.loss_grad()
        self.adjoint()
        self.update()

    def capture(self, steps: int):
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    self.step()
        torch.cuda.current_stream().wait_stream(s)
        self.graph, self.graph_steps = g, steps
        return g

    def run(self, steps: int):
        if self.graph is not None and steps % self.graph_steps == 0:
            for _ in range(steps // self.graph_steps):
                self.graph.replay()
        else:
            for _ in range(steps):
                self.step()


class BatchedSolver:
    """Independent scans solved together (many reconstructions at once): one PixelGridSolver per scan, each
    with its own captured step graph, replayed on its own HIP stream so that the scans' kernels overlap and
    fill the chip where one scan's small kernels and tails would leave it idle.  Each scan's results are the
    ones it gets alone (the kernels are deterministic and share no buffers)."""

    def __init__(self, solvers, graph_steps: int = 10, autotune: bool = False):
        self.solvers = list(solvers)
        self.graph_steps = graph_steps
        self.streams = [torch.cuda.Stream() for _ in self.solvers]
        # ray tilings timed per scan shape before the graphs record them
        self.tilings = [s.autotune() for s in self.solvers] if autotune else None
        for s in self.solvers:
            s.step()
        torch.cuda.synchronize()
        for s in self.solvers:
            s.capture(graph_steps)
        torch.cuda.synchronize()

    def run(self, steps: int):
        """Advance every scan by `steps` (a multiple of graph_steps), all scans concurrently."""
        cur = torch.cuda.current_stream()
        for s, st in zip(self.solvers, self.streams):
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                s.run(steps)
        for st in self.streams:
            cur.wait_stream(st)

    def run_sequential(self, steps: int):
        """The same work, one scan after another on the current stream (the reference for the overlap)."""
        for s in self.solvers:
            s.run(steps)


class GroupedBatchSolver:
    """Independent scans advanced together with one launch per stage over all scans of a group
    (pact_batch_step): five launches per step for the whole group instead of five per scan.  Each scan keeps
    its own buffers (those of its PixelGridSolver) and the partition of work it has alone, so its states equal,
    bit for bit, those it reaches alone.  With groups > 1 the scans are dealt to that many groups of about
    equal work (largest first), each group with its own plan and graph replayed on its own stream, so that one
    group's stages overlap another's.  With persistent=True each group's step is one launch that takes the
    stages' blocks from a queue (pact_batch_step_persistent).  Every scan must take the whole-grid or banded
    adjoint."""

    def __init__(self, solvers, graph_steps: int = 10, autotune: bool = False, groups: int = 1,
                 persistent: bool = False):
        self.solvers = list(solvers)
        self.graph_steps = graph_steps
        self._step_fn = pact.batch_step_persistent if persistent else pact.batch_step
        if any(s.ws_adj_bytes == 0 for s in self.solvers):
            raise ValueError("a scan takes the tiled adjoint, which the batched step does not run")
        # ray tilings timed per scan shape before the plan records them
        self.tilings = [s.autotune() for s in self.solvers] if autotune else None
        for s in self.solvers:               # every scan starts on its buffer 0 (the plan's parity 0)
            if s._cur != 0:
                s._bufs[0].copy_(s._bufs[s._cur])
                s._staged[0].copy_(s._staged[s._cur])
                s._cur = 0
        work = [s.scan.centres.shape[0] * s.g.n_elem * s.n_samples for s in self.solvers]
        n_groups = max(1, min(groups, len(self.solvers)))
        members, load = [[] for _ in range(n_groups)], [0] * n_groups
        for k in sorted(range(len(self.solvers)), key=lambda k: -work[k]):
            j = load.index(min(load))
            members[j].append(k)
            load[j] += work[k]
        self.groups = []
        for ks in members:
            scans = (pact.BatchScan * len(ks))()
            for q, k in enumerate(ks):
                scans[q] = self._describe(self.solvers[k])
            plan, table = pact.batch_plan(scans)
            self.groups.append({"members": ks, "scans": scans, "plan": plan, "table": table, "graph": None,
                                "stream": torch.cuda.Stream()})
        self.parity = 0
        self.step()
        torch.cuda.synchronize()
        self.capture(graph_steps)
        torch.cuda.synchronize()

    @staticmethod
    def _describe(s: "PixelGridSolver") -> "pact.BatchScan":
        g, sd = s.g, s.scan
        ptr = lambda t: t.data_ptr()  # noqa: E731
        d = pact.BatchScan()
        d.sosg, d.ring = g.sosg, g.ring
        d.N, d.M, d.P, d.n_samples = sd.centres.shape[0], sd.M, g.P, s.n_samples
        d.px, d.v0, d.support_radius, d.eps = g.px, sd.v0, s.support, s.eps
        d.lam, d.lr, d.b1, d.b2, d.adam_eps = s.lam, s.lr, s.b1, s.b2, s.adam_eps
        d.centres, d.T, d.w, d.dL_dw = ptr(sd.centres), ptr(sd.T), ptr(s.w), ptr(s.gw)
        d.patch_loss, d.loss = ptr(s.ws_loss), ptr(s.loss)
        d.sos[0], d.sos[1] = ptr(s._bufs[0]), ptr(s._bufs[1])
        d.staged[0], d.staged[1] = ptr(s._staged[0]), ptr(s._staged[1])
        d.m, d.v, d.t, d.mask, d.grad = ptr(s.m), ptr(s.v), ptr(s.t), ptr(s.mask), ptr(s.grad)
        d.partial, d.partial_bytes = ptr(s.ws_adj), s.ws_adj.numel()
        return d

    def _flip(self):
        self.parity ^= 1
        for s in self.solvers:
            s._cur = self.parity

    def step(self, with_loss: bool = True):
        """One step of every scan, every group on the current stream."""
        for gr in self.groups:
            self._step_fn(gr["plan"], self.parity, with_loss)
        self._flip()

    def capture(self, steps: int):
        """Capture `steps` (even) batched steps of each group into a HIP graph of its own; the scalar losses on
        the last step only."""
        if steps % 2:
            raise ValueError("capture an even number of steps (the SOS buffers alternate)")
        p0 = self.parity
        for gr in self.groups:
            g = torch.cuda.CUDAGraph()
            st = torch.cuda.Stream()
            st.wait_stream(torch.cuda.current_stream())
            par = p0
            with torch.cuda.stream(st):
                with torch.cuda.graph(g, stream=st):
                    for k in range(steps):
                        self._step_fn(gr["plan"], par, k == steps - 1)
                        par ^= 1
            torch.cuda.current_stream().wait_stream(st)
            gr["graph"] = g
        self.parity = p0                      # capturing does not run the steps
        for s in self.solvers:
            s._cur = p0

    def run(self, steps: int):
        """Advance every scan by `steps` steps: graph replays (each group on its own stream) where the captured
        graphs divide the count, else eager steps."""
        if all(gr["graph"] is not None for gr in self.groups) and steps % self.graph_steps == 0:
            cur = torch.cuda.current_stream()
            for gr in self.groups:
                gr["stream"].wait_stream(cur)
                with torch.cuda.stream(gr["stream"]):
                    for _ in range(steps // self.graph_steps):
                        gr["graph"].replay()
            for gr in self.groups:
                cur.wait_stream(gr["stream"])
        else:
            for _ in range(steps):
                self.step()

