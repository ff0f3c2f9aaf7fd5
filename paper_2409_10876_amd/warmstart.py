"""Learned warm start of the SOS optimisation.

The paper's method is self-supervised and needs no training data (Sec. 3.3).  This module adds a small
convolutional network that maps a scan's delay-and-sum stack (Eq. DAS), averaged down to the SOS node
grid, to a starting SOS for the plain optimisation of Eq. jr.  The plain optimisation from the uniform
v0 stays the fallback and the reference the result is compared with: the warm start only changes where it
begins.

* ``WarmStartNet``: the network (8 convolutions of 3 x 3, 64 channels, two 2 x 2 poolings, two
  nearest-neighbour doublings with additive skips), BF16 activations on MFMA with FP32 accumulation,
  its hand-written backward pass and an Adam step, all through libpact calls on torch's current stream.
* ``ScanSimulator``: training and evaluation scans from the method's own forward model: the SOS node
  grid -> wavefront errors from every source (pact_sos_to_delays, Eq. wf) -> arrival times (Eq. TOF) and
  Ricker channel data (pact_ricker_channels) -> delay-and-sum stack (pact_das_stack) -> network input.
* ``save`` / ``load_params``: the trained parameters and the input scale in a safetensors file.

Parameter vector (float32): for each convolution l = 1..8, W_l [co][3][3][ci] then b_l [co], with the
channel counts of ``ARCH``.  The input has 16 channels (the stack's delays, then zeros) and the last layer
16 outputs of which only channel 0 is used; the weights of the unused channels start at zero and, their
gradients being zero, stay there.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import pact
from .pact import BF16, F32

# (input channels, output channels, relu) of the eight convolutions
ARCH = ((16, 64, True), (64, 64, True), (64, 64, True), (64, 64, True),
        (64, 64, True), (64, 64, True), (64, 64, True), (64, 16, False))
IN_CHANNELS = 16
OUT_SCALE = 0.05          # mm/us of SOS per unit of network output
FACTOR = 4                # image pixels per SOS node along each axis


def param_layout():
    """[(offset of W_l, offset of b_l, ci, co)] and the total count."""
    out, o = [], 0
    for ci, co, _ in ARCH:
        out.append((o, o + co * 9 * ci, ci, co))
        o += co * 9 * ci + co
    return out, o


LAYOUT, N_PARAMS = param_layout()


def init_params(n_inputs: int, seed: int = 0) -> np.ndarray:
    """He-uniform weights over the real fan-in (n_inputs input channels for the first layer, one output
    channel for the last), zero biases, zero weights on the padded channels."""
    rng = np.random.default_rng(3000 + seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    for l, (ow, ob, ci, co) in enumerate(LAYOUT):
        ci_real = n_inputs if l == 0 else ci
        co_real = 1 if l == len(LAYOUT) - 1 else co
        lim = math.sqrt(6.0 / (9 * ci_real)) * (0.1 if l == len(LAYOUT) - 1 else 1.0)
        W = np.zeros((co, 3, 3, ci), dtype=np.float32)
        W[:co_real, :, :, :ci_real] = rng.uniform(-lim, lim, (co_real, 3, 3, ci_real))
        p[ow:ob] = W.reshape(-1)
    return p


class WarmStartNet:
    """The initialiser on one device, with buffers for up to `batch` images of H x W nodes (multiples of 4)."""

    def __init__(self, batch: int, H: int, W: int, params=None, n_inputs: int = 11, device="cuda", seed: int = 0):
        if H % 4 or W % 4:
            raise ValueError("H and W must be multiples of 4 (two poolings)")
        self.batch, self.H, self.W = int(batch), int(H), int(W)
        dev = torch.device(device)
        self.device = dev
        p = init_params(n_inputs, seed) if params is None else params
        self.params = torch.as_tensor(p, dtype=F32).to(dev).contiguous().clone()
        if self.params.numel() != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters, got {self.params.numel()}")
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = torch.zeros(2, dtype=torch.int32, device=dev)
        self.packed = [(torch.empty(pact.conv3x3_packed_count(ci, co), dtype=BF16, device=dev),
                        torch.empty(pact.conv3x3_packed_count(co, ci), dtype=BF16, device=dev))
                       for (_, _, ci, co) in LAYOUT]
        self.pack()
        B, h, w = self.batch, self.H, self.W

        def buf(s, c=64):
            return torch.empty(B, h // s, w // s, c, dtype=BF16, device=dev)

        # forward activations (kept for the backward pass)
        self.a1, self.a2, self.u6, self.a7 = buf(1), buf(1), buf(1), buf(1)
        self.p2, self.a3, self.a4, self.u5, self.a6 = buf(2), buf(2), buf(2), buf(2), buf(2)
        self.p4, self.a5 = buf(4), buf(4)
        self.z = buf(1, ARCH[-1][1])
        # backward buffers
        self.gz = buf(1, ARCH[-1][1])
        self.gf = [buf(1), buf(1), buf(1)]
        self.gh = [buf(2), buf(2), buf(2)]
        self.gq = [buf(4), buf(4)]
        self.loss = torch.zeros(1, dtype=F32, device=dev)
        need = max(pact.conv3x3_wgrad_workspace_size(B, h // s, w // s, ci, co)
                   for s in (1, 2, 4) for (_, _, ci, co) in LAYOUT)
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.ws_loss = torch.empty(max(1, pact.warm_loss_workspace_size(B, h, w)), dtype=torch.uint8, device=dev)

    # ---- parameters ----
    def weights(self, l: int):
        ow, ob, ci, co = LAYOUT[l]
        return self.params[ow:ob].view(co, 3, 3, ci), self.params[ob:ob + co]

    def grad_slice(self, l: int):
        ow, ob, ci, co = LAYOUT[l]
        return self.grad[ow:ob + co]

    def pack(self):
        for l, (fwd, adj) in enumerate(self.packed):
            _, _, ci, co = LAYOUT[l]
            pact.conv3x3_pack(self.weights(l)[0], ci, co, packed=fwd, packed_adjoint=adj)

    # ---- forward / backward ----
    def _conv(self, l, x, out, relu=None):
        _, _, ci, co = LAYOUT[l]
        return pact.conv3x3(x, self.packed[l][0], co, bias=self.weights(l)[1],
                            relu=ARCH[l][2] if relu is None else relu, out=out)

    def _conv_adj(self, l, g, out, mask=None):
        _, _, ci, co = LAYOUT[l]
        return pact.conv3x3(g, self.packed[l][1], ci, mask=mask, out=out)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x [n][H][W][16] bf16 (n <= batch) -> z [n][H][W][16] bf16 (channel 0 is the output)."""
        n = x.shape[0]
        if n > self.batch or tuple(x.shape[1:]) != (self.H, self.W, IN_CHANNELS):
            raise ValueError(f"input shape {tuple(x.shape)} does not fit the network's buffers")
        a1, a2, p2, a3, a4 = self.a1[:n], self.a2[:n], self.p2[:n], self.a3[:n], self.a4[:n]
        p4, a5, u5, a6, u6, a7, z = self.p4[:n], self.a5[:n], self.u5[:n], self.a6[:n], self.u6[:n], self.a7[:n], self.z[:n]
        self._conv(0, x, a1)
        self._conv(1, a1, a2)
        pact.pool2(a2, out=p2)
        self._conv(2, p2, a3)
        self._conv(3, a3, a4)
        pact.pool2(a4, out=p4)
        self._conv(4, p4, a5)
        pact.up2_add(a5, a4, out=u5)
        self._conv(5, u5, a6)
        pact.up2_add(a6, a2, out=u6)
        self._conv(6, u6, a7)
        self._conv(7, a7, z)
        return z

    def backward(self, x: torch.Tensor, gz: torch.Tensor):
        """Parameter gradient (into self.grad) for the output gradient gz [n][H][W][16], after forward(x)."""
        n = x.shape[0]
        a1, a2, p2, a3, a4 = self.a1[:n], self.a2[:n], self.p2[:n], self.a3[:n], self.a4[:n]
        p4, a5, u5, a6, u6, a7 = self.p4[:n], self.a5[:n], self.u5[:n], self.a6[:n], self.u6[:n], self.a7[:n]
        fA, fB, fC = (t[:n] for t in self.gf)
        hA, hB, hC = (t[:n] for t in self.gh)
        qA, qB = (t[:n] for t in self.gq)
        wg = lambda l, inp, g: pact.conv3x3_wgrad(inp, g, out=self.grad_slice(l), ws=self.ws)  # noqa: E731
        wg(7, a7, gz)
        g7 = self._conv_adj(7, gz, fA, mask=a7)            # dL/d(pre-activation of layer 7)
        wg(6, u6, g7)
        g_u6 = self._conv_adj(6, g7, fB)                    # dL/du6 (also the skip's gradient into a2)
        g6 = pact.up2_add_adjoint(g_u6, mask_low=a6, out=hA)
        wg(5, u5, g6)
        g_u5 = self._conv_adj(5, g6, hB)                    # dL/du5 (also the skip's gradient into a4)
        g5 = pact.up2_add_adjoint(g_u5, mask_low=a5, out=qA)
        wg(4, p4, g5)
        g_p4 = self._conv_adj(4, g5, qB)
        g4 = pact.pool2_adjoint(g_p4, skip=g_u5, mask=a4, out=hC)
        wg(3, a3, g4)
        g3 = self._conv_adj(3, g4, hA, mask=a3)
        wg(2, p2, g3)
        g_p2 = self._conv_adj(2, g3, hB)
        g2 = pact.pool2_adjoint(g_p2, skip=g_u6, mask=a2, out=fA)
        wg(1, a1, g2)
        g1 = self._conv_adj(1, g2, fC, mask=a1)
        wg(0, x, g1)
        return self.grad

    def loss_grad(self, x, target, mask, n_free: int):
        """Forward, the mean squared error over the free nodes (target in output units) and its gradient."""
        n = x.shape[0]
        z = self.forward(x)
        gz = self.gz[:n]
        pact.warm_loss(z, target, mask, 1.0 / (n * n_free), loss=self.loss, g=gz, ws=self.ws_loss)
        self.backward(x, gz)
        return self.loss

    def loss_only(self, x, target, mask, n_free: int):
        """Forward and the mean squared error (no backward pass)."""
        n = x.shape[0]
        z = self.forward(x)
        pact.warm_loss(z, target, mask, 1.0 / (n * n_free), loss=self.loss, g=self.gz[:n], ws=self.ws_loss)
        return self.loss

    def train_step(self, x, target, mask, n_free: int, lr: float):
        self.loss_grad(x, target, mask, n_free)
        pact.adam_step(self.params, self.m, self.v, self.t, None, self.grad, lr)
        self.pack()
        return self.loss

    def predict_sos(self, x, mask, v0: float, out=None):
        """SOS node grids [n][H][W]: v0 + OUT_SCALE z on the free nodes, v0 elsewhere."""
        z = self.forward(x)
        return pact.warm_sos(z, mask, v0, OUT_SCALE, out=out)


class ScanSimulator:
    """Scans of a fixed geometry from the method's own forward model (see the module docstring)."""

    def __init__(self, geom: pact.Geometry, delays, fs: float, n_t: int, t0: float, v0: float,
                 n_samples: int = 512, device="cuda"):
        self.g = geom
        self.d = torch.as_tensor(delays, dtype=F32).to(device).contiguous()
        self.fs, self.n_t, self.t0, self.v0, self.n_samples = float(fs), int(n_t), float(t0), float(v0), int(n_samples)
        self.device = torch.device(device)
        self.S = torch.empty(geom.n_elem, self.n_t, dtype=F32, device=self.device)
        self.stack = torch.empty(self.d.numel(), geom.ny, geom.nx, dtype=F32, device=self.device)

    def channels(self, sos, blobs):
        """Channel data [n_elem][n_t] of the blobs [n][4] (x, y, sigma, amp) through the SOS node grid."""
        src = blobs[:, :2].contiguous()
        w = pact.sos_to_delays(sos, self.g, self.v0, src, self.n_samples)
        return pact.ricker_channels(w, src, blobs[:, 3].contiguous(), blobs[:, 2].contiguous(), self.g, self.v0,
                                    self.n_t, self.fs, self.t0, out=self.S)

    def das(self, sos, blobs):
        self.channels(sos, blobs)
        return pact.das_stack(self.S, self.fs, self.t0, self.g, self.v0, self.d, out=self.stack)

    def network_input(self, stack, scale: float, out=None):
        return pact.warm_input(stack, FACTOR, scale, IN_CHANNELS, out=out)


def input_scale(sim: ScanSimulator, sos_list, blob_list) -> float:
    """1 / RMS of the averaged stacks of a few scans (fixed for the life of a trained network)."""
    acc, cnt = 0.0, 0
    for sos, blobs in zip(sos_list, blob_list):
        x = sim.network_input(sim.das(sos, blobs), 1.0).float()
        acc += float((x[..., :sim.d.numel()] ** 2).sum())
        cnt += x[..., :sim.d.numel()].numel()
    return 1.0 / math.sqrt(acc / cnt)


def save(path: str, params: torch.Tensor, scale: float, meta: dict | None = None):
    from safetensors.torch import save_file
    md = {"input_scale": repr(float(scale)), "n_params": str(N_PARAMS)}
    md.update({k: str(v) for k, v in (meta or {}).items()})
    save_file({"params": params.detach().float().cpu().contiguous()}, path, metadata=md)


def load_params(path: str):
    """(params float32 numpy, input scale, metadata)."""
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        md = f.metadata()
        p = f.get_tensor("params").numpy()
    return p, float(md["input_scale"]), md


def now() -> float:
    torch.cuda.synchronize()
    return time.perf_counter()
