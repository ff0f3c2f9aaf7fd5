"""Learned warm start of the SOS optimisation: FP64 reference of the initialiser network, its loss and
gradients, its input preparation, and the synthetic channel model that builds its training set.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's method is self-supervised and uses no training data (Sec. 1, Sec. 3.3); this part is an
addition around it.  A small convolutional network maps the delay-and-sum stack (Eq. DAS) of a scan,
averaged down to the SOS node grid, to an SOS map that starts the plain optimisation of Eq. jr in place
of the uniform v0.  The network is trained on scans that the method's own forward model generates
(Eq. TOF for the arrival times, Eq. DAS for the stack).

Readings taken (none of this is in the paper):

* Network (8 convolutions, 64 channels): every convolution is 3 x 3, stride 1, zero padding 1, with a
  bias; ReLU after the first seven.  Resolution schedule with 2 x 2 average pooling on the way down,
  nearest-neighbour doubling on the way up, and additive skips:
      a1 = relu(c1(x)); a2 = relu(c2(a1)); p2 = pool(a2)
      a3 = relu(c3(p2)); a4 = relu(c4(a3)); p4 = pool(a4)
      a5 = relu(c5(p4)); u5 = up(a5) + a4
      a6 = relu(c6(u5)); u6 = up(a6) + a2
      a7 = relu(c7(u6)); z = c8(a7)
  Channel counts are padded to what the kernels take: the input has 16 channels (the stack's delays,
  then zeros) and c8 has 16 output channels of which only channel 0 is used (the other rows of its
  weights and bias stay zero).  Tensors are NHWC: [batch][row][column][channel].
* Weights W_l [co][ky][kx][ci] (tap (ky, kx) reads the input at row + ky - 1, column + kx - 1);
  parameter vector = W1, b1, W2, b2, ..., W8, b8, row-major.
* Output: SOS = v0 + s z[..., 0] with s = 0.05 mm/us; training loss = mean over the batch's free
  (masked) nodes of (z[..., 0] - t)^2 with t = (v_true - v0) / s.
* Precision on the device: BF16 weights and activations, FP32 accumulation and bias.  With
  ``bf16=True`` the forward pass here also rounds every stored activation (a_l, p_l, u_l, z) to the
  nearest bfloat16; the weights passed in are BF16 values.  float64 otherwise.
* Input: the stack's M images averaged over f x f pixel blocks (f = 4 takes the 560^2 image grid to
  the 140^2 SOS grid) and multiplied by a fixed scale.
* Channel model of the training scans: the arrival time of source b at element n is Eq. TOF along the
  straight ray, T = (|r_n - c_b| - w_bn) / v0 with w_bn the wavefront error of Eq. wf from c_b to r_n
  (because integral dl / v = (1 / v0) integral (1 - (1 - v0 / v)) dl); the trace is a sum of even
  Ricker pulses A_b (1 - u^2) exp(-u^2 / 2), u = v0 (t - T_bn) / sigma_b, over |u| <= 8.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as Fn

F64 = torch.float64

# (input channels, output channels, relu) of the eight convolutions
ARCH = ((16, 64, True), (64, 64, True), (64, 64, True), (64, 64, True),
        (64, 64, True), (64, 64, True), (64, 64, True), (64, 16, False))
OUT_SCALE = 0.05      # mm/us per unit of the network output


def layout():
    out = []
    for l, (ci, co, _) in enumerate(ARCH, start=1):
        out += [(f"W{l}", (co, 3, 3, ci)), (f"b{l}", (co,))]
    return out


def n_params() -> int:
    return sum(math.prod(s) for _, s in layout())


def unpack(params: torch.Tensor) -> dict:
    out, o = {}, 0
    for name, shape in layout():
        k = math.prod(shape)
        out[name] = params[o:o + k].reshape(shape)
        o += k
    assert o == params.numel()
    return out


def round_bf16(x: torch.Tensor) -> torch.Tensor:
    """Nearest bfloat16 (ties to even) of the float32 value, returned as float64.  Under reverse mode the
    rounding passes the gradient unchanged (x + (round(x) - x) with the difference held constant; the
    sum is exactly round(x) because the difference is exact)."""
    r = x.detach().to(torch.float32).to(torch.bfloat16).to(F64)
    return x + (r - x.detach()) if x.requires_grad else r


def conv3x3(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor | None) -> torch.Tensor:
    """y[n, r, c, o] = b[o] + sum_{ky, kx, i} W[o, ky, kx, i] x[n, r + ky - 1, c + kx - 1, i], zero outside.

    torch's conv2d (a cross-correlation) is the library routine for the sum; NHWC <-> NCHW around it."""
    y = Fn.conv2d(x.permute(0, 3, 1, 2), W.permute(0, 3, 1, 2), b, padding=1)
    return y.permute(0, 2, 3, 1)


def conv3x3_loops(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor | None) -> torch.Tensor:
    """The same sum written out with explicit shifts (for small cases)."""
    n, H, Wd, _ = x.shape
    co = W.shape[0]
    xp = torch.zeros(n, H + 2, Wd + 2, x.shape[3], dtype=x.dtype)
    xp[:, 1:H + 1, 1:Wd + 1] = x
    y = torch.zeros(n, H, Wd, co, dtype=x.dtype)
    for ky in range(3):
        for kx in range(3):
            y += torch.einsum("nrci,oi->nrco", xp[:, ky:ky + H, kx:kx + Wd], W[:, ky, kx, :])
    if b is not None:
        y += b
    return y


def pool2(a: torch.Tensor) -> torch.Tensor:
    """2 x 2 average (even sizes)."""
    n, H, W, C = a.shape
    return a.reshape(n, H // 2, 2, W // 2, 2, C).mean(dim=(2, 4))


def up2(a: torch.Tensor) -> torch.Tensor:
    """Nearest-neighbour doubling."""
    return a.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)


def forward(params: torch.Tensor, x: torch.Tensor, bf16: bool = False, keep: bool = False):
    """Network output z [n][H][W][16] for the input x [n][H][W][16] (H, W multiples of 4).  With
    keep=True also the dict of stored activations."""
    net = unpack(params)
    rnd = round_bf16 if bf16 else (lambda t: t)

    def conv(t, l, relu):
        y = conv3x3(t, net[f"W{l}"], net[f"b{l}"])
        return rnd(torch.relu(y) if relu else y)

    act = {}
    act["a1"] = conv(x, 1, True)
    act["a2"] = conv(act["a1"], 2, True)
    act["p2"] = rnd(pool2(act["a2"]))
    act["a3"] = conv(act["p2"], 3, True)
    act["a4"] = conv(act["a3"], 4, True)
    act["p4"] = rnd(pool2(act["a4"]))
    act["a5"] = conv(act["p4"], 5, True)
    act["u5"] = rnd(up2(act["a5"]) + act["a4"])
    act["a6"] = conv(act["u5"], 6, True)
    act["u6"] = rnd(up2(act["a6"]) + act["a2"])
    act["a7"] = conv(act["u6"], 7, True)
    z = conv(act["a7"], 8, False)
    return (z, act) if keep else z


def target(v_true: torch.Tensor, v0: float) -> torch.Tensor:
    return (v_true - v0) / OUT_SCALE


def loss(z: torch.Tensor, t: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """Mean over the batch's free nodes of (z[..., 0] - t)^2; t [n][H][W], mask [H][W] (1 = free)."""
    m = mask.to(F64)
    return (m * (z[..., 0] - t) ** 2).sum() / (z.shape[0] * m.sum())


def loss_and_grad(params: torch.Tensor, x: torch.Tensor, t: torch.Tensor, mask: torch.Tensor, bf16: bool = False):
    """Loss and its gradient with respect to the parameter vector, by reverse mode in float64.  With
    bf16=True the forward pass rounds its stored activations (the gradient passes each rounding as the
    identity, so it is the float64 gradient at the rounded activations)."""
    p = params.detach().clone().requires_grad_(True)
    L = loss(forward(p, x, bf16=bf16), t, mask)
    (g,) = torch.autograd.grad(L, p)
    return L.detach(), g


def conv_adjoints(x: torch.Tensor, W: torch.Tensor, g: torch.Tensor):
    """Adjoints of y = conv3x3(x, W, b) for the output gradient g: (dL/dx, dL/dW, dL/db), by reverse mode."""
    xx = x.detach().clone().requires_grad_(True)
    WW = W.detach().clone().requires_grad_(True)
    bb = torch.zeros(W.shape[0], dtype=F64, requires_grad=True)
    y = conv3x3(xx, WW, bb)
    return torch.autograd.grad(y, (xx, WW, bb), g)


def prepare_input(stack: torch.Tensor, factor: int, scale: float, channels: int = 16) -> torch.Tensor:
    """stack [M][H][W] -> [H/f][W/f][channels]: f x f block means times scale, zero channels beyond M."""
    M, H, W = stack.shape
    blk = stack.reshape(M, H // factor, factor, W // factor, factor).mean(dim=(2, 4)) * scale
    out = torch.zeros(H // factor, W // factor, channels, dtype=F64)
    out[..., :M] = blk.permute(1, 2, 0)
    return out


def arrival_times(w: torch.Tensor, sources: torch.Tensor, elements: torch.Tensor, v0: float) -> torch.Tensor:
    """T[b][n] = (|r_n - c_b| - w[b][n]) / v0 (Eq. TOF through Eq. wf)."""
    dist = torch.linalg.norm(elements[None, :, :] - sources[:, None, :], dim=-1)
    return (dist - w) / v0


def ricker_channels(T: torch.Tensor, amp: torch.Tensor, sigma: torch.Tensor, v0: float, n_t: int, fs: float,
                    t0: float = 0.0) -> torch.Tensor:
    """S[n][t] = sum_b A_b (1 - u^2) exp(-u^2 / 2) over |u| <= 8, u = v0 (t0 + t / fs - T[b][n]) / sigma_b."""
    n_src, n_elem = T.shape
    time = t0 + torch.arange(n_t, dtype=F64) / fs
    S = torch.zeros(n_elem, n_t, dtype=F64)
    for b in range(n_src):
        u = v0 * (time[None, :] - T[b][:, None]) / sigma[b]
        S += torch.where(u.abs() <= 8.0, amp[b] * (1 - u * u) * torch.exp(-0.5 * u * u), torch.zeros((), dtype=F64))
    return S
