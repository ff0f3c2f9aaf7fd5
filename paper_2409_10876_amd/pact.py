"""Thin ctypes binding of libpact (see include/pact.h for every call's contract).

Argument marshalling only: each function checks tensor devices, dtypes,
shapes and contiguity, passes raw device pointers and torch's current HIP
stream, and raises PactError on a negative status.  All arithmetic runs in
the library's HIP kernels.  torch is imported first so that the library binds
to the same HIP runtime as torch.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpact.so")


class PactError(RuntimeError):
    pass


class Ring(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int), ("radius", ctypes.c_float), ("phi0", ctypes.c_float)]


class Grid(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int), ("nx", ctypes.c_int), ("spacing", ctypes.c_float)]


class Patches(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int), ("stride", ctypes.c_int), ("fwhm", ctypes.c_float)]


_P = ctypes.c_void_p


class BatchScan(ctypes.Structure):
    """pact_batch_scan (include/pact.h): one scan of a batched solve."""
    _fields_ = [("sosg", Grid), ("ring", Ring), ("N", ctypes.c_int), ("M", ctypes.c_int), ("P", ctypes.c_int),
                ("n_samples", ctypes.c_int), ("px", ctypes.c_float), ("v0", ctypes.c_float),
                ("support_radius", ctypes.c_float), ("eps", ctypes.c_float), ("lam", ctypes.c_float),
                ("lr", ctypes.c_float), ("b1", ctypes.c_float), ("b2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("centres", ctypes.c_void_p), ("T", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("dL_dw", ctypes.c_void_p), ("patch_loss", ctypes.c_void_p), ("loss", ctypes.c_void_p),
                ("sos", ctypes.c_void_p * 2), ("staged", ctypes.c_void_p * 2), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("t", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("partial", ctypes.c_void_p), ("partial_bytes", ctypes.c_size_t)]
# geometry structs are passed by pointer (passing small float-bearing structs by value through libffi is not
# reliable); ctypes applies byref() to a struct instance given for a POINTER argument
_PRING = ctypes.POINTER(Ring)
_PGRID = ctypes.POINTER(Grid)
_PPATCH = ctypes.POINTER(Patches)
_I = ctypes.c_int
_F = ctypes.c_float
_Z = ctypes.c_size_t

_SIGS = {
    "pact_batch_plan_bytes": (_Z, [_I]),
    "pact_batch_table_bytes": (_Z, [_I]),
    "pact_batch_plan": (_I, [_P, _I, _P, _Z, _P, _Z, _P]),
    "pact_batch_step": (_I, [_P, _I, _I, _P]),
    "pact_batch_step_persistent": (_I, [_P, _I, _I, _P]),
    "pact_last_error": (ctypes.c_char_p, []),
    "pact_version": (_I, []),
    "pact_patch_count": (_I, [_PGRID, _PPATCH, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "pact_patch_centres": (_I, [_PGRID, _PPATCH, _P]),
    "pact_das_stack": (_I, [_P, _I, _F, _F, _PRING, _F, _P, _I, _PGRID, _P, _P]),
    "pact_patch_fft": (_I, [_P, _I, _PGRID, _PPATCH, _I, _P, _P]),
    "pact_ifft2_real": (_I, [_P, _I, _I, _P, _P]),
    "pact_sos_to_delays": (_I, [_P, _PGRID, _F, _P, _I, _PRING, _I, _F, _P, _P, _P]),
    "pact_staged_contrast_floats": (_Z, [_PGRID]),
    "pact_stage_contrast": (_I, [_P, _PGRID, _F, _F, _P, _P]),
    "pact_sos_to_delays_adjoint_workspace_size": (_Z, [_PGRID, _I, _PRING]),
    "pact_sos_to_delays_adjoint": (_I, [_P, _PGRID, _F, _P, _I, _PRING, _I, _F, _P, _P, _P, _P, _I, _P, _Z, _P]),
    "pact_delays_to_psf": (_I, [_P, _P, _I, _PRING, _P, _I, _I, _F, _P, _P, _P]),
    "pact_delays_to_psf_adjoint": (_I, [_P, _P, _I, _PRING, _P, _I, _I, _F, _P, _P, _P]),
    "pact_multichannel_deconv": (_I, [_P, _P, _I, _I, _I, _F, _P, _P]),
    "pact_multichannel_deconv_adjoint": (_I, [_P, _P, _I, _I, _I, _F, _P, _P, _P]),
    "pact_residual_loss_workspace_size": (_Z, [_I, _I]),
    "pact_residual_loss": (_I, [_P, _P, _P, _I, _I, _I, _F, _P, _P, _P, _P, _Z, _P]),
    "pact_loss_and_grad_workspace_size": (_Z, [_I, _I, _I, _I]),
    "pact_loss_and_grad": (_I, [_P, _P, _P, _I, _PRING, _P, _I, _I, _F, _F, _P, _P, _P, _P, _Z, _P]),
    "pact_projected_spectra_floats": (_Z, [_I, _I]),
    "pact_project_spectra": (_I, [_P, _I, _I, _I, _F, _P, _P, _PRING, _P, _P]),
    "pact_loss_and_grad_projected": (_I, [_P, _P, _P, _I, _PRING, _I, _I, _F, _F, _P, _P, _P, _P, _Z, _P]),
    "pact_loss_and_grad_noalloc": (_I, [_P, _P, _P, _I, _PRING, _P, _I, _I, _F, _F, _P, _P, _P, _P]),
    "pact_tv_grad": (_I, [_P, _P, _PGRID, _F, _P, _P, _P]),
    "pact_adam_step": (_I, [_P, _P, _P, _P, _P, _I, _P, _F, _F, _F, _F, _P]),
    "pact_stitch": (_I, [_P, _I, _PGRID, _PPATCH, _P, _P]),
    "pact_siren_sos": (_I, [_P, _I, _F, _P, _PGRID, _F, _F, _P, _P]),
    "pact_siren_sos_adjoint_workspace_size": (_Z, [_PGRID, _I]),
    "pact_siren_sos_adjoint": (_I, [_P, _I, _F, _P, _PGRID, _F, _P, _P, _P, _Z, _P]),
    "pact_tv_adam_step": (_I, [_P, _P, _P, _P, _P, _P, _PGRID, _P, _F, _P, _F, _F, _F, _F, _P]),
    "pact_sos_adjoint_tv_adam_step": (_I, [_P, _P, _P, _P, _P, _P, _PGRID, _F, _P, _I, _PRING, _I, _F, _P, _P, _P,
                                           _F, _P, _F, _F, _F, _F, _P, _P, _Z, _P]),
    "pact_nf_param_count": (_Z, [_I, _I]),
    "pact_nf_packed_count": (_Z, [_I, _I]),
    "pact_nf_pack": (_I, [_P, _I, _I, _P, _P]),
    "pact_nf_activation_bytes": (_Z, [_I, _PRING, _I]),
    "pact_nf_sos_to_delays": (_I, [_P, _P, _P, _I, _I, _F, _F, _F, _P, _I, _PRING, _I, _P, _P, _Z, _P]),
    "pact_nf_sos_to_delays_adjoint_workspace_size": (_Z, [_I, _I]),
    "pact_nf_sos_to_delays_adjoint": (_I, [_P, _P, _P, _I, _I, _F, _F, _F, _P, _I, _PRING, _I, _P, _P, _P, _P,
                                           _Z, _P, _Z, _P]),
    "pact_rays_autotune": (_I, [_P, _PGRID, _F, _P, _I, _PRING, _I, _F, _P, _P, _P, _P, _Z, _P, _P]),
    "pact_conv3x3_packed_count": (_Z, [_I, _I]),
    "pact_conv3x3_pack": (_I, [_P, _I, _I, _P, _P, _P]),
    "pact_conv3x3_bf16": (_I, [_P, _I, _I, _I, _I, _P, _P, _I, _I, _P, _P, _P]),
    "pact_conv3x3_wgrad_workspace_size": (_Z, [_I, _I, _I, _I, _I]),
    "pact_conv3x3_wgrad_bf16": (_I, [_P, _P, _I, _I, _I, _I, _I, _P, _P, _Z, _P]),
    "pact_pool2_bf16": (_I, [_P, _I, _I, _I, _I, _P, _P]),
    "pact_up2_add_bf16": (_I, [_P, _P, _I, _I, _I, _I, _P, _P]),
    "pact_up2_add_adjoint_bf16": (_I, [_P, _P, _I, _I, _I, _I, _P, _P]),
    "pact_pool2_adjoint_bf16": (_I, [_P, _P, _P, _I, _I, _I, _I, _P, _P]),
    "pact_warm_input": (_I, [_P, _I, _I, _I, _I, _F, _I, _P, _P]),
    "pact_warm_loss_workspace_size": (_Z, [_I, _I, _I]),
    "pact_warm_loss": (_I, [_P, _I, _I, _I, _I, _P, _P, _F, _P, _P, _P, _Z, _P]),
    "pact_warm_sos": (_I, [_P, _I, _I, _I, _I, _P, _F, _F, _P, _P]),
    "pact_ricker_channels": (_I, [_P, _P, _P, _P, _I, _PRING, _F, _I, _F, _F, _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpact.so (built in-tree by paper_2409_10876_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PactError(f"{path} is missing: build it with `python -m paper_2409_10876_amd.build` "
                        "(there is no fallback implementation)")
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int, what: str):
    if status != 0:
        msg = load().pact_last_error().decode(errors="replace")
        raise PactError(f"{what} failed with status {status}: {msg}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, name="tensor", numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


F32, C64, U8, I32, BF16 = torch.float32, torch.complex64, torch.uint8, torch.int32, torch.bfloat16


@dataclass(frozen=True)
class Geometry:
    """Scan geometry in the units of the C ABI (mm, us, mm/us)."""
    n_elem: int
    radius: float
    phi0: float
    ny: int
    nx: int
    px: float
    P: int
    stride: int
    fwhm: float
    sos_ny: int
    sos_nx: int
    sos_spacing: float

    @property
    def ring(self) -> Ring:
        return Ring(self.n_elem, self.radius, self.phi0)

    @property
    def img(self) -> Grid:
        return Grid(self.ny, self.nx, self.px)

    @property
    def sosg(self) -> Grid:
        return Grid(self.sos_ny, self.sos_nx, self.sos_spacing)

    @property
    def patches(self) -> Patches:
        return Patches(self.P, self.stride, self.fwhm)

    @property
    def n_patches(self) -> int:
        a, b = patch_count(self)
        return a * b


def patch_count(g: Geometry):
    npy, npx = ctypes.c_int(), ctypes.c_int()
    _check(load().pact_patch_count(g.img, g.patches, ctypes.byref(npy), ctypes.byref(npx)), "pact_patch_count")
    return npy.value, npx.value


def patch_centres(g: Geometry, device="cuda") -> torch.Tensor:
    N = g.n_patches
    host = (ctypes.c_float * (2 * N))()
    _check(load().pact_patch_centres(g.img, g.patches, ctypes.cast(host, ctypes.c_void_p)), "pact_patch_centres")
    return torch.tensor(list(host), dtype=F32).view(N, 2).to(device)


def das_stack(S, fs, t0, g: Geometry, v0, d, out=None):
    n_elem, n_t = S.shape
    assert n_elem == g.n_elem, "S rows must match the ring"
    M = d.numel()
    out = torch.empty(M, g.ny, g.nx, dtype=F32, device=S.device) if out is None else out
    _check(load().pact_das_stack(_ptr(S, F32, "S"), n_t, fs, t0, g.ring, v0, _ptr(d, F32, "d"), M, g.img,
                                 _ptr(out, F32, "stack", M * g.ny * g.nx), _stream()), "pact_das_stack")
    return out


def patch_fft(stack, g: Geometry, half=True, out=None):
    M = stack.shape[0]
    N = g.n_patches
    W = g.P // 2 + 1 if half else g.P
    out = torch.empty(N, M, g.P, W, dtype=C64, device=stack.device) if out is None else out
    _check(load().pact_patch_fft(_ptr(stack, F32, "stack", M * g.ny * g.nx), M, g.img, g.patches, int(half),
                                 _ptr(out, C64, "Y", N * M * g.P * W), _stream()), "pact_patch_fft")
    return out


def ifft2_real(X, out=None):
    P = X.shape[-1]
    B = X.numel() // (P * P)
    out = torch.empty(X.shape, dtype=F32, device=X.device) if out is None else out
    _check(load().pact_ifft2_real(_ptr(X, C64, "X"), B, P, _ptr(out, F32, "x", B * P * P), _stream()),
           "pact_ifft2_real")
    return out


def sos_to_delays(sos, g: Geometry, v0, centres, n_samples, out=None, support=0.0, staged=None):
    """support: radius (mm) of the circular mask outside which the SOS is v0 (0: none); staged: the staged
    contrast grid of sos (stage_contrast) or None; see include/pact.h."""
    N = centres.shape[0]
    out = torch.empty(N, g.n_elem, dtype=F32, device=sos.device) if out is None else out
    _check(load().pact_sos_to_delays(_ptr(sos, F32, "sos", g.sos_ny * g.sos_nx), g.sosg, v0,
                                     _ptr(centres, F32, "centres", 2 * N), N, g.ring, n_samples, float(support),
                                     _ptr(staged, F32, "staged", staged_contrast_floats(g)),
                                     _ptr(out, F32, "w", N * g.n_elem), _stream()), "pact_sos_to_delays")
    return out


def staged_contrast_floats(g: Geometry) -> int:
    return int(load().pact_staged_contrast_floats(g.sosg))


def stage_contrast(sos, g: Geometry, v0, support=0.0, out=None):
    """The contrast grid the ray kernels hold in LDS, formed once (see include/pact.h): float
    [(sos_ny + 2) (sos_nx + 2)]."""
    n = staged_contrast_floats(g)
    out = torch.empty(n, dtype=F32, device=sos.device) if out is None else out
    _check(load().pact_stage_contrast(_ptr(sos, F32, "sos", g.sos_ny * g.sos_nx), g.sosg, v0, float(support),
                                      _ptr(out, F32, "staged", n), _stream()), "pact_stage_contrast")
    return out


def sos_to_delays_adjoint_workspace_size(g: Geometry, N: int) -> int:
    return load().pact_sos_to_delays_adjoint_workspace_size(g.sosg, N, g.ring)


def sos_to_delays_adjoint(sos, g: Geometry, v0, centres, n_samples, dL_dw, out=None, scale=None, accumulate=False,
                          ws=None, support=0.0, staged=None):
    N = centres.shape[0]
    out = torch.empty(g.sos_ny, g.sos_nx, dtype=F32, device=sos.device) if out is None else out
    need = sos_to_delays_adjoint_workspace_size(g, N)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=sos.device) if ws is None else ws
    _check(load().pact_sos_to_delays_adjoint(
        _ptr(sos, F32, "sos", g.sos_ny * g.sos_nx), g.sosg, v0, _ptr(centres, F32, "centres", 2 * N), N, g.ring,
        n_samples, float(support), _ptr(staged, F32, "staged", staged_contrast_floats(g)),
        _ptr(dL_dw, F32, "dL_dw", N * g.n_elem), _ptr(scale, F32, "scale", 1),
        _ptr(out, F32, "dL_dsos", g.sos_ny * g.sos_nx), int(accumulate), _ptr(ws, name="ws"), ws.numel(),
        _stream()), "pact_sos_to_delays_adjoint")
    return out


def rays_autotune(sos, g: Geometry, v0, centres, n_samples, dL_dw, w, dL_dsos, ws, support=0.0):
    """Time the ray tilings on this geometry and keep the fastest (see include/pact.h); returns
    (forward lanes per ray, adjoint segments per ray).  w, dL_dsos and ws are overwritten."""
    N = centres.shape[0]
    n = g.sos_ny * g.sos_nx
    out = (ctypes.c_int * 2)()
    _check(load().pact_rays_autotune(_ptr(sos, F32, "sos", n), g.sosg, v0, _ptr(centres, F32, "centres", 2 * N), N,
                                     g.ring, n_samples, float(support), _ptr(dL_dw, F32, "dL_dw", N * g.n_elem),
                                     _ptr(w, F32, "w", N * g.n_elem), _ptr(dL_dsos, F32, "dL_dsos", n),
                                     _ptr(ws, name="ws"), ws.numel(), ctypes.cast(out, ctypes.c_void_p), _stream()),
           "pact_rays_autotune")
    return out[0], out[1]


def delays_to_psf(w, centres, g: Geometry, d, with_psf=False, H=None, h=None):
    N = w.shape[0]
    M = d.numel()
    P = g.P
    H = torch.empty(N, M, P, P, dtype=C64, device=w.device) if H is None else H
    if with_psf and h is None:
        h = torch.empty(N, M, P, P, dtype=F32, device=w.device)
    _check(load().pact_delays_to_psf(_ptr(w, F32, "w", N * g.n_elem), _ptr(centres, F32, "centres", 2 * N), N,
                                     g.ring, _ptr(d, F32, "d", M), M, P, g.px, _ptr(H, C64, "H", N * M * P * P),
                                     _ptr(h, F32, "h", N * M * P * P) if with_psf else None, _stream()),
           "pact_delays_to_psf")
    return (H, h) if with_psf else H


def delays_to_psf_adjoint(w, centres, g: Geometry, d, dL_dH, out=None):
    N = w.shape[0]
    M = d.numel()
    out = torch.empty(N, g.n_elem, dtype=F32, device=w.device) if out is None else out
    _check(load().pact_delays_to_psf_adjoint(_ptr(w, F32, "w", N * g.n_elem), _ptr(centres, F32, "centres", 2 * N),
                                             N, g.ring, _ptr(d, F32, "d", M), M, g.P, g.px,
                                             _ptr(dL_dH, C64, "dL_dH", N * M * g.P * g.P),
                                             _ptr(out, F32, "dL_dw", N * g.n_elem), _stream()),
           "pact_delays_to_psf_adjoint")
    return out


def multichannel_deconv(Y, H, eps, out=None):
    N, M, P, _ = Y.shape
    out = torch.empty(N, P, P, dtype=C64, device=Y.device) if out is None else out
    _check(load().pact_multichannel_deconv(_ptr(Y, C64, "Y"), _ptr(H, C64, "H", Y.numel()), N, M, P, eps,
                                           _ptr(out, C64, "X", N * P * P), _stream()), "pact_multichannel_deconv")
    return out


def multichannel_deconv_adjoint(Y, H, eps, dL_dX, out=None):
    N, M, P, _ = Y.shape
    out = torch.empty_like(H) if out is None else out
    _check(load().pact_multichannel_deconv_adjoint(_ptr(Y, C64, "Y"), _ptr(H, C64, "H", Y.numel()), N, M, P, eps,
                                                   _ptr(dL_dX, C64, "dL_dX", N * P * P),
                                                   _ptr(out, C64, "dL_dH", Y.numel()), _stream()),
           "pact_multichannel_deconv_adjoint")
    return out


def residual_loss(Y, H, X, px, with_grads=True):
    N, M, P, _ = Y.shape
    loss = torch.empty(1, dtype=F32, device=Y.device)
    gH = torch.empty_like(H) if with_grads else None
    gX = torch.empty_like(X) if with_grads else None
    need = load().pact_residual_loss_workspace_size(N, P)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=Y.device)
    _check(load().pact_residual_loss(_ptr(Y, C64, "Y"), _ptr(H, C64, "H", Y.numel()), _ptr(X, C64, "X", N * P * P),
                                     N, M, P, px, _ptr(loss, F32, "loss"), _ptr(gH, C64, "dL_dH"),
                                     _ptr(gX, C64, "dL_dX"), _ptr(ws, name="ws"), ws.numel(), _stream()),
           "pact_residual_loss")
    return loss, gH, gX


def loss_and_grad_workspace_size(N, M, P, n_elem) -> int:
    return load().pact_loss_and_grad_workspace_size(N, M, P, n_elem)


def loss_and_grad(Y_half, w, centres, g: Geometry, d, eps, loss=None, dL_dw=None, want_grad=True, X=None,
                  ws=None, want_loss=True):
    """want_loss False: the scalar loss is not formed (one launch fewer); returns (None, dL_dw)."""
    N, M, P, Wh = Y_half.shape
    assert Wh == P // 2 + 1 and P == g.P
    dev = Y_half.device
    if want_loss:
        loss = torch.empty(1, dtype=F32, device=dev) if loss is None else loss
    else:
        loss = None
    if want_grad and dL_dw is None:
        dL_dw = torch.empty(N, g.n_elem, dtype=F32, device=dev)
    need = loss_and_grad_workspace_size(N, M, P, g.n_elem)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev) if ws is None else ws
    _check(load().pact_loss_and_grad(_ptr(Y_half, C64, "Y_half"), _ptr(w, F32, "w", N * g.n_elem),
                                     _ptr(centres, F32, "centres", 2 * N), N, g.ring, _ptr(d, F32, "d", M), M, P,
                                     g.px, eps, _ptr(loss, F32, "loss", 1),
                                     _ptr(dL_dw, F32, "dL_dw", N * g.n_elem) if want_grad else None,
                                     _ptr(X, C64, "X", N * P * P), _ptr(ws, name="ws"), ws.numel(), _stream()),
           "pact_loss_and_grad")
    return loss, dL_dw


def project_spectra(Y_half, g: Geometry, d, centres, out=None):
    """Step-invariant projections of the half spectra and the ring hits of every patch and bin (see
    include/pact.h): float [pact_projected_spectra_floats(N, P)]."""
    N, M, P, Wh = Y_half.shape
    assert Wh == P // 2 + 1 and P == g.P
    n = int(load().pact_projected_spectra_floats(N, P))
    out = torch.empty(n, dtype=F32, device=Y_half.device) if out is None else out
    _check(load().pact_project_spectra(_ptr(Y_half, C64, "Y_half"), N, M, P, g.px, _ptr(d, F32, "d", M),
                                       _ptr(centres, F32, "centres", 2 * N), g.ring, _ptr(out, F32, "T", n),
                                       _stream()), "pact_project_spectra")
    return out


def loss_and_grad_projected(T, M, w, centres, g: Geometry, eps, loss=None, dL_dw=None, want_grad=True, X=None,
                            ws=None, want_loss=True):
    """pact_loss_and_grad from projected spectra T (project_spectra) with M delays."""
    N = centres.shape[0]
    P = g.P
    dev = T.device
    loss = (torch.empty(1, dtype=F32, device=dev) if loss is None else loss) if want_loss else None
    if want_grad and dL_dw is None:
        dL_dw = torch.empty(N, g.n_elem, dtype=F32, device=dev)
    need = loss_and_grad_workspace_size(N, M, P, g.n_elem)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev) if ws is None else ws
    n = int(load().pact_projected_spectra_floats(N, P))
    _check(load().pact_loss_and_grad_projected(_ptr(T, F32, "T", n), _ptr(w, F32, "w", N * g.n_elem),
                                               _ptr(centres, F32, "centres", 2 * N), N, g.ring, M, P, g.px, eps,
                                               _ptr(loss, F32, "loss", 1),
                                               _ptr(dL_dw, F32, "dL_dw", N * g.n_elem) if want_grad else None,
                                               _ptr(X, C64, "X", N * P * P), _ptr(ws, name="ws"), ws.numel(),
                                               _stream()), "pact_loss_and_grad_projected")
    return loss, dL_dw


def loss_and_grad_noalloc(Y_half, w, centres, g: Geometry, d, eps, loss, dL_dw=None, X=None):
    """pact_loss_and_grad without a workspace (the library's own scratch; allocates nothing, so loss and dL_dw
    must be given)."""
    N, M, P, Wh = Y_half.shape
    assert Wh == P // 2 + 1 and P == g.P
    _check(load().pact_loss_and_grad_noalloc(_ptr(Y_half, C64, "Y_half"), _ptr(w, F32, "w", N * g.n_elem),
                                             _ptr(centres, F32, "centres", 2 * N), N, g.ring, _ptr(d, F32, "d", M), M,
                                             P, g.px, eps, _ptr(loss, F32, "loss", 1),
                                             _ptr(dL_dw, F32, "dL_dw", N * g.n_elem), _ptr(X, C64, "X", N * P * P),
                                             _stream()), "pact_loss_and_grad_noalloc")
    return loss, dL_dw


def tv_grad(sos, mask, g: Geometry, lam, grad, loss):
    n = g.sos_ny * g.sos_nx
    _check(load().pact_tv_grad(_ptr(sos, F32, "sos", n), _ptr(mask, U8, "mask", n), g.sosg, lam,
                               _ptr(grad, F32, "grad", n), _ptr(loss, F32, "loss", 1), _stream()), "pact_tv_grad")


def adam_step(sos, m, v, t, mask, grad, lr, b1=0.9, b2=0.999, eps=1e-8):
    """mask None: every entry is free."""
    n = sos.numel()
    _check(load().pact_adam_step(_ptr(sos, F32, "sos"), _ptr(m, F32, "m", n), _ptr(v, F32, "v", n),
                                 _ptr(t, I32, "t", 2), _ptr(mask, U8, "mask", n), n, _ptr(grad, F32, "grad", n),
                                 lr, b1, b2, eps, _stream()), "pact_adam_step")


def stitch(patches, g: Geometry, out=None):
    """Gaussian-weighted stitching of patch images [N][P][P] into the image [ny][nx]."""
    N = patches.shape[0]
    out = torch.empty(g.ny, g.nx, dtype=F32, device=patches.device) if out is None else out
    _check(load().pact_stitch(_ptr(patches, F32, "patches", N * g.P * g.P), N, g.img, g.patches,
                              _ptr(out, F32, "image", g.ny * g.nx), _stream()), "pact_stitch")
    return out


def siren_sos(params, hidden, omega0, mask, g: Geometry, mask_radius, v0, out=None):
    """The paper's sinusoidal network on the SOS-grid nodes -> SOS node grid [sos_ny][sos_nx]."""
    n = g.sos_ny * g.sos_nx
    out = torch.empty(g.sos_ny, g.sos_nx, dtype=F32, device=params.device) if out is None else out
    _check(load().pact_siren_sos(_ptr(params, F32, "params", 4 * hidden + 3), hidden, omega0,
                                 _ptr(mask, U8, "mask", n), g.sosg, mask_radius, v0, _ptr(out, F32, "sos", n),
                                 _stream()), "pact_siren_sos")
    return out


def siren_sos_adjoint(params, hidden, omega0, mask, g: Geometry, mask_radius, dL_dsos, out=None, ws=None):
    n = g.sos_ny * g.sos_nx
    out = torch.empty(4 * hidden + 3, dtype=F32, device=params.device) if out is None else out
    need = int(load().pact_siren_sos_adjoint_workspace_size(g.sosg, hidden))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=params.device) if ws is None else ws
    _check(load().pact_siren_sos_adjoint(_ptr(params, F32, "params", 4 * hidden + 3), hidden, omega0,
                                         _ptr(mask, U8, "mask", n), g.sosg, mask_radius,
                                         _ptr(dL_dsos, F32, "dL_dsos", n), _ptr(out, F32, "dL_dparams", 4 * hidden + 3),
                                         _ptr(ws, name="ws"), ws.numel(), _stream()), "pact_siren_sos_adjoint")
    return out


def tv_adam_step(sos_in, sos_out, m, v, t, mask, g: Geometry, grad, lam, loss, lr, b1=0.9, b2=0.999, eps=1e-8):
    """loss None: the TV value is not added to a loss."""
    n = g.sos_ny * g.sos_nx
    _check(load().pact_tv_adam_step(_ptr(sos_in, F32, "sos_in", n), _ptr(sos_out, F32, "sos_out", n),
                                    _ptr(m, F32, "m", n), _ptr(v, F32, "v", n), _ptr(t, I32, "t", 2),
                                    _ptr(mask, U8, "mask", n), g.sosg, _ptr(grad, F32, "grad", n), lam,
                                    _ptr(loss, F32, "loss", 1), lr, b1, b2, eps, _stream()), "pact_tv_adam_step")
    return sos_out


def sos_adjoint_tv_adam_step(sos_in, sos_out, m, v, t, mask, g: Geometry, v0, centres, n_samples, dL_dw, lam, loss,
                             lr, b1=0.9, b2=0.999, eps=1e-8, support=0.0, grad=None, ws=None, staged_in=None,
                             staged_out=None):
    """Ray adjoint, TV and Adam in two launches (see include/pact.h); loss None: no TV value added."""
    N = centres.shape[0]
    n = g.sos_ny * g.sos_nx
    need = sos_to_delays_adjoint_workspace_size(g, N)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=sos_in.device) if ws is None else ws
    _check(load().pact_sos_adjoint_tv_adam_step(
        _ptr(sos_in, F32, "sos_in", n), _ptr(sos_out, F32, "sos_out", n), _ptr(m, F32, "m", n), _ptr(v, F32, "v", n),
        _ptr(t, I32, "t", 2), _ptr(mask, U8, "mask", n), g.sosg, v0, _ptr(centres, F32, "centres", 2 * N), N, g.ring,
        n_samples, float(support), _ptr(staged_in, F32, "staged_in", staged_contrast_floats(g)),
        _ptr(staged_out, F32, "staged_out", staged_contrast_floats(g)), _ptr(dL_dw, F32, "dL_dw", N * g.n_elem), lam,
        _ptr(loss, F32, "loss", 1), lr, b1, b2, eps, _ptr(grad, F32, "grad", n), _ptr(ws, name="ws"), ws.numel(),
        _stream()),
        "pact_sos_adjoint_tv_adam_step")
    return sos_out


# ---- neural-field SOS ----

@dataclass(frozen=True)
class NfNet:
    """Neural-field network sizes and SOS mapping (see include/pact.h)."""
    n_freq: int = 128
    width: int = 128
    amp: float = 0.15
    mask_radius: float = 26.0

    @property
    def n_params(self) -> int:
        return int(load().pact_nf_param_count(self.n_freq, self.width))

    @property
    def n_packed(self) -> int:
        return int(load().pact_nf_packed_count(self.n_freq, self.width))


def nf_pack(params, net: NfNet, out=None):
    out = torch.empty(net.n_packed, dtype=BF16, device=params.device) if out is None else out
    _check(load().pact_nf_pack(_ptr(params, F32, "params", net.n_params), net.n_freq, net.width,
                               _ptr(out, BF16, "packed", net.n_packed), _stream()), "pact_nf_pack")
    return out


def nf_activation_bytes(N: int, g: Geometry, n_samples: int) -> int:
    return int(load().pact_nf_activation_bytes(N, g.ring, n_samples))


def nf_sos_to_delays(B, params, packed, net: NfNet, v0, centres, g: Geometry, n_samples, out=None, act=None):
    """act: optional uint8 device buffer of nf_activation_bytes() bytes that receives the activations."""
    N = centres.shape[0]
    out = torch.empty(N, g.n_elem, dtype=F32, device=params.device) if out is None else out
    _check(load().pact_nf_sos_to_delays(
        _ptr(B, F32, "B", 2 * net.n_freq), _ptr(params, F32, "params", net.n_params),
        _ptr(packed, BF16, "packed", net.n_packed), net.n_freq, net.width, net.amp, net.mask_radius, v0,
        _ptr(centres, F32, "centres", 2 * N), N, g.ring, n_samples, _ptr(out, F32, "w", N * g.n_elem),
        _ptr(act, name="act"), act.numel() if act is not None else 0, _stream()), "pact_nf_sos_to_delays")
    return out


def nf_sos_to_delays_adjoint_workspace_size(net: NfNet) -> int:
    return int(load().pact_nf_sos_to_delays_adjoint_workspace_size(net.n_freq, net.width))


def nf_sos_to_delays_adjoint(B, params, packed, net: NfNet, v0, centres, g: Geometry, n_samples, dL_dw, out=None,
                             scale=None, ws=None, act=None):
    N = centres.shape[0]
    out = torch.empty(net.n_params, dtype=F32, device=params.device) if out is None else out
    need = nf_sos_to_delays_adjoint_workspace_size(net)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=params.device) if ws is None else ws
    _check(load().pact_nf_sos_to_delays_adjoint(
        _ptr(B, F32, "B", 2 * net.n_freq), _ptr(params, F32, "params", net.n_params),
        _ptr(packed, BF16, "packed", net.n_packed), net.n_freq, net.width, net.amp, net.mask_radius, v0,
        _ptr(centres, F32, "centres", 2 * N), N, g.ring, n_samples, _ptr(dL_dw, F32, "dL_dw", N * g.n_elem),
        _ptr(scale, F32, "scale", 1), _ptr(out, F32, "dL_dparams", net.n_params), _ptr(act, name="act"),
        act.numel() if act is not None else 0, _ptr(ws, name="ws"), ws.numel(), _stream()),
        "pact_nf_sos_to_delays_adjoint")
    return out


# ---- learned warm start: convolution layers and the training-scan generator ----

def conv3x3_packed_count(ci: int, co: int) -> int:
    return int(load().pact_conv3x3_packed_count(ci, co))


def conv3x3_pack(weights, ci, co, packed=None, packed_adjoint=None, adjoint=True):
    """weights [co][3][3][ci] float -> (packed [co][K] bf16, packed adjoint [ci][K'] bf16 or None)."""
    dev = weights.device
    packed = torch.empty(conv3x3_packed_count(ci, co), dtype=BF16, device=dev) if packed is None else packed
    if adjoint and packed_adjoint is None:
        packed_adjoint = torch.empty(conv3x3_packed_count(co, ci), dtype=BF16, device=dev)
    _check(load().pact_conv3x3_pack(_ptr(weights, F32, "weights", co * 9 * ci), ci, co,
                                    _ptr(packed, BF16, "packed", conv3x3_packed_count(ci, co)),
                                    _ptr(packed_adjoint, BF16, "packed_adjoint", conv3x3_packed_count(co, ci)),
                                    _stream()), "pact_conv3x3_pack")
    return packed, packed_adjoint


def conv3x3(x, packed, co, bias=None, relu=False, mask=None, out=None):
    """x [n][H][W][ci] bf16 -> [n][H][W][co] bf16."""
    n, H, W, ci = x.shape
    out = torch.empty(n, H, W, co, dtype=BF16, device=x.device) if out is None else out
    _check(load().pact_conv3x3_bf16(_ptr(x, BF16, "x"), n, H, W, ci,
                                    _ptr(packed, BF16, "packed", conv3x3_packed_count(ci, co)),
                                    _ptr(bias, F32, "bias", co), co, int(relu),
                                    _ptr(mask, BF16, "mask", n * H * W * co),
                                    _ptr(out, BF16, "y", n * H * W * co), _stream()), "pact_conv3x3_bf16")
    return out


def conv3x3_wgrad_workspace_size(n, H, W, ci, co) -> int:
    return int(load().pact_conv3x3_wgrad_workspace_size(n, H, W, ci, co))


def conv3x3_wgrad(x, g, out=None, ws=None):
    """Weight and bias gradients [co * 9 * ci + co] (float) from input x and output gradient g."""
    n, H, W, ci = x.shape
    co = g.shape[3]
    out = torch.empty(co * 9 * ci + co, dtype=F32, device=x.device) if out is None else out
    need = conv3x3_wgrad_workspace_size(n, H, W, ci, co)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device) if ws is None else ws
    _check(load().pact_conv3x3_wgrad_bf16(_ptr(x, BF16, "x"), _ptr(g, BF16, "g", n * H * W * co), n, H, W, ci, co,
                                          _ptr(out, F32, "grad", co * 9 * ci + co), _ptr(ws, name="ws"), ws.numel(),
                                          _stream()), "pact_conv3x3_wgrad_bf16")
    return out


def pool2(x, out=None):
    n, H, W, C = x.shape
    out = torch.empty(n, H // 2, W // 2, C, dtype=BF16, device=x.device) if out is None else out
    _check(load().pact_pool2_bf16(_ptr(x, BF16, "x"), n, H, W, C, _ptr(out, BF16, "y", n * (H // 2) * (W // 2) * C),
                                  _stream()), "pact_pool2_bf16")
    return out


def up2_add(x, skip, out=None):
    n, H, W, C = skip.shape
    out = torch.empty_like(skip) if out is None else out
    _check(load().pact_up2_add_bf16(_ptr(x, BF16, "x", n * (H // 2) * (W // 2) * C), _ptr(skip, BF16, "skip"), n, H,
                                    W, C, _ptr(out, BF16, "y", n * H * W * C), _stream()), "pact_up2_add_bf16")
    return out


def up2_add_adjoint(g_high, mask_low=None, out=None):
    n, H, W, C = g_high.shape
    out = torch.empty(n, H // 2, W // 2, C, dtype=BF16, device=g_high.device) if out is None else out
    cnt = n * (H // 2) * (W // 2) * C
    _check(load().pact_up2_add_adjoint_bf16(_ptr(g_high, BF16, "g_high"), _ptr(mask_low, BF16, "mask_low", cnt), n,
                                            H, W, C, _ptr(out, BF16, "g_low", cnt), _stream()),
           "pact_up2_add_adjoint_bf16")
    return out


def pool2_adjoint(g_low, skip=None, mask=None, out=None):
    n, h, w, C = g_low.shape
    H, W = 2 * h, 2 * w
    cnt = n * H * W * C
    out = torch.empty(n, H, W, C, dtype=BF16, device=g_low.device) if out is None else out
    _check(load().pact_pool2_adjoint_bf16(_ptr(g_low, BF16, "g_low"), _ptr(skip, BF16, "skip", cnt),
                                          _ptr(mask, BF16, "mask", cnt), n, H, W, C, _ptr(out, BF16, "g_high", cnt),
                                          _stream()), "pact_pool2_adjoint_bf16")
    return out


def warm_input(stack, factor, scale, channels=16, out=None):
    """DAS stack [M][H][W] float -> network input [H/f][W/f][channels] bf16."""
    M, H, W = stack.shape
    out = torch.empty(H // factor, W // factor, channels, dtype=BF16, device=stack.device) if out is None else out
    _check(load().pact_warm_input(_ptr(stack, F32, "stack"), M, H, W, factor, scale, channels,
                                  _ptr(out, BF16, "x", (H // factor) * (W // factor) * channels), _stream()),
           "pact_warm_input")
    return out


def warm_loss_workspace_size(n, H, W) -> int:
    return int(load().pact_warm_loss_workspace_size(n, H, W))


def warm_loss(z, target, mask, norm, loss=None, g=None, ws=None):
    n, H, W, C = z.shape
    dev = z.device
    loss = torch.empty(1, dtype=F32, device=dev) if loss is None else loss
    g = torch.empty_like(z) if g is None else g
    need = warm_loss_workspace_size(n, H, W)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev) if ws is None else ws
    _check(load().pact_warm_loss(_ptr(z, BF16, "z"), n, H, W, C, _ptr(target, F32, "target", n * H * W),
                                 _ptr(mask, U8, "mask", H * W), norm, _ptr(loss, F32, "loss", 1),
                                 _ptr(g, BF16, "g", n * H * W * C), _ptr(ws, name="ws"), ws.numel(), _stream()),
           "pact_warm_loss")
    return loss, g


def warm_sos(z, mask, v0, scale, out=None):
    n, H, W, C = z.shape
    out = torch.empty(n, H, W, dtype=F32, device=z.device) if out is None else out
    _check(load().pact_warm_sos(_ptr(z, BF16, "z"), n, H, W, C, _ptr(mask, U8, "mask", H * W), v0, scale,
                                _ptr(out, F32, "sos", n * H * W), _stream()), "pact_warm_sos")
    return out


def ricker_channels(w, sources, amp, sigma, g: Geometry, v0, n_t, fs, t0=0.0, out=None):
    """Channel data [n_elem][n_t] of Ricker sources with wavefront errors w [n_src][n_elem]."""
    n_src = sources.shape[0]
    out = torch.empty(g.n_elem, n_t, dtype=F32, device=w.device) if out is None else out
    _check(load().pact_ricker_channels(_ptr(w, F32, "w", n_src * g.n_elem), _ptr(sources, F32, "sources", 2 * n_src),
                                       _ptr(amp, F32, "amp", n_src), _ptr(sigma, F32, "sigma", n_src), n_src, g.ring,
                                       v0, n_t, fs, t0, _ptr(out, F32, "S", g.n_elem * n_t), _stream()),
           "pact_ricker_channels")
    return out


# ---- batched solves: one launch per stage over many scans ----

def batch_plan(scans):
    """Plan a batched step over `scans` (a ctypes array of BatchScan): returns (host plan buffer, device table)."""
    n = len(scans)
    lib = load()
    plan = ctypes.create_string_buffer(int(lib.pact_batch_plan_bytes(n)))
    nb = int(lib.pact_batch_table_bytes(n))
    if nb == 0:
        raise PactError(f"pact_batch_table_bytes: {n} scans not supported")
    table = torch.empty(nb, dtype=torch.uint8, device="cuda")
    _check(lib.pact_batch_plan(ctypes.cast(scans, ctypes.c_void_p), n, ctypes.cast(plan, ctypes.c_void_p), len(plan),
                               _ptr(table, name="table"), nb, _stream()), "pact_batch_plan")
    return plan, table


def batch_step(plan, parity, with_loss=True):
    _check(load().pact_batch_step(ctypes.cast(plan, ctypes.c_void_p), int(parity), int(bool(with_loss)), _stream()),
           "pact_batch_step")


def batch_step_persistent(plan, parity, with_loss=True):
    _check(load().pact_batch_step_persistent(ctypes.cast(plan, ctypes.c_void_p), int(parity), int(bool(with_loss)),
                                             _stream()), "pact_batch_step_persistent")

