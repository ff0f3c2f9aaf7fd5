"""The C ABI without a GPU: the library loads, exports every symbol include/pact.h declares, computes the
host-side geometry, and rejects bad arguments with the documented status codes before enqueuing anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pact.h")

FAKE = ctypes.c_void_p(0x1000)     # never dereferenced: every call below fails its host-side checks first


@pytest.fixture(scope="module")
def P():
    import paper_2409_10876_amd as P
    return P


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"PACT_API\s+[\w\s\*]+?\b(pact_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(P):
    names = _declared()
    assert len(names) >= 20
    lib = P.pact.load()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.pact.exported_symbols()) == names
    assert lib.pact_version() == 2


def test_patch_geometry_matches_oracle(P):
    from oracle.geometry import patch_centres
    for scan in (synth.TINY, synth.PAPER):
        g = P.geometry_from(scan)
        assert P.pact.patch_count(g) == (scan.n_patch_y, scan.n_patch_x)
        got = P.pact.patch_centres(g, device="cpu").numpy()
        want = patch_centres(scan.ny, scan.nx, float(np.float32(scan.px)), scan.P, scan.stride).numpy()
        np.testing.assert_allclose(got, want, atol=1e-6)


def _status(P, name, *args):
    lib = P.pact.load()
    s = getattr(lib, name)(*args)
    return s, lib.pact_last_error().decode()


def test_argument_errors(P):
    pt = P.pact
    ring = pt.Ring(256, 50.0, 0.0)
    img = pt.Grid(128, 128, 0.2)
    sosg = pt.Grid(32, 32, 0.8)
    s, msg = _status(P, "pact_sos_to_delays", None, sosg, 1.5, FAKE, 49, ring, 256, 0.0, None, FAKE, None)
    assert s == -1 and "null" in msg
    s, msg = _status(P, "pact_sos_to_delays", FAKE, sosg, 1.5, FAKE, 49, pt.Ring(0, 50.0, 0.0), 256, 0.0, None,
                     FAKE, None)
    assert s == -1 and "n_elem" in msg
    s, msg = _status(P, "pact_sos_to_delays", FAKE, pt.Grid(300, 300, 0.1), 1.5, FAKE, 49, ring, 256, 0.0, None,
                     FAKE, None)
    assert s == -4 and "LDS" in msg
    s, msg = _status(P, "pact_sos_to_delays", FAKE, sosg, 1.5, FAKE, 49, ring, 256, -1.0, None, FAKE, None)
    assert s == -1 and "support_radius" in msg
    s, msg = _status(P, "pact_patch_fft", FAKE, 5, img, pt.Patches(120, 8, 1.0), 1, FAKE, None)
    assert s == -4
    s, msg = _status(P, "pact_patch_fft", FAKE, 5, img, pt.Patches(200, 8, 1.0), 1, FAKE, None)
    assert s == -1 and "larger" in msg
    s, msg = _status(P, "pact_loss_and_grad", FAKE, FAKE, FAKE, 49, ring, FAKE, 17, 32, 0.2, 1e-6, FAKE, FAKE, None,
                     FAKE, 1 << 30, None)
    assert s == -4 and "M = 17" in msg
    s, msg = _status(P, "pact_loss_and_grad", FAKE, FAKE, FAKE, 49, ring, FAKE, 5, 32, 0.2, 1e-6, FAKE, FAKE, None,
                     FAKE, 16, None)
    assert s == -3 and "workspace" in msg
    s, msg = _status(P, "pact_sos_to_delays_adjoint", FAKE, sosg, 1.5, FAKE, 49, ring, 0, 0.0, None, FAKE, None,
                     FAKE, 0, None, 0, None)
    assert s == -1 and "n_samples" in msg
    s, msg = _status(P, "pact_sos_to_delays_adjoint", FAKE, None, 1.5, FAKE, 49, ring, 256, 0.0, None, FAKE, None,
                     FAKE, 0, None, 0, None)
    assert s == -1 and "geometry" in msg
    s, msg = _status(P, "pact_residual_loss", FAKE, FAKE, FAKE, 4, 3, 8, 0.1, FAKE, None, None, FAKE, 0, None)
    assert s == -3
    s, msg = _status(P, "pact_adam_step", FAKE, FAKE, FAKE, FAKE, FAKE, 10, FAKE, 1e-3, 1.0, 0.999, 1e-8, None)
    assert s == -1 and "betas" in msg
    s, msg = _status(P, "pact_multichannel_deconv", FAKE, FAKE, 4, 3, 8, -1.0, FAKE, None)
    assert s == -1 and "eps" in msg
    s, msg = _status(P, "pact_das_stack", FAKE, 100, 40.0, 0.0, ring, 0.0, FAKE, 5, img, FAKE, None)
    assert s == -1
    s, msg = _status(P, "pact_stage_contrast", FAKE, sosg, 1.5, -1.0, FAKE, None)
    assert s == -1 and "support_radius" in msg
    s, msg = _status(P, "pact_stage_contrast", FAKE, None, 1.5, 0.0, FAKE, None)
    assert s == -1 and "geometry" in msg
    assert P.pact.load().pact_staged_contrast_floats(sosg) == 34 * 34


def test_workspace_sizes(P):
    pt = P.pact
    # one workgroup per patch: the patch losses, added in order by a second kernel
    assert pt.loss_and_grad_workspace_size(169, 11, 80, 512) == 169 * 4
    assert P.pact.load().pact_residual_loss_workspace_size(0, 8) == 0


def test_binding_refuses_host_tensors(P):
    import torch
    g = P.geometry_from(synth.TINY)
    with pytest.raises(ValueError):
        P.pact.sos_to_delays(torch.zeros(32, 32), g, 1.5, torch.zeros(49, 2), 256, out=torch.zeros(49, 256))


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: without libpact.so every call raises PactError."""
    import paper_2409_10876_amd.pact as pt
    saved = pt._lib
    try:
        pt._lib = None
        with pytest.raises(pt.PactError, match="missing"):
            pt.load(str(tmp_path / "libpact.so"))
    finally:
        pt._lib = saved


def test_warm_start_argument_errors(P):
    pt = P.pact
    ring = pt.Ring(512, 110.0, 0.0)
    # channel pairs that are not built, null pointers, empty shapes
    s, msg = _status(P, "pact_conv3x3_bf16", FAKE, 2, 8, 8, 32, FAKE, None, 64, 1, None, FAKE, None)
    assert s == -4 and "not built" in msg
    s, msg = _status(P, "pact_conv3x3_bf16", None, 2, 8, 8, 64, FAKE, None, 64, 1, None, FAKE, None)
    assert s == -1 and "null" in msg
    s, msg = _status(P, "pact_conv3x3_bf16", FAKE, 0, 8, 8, 64, FAKE, None, 64, 1, None, FAKE, None)
    assert s == -1
    s, msg = _status(P, "pact_conv3x3_pack", FAKE, 16, 16, FAKE, None, None)
    assert s == -4
    assert pt.load().pact_conv3x3_packed_count(16, 64) == 64 * 160
    assert pt.load().pact_conv3x3_packed_count(64, 16) == 16 * 576
    # weight gradient: workspace too small
    s, msg = _status(P, "pact_conv3x3_wgrad_bf16", FAKE, FAKE, 2, 8, 8, 64, 64, FAKE, FAKE, 16, None)
    assert s == -3 and "workspace" in msg
    # resampling needs even sizes and channel counts that are multiples of 8
    s, msg = _status(P, "pact_pool2_bf16", FAKE, 1, 7, 8, 64, FAKE, None)
    assert s == -1 and "even" in msg
    s, msg = _status(P, "pact_up2_add_bf16", FAKE, FAKE, 1, 8, 8, 12, FAKE, None)
    assert s == -1 and "multiple of 8" in msg
    s, msg = _status(P, "pact_warm_input", FAKE, 20, 560, 560, 4, 1.0, 16, FAKE, None)
    assert s == -1
    s, msg = _status(P, "pact_warm_loss", FAKE, 2, 140, 140, 16, FAKE, FAKE, 1.0, FAKE, FAKE, FAKE, 4, None)
    assert s == -3 and "workspace" in msg
    s, msg = _status(P, "pact_ricker_channels", FAKE, FAKE, FAKE, FAKE, 0, ring, 1.5, 4096, 40.0, 0.0, FAKE, None)
    assert s == -1
    s, msg = _status(P, "pact_ricker_channels", FAKE, FAKE, FAKE, FAKE, 4, pt.Ring(0, 110.0, 0.0), 1.5, 4096, 40.0,
                     0.0, FAKE, None)
    assert s == -1 and "n_elem" in msg


def test_nf_activation_buffer_too_small(P):
    pt = P.pact
    ring = pt.Ring(512, 110.0, 0.0)
    need = pt.load().pact_nf_activation_bytes(169, ring, 256)
    # h1..h4, f and the adjoint's layer-1 gradients: 32 KB + 128 + 8 KB per 32 samples
    assert need == 169 * 512 * 8 * (32768 + 128 + 8192)
    s, msg = _status(P, "pact_nf_sos_to_delays", FAKE, FAKE, FAKE, 128, 128, 0.15, 26.0, 1.5, FAKE, 169, ring, 256,
                     FAKE, FAKE, need - 1, None)
    assert s == -3 and "activation buffer" in msg


def test_batch_scan_layout_matches_the_header(P, tmp_path):
    """The binding's pact_batch_scan has the C layout (offsets from a host program compiled against the
    header)."""
    import shutil
    import subprocess
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    bs = P.pact.BatchScan
    names = [f[0] for f in bs._fields_]
    c_names = ["lambda" if n == "lam" else n for n in names]
    src = tmp_path / "layout.cpp"
    src.write_text('#include <cstddef>\n#include <cstdio>\n#include "pact.h"\nint main() {\n'
                   '  printf("%zu\\n", sizeof(pact_batch_scan));\n' +
                   "".join(f'  printf("%zu\\n", offsetof(pact_batch_scan, {n}));\n' for n in c_names) + "}\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cxx, "-I", include, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(bs)
    assert got[1:] == [getattr(bs, n).offset for n in names]


def test_batch_argument_errors(P):
    lib = P.pact.load()
    plan = ctypes.create_string_buffer(int(lib.pact_batch_plan_bytes(1)))
    assert lib.pact_batch_table_bytes(0) == 0 and lib.pact_batch_table_bytes(257) == 0
    assert lib.pact_batch_table_bytes(32) > 0
    s = lib.pact_batch_plan(None, 1, plan, len(plan), FAKE, 1 << 20, None)
    assert s == -1 and "null" in lib.pact_last_error().decode()
    scans = (P.pact.BatchScan * 1)()
    s = lib.pact_batch_plan(ctypes.cast(scans, ctypes.c_void_p), 300, plan, len(plan), FAKE, 1 << 20, None)
    assert s == -4 and "256" in lib.pact_last_error().decode()
    # a buffer that pact_batch_plan did not fill is refused before anything is launched
    s = lib.pact_batch_step(plan, 0, 1, None)
    assert s == -1 and "plan" in lib.pact_last_error().decode()
    s = lib.pact_batch_step_persistent(plan, 0, 1, None)
    assert s == -1 and "plan" in lib.pact_last_error().decode()
    s = lib.pact_batch_step_persistent(None, 0, 1, None)
    assert s == -1 and "null" in lib.pact_last_error().decode()

