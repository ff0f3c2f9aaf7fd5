"""Benchmark: forward+adjoint SOS-optimisation steps per second on the paper-shaped workload.

One bench step = one reconstruction job on a synthetic 560^2 scan (512-element ring of radius 110 mm,
4096 samples at 40 MHz, 11 delays, 169 patches of 80^2, 140^2 SOS grid, 256 samples per ray): the DAS
stack and the windowed patch spectra once, then 500 forward+adjoint optimisation steps (wavefronts,
fused deconvolution/loss/gradient, ray adjoint, TV, Adam), replayed from HIP graphs.  Channel data are
resident in HBM before the timed region.  value = optimisation steps per second over the whole job
(DAS and FFT included once per job).

Also reported: the roofline of the fused loss kernel (algorithmic bytes of the half spectra per launch
over its average launch time, measured with HIP events inside the timed region) and the FP64 oracle
timed on this host's cores on a bounded sample (a few optimisation steps at the same scale).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X published FP32 vector peak (it counts packed FP32 instructions); the roofline fractions of the
# ALU-bound stages are quoted against it.
FP32_PUBLISHED_PEAK_TFLOPS = 157.3
# The issue-rate bound of these kernels, reported beside it: packed FP32 is disabled, so one wave64 FP32 FMA
# per cycle per CU, 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.
ALU_ISSUE_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
COPY_REF_BYTES = 256 << 20
MFMA_BF16_PEAK_TFLOPS = 2500.0                            # dense BF16 MFMA, MI355X
# Algorithmic FP32 operations per ray sample (FMA = 2), from the definitions of the two ray maps:
#   forward: position 4, cell fractions 2, bilinear contrast 6, v0 + delta 1, delta / v 2, accumulate 1
#   adjoint: position 4, cell fractions 2, bilinear contrast 6, v0 + delta 1, v0 / v^2 and the ray weight 3,
#            four bilinear shares 6, four accumulations 4
FLOPS_PER_SAMPLE_FWD = 16
FLOPS_PER_SAMPLE_ADJ = 26
METRIC = "fwd+adjoint SOS-opt steps/s (patches×delays/s); time-to-SOS-RMSE, plain vs warm"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed reconstruction jobs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed reconstruction jobs")
    ap.add_argument("--opt-steps", type=int, default=500, help="optimisation steps per job")
    ap.add_argument("--graph-steps", type=int, default=50, help="optimisation steps per captured HIP graph")
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny"])
    ap.add_argument("--timing-steps", type=int, default=100, help="eager steps timed per stage with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=15, help="oracle steps timed for the CPU baseline")
    ap.add_argument("--nf-steps", type=int, default=3, help="neural-field optimisation steps timed (0: skip)")
    ap.add_argument("--warm-scans", type=int, default=100,
                    help="held-out scans of the learned warm-start comparison (0: skip)")
    ap.add_argument("--batch-scans", type=int, default=32,
                    help="also time this many independent uneven scans solved together (0: skip)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run one plain 256 MiB device copy kernel first (the reference for HBM counter scaling)")
    return ap.parse_args()


def traffic_bytes(stage):
    """HBM bytes per launch of a stage from the committed rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy reference), or None when the stage's kernel source has changed since."""
    import hashlib
    rec = TRAFFIC.get(stage)
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2409_10876_amd", "csrc", rec["source"])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return rec["bytes"] if digest == rec["sha256_16"] else None


# Measured HBM traffic per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that make a plain 256 MiB
# copy kernel read as 256 MiB; rocprofv3 counter runs recorded under profiles/), keyed to the kernel source
# it was taken on.
TRAFFIC = {
    "sos_to_delays": {"source": "rays.hip", "sha256_16": "7d4719c27ab48eee", "bytes": 1127302},
    "loss_and_grad": {"source": "loss.hip", "sha256_16": "0fa16bc95a50c044", "bytes": 16833422},
    "sos_to_delays_adjoint": {"source": "rays.hip", "sha256_16": "7d4719c27ab48eee", "bytes": 33810707},
    "adjoint_tv_adam": {"source": "rays.hip", "sha256_16": "7d4719c27ab48eee", "bytes": 34861434},
}


def active_samples(scan, support, centres):
    """Ray samples (all patches and elements) that can touch a node inside the support disc: those within the
    support radius grown by a cell diagonal, at the midpoints of each ray's part inside the SOS box (all samples
    without a support).  FP64, from the geometry alone (centres: the scan's patch centres, [N][2])."""
    import numpy as np
    total = scan.n_patches * scan.n_elem * scan.n_samples
    if not support > 0:
        return total
    c = np.asarray(centres, dtype=np.float64)
    phi = scan.phi0 + 2 * np.pi * np.arange(scan.n_elem) / scan.n_elem
    e = scan.radius * np.stack([np.cos(phi), np.sin(phi)], -1)
    h = 0.5 * (scan.sos_n + 1) * scan.sos_spacing
    rc = support + np.sqrt(2.0) * scan.sos_spacing
    mid = (np.arange(scan.n_samples) + 0.5) / scan.n_samples
    n = 0
    for ci in c:
        d = e - ci
        L0 = np.linalg.norm(d, axis=-1)
        u = d / L0[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            tx = np.where(u[:, 0] != 0, (np.sign(u[:, 0]) * h - ci[0]) / u[:, 0], np.inf)
            ty = np.where(u[:, 1] != 0, (np.sign(u[:, 1]) * h - ci[1]) / u[:, 1], np.inf)
        L = np.minimum(np.minimum(L0, tx), ty)
        p = ci[None, None, :] + (L[:, None] * mid[None, :])[..., None] * u[:, None, :]
        n += int((np.linalg.norm(p, axis=-1) <= rc).sum())
    return n


def cpu_baseline(scan, inp, n_steps):
    """The FP64 oracle, as it stands, on this host: n_steps full optimisation steps (rays, deconvolution loss,
    reverse-mode gradient, TV, Adam) on spectra of the same shape."""
    import numpy as np
    import torch
    from oracle import loss as Oloss, adam as Oadam
    from oracle.geometry import patch_centres

    rng = np.random.default_rng(0)
    N = scan.n_patches
    Y = torch.fft.fft2(torch.tensor(rng.normal(size=(N, scan.M, scan.P, scan.P))))
    geom = dict(sos_spacing=scan.sos_spacing, v0=scan.v0, centres=patch_centres(scan.ny, scan.nx, scan.px, scan.P,
                                                                                  scan.stride),
                n_elem=scan.n_elem, radius=scan.radius, phi0=scan.phi0, n_samples=scan.n_samples,
                delays=np.asarray(scan.delays), px=scan.px, eps=scan.eps)
    opt = Oadam.Adam(torch.full((scan.sos_n, scan.sos_n), scan.v0, dtype=torch.float64), inp.mask, lr=scan.lr)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        _, gv, _, _ = Oloss.loss_and_grad(opt.p, inp.mask, Y, geom, scan.lam_tv)
        opt.step(gv)
    dt = time.perf_counter() - t0
    cores = torch.get_num_threads()
    # the same on one core, one step
    torch.set_num_threads(1)
    t1 = time.perf_counter()
    _, gv, _, _ = Oloss.loss_and_grad(opt.p, inp.mask, Y, geom, scan.lam_tv)
    opt.step(gv)
    dt1 = time.perf_counter() - t1
    torch.set_num_threads(cores)
    return {"value": n_steps / dt, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_steps} full FP64 oracle optimisation steps at the same workload "
                      f"({N} patches x {scan.M} delays, {scan.n_elem} elements, {scan.sos_n}^2 SOS grid, "
                      f"{scan.n_samples} samples/ray) in {dt:.1f} s; DAS/FFT not included",
            "patches_x_delays_per_s": n_steps * N * scan.M / dt,
            "job_s_extrapolated": scan.steps * dt / n_steps,
            "single_core": {"value": 1.0 / dt1, "unit": "steps/s", "cores": 1, "sample": f"1 step in {dt1:.1f} s"},
            "host_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


# The paper's own end-to-end times (Table 1 and Fig. 3d), on its hardware and its data (five k-Wave
# phantoms, 16 delays, a 200k-pixel SOS map): context, not a target, since the workloads differ.
PAPER_CONTEXT = {
    "hardware": "one NVIDIA RTX A6000, PyTorch, precision not stated",
    "reconstruction_s": {"neural field (10 epochs)": 40.3, "pixel grid + TV (30 epochs)": 113.3},
    "deconvolution_with_true_sos_s": 2.6, "das_s": 0.13,
    "deconvolution_vs_channels_s": {"4": 0.9, "32": 5.0},
    "source": "Table 1 and Fig. 3d of the paper",
}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2409_10876_amd as P
    from paper_2409_10876_amd import pact

    scan = synth.PAPER if args.workload == "paper" else synth.TINY
    dev = torch.device("cuda:0")
    if args.copy_ref:
        # elementwise copy kernel: reads and writes COPY_REF_BYTES each
        x = torch.ones(COPY_REF_BYTES // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
        print(f"[bench] copy reference: {COPY_REF_BYTES} bytes read and written by one elementwise kernel", flush=True)
    t_setup = time.perf_counter()
    inp = synth.make_inputs(scan, seed=0)
    print(f"[bench] inputs ready ({time.perf_counter() - t_setup:.1f} s): {synth.describe(scan)}", flush=True)

    sd = P.prepare_scan(scan, inp.S, np.asarray(scan.delays, dtype=np.float32), device=dev)
    # the mask is the disc of free nodes within mask_radius: the rays skip the samples that touch fixed nodes only
    solver = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples,
                               support_radius=scan.mask_radius)
    sos0 = solver.sos.clone()

    G = args.graph_steps
    assert args.opt_steps % G == 0, "--opt-steps must be a multiple of --graph-steps"
    solver.step()
    torch.cuda.synchronize()
    solver.capture(G)
    torch.cuda.synchronize()
    print("[bench] step graph captured", flush=True)

    def job():
        sd.prepare()
        solver.set_sos(sos0)
        solver.m.zero_()
        solver.v.zero_()
        solver.t.zero_()
        solver.run(args.opt_steps)

    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    print("[bench] warmup done", flush=True)

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        job()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(stop)
    elapsed = max(wall, gpu_ms / 1e3)
    opt_steps = args.steps * args.opt_steps
    value = opt_steps / elapsed
    print(f"[bench] {opt_steps} steps in {elapsed:.3f} s ({1e6 * elapsed / opt_steps:.1f} us/step)", flush=True)

    # Per-stage timing, same process and data: HIP events on the launch stream around each stage of
    # optimisation steps run eagerly (ROCm does not allow timing events inside captured graphs).
    # the step's launches as the captured graph runs them (the scalar loss only on a graph's last step), and the
    # ray adjoint on its own (its kernels are the dominant ones)
    stages = {"sos_to_delays": solver.delays, "loss_and_grad": lambda: solver.loss_grad(with_loss=False),
              "adjoint_tv_adam": lambda: solver.adjoint_update(with_loss=False),
              "sos_to_delays_adjoint": solver.adjoint}
    reps = args.timing_steps
    evs = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
           for k in stages}
    das_ev = tuple(torch.cuda.Event(enable_timing=True) for _ in range(4))
    # keep the GPU busy while Python enqueues the timing pass, so that each event pair brackets only the work
    # between them (no host launch gaps)
    torch.cuda._sleep(int(args.timing_steps * 2_000_000))
    das_ev[0].record()
    sd.stack = P.pact.das_stack(sd.S, sd.fs, sd.t0, sd.geom, sd.v0, sd.d, out=sd.stack)
    das_ev[1].record()
    sd.Y = P.pact.patch_fft(sd.stack, sd.geom, half=True, out=sd.Y)
    das_ev[2].record()
    sd.T = P.pact.project_spectra(sd.Y, sd.geom, sd.d, sd.centres, out=sd.T)
    das_ev[3].record()
    for r in range(reps):
        for k, fn in stages.items():
            evs[k][r][0].record()
            fn()
            evs[k][r][1].record()
    torch.cuda.synchronize()
    breakdown = {k: 1e3 * sum(a.elapsed_time(b) for a, b in v) / reps for k, v in evs.items()}
    breakdown["das_stack_once"] = 1e3 * das_ev[0].elapsed_time(das_ev[1])
    breakdown["patch_fft_once"] = 1e3 * das_ev[1].elapsed_time(das_ev[2])
    breakdown["project_spectra_once"] = 1e3 * das_ev[2].elapsed_time(das_ev[3])
    N, M, Pp = scan.n_patches, scan.M, scan.P
    G2 = scan.sos_n * scan.sos_n
    # the ray samples the method needs: those that can touch a free node (the others add exactly zero)
    samples = active_samples(scan, solver.support, sd.centres.cpu().numpy())
    rays_io = N * scan.n_elem * 4
    n_virtual = Pp * (Pp // 2 + 1) + (Pp // 2 - 1 if Pp % 2 == 0 else 0)
    # per stage: (kernels, bound, algorithmic work per launch, unit of the work)
    work = {
        "sos_to_delays": ("rays_fwd_kernel", "alu", samples * FLOPS_PER_SAMPLE_FWD, "flop"),
        # the projected spectra (five floats per patch and bin) once, w in, dL/dw out
        # per patch and bin the five projections, per patch and virtual bin the two ring hits, w in, dL/dw out
        "loss_and_grad": ("loss_proj_kernel", "hbm", N * Pp * (Pp // 2 + 1) * 20 + N * n_virtual * 8 + 2 * rays_io,
                          "byte"),
        "sos_to_delays_adjoint": ("rays_adj_grid_kernel + rays_adj_reduce_kernel", "alu",
                                  samples * FLOPS_PER_SAMPLE_ADJ, "flop"),
        # the step's last two launches: the grid adjoint, then its partials' sum fused with TV and Adam
        "adjoint_tv_adam": ("rays_adj_grid_kernel + adj_reduce_tv_adam_kernel", "alu",
                            samples * FLOPS_PER_SAMPLE_ADJ, "flop"),
    }
    rooflines = {}
    for k, (kern, bound, units, unit) in work.items():
        us = breakdown[k]
        if unit == "byte":
            ach, peak, u = units / (us * 1e-6) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, u = units / (us * 1e-6) / 1e12, FP32_PUBLISHED_PEAK_TFLOPS, "TFLOP/s"
        rooflines[k] = {"bound": bound, "kernel": kern, "achieved": ach, "peak": peak, "unit": u, "frac": ach / peak,
                        "traffic": traffic_bytes(k), "alg_" + unit + "s_per_launch": units, "avg_launch_us": us}
        if unit == "flop":
            rooflines[k]["issue_peak"] = ALU_ISSUE_PEAK_TFLOPS
            rooflines[k]["frac_of_issue_peak"] = ach / ALU_ISSUE_PEAK_TFLOPS
    dominant = max(work, key=lambda k: breakdown[k])
    # the step as a whole against the HBM roofline: the bytes one optimisation step must move (the projected
    # spectra and ring hits once, w and dL/dw written and read, the SOS read by both ray kernels and TV + Adam
    # and written, the gradient written and read, Adam's m and v read and written, the mask) over the
    # graph-replayed time per step
    step_bytes = work["loss_and_grad"][2] + 2 * rays_io + G2 * 4 * (3 + 1 + 1 + 4) + G2
    us_step = 1e6 * elapsed / opt_steps
    print("[bench] stage times (us): " + ", ".join(f"{k} {v:.1f}" for k, v in breakdown.items()), flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": synth.describe(scan),
                   "bench_step": f"one job = das_stack + patch_fft once + {args.opt_steps} optimisation steps",
                   "opt_steps_per_job": args.opt_steps, "patches": N, "delays": M, "n_elem": scan.n_elem,
                   "sos_grid": scan.sos_n, "n_samples": scan.n_samples, "graph_steps": G},
        "patches_x_delays_per_s": value * N * M,
        "ms_per_opt_step": 1e3 * elapsed / opt_steps,
        "roofline": dict(rooflines[dominant], stage=dominant,
                         timing=f"HIP events around {reps} eager launches on the launch stream"),
        "rooflines": rooflines,
        "hbm_frac_step": step_bytes / (us_step * 1e-6) / (HBM_PEAK_GBS * 1e9),
        "step_alg_bytes": step_bytes,
        "ray_samples": {"needed": samples, "all": N * scan.n_elem * scan.n_samples,
                        "note": "the rays skip the samples that touch only fixed nodes (SOS v0, outside the mask)"},
        "stage_us": breakdown,
    }
    out["reconstruction"] = reconstruction_quality(P, sd, solver, inp, scan, elapsed / args.steps)
    rq = out["reconstruction"]
    af = rq["ip_image"]["aberration_free"]
    print(f"[bench] SOS RMSE {rq['sos_rmse_initial_m_per_s']:.2f} -> {rq['sos_rmse_m_per_s']:.2f} m/s; image PSNR / SSIM "
          "against the aberration-free image: " + ", ".join(f"{k} {v['psnr_db']:.2f} dB / {v['ssim']:.3f}"
                                                            for k, v in af.items()), flush=True)
    out["precision"] = precision_leg(P, sd, solver, scan, inp.mask)
    out["delay_sweep"] = delay_sweep(P, sd, scan, solver)
    out["paper_neural_field"] = siren_leg(P, sd, scan, inp, reps=args.timing_steps)
    if args.nf_steps > 0:
        out["neural_field"] = nf_leg(P, sd, scan, args.nf_steps)
    if args.batch_scans > 0:
        out["batched"] = batch_leg(P, args.batch_scans)
    if args.warm_scans > 0:
        out["warm_start"] = warm_leg(P, args.warm_scans)
        sm = out["warm_start"].get("summary")
        if sm and sm.get("t_warm_to_rmse_s"):
            # the metric's second half: time for each start to reach the plain method's final SOS error
            out["time_to_sos_rmse"] = {
                "target": "the SOS RMSE of the plain method after its 500 steps, per held-out scan",
                "plain_s": sm["t_plain_to_rmse_s"], "warm_s": sm["t_warm_to_rmse_s"],
                "speedup": sm["t_plain_to_rmse_s"] / sm["t_warm_to_rmse_s"],
                "rmse_plain_m_per_s": sm["rmse_plain"], "rmse_warm_start_m_per_s": sm["rmse_net"],
                "scans": sm["n_scans"], "reached_fraction": sm["rmse_target_reached_fraction"],
                "equal_loss_reached_fraction": sm.get("equal_loss_reached_fraction"),
                "loss_split_where_equal_loss_not_reached": sm.get("loss_split_not_reached")}
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", flush=True)
        out["cpu_baseline"] = cpu_baseline(scan, inp, args.cpu_steps)
    out["paper_context"] = dict(PAPER_CONTEXT, this_job_s=elapsed / args.steps,
                                this_job="das_stack + patch_fft + 500 pixel-grid steps on the paper-shaped scan")
    print(json.dumps(out), flush=True)


def precision_leg(P, sd, solver, scan, mask):
    """FP32 error of every quantity the step produces, against the FP64 oracle at the same state (the SOS after
    the timed jobs): the half spectra Y (oracle: FP64 windowed FFT of the GPU's DAS stack), and w, the data
    loss, dL/dw and dL/dv (oracle: its own Y, rays, deconvolution loss and reverse-mode gradient).  Relative
    L2 errors over every element (the loss: relative error)."""
    import numpy as np
    import torch
    from oracle import deconv as Odec, loss as Oloss, patches as Opatch, psf as Opsf
    from oracle.geometry import patch_centres
    F64 = torch.float64
    t0 = time.perf_counter()
    g = sd.geom
    sos = solver.sos.clone()
    rho = solver.support
    w = P.pact.sos_to_delays(sos, g, scan.v0, sd.centres, scan.n_samples, support=rho)
    loss, gw = sd.loss_and_grad(w, scan.eps)
    gv = P.pact.sos_to_delays_adjoint(sos, g, scan.v0, sd.centres, scan.n_samples, gw, support=rho)
    torch.cuda.synchronize()
    stack = sd.stack.cpu().double().numpy()
    Y = Opatch.patch_spectra(stack, scan.P, scan.stride, scan.px, scan.fwhm)
    geom = dict(sos_spacing=scan.sos_spacing, v0=scan.v0,
                centres=patch_centres(scan.ny, scan.nx, scan.px, scan.P, scan.stride), n_elem=scan.n_elem,
                radius=scan.radius, phi0=scan.phi0, n_samples=scan.n_samples, delays=np.asarray(scan.delays),
                px=scan.px, eps=scan.eps)
    ones = np.ones((scan.sos_n, scan.sos_n), dtype=bool)
    L, gv_o, gw_o, w_o = Oloss.loss_and_grad(sos.cpu().to(F64), ones, Y, geom, 0.0)
    # the transfer functions H (Eq. TF) and the deconvolved spectra X (Eq. multi-deconv), which the step's
    # fused loss never stores: the standalone entry points against the oracle's, each from its own w
    d32 = torch.tensor(np.asarray(scan.delays), dtype=torch.float32, device="cuda")
    H = P.pact.delays_to_psf(w, sd.centres, g, d32)
    X = torch.empty(sd.centres.shape[0], scan.P, scan.P, dtype=torch.complex64, device="cuda")
    P.pact.loss_and_grad(sd.Y, w, sd.centres, g, d32, scan.eps, want_grad=False, X=X)
    torch.cuda.synchronize()
    H_o = Opsf.transfer_functions(w_o, geom["centres"], scan.radius, scan.phi0, geom["delays"], scan.P, scan.px)
    X_o = Odec.multichannel_deconv(torch.as_tensor(Y), H_o, scan.eps)
    rel = lambda a, b: (torch.linalg.vector_norm(a.cpu().to(b.dtype) - b) / torch.linalg.vector_norm(b)).item()
    free = torch.as_tensor(np.asarray(mask)).bool()
    out = {"Y_half": rel(sd.Y, Opatch.half_spectrum(Y)), "w": rel(w, w_o), "H": rel(H, H_o), "X": rel(X, X_o),
           "loss": abs(loss.item() - L.item()) / abs(L.item()), "dL_dw": rel(gw, gw_o),
           "dL_dsos": rel(gv.cpu()[free], gv_o[free]),
           "measure": "relative L2 over every element (loss: relative error; dL/dsos: over the free nodes, the "
                      "ones the step updates), FP32 GPU against the FP64 oracle; H and X from the standalone "
                      "entry points (the step's loss forms neither)",
           "support_radius_mm": rho, "state": "the SOS after the timed jobs", "oracle_s": time.perf_counter() - t0}
    print("[bench] precision vs FP64 oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()
                                                           if isinstance(v, float) and k != "oracle_s"), flush=True)
    return out


def reconstruction_quality(P, sd, solver, inp, scan, job_s):
    """The state after the last timed job: SOS error on the free nodes, and the stitched deconvolved image
    (Supp. S1.4) against three references (PSNR / SSIM after scaling to the reference's range):
    - the aberration-free image: the same blobs in a uniform medium (SOS v0 everywhere), the same processing
      (DAS, patch spectra, deconvolution with w = 0, stitching).  It is what a perfect SOS correction gives, and
      it is band-limited like every reconstruction;
    - the deconvolution of the same data with the true SOS (Table 1's oracle row);
    - the synthetic initial pressure itself (unfiltered blobs, which no band-limited image matches)."""
    import numpy as np
    import torch
    import synth
    from synth.phantoms import SosPhantom
    from paper_2409_10876_amd import metrics
    g = sd.geom
    N = sd.centres.shape[0]
    X = torch.empty(N, g.P, g.P, dtype=torch.complex64, device=sd.S.device)

    def image(scan_data, w):
        scan_data.loss_and_grad(w, solver.eps, X=X)
        return P.pact.stitch(P.pact.ifft2_real(X), g)

    solver.delays()
    img = image(sd, solver.w)
    w0 = torch.zeros_like(solver.w)
    img0 = image(sd, w0)                                    # no SOS correction (uniform v0)
    mask = torch.tensor(inp.mask).bool()
    vt = torch.tensor(inp.sos_true)
    v_true = torch.where(mask, vt, torch.full_like(vt, scan.v0)).to(torch.float32).to(sd.S.device).contiguous()
    w_true = P.pact.sos_to_delays(v_true, g, scan.v0, sd.centres, scan.n_samples)
    img_true = image(sd, w_true)                            # deconvolution with the true SOS
    # the same blobs in a uniform medium, through the same processing
    S_free = synth.channel_data(scan, SosPhantom("uniform", scan.v0, {}), inp.blobs, rng=np.random.default_rng(0))
    sd_free = P.prepare_scan(scan, S_free, np.asarray(scan.delays, dtype=np.float32), device=sd.S.device)
    img_free = image(sd_free, w0)
    das = sd.stack[len(scan.delays) // 2]                   # the d = 0 DAS image
    torch.cuda.synchronize()
    rmse = lambda v: 1e3 * torch.sqrt(((v.cpu().double() - vt)[mask] ** 2).mean()).item()  # noqa: E731
    refs = {"aberration_free": img_free.cpu(), "true_sos_deconv": img_true.cpu(),
            "synthetic_truth": torch.tensor(inp.ip_true)}
    images = {"reconstructed": img, "true_sos_deconv": img_true, "uniform_sos": img0, "das_d0": das}
    q = {}
    for rname, ref in refs.items():
        q[rname] = {}
        for name, im in images.items():
            if name == rname:
                continue
            a, b = metrics.normalise(im.cpu().double(), ref.double())
            q[rname][name] = {"psnr_db": metrics.psnr(a, b), "ssim": metrics.ssim(a, b)}
    del sd_free
    return {"sos_rmse_m_per_s": rmse(solver.sos), "sos_rmse_initial_m_per_s": rmse(torch.full_like(vt, scan.v0)),
            "time_to_rmse_s": job_s, "ip_image": q,
            "note": "plain method after one timed job; IP figures after scaling to each reference's range"}


def delay_sweep(P, sd, scan, solver, counts=(4, 8, 11, 16), reps=20):
    """Fused loss-and-gradient time against the number of delay channels M (the paper's M-vs-time trend), on
    spectra of the same patch geometry: the direct form, which reads the M spectra at every step, and the
    projected form the step uses (its per-step work does not depend on M; the projection runs once per scan)."""
    import torch
    g = sd.geom
    N = sd.centres.shape[0]
    out = {}

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1_000_000)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return 1e3 * a.elapsed_time(b) / reps

    for M in counts:
        d = torch.linspace(-0.8, 0.8, M, device=sd.S.device)
        Y = torch.randn(N, M, g.P, g.P // 2 + 1, dtype=torch.complex64, device=sd.S.device)
        ws = torch.empty(max(1, P.pact.loss_and_grad_workspace_size(N, M, g.P, g.n_elem)), dtype=torch.uint8,
                         device=sd.S.device)
        gw = torch.empty_like(solver.w)
        T = P.pact.project_spectra(Y, g, d, sd.centres)
        us_direct = timed(lambda: P.pact.loss_and_grad(Y, solver.w, sd.centres, g, d, solver.eps, dL_dw=gw, ws=ws,
                                                       want_loss=False))
        us_proj = timed(lambda: P.pact.loss_and_grad_projected(T, M, solver.w, sd.centres, g, solver.eps, dL_dw=gw,
                                                               ws=ws, want_loss=False))
        us_once = timed(lambda: P.pact.project_spectra(Y, g, d, sd.centres, out=T))
        out[str(M)] = {"direct_us": us_direct, "direct_GB_per_s": N * M * g.P * (g.P // 2 + 1) * 8 / (us_direct * 1e-6) / 1e9,
                       "projected_us": us_proj, "project_once_us": us_once}
        del Y, ws, T
    print("[bench] delay sweep (us, direct / projected / projection once): " + ", ".join(
        f"M={k} {v['direct_us']:.1f}/{v['projected_us']:.1f}/{v['project_once_us']:.0f}" for k, v in out.items()),
        flush=True)
    return out


def siren_leg(P, sd, scan, inp, reps=100, graph_steps=50):
    """The paper's own neural-field form on the same scan: a 2 -> 256 -> 1 sinusoidal network (1027
    parameters) on the SOS-grid nodes, then the pixel-grid path; Adam on the network.  Graph-replayed steps
    per second, and each stage with HIP events."""
    import torch
    import synth
    solver = P.SirenSolver(sd, inp.mask, synth.nf.siren_params(256, 30.0), 256, 30.0, scan.mask_radius, lr=5e-3,
                           support_radius=scan.mask_radius,
                           eps=scan.eps, n_samples=scan.n_samples)
    solver.step()
    torch.cuda.synchronize()
    solver.capture(graph_steps)
    solver.run(graph_steps)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    solver.run(4 * graph_steps)
    b.record()
    torch.cuda.synchronize()
    us_step = 1e3 * a.elapsed_time(b) / (4 * graph_steps)
    stages = {"siren_sos": solver.sos_grid, "sos_to_delays": solver.delays, "loss_and_grad": solver.loss_grad,
              "adjoints (rays + network)": solver.adjoint, "adam_step": solver.update}
    evs = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
           for k in stages}
    torch.cuda._sleep(int(reps * 2_000_000))
    for r in range(reps):
        for k, fn in stages.items():
            evs[k][r][0].record()
            fn()
            evs[k][r][1].record()
    torch.cuda.synchronize()
    us = {k: 1e3 * sum(x.elapsed_time(y) for x, y in v) / reps for k, v in evs.items()}
    print(f"[bench] paper neural field: {us_step:.1f} us/step; " + ", ".join(f"{k} {v:.1f}" for k, v in us.items()),
          flush=True)
    return {"steps_per_s": 1e6 / us_step, "us_per_step": us_step, "stage_us": us,
            "config": "sinusoidal network 2 -> 256 -> 1 (1027 parameters, omega0 30) on the 140^2 SOS nodes, "
                      "then the pixel-grid path; no TV"}


def batch_leg(P, n_scans, steps=100, graph_steps=10):
    """Independent scans of uneven sizes (256^2 .. 768^2 px, 256 .. 1024 elements, 7 .. 15 delays, 64^2 or
    80^2 patches) solved together, three ways: per-scan step graphs replayed one scan after another, the same
    graphs on one stream each, and one launch per stage over all scans (five launches per batched step, captured
    in one graph; also over 2 and 4 groups of scans on their own streams).  Reports optimisation steps per second
    summed over the scans."""
    import numpy as np
    import torch
    import synth
    t0 = time.perf_counter()
    scans = synth.configs.batch_scans(n_scans)
    solvers = []
    for k, sc in enumerate(scans):
        inp = synth.make_inputs(sc, seed=sc.seed)
        sd = P.prepare_scan(sc, inp.S, np.asarray(sc.delays, dtype=np.float32))
        solvers.append(P.PixelGridSolver(sd, inp.mask, eps=sc.eps, lam=sc.lam_tv, lr=sc.lr, n_samples=sc.n_samples,
                                         support_radius=sc.mask_radius))
    print(f"[bench] batch: {n_scans} scans prepared in {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    batch = P.BatchedSolver(solvers, graph_steps=graph_steps, autotune=True)
    print(f"[bench] batch: ray tilings autotuned per scan shape in {time.perf_counter() - t0:.1f} s", flush=True)
    # one launch per stage over all scans, and over each of 2 and 4 groups of scans on their own streams
    grouped = {("grouped" if g == 1 else f"grouped_{g}_streams"): P.GroupedBatchSolver(solvers, graph_steps=graph_steps,
                                                                                       groups=g) for g in (1, 2, 4)}
    batch.run(graph_steps)
    batch.run_sequential(graph_steps)
    for gs in grouped.values():
        gs.run(graph_steps)
    torch.cuda.synchronize()
    out = {}
    forms = [("sequential", batch.run_sequential), ("concurrent", batch.run)] + \
        [(name, gs.run) for name, gs in grouped.items()]
    for name, fn in forms:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(steps)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        out[name] = {"ms": ms, "scan_steps_per_s": n_scans * steps / (ms * 1e-3)}
    out["speedup"] = out["sequential"]["ms"] / out["concurrent"]["ms"]
    out["speedup_grouped"] = out["sequential"]["ms"] / out["grouped"]["ms"]
    out["scans"] = [{"px": s.ny, "n_elem": s.n_elem, "M": s.M, "P": s.P, "patches": s.n_patches, "sos_n": s.sos_n,
                     "ray_tiling": list(t)} for s, t in zip(scans, batch.tilings)]
    best = min((k for k, _ in forms if k != "sequential"), key=lambda k: out[k]["ms"])
    out["fastest"] = best
    out["patches_x_delays_per_s"] = sum(s.n_patches * s.M for s in scans) * steps / (out[best]["ms"] * 1e-3)
    print(f"[bench] batch: {n_scans} scans x {steps} steps: sequential {out['sequential']['ms']:.1f} ms, "
          f"concurrent streams {out['concurrent']['ms']:.1f} ms, grouped launches {out['grouped']['ms']:.1f} ms, "
          f"in 2 groups {out['grouped_2_streams']['ms']:.1f} ms, in 4 groups {out['grouped_4_streams']['ms']:.1f} ms",
          flush=True)
    return out


WARM_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2409_10876_amd", "weights",
                            "warm_start.safetensors")
WARM_LEVELS = (1, 1, 2, 2, 4, 2, 1, 1)       # resolution divisor of each convolution's grid


def warm_flops(batch, G, real=False):
    """MFMA flops of one training step of the warm-start network (forward, input gradients of layers 2..8,
    weight gradients), as executed (K padded to 32) or with the real channel counts (11 inputs, 1 output)."""
    from paper_2409_10876_amd import warmstart as W
    kpad = lambda c: (9 * c + 31) // 32 * 32          # noqa: E731
    tot = 0
    for l, ((ci, co, _), s) in enumerate(zip(W.ARCH, WARM_LEVELS)):
        px = batch * (G // s) ** 2
        if real:
            ci = 11 if l == 0 else ci
            co = 1 if l == 7 else co
            tot += 2 * px * co * 9 * ci * (2 if l == 0 else 3)
        else:
            tot += 2 * px * co * kpad(ci) + 2 * px * co * 9 * ci + (2 * px * ci * kpad(co) if l > 0 else 0)
    return tot


def warm_leg(P, n_scans, batch=32, reps=20):
    """Learned warm start (an addition to the paper's self-supervised method): the committed trained
    initialiser on held-out scans of the paper-shaped geometry, plain optimisation from v0 against the
    network's SOS followed by the same steps; the training step and the main convolution kernel against
    the dense BF16 MFMA peak."""
    import numpy as np
    import torch
    import synth
    from synth.warm import WARM, phantom_batch
    from paper_2409_10876_amd import train_warm_start as T, warmstart as W
    if not os.path.exists(WARM_WEIGHTS):
        return {"skipped": "no trained weights at paper_2409_10876_amd/weights/warm_start.safetensors"}
    dev = torch.device("cuda:0")
    params, scale, meta = W.load_params(WARM_WEIGHTS)
    scan = synth.PAPER
    G = scan.sos_n
    sim = T.make_sim(scan, dev)
    net = W.WarmStartNet(1, G, G, params=params, n_inputs=scan.M, device=dev)
    rows = []
    for i in range(WARM.n_train, WARM.n_train + n_scans):
        sos, blobs = phantom_batch(scan, [i])
        rows.append(T.evaluate_scan(net, sim, scan, sos[0], blobs[0], scale, device=dev))
    summary = T.summarise(rows)
    curves = {k: np.mean([r[k] for r in rows], axis=0).tolist() for k in ("rmse_curve_plain", "rmse_curve_warm")}
    # training step and convolution timing at the training batch (synthetic inputs, the trained weights)
    tnet = W.WarmStartNet(batch, G, G, params=params, n_inputs=scan.M, device=dev)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = torch.zeros(batch, G, G, 16)
    x[..., :scan.M] = torch.randn(batch, G, G, scan.M, generator=g)
    x = x.to(torch.bfloat16).to(dev)
    tg = torch.randn(batch, G, G, generator=g).to(dev)
    mask = torch.from_numpy(synth.free_node_mask(scan)).to(dev)
    n_free = int(mask.sum())
    for _ in range(3):
        tnet.train_step(x, tg, mask, n_free, 1e-4)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        tnet.train_step(x, tg, mask, n_free, 1e-4)
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / reps
    fl, fl_real = warm_flops(batch, G), warm_flops(batch, G, real=True)
    # the 64 -> 64 convolution at full resolution (layers 2 and 7), one launch timed on the launch stream
    conv = lambda: P.pact.conv3x3(tnet.a1, tnet.packed[1][0], 64, bias=tnet.weights(1)[1], relu=True,  # noqa: E731
                                  out=tnet.a2)
    conv()
    a.record()
    for _ in range(reps):
        conv()
    b.record()
    torch.cuda.synchronize()
    us_conv = 1e3 * a.elapsed_time(b) / reps
    conv_flops = 2 * batch * G * G * 64 * 576
    wg = lambda: P.pact.conv3x3_wgrad(tnet.a1, tnet.gf[2], out=tnet.grad_slice(1), ws=tnet.ws)  # noqa: E731
    wg()
    a.record()
    for _ in range(reps):
        wg()
    b.record()
    torch.cuda.synchronize()
    us_wg = 1e3 * a.elapsed_time(b) / reps
    # the FP64 oracle of the network: forward and reverse mode for one image of the training shape
    from oracle import warmstart as Ow
    F64 = torch.float64
    xo = x[:1].float().cpu().to(F64)
    n_oracle = 8
    t0 = time.perf_counter()
    for _ in range(n_oracle):
        Ow.loss_and_grad(torch.tensor(params, dtype=F64), xo, tg[:1].cpu().to(F64), mask.cpu())
    dt_oracle = (time.perf_counter() - t0) / n_oracle
    print(f"[bench] warm start: rmse v0 {summary['rmse_v0']:.2f} net {summary['rmse_net']:.2f} plain "
          f"{summary['rmse_plain']:.2f} m/s; train step {ms_step:.2f} ms; conv 64->64 {us_conv:.1f} us; "
          f"weight gradient {us_wg:.1f} us", flush=True)
    return {
        "held_out_scans": n_scans, "summary": summary, "mean_rmse_curves_per_10_steps": curves,
        "weights": {k: meta[k] for k in meta}, "network": "8 conv 3x3, 64 channels, 2 poolings, 2 doublings with "
        "skips; BF16 MFMA, FP32 accumulation; input: 11-delay DAS stack averaged to 140^2",
        "cpu_oracle": {"value": 1.0 / dt_oracle, "unit": "images/s (forward + reverse-mode gradient)",
                       "cores": torch.get_num_threads(), "kind": "oracle",
                       "sample": f"{n_oracle} passes over one {G}x{G} image, float64, "
                                 f"{n_oracle * dt_oracle:.2f} s in all",
                       "gpu_images_per_s_training": batch / (ms_step * 1e-3)},
        "train_step": {"batch": batch, "ms": ms_step, "mfma_flops_executed": fl, "mfma_flops_real_channels": fl_real,
                       "tflops_executed": fl / (ms_step * 1e-3) / 1e12, "frac_of_bf16_peak": fl / (ms_step * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS},
        "conv3x3_64x64": {"kernel": "conv3x3_kernel<64,64>", "shape": f"{batch}x{G}x{G}x64", "us": us_conv,
                          "tflops": conv_flops / (us_conv * 1e-6) / 1e12,
                          "frac_of_bf16_peak": conv_flops / (us_conv * 1e-6) / 1e12 / MFMA_BF16_PEAK_TFLOPS},
        "conv3x3_wgrad_64x64": {"kernel": "conv3x3_wgrad_kernel<64,64> + sum_partials1/2", "us": us_wg,
                                "tflops": conv_flops / (us_wg * 1e-6) / 1e12,
                                "frac_of_bf16_peak": conv_flops / (us_wg * 1e-6) / 1e12 / MFMA_BF16_PEAK_TFLOPS},
    }


def nf_oracle_rate(scan, cfg, n_centres=16, n_elem=64):
    """The FP64 oracle of the neural field (forward and the layer-by-layer backward) on a bounded sample of
    rays of the same workload: ray samples per second on this host."""
    import numpy as np
    import torch
    import synth
    from oracle import nf as Onf
    from oracle.geometry import patch_centres
    F64 = torch.float64
    B = torch.tensor(synth.nf.frequencies(cfg), dtype=F64)
    params = torch.tensor(synth.nf.init_params(cfg), dtype=F64)
    c = patch_centres(scan.ny, scan.nx, scan.px, scan.P, scan.stride)[:n_centres]
    phi = scan.phi0 + 2 * np.pi * np.arange(0, scan.n_elem, scan.n_elem // n_elem)[:n_elem] / scan.n_elem
    ring = torch.tensor(np.stack([scan.radius * np.cos(phi), scan.radius * np.sin(phi)], -1), dtype=F64)
    gw = torch.ones(n_centres, n_elem, dtype=F64)
    t0 = time.perf_counter()
    Onf.sos_to_delays(params, B, c, ring, scan.mask_radius, scan.v0, cfg.amp, scan.n_samples)
    Onf.sos_to_delays_vjp(params, B, c, ring, scan.mask_radius, scan.v0, cfg.amp, scan.n_samples, gw)
    dt = time.perf_counter() - t0
    pts = n_centres * n_elem * scan.n_samples
    return {"value": pts / dt, "unit": "ray samples/s (forward + backward)", "cores": torch.get_num_threads(),
            "kind": "oracle", "sample": f"{n_centres} patch centres x {n_elem} elements x {scan.n_samples} samples "
                                        f"in {dt:.2f} s"}


def nf_bf16_error(solver, scan, cfg, n_centres=4, n_elem=32):
    """The BF16 error of the neural-field delays at the initial parameters, on a sample of rays, as relative L2
    of the GPU's w against the FP64 oracle network: with the FP32 master weights (the whole precision error of
    the workload: BF16 weights and activations), with the weights rounded to BF16 as the kernels use them (the
    activations' rounding alone), and with the kernels' BF16 rounding points too (what is left is FP32 against
    FP64 arithmetic: the logic)."""
    import numpy as np
    import torch
    import synth
    from oracle import nf as Onf
    F64 = torch.float64
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    solver.pack()
    solver.delays()
    stride = scan.n_elem // n_elem
    w = solver.w[:n_centres, ::stride][:, :n_elem].cpu().double()
    B = torch.tensor(np.asarray(synth.nf.frequencies(cfg), dtype=np.float32), dtype=F64)
    params = torch.tensor(np.asarray(synth.nf.init_params(cfg), dtype=np.float32), dtype=F64)
    blocks = Onf.unpack(params, cfg.n_freq, cfg.width)
    for name in ("W1", "W2", "W3", "W4", "w5"):
        blocks[name] = Onf.round_bf16(blocks[name])
    params_bf16 = Onf.pack(blocks, cfg.n_freq, cfg.width)
    c = solver.scan.centres[:n_centres].cpu().double()
    phi = f32(scan.phi0) + 2 * np.pi * np.arange(0, scan.n_elem, stride)[:n_elem] / scan.n_elem
    ring = torch.tensor(np.stack([f32(scan.radius) * np.cos(phi), f32(scan.radius) * np.sin(phi)], -1), dtype=F64)
    rel = lambda a, b: (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()  # noqa: E731
    out = {}
    for name, p, bf in (("w_vs_fp64_network", params, False), ("w_vs_fp64_network_bf16_weights", params_bf16, False),
                        ("w_vs_bf16_rounding_oracle", params_bf16, True)):
        out[name] = rel(w, Onf.sos_to_delays(p, B, c, ring, f32(scan.mask_radius), f32(scan.v0), f32(cfg.amp),
                                             scan.n_samples, bf16=bf))
    out["sample"] = f"{n_centres} patch centres x {n_elem} elements (every {stride}th), initial parameters"
    print(f"[bench] neural field BF16 error: w rel L2 {out['w_vs_fp64_network']:.2e} vs the FP64 network, "
          f"{out['w_vs_fp64_network_bf16_weights']:.2e} with its weights in BF16, "
          f"{out['w_vs_bf16_rounding_oracle']:.2e} vs the BF16-rounding oracle", flush=True)
    return out


def nf_leg(P, sd, scan, steps):
    """The neural-field workload on the same scan: Fourier features (128 frequencies) -> 4 x 128 ReLU -> SOS at
    every ray sample, BF16 MFMA.  Times `steps` optimisation steps and each stage (HIP events on the launch
    stream), and reports the network kernels against the dense BF16 MFMA peak."""
    import torch
    import synth
    cfg = synth.nf.NF
    net = P.pact.NfNet(cfg.n_freq, cfg.width, cfg.amp, scan.mask_radius)
    solver = P.NeuralFieldSolver(sd, synth.nf.frequencies(cfg), synth.nf.init_params(cfg), net, lr=scan.lr,
                                 eps=scan.eps, n_samples=scan.n_samples)
    bf16_error = nf_bf16_error(solver, scan, cfg)
    solver.step()
    torch.cuda.synchronize()
    stages = {"nf_pack": solver.pack, "nf_sos_to_delays": solver.delays, "loss_and_grad": solver.loss_grad,
              "nf_sos_to_delays_adjoint": solver.adjoint, "adam_step": solver.update}
    evs = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
           for k in stages}
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(2_000_000)
    t0.record()
    for r in range(steps):
        for k, fn in stages.items():
            evs[k][r][0].record()
            fn()
            evs[k][r][1].record()
    t1.record()
    torch.cuda.synchronize()
    us = {k: 1e3 * sum(a.elapsed_time(b) for a, b in v) / steps for k, v in evs.items()}
    step_ms = t0.elapsed_time(t1) / steps
    H, K = cfg.width, 2 * cfg.n_freq
    pts = scan.n_patches * scan.n_elem * scan.n_samples
    fwd = 2 * (H * K + 3 * H * H + H)                     # MFMA/FMA flops per point, forward
    # algorithmic backward per point: weight gradients of all layers + input gradients of layers 2-4 + head
    bwd = 2 * (H * K + 3 * H * H) + 2 * 3 * H * H + 2 * H
    peak = MFMA_BF16_PEAK_TFLOPS
    roof = {
        "nf_sos_to_delays": {"bound": "mfma", "achieved": pts * fwd / (us["nf_sos_to_delays"] * 1e-6) / 1e12,
                             "peak": peak, "unit": "TFLOP/s", "alg_flops_per_launch": pts * fwd,
                             "avg_launch_us": us["nf_sos_to_delays"]},
        "nf_sos_to_delays_adjoint": {"bound": "mfma",
                                     "achieved": pts * bwd / (us["nf_sos_to_delays_adjoint"] * 1e-6) / 1e12,
                                     "peak": peak, "unit": "TFLOP/s", "alg_flops_per_launch": pts * bwd,
                                     "avg_launch_us": us["nf_sos_to_delays_adjoint"],
                                     "note": "from the activations stored by the forward pass: one kernel for the head and layers 4..2 (writing the layer-1 pre-activation gradients), one for layer 1"},
    }
    for v in roof.values():
        v["frac"] = v["achieved"] / v["peak"]
    print(f"[bench] neural field: {step_ms:.2f} ms/step; " + ", ".join(f"{k} {v:.0f} us" for k, v in us.items()),
          flush=True)
    gpu_pts = pts / ((us["nf_sos_to_delays"] + us["nf_sos_to_delays_adjoint"]) * 1e-6)
    return {"steps_per_s": 1e3 / step_ms, "ms_per_step": step_ms, "steps_timed": steps, "stage_us": us,
            "rooflines": roof, "dtype": "bf16 MFMA, f32 accumulate",
            "points_per_s_fwd_adj": gpu_pts, "cpu_oracle": nf_oracle_rate(scan, cfg), "bf16_error": bf16_error,
            "config": f"Fourier features {cfg.n_freq} (sigma {cfg.sigma} /mm) -> {cfg.depth} x {cfg.width} ReLU -> "
                      f"SOS, {pts} ray samples per step"}


if __name__ == "__main__":
    main()
