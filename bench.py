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
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps timed for the CPU baseline")
    return ap.parse_args()


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
    return {"value": n_steps / dt, "unit": "steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n_steps} full FP64 oracle optimisation steps at the same workload "
                      f"({N} patches x {scan.M} delays, {scan.n_elem} elements, {scan.sos_n}^2 SOS grid, "
                      f"{scan.n_samples} samples/ray) in {dt:.1f} s; DAS/FFT not included",
            "patches_x_delays_per_s": n_steps * N * scan.M / dt}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2409_10876_amd as P
    from paper_2409_10876_amd import pact

    scan = synth.PAPER if args.workload == "paper" else synth.TINY
    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    inp = synth.make_inputs(scan, seed=0)
    print(f"[bench] inputs ready ({time.perf_counter() - t_setup:.1f} s): {synth.describe(scan)}", flush=True)

    sd = P.prepare_scan(scan, inp.S, np.asarray(scan.delays, dtype=np.float32), device=dev)
    solver = P.PixelGridSolver(sd, inp.mask, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples)
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
        solver.sos.copy_(sos0)
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
    stages = {"sos_to_delays": solver.delays, "loss_and_grad": solver.loss_grad,
              "sos_to_delays_adjoint": solver.adjoint, "tv_grad": solver.regularise, "adam_step": solver.update}
    reps = args.timing_steps
    evs = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
           for k in stages}
    das_ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
              torch.cuda.Event(enable_timing=True))
    # keep the GPU busy while Python enqueues the timing pass, so that each event pair brackets only the work
    # between them (no host launch gaps)
    torch.cuda._sleep(int(args.timing_steps * 2_000_000))
    das_ev[0].record()
    sd.stack = P.pact.das_stack(sd.S, sd.fs, sd.t0, sd.geom, sd.v0, sd.d, out=sd.stack)
    das_ev[1].record()
    sd.Y = P.pact.patch_fft(sd.stack, sd.geom, half=True, out=sd.Y)
    das_ev[2].record()
    for r in range(reps):
        for k, fn in stages.items():
            evs[k][r][0].record()
            fn()
            evs[k][r][1].record()
    torch.cuda.synchronize()
    breakdown = {k: 1e3 * sum(a.elapsed_time(b) for a, b in v) / reps for k, v in evs.items()}
    breakdown["das_stack_once"] = 1e3 * das_ev[0].elapsed_time(das_ev[1])
    breakdown["patch_fft_once"] = 1e3 * das_ev[1].elapsed_time(das_ev[2])
    loss_us = breakdown["loss_and_grad"]
    N, M, Pp = scan.n_patches, scan.M, scan.P
    y_bytes = N * M * Pp * (Pp // 2 + 1) * 8                # half spectra, complex64: read once per launch
    other = (N * scan.n_elem * 4) * 2 + 4                   # w read, dL/dw written, loss
    alg_bytes = y_bytes + other
    achieved = alg_bytes / (loss_us * 1e-6) / 1e9
    print("[bench] stage times (us): " + ", ".join(f"{k} {v:.1f}" for k, v in breakdown.items()), flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{scan.name}: {synth.describe(scan)}",
                   "bench_step": f"one job = das_stack + patch_fft once + {args.opt_steps} optimisation steps",
                   "opt_steps_per_job": args.opt_steps, "patches": N, "delays": M, "n_elem": scan.n_elem,
                   "sos_grid": scan.sos_n, "n_samples": scan.n_samples, "graph_steps": G},
        "patches_x_delays_per_s": value * N * M,
        "ms_per_opt_step": 1e3 * elapsed / opt_steps,
        "roofline": {"bound": "hbm", "kernel": "pact_loss_and_grad (loss_grad_kernel + loss_finish_kernel)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": alg_bytes, "avg_launch_us": loss_us,
                     "timing": f"HIP events around {reps} eager launches on the launch stream"},
        "stage_us": breakdown,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", flush=True)
        out["cpu_baseline"] = cpu_baseline(scan, inp, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
