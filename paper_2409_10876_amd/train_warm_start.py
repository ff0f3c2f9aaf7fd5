"""Train the warm-start network on scans from the method's own forward model, and compare the
warm-started optimisation with the plain one on held-out scans.

    python -m paper_2409_10876_amd.train_warm_start --out weights.safetensors            # train + evaluate
    python -m paper_2409_10876_amd.train_warm_start --weights weights.safetensors --n-train 0   # evaluate

Scans have the paper-shaped geometry (560^2 image at 0.1 mm, 512-element ring of radius 110 mm, 11
delays, 140^2 SOS nodes); phantoms come from ``synth.warm`` (seeded ellipse SOS maps of 1.450 - 1.620
mm/us and 100 initial-pressure blobs).  The whole training set lives in HBM (BF16 network inputs and FP32
targets, about 14 GB for 20 000 scans).

Evaluation per held-out scan:
* plain: ``steps`` optimisation steps from v0 (the paper's method); its final loss L_plain.
* warm: the network's SOS, then plain steps until the loss (data term plus TV) is at most L_plain.
The time of each (network inference included for the warm start) and the SOS RMSE on the free nodes
are reported.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

import synth
from synth.warm import WARM, phantom_batch

from . import pact
from .solver import PixelGridSolver, ScanData, geometry_from
from .warmstart import IN_CHANNELS, OUT_SCALE, ScanSimulator, WarmStartNet, input_scale, load_params, save


def log(msg: str):
    print(f"[warm] {msg}", flush=True)


def make_sim(scan, device) -> ScanSimulator:
    return ScanSimulator(geometry_from(scan), np.asarray(scan.delays, dtype=np.float32), scan.fs, scan.n_t, scan.t0,
                         scan.v0, n_samples=512, device=device)


def build_set(sim, scan, indices, scale, device, chunk=256, every=2000):
    """Network inputs [n][G][G][16] (BF16) and targets [n][G][G] (output units) of the given phantoms."""
    G = scan.sos_n
    n = len(indices)
    X = torch.zeros(n, G, G, IN_CHANNELS, dtype=torch.bfloat16, device=device)
    T = torch.empty(n, G, G, dtype=torch.float32, device=device)
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        idx = indices[c0:c0 + chunk]
        sos, blobs = phantom_batch(scan, idx)
        sos_d = torch.from_numpy(sos).to(device)
        blobs_d = torch.from_numpy(blobs).to(device)
        T[c0:c0 + len(idx)] = (sos_d - scan.v0) / OUT_SCALE
        for k in range(len(idx)):
            stack = sim.das(sos_d[k], blobs_d[k])
            sim.network_input(stack, scale, out=X[c0 + k])
        if (c0 // chunk) % max(1, every // chunk) == 0 or c0 + chunk >= n:
            torch.cuda.synchronize()
            log(f"scans {min(c0 + chunk, n)}/{n} ({time.perf_counter() - t0:.1f} s)")
    return X, T


def train(net, X, T, mask, n_free, epochs, batch, lr, Xv=None, Tv=None, seed=0, every=200):
    n = X.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    gen = torch.Generator().manual_seed(seed)
    xb = torch.empty((batch,) + tuple(X.shape[1:]), dtype=X.dtype, device=X.device)
    tb = torch.empty((batch,) + tuple(T.shape[1:]), dtype=T.dtype, device=T.device)
    history = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(X.device)
        run = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(T, 0, idx, out=tb)
            # constant rate, then a tenth of it for the last fifth of the steps
            rate = lr if step < 0.8 * total else 0.1 * lr
            net.train_step(xb, tb, mask, n_free, rate)
            step += 1
            if step % every == 0:
                run = float(net.loss)
                log(f"epoch {ep} step {step}/{total} loss {run:.4f} ({time.perf_counter() - t0:.1f} s)")
        last = float(net.loss)                       # the epoch's last training batch
        val = validate(net, Xv, Tv, mask, n_free, batch) if Xv is not None else None
        history.append({"epoch": ep, "train_loss_last_batch": last, "val_loss": val,
                        "elapsed_s": time.perf_counter() - t0})
        log(f"epoch {ep} done: train {last:.4f} val {val if val is None else round(val, 4)} "
            f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return history, time.perf_counter() - t0, total


def validate(net, X, T, mask, n_free, batch):
    tot, cnt = 0.0, 0
    for c0 in range(0, X.shape[0], batch):
        xb, tb = X[c0:c0 + batch], T[c0:c0 + batch]
        tot += float(net.loss_only(xb, tb, mask, n_free)) * xb.shape[0]
        cnt += xb.shape[0]
    return tot / cnt


def _reset(solver, sos_init):
    solver.set_sos(sos_init)
    solver.m.zero_()
    solver.v.zero_()
    solver.t.zero_()


def evaluate_scan(net, sim, scan, sos_true, blobs, scale, steps=500, chunk=10, device="cuda"):
    """Plain and warm-started optimisation of one scan (see the module docstring).  Both runs go the full
    `steps`, read the loss and keep a copy of the SOS after every chunk of steps, so that the time to a
    given loss or SOS error can be read off either run."""
    dev = torch.device(device)
    mask_np = synth.free_node_mask(scan)
    mask = torch.from_numpy(mask_np).to(dev)
    sos_d = torch.from_numpy(sos_true).to(dev)
    blobs_d = torch.from_numpy(blobs).to(dev)
    sim.channels(sos_d, blobs_d)
    sd = ScanData(sim.g, sim.S.clone(), sim.d, sim.fs, sim.t0, sim.v0)
    sd.prepare()
    vt = torch.from_numpy(sos_true).double()
    m = torch.from_numpy(mask_np).bool()

    def rmse(v):
        return 1e3 * math.sqrt(float(((v.detach().cpu().double() - vt)[m] ** 2).mean()))

    G = scan.sos_n
    n_chunks = steps // chunk
    v0 = torch.full((G, G), scan.v0, dtype=torch.float32, device=dev)
    solvers = []
    for _ in range(2):
        s = PixelGridSolver(sd, mask_np, eps=scan.eps, lam=scan.lam_tv, lr=scan.lr, n_samples=scan.n_samples,
                            support_radius=scan.mask_radius)
        s.step()
        s.capture(chunk)
        solvers.append(s)
    plain, warm = solvers
    snaps = torch.empty(2, n_chunks + 1, G, G, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def run(solver, snap, t_start):
        losses, times = [], []
        for k in range(n_chunks):
            solver.run(chunk)
            snap[k + 1].copy_(solver.sos)
            losses.append(float(solver.loss))            # loss of the chunk's last step (before its update)
            times.append(time.perf_counter() - t_start)
        return losses, times

    # plain: from v0
    _reset(plain, v0)
    snaps[0, 0].copy_(v0)
    t0 = time.perf_counter()
    loss_p, time_p = run(plain, snaps[0], t0)
    # warm: network inference, then the same steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = sim.network_input(sd.stack, scale)
    sos_net = net.predict_sos(x[None], mask, scan.v0)[0]
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    _reset(warm, sos_net)
    snaps[1, 0].copy_(sos_net)
    loss_w, time_w = run(warm, snaps[1], t0)
    torch.cuda.synchronize()
    rm_p = [rmse(snaps[0, k]) for k in range(n_chunks + 1)]
    rm_w = [rmse(snaps[1, k]) for k in range(n_chunks + 1)]
    # the loss split into its data term and lambda * TV at the network's SOS and at both final SOS grids
    terms = {name: loss_terms(plain, snaps[i, k].contiguous())
             for name, i, k in (("net", 1, 0), ("plain_final", 0, n_chunks), ("warm_final", 1, n_chunks))}
    L_plain = loss_p[-1]
    eq = next((k for k, L in enumerate(loss_w) if L <= L_plain), None)
    target = rm_p[-1]
    first_p = next(k for k, r in enumerate(rm_p) if r <= target)
    first_w = next((k for k, r in enumerate(rm_w) if r <= target), None)
    t_at = lambda times, k, t_first: t_first if k == 0 else times[k - 1]        # noqa: E731
    return {"rmse_v0": rm_p[0], "rmse_net": rm_w[0], "rmse_plain": rm_p[-1], "rmse_warm_final": rm_w[-1],
            "loss_plain": L_plain, "steps_plain": steps,
            "steps_warm_to_equal_loss": None if eq is None else (eq + 1) * chunk,
            "rmse_warm_at_equal_loss": None if eq is None else rm_w[eq + 1],
            "t_plain_s": time_p[-1], "t_inference_s": t_inf,
            "t_warm_to_equal_loss_s": None if eq is None else time_w[eq],
            "t_plain_to_rmse_s": t_at(time_p, first_p, 0.0),
            "t_warm_to_rmse_s": None if first_w is None else t_at(time_w, first_w, t_inf),
            "rmse_curve_plain": rm_p, "rmse_curve_warm": rm_w, "loss_curve_plain": loss_p, "loss_curve_warm": loss_w,
            **{f"data_{n}": t[0] for n, t in terms.items()}, **{f"lam_tv_{n}": t[1] for n, t in terms.items()}}


def loss_terms(solver, sos):
    """The two parts of the step's loss (Eq. jr) at an SOS grid: the data term of the fused deconvolution loss
    and lambda * TV."""
    w = pact.sos_to_delays(sos, solver.g, solver.scan.v0, solver.scan.centres, solver.n_samples,
                           support=solver.support)
    data, _ = solver.scan.loss_and_grad(w, solver.eps, want_grad=False)
    tvl = torch.zeros(1, dtype=torch.float32, device=sos.device)
    pact.tv_grad(sos.contiguous(), solver.mask, solver.g, solver.lam, torch.zeros_like(sos), tvl)
    return float(data), float(tvl)


def summarise(rows):
    def mean(key):
        vals = [r[key] for r in rows if r[key] is not None]
        return float(np.mean(vals)) if vals else None
    out = {k: mean(k) for k in ("rmse_v0", "rmse_net", "rmse_plain", "rmse_warm_final", "t_plain_s",
                                "t_inference_s", "t_plain_to_rmse_s", "t_warm_to_rmse_s")}
    reached = [r for r in rows if r["steps_warm_to_equal_loss"] is not None]
    out["equal_loss_reached_fraction"] = len(reached) / len(rows)
    if reached:
        out["steps_warm_to_equal_loss_mean_where_reached"] = float(np.mean([r["steps_warm_to_equal_loss"] for r in reached]))
        out["t_warm_to_equal_loss_s_mean_where_reached"] = float(np.mean([r["t_warm_to_equal_loss_s"] for r in reached]))
        out["rmse_warm_at_equal_loss_mean_where_reached"] = float(np.mean([r["rmse_warm_at_equal_loss"] for r in reached]))
        out["rmse_plain_mean_where_reached"] = float(np.mean([r["rmse_plain"] for r in reached]))
    # where the warm run stays above the plain run's final loss: which part of the loss keeps it there
    missed = [r for r in rows if r["steps_warm_to_equal_loss"] is None]
    for grp, rs in (("not_reached", missed), ("reached", reached)):
        if rs:
            out[f"loss_split_{grp}"] = {
                k: float(np.mean([r[k] for r in rs]))
                for k in ("data_net", "lam_tv_net", "data_plain_final", "lam_tv_plain_final", "data_warm_final",
                          "lam_tv_warm_final")}
    rr = [r for r in rows if r["t_warm_to_rmse_s"] is not None]
    out["rmse_target_reached_fraction"] = len(rr) / len(rows)
    if rr:
        out["speedup_time_to_plain_final_rmse"] = float(np.mean([r["t_plain_to_rmse_s"] for r in rr]) /
                                                        np.mean([r["t_warm_to_rmse_s"] for r in rr]))
    out["n_scans"] = len(rows)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n-train", type=int, default=WARM.n_train)
    ap.add_argument("--n-eval", type=int, default=WARM.n_eval)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--steps", type=int, default=500, help="plain optimisation steps")
    ap.add_argument("--weights", default=None, help="trained parameters to start from / evaluate")
    ap.add_argument("--out", default=None, help="where to save the trained parameters")
    ap.add_argument("--summary", default=None, help="JSON file for the results")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    scan = synth.PAPER
    G = scan.sos_n
    sim = make_sim(scan, dev)
    mask = torch.from_numpy(synth.free_node_mask(scan)).to(dev)
    n_free = int(mask.sum())
    params, scale = None, None
    if args.weights:
        params, scale, _ = load_params(args.weights)
    if scale is None:
        sos, blobs = phantom_batch(scan, list(range(16)))
        scale = input_scale(sim, [torch.from_numpy(s).to(dev) for s in sos], [torch.from_numpy(b).to(dev) for b in blobs])
        log(f"input scale {scale:.4g}")
    net = WarmStartNet(args.batch, G, G, params=params, n_inputs=scan.M, device=dev)
    result = {"n_train": args.n_train, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
              "input_scale": scale}
    eval_idx = list(range(WARM.n_train, WARM.n_train + args.n_eval))
    if args.n_train > 0:
        t0 = time.perf_counter()
        X, T = build_set(sim, scan, list(range(args.n_train)), scale, dev)
        Xv, Tv = build_set(sim, scan, eval_idx, scale, dev)
        result["data_s"] = time.perf_counter() - t0
        log(f"training set ready: {args.n_train} scans in {result['data_s']:.1f} s")
        hist, t_train, n_steps = train(net, X, T, mask, n_free, args.epochs, args.batch, args.lr, Xv, Tv)
        result.update(history=hist, train_s=t_train, train_steps=n_steps, ms_per_train_step=1e3 * t_train / n_steps)
        del X, T
        torch.cuda.empty_cache()
        if args.out:
            save(args.out, net.params, scale, {"n_train": args.n_train, "epochs": args.epochs})
            log(f"saved {args.out}")
    rows = []
    for k, i in enumerate(eval_idx):
        sos, blobs = phantom_batch(scan, [i])
        r = evaluate_scan(net, sim, scan, sos[0], blobs[0], scale, steps=args.steps, device=dev)
        rows.append(r)
        log(f"eval {k + 1}/{len(eval_idx)}: rmse v0 {r['rmse_v0']:.2f} net {r['rmse_net']:.2f} plain "
            f"{r['rmse_plain']:.2f} warm(final) {r['rmse_warm_final']:.2f} m/s; warm steps to equal loss "
            f"{r['steps_warm_to_equal_loss']}; time to plain's final rmse: warm {r['t_warm_to_rmse_s']} "
            f"plain {r['t_plain_to_rmse_s']:.4f} s")
    result["eval"] = summarise(rows)
    result["eval_rows"] = [{k: v for k, v in r.items() if not k.endswith("_curve_plain") and not k.endswith("_curve_warm")}
                           for r in rows]
    # mean curves over the held-out scans (per chunk of steps)
    for key in ("rmse_curve_plain", "rmse_curve_warm", "loss_curve_plain", "loss_curve_warm"):
        result[key + "_mean"] = np.mean([r[key] for r in rows], axis=0).tolist()
    log("summary " + json.dumps(result["eval"]))
    if args.summary:
        with open(args.summary, "w") as f:
            json.dump(result, f, indent=1)


if __name__ == "__main__":
    main()
