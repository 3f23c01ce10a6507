#!/usr/bin/env python
"""Benchmark of the ICRS hot path on one MI355X: magnified epochs per second.

Workload: 2048 binary planetary-regime events (log10 q in [-5,-2], s in [0.5,2], u0 in
[0,0.3], linear limb darkening u in [0.3,0.7]) with rho = 1e-3 and 100..5000 epochs each,
clustered within +-3 rho tE of caustic crossings (about 5.1 million epochs); 128 limb points,
FP32 ray loop, FP32 Ehrlich-Aberth with FP64 polish.  One step is one full pass of the path
over the whole batch with inputs resident in HBM.  Grids come from the autotuner, untimed,
on a 1% calibration subset of the same batch:
  * plain grid: the smallest grid whose median error is within 1e-4 of the grid-free disk
    quadrature (icrs_disk_magnification, on the calibration epochs where no caustic crosses
    the disk: the metric's accuracy, measured against the true magnification);
  * learned grid and drift gate: the fastest pair whose median error is within 1e-4 of the
    same reference and whose 99th percentile is no worse than the plain path's.
Lines:
  * batched+learned (the headline `value`): the batch uploaded once (icrs_prepare), each step
    one replay of a captured HIP graph of the learned path (centre images, 16 check points,
    the bounds network on the matrix cores, per-image boxes, rays, drift gate, and the plain
    path for every epoch the checks hand back -- list sizes stay on the device);
  * plain: one eager icrs_magnification call per step over the batch (profiled: the main ray
    pass is one launch per step); batched+plain: the same path as a graph replay;
    plain_per_event: one call per event on the first 128 events.

Printed: one JSON line with the throughputs, the dominant kernel's roofline position (timed
live with HIP events on the library's stream), the oracle's CPU throughput on a sample of the
same epochs, and, on that sample, each path's agreement with the oracle and its error
against the oracle's grid-free source-disk quadrature (the exact finite-source magnification
where no caustic crosses the disk), with the 1e-4 accuracy bar stated as met or not; and the
learned path against the plain path on every epoch.
"""
from __future__ import annotations

import argparse
import json
from concurrent.futures import ThreadPoolExecutor
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "magnified epochs/sec at rho=1e-3 LD (rel err<=1e-4), plain vs batched+learned"
FLOPS_PER_RAY = {2: 35.0, 3: 48.0}          # algorithmic flop-equivalents per ray
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}  # MI355X vector peaks
def kernel_name(rays, n_theta):
    """The ray kernel instantiation a grid of n_theta columns runs on (2, 4, 8, 12 or 16 columns per lane)."""
    j = (n_theta + 63) // 64
    jmax = 2 if j <= 2 else 4 if j <= 4 else 8 if j <= 8 else 12 if j <= 12 else 16
    exact = n_theta % 64 == 0 and j == jmax
    m = "MapF32" if rays == "fp32" else "MapF64"
    return f"rays_kernel<2, {jmax}, {'true' if exact else 'false'}, {m}<2, {jmax}>>"


# HBM bytes per launch of the main ray kernel from rocprofv3 FETCH_SIZE + WRITE_SIZE passes,
# scaled by the same counters' reading on a plain copy kernel of known size (FETCH reads 2.0x
# low, WRITE 1.0x on this machine); keyed by (ray precision, events, path, N_r, N_theta).
# Filled in from measured counter runs of the current kernels; absent (null) otherwise.
TRAFFIC = {("fp32", 2048, "plain", 192, 512): 2.3785e11,      # FETCH 68574614 KiB x 2.0 + WRITE 95127772 KiB
           ("fp32", 2048, "fallback", 192, 512): 1.9308e11,   # FETCH 55158908 KiB x 2.0 + WRITE 78235439 KiB
           ("fp32", 2048, "learned", 32, 128): 5.8938e10}     # FETCH 18143603 KiB x 2.0 + WRITE 21269333 KiB


def cpu_baseline(w, mags, budget_s, seed=0):
    """The FP64 oracle on a bounded sample of the same epochs, on all host threads (median of
    three timings) and on one (median of three); on the same sample, each GPU path against the oracle and against the oracle's source-disk
    quadrature (epochs where no caustic crosses the disk and two resolutions agree)."""
    from oracle import oracle as O
    rng = np.random.default_rng(seed)
    ev_of = np.repeat(np.arange(w.n_events), np.diff(w.offsets))

    threads = O.num_threads()

    def run(idx, workers):
        """Oracle magnifications of the sampled epochs, one event per job on `workers` host
        threads (each job's OpenMP region held to one thread); returns (idx, mag, seconds)."""
        idx = np.sort(idx)
        out = np.empty(idx.size)
        ev = np.unique(ev_of[idx])

        def one(i):
            O.set_num_threads(1)
            sel = idx[ev_of[idx] == i]
            out[np.searchsorted(idx, sel)] = O.magnification(w.n_lens, w.params[i], w.t[sel], n_limb=w.n_limb,
                                                             n_r=w.n_r, n_theta=w.n_theta)["mag"]

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, ev))
        return idx, out, time.perf_counter() - t0

    _, _, dt = run(rng.choice(w.n_epochs, size=4 * threads, replace=False), threads)
    n = int(np.clip(budget_s / max(dt / (4 * threads), 1e-6), 96, 30000)) // 3 * 3
    idx = np.sort(rng.choice(w.n_epochs, size=n, replace=False))
    # all threads: three disjoint thirds of the sample, the rate the median of the three
    parts = [run(idx[k::3], threads) for k in range(3)]
    rates = sorted(p[0].size / p[2] for p in parts)
    mag = np.empty(idx.size)
    for p_idx, p_mag, _ in parts:
        mag[np.searchsorted(idx, p_idx)] = p_mag
    dt = sum(p[2] for p in parts)
    # one thread: three small samples, median
    n1 = 24
    one = sorted(n1 / run(rng.choice(w.n_epochs, size=n1, replace=False), 1)[2] for _ in range(3))
    ref = np.full(idx.size, np.nan)
    for i in np.unique(ev_of[idx]):
        sel = np.nonzero(ev_of[idx] == i)[0]
        m1, ch = O.disk_mag(w.n_lens, w.params[i], w.t[idx[sel]], n_x=16, n_phi=96)
        m2, _ = O.disk_mag(w.n_lens, w.params[i], w.t[idx[sel]], n_x=24, n_phi=144)
        ok = (ch == 0) & (np.abs(m1 / m2 - 1.0) < 1e-7)
        ref[sel[ok]] = m2[ok]
    good = np.isfinite(ref)
    acc = {"n_sampled": int(idx.size), "n_disk_reference": int(good.sum())}
    for name, g in mags.items():
        rel = np.abs(g[idx] / mag - 1.0)
        err = np.abs(g[idx][good] / ref[good] - 1.0)
        acc[name] = {"vs_oracle_max": float(rel.max()), "vs_oracle_median": float(np.median(rel)),
                     "vs_disk_median": float(np.median(err)), "vs_disk_p99": float(np.quantile(err, 0.99)),
                     "vs_disk_max": float(err.max()), "vs_disk_frac_le_1e-4": float(np.mean(err <= 1e-4))}
    return {
        "value": rates[1], "unit": "epochs/s", "cores": threads, "kind": "oracle",
        "single_core": {"value": one[1], "unit": "epochs/s", "cores": 1, "runs": one, "epochs_per_run": n1},
        "runs": rates,
        "sample": f"{idx.size} epochs drawn uniformly (seed {seed}) from the same workload, timed as three "
                  f"disjoint thirds (median rate), FP64 oracle (plain path), {w.n_r}x{w.n_theta} grids, "
                  f"{dt:.1f} s on {threads} threads; single core: median of three runs of {n1} epochs",
    }, acc, (idx[good], ref[good])


PLAIN_LADDER = [(128, 512), (256, 512), (128, 1024), (256, 1024), (512, 1024)]
LEARNED_LADDER = [(64, 256), (128, 512), (256, 512), (128, 1024), (256, 1024)]


def accuracy_sweep(w, model, gate_rel, idx, ref, every=10, gate_slack=0.0):
    """Throughput against true accuracy: each path on a ladder of grids, its error against the
    grid-free disk quadrature on the sampled epochs, and its rate on every `every`-th epoch of
    the workload (inputs resident, one warm-up call, then one timed call).  The learned rungs
    hand their fallback epochs to the plain grid of the same rung.  Picks, per path, the
    fastest grid whose median error is at most 1e-4."""
    import torch
    from paper_2510_02639_amd import icrs, workloads
    ev_of = np.repeat(np.arange(w.n_events), np.diff(w.offsets))
    one = workloads.Workload("sampled", 2, w.params[ev_of[idx]], np.arange(idx.size + 1, dtype=np.int64), w.t[idx],
                             w.n_limb, w.n_r, w.n_theta, "fp32", "fp32")
    sub = w.sample_epochs(every)
    t_one = torch.tensor(one.t, device="cuda")
    t_sub = torch.tensor(sub.t, device="cuda")
    out = {"reference": f"grid-free source-disk quadrature of the oracle on {idx.size} sampled epochs",
           "rate_subset_epochs": int(sub.n_epochs)}

    def stats(m):
        e = np.abs(m / ref - 1.0)
        return {"median": float(np.median(e)), "p90": float(np.quantile(e, 0.9)),
                "p99": float(np.quantile(e, 0.99)), "frac_le_1e-4": float(np.mean(e <= 1e-4))}

    def rate(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return sub.n_epochs / (time.perf_counter() - t0)

    for name, ladder in (("plain", PLAIN_LADDER), ("batched+learned", LEARNED_LADDER)):
        rows = []
        for rung, (n_r, n_theta) in enumerate(ladder):
            pg = PLAIN_LADDER[rung]
            hg = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=pg[0], n_theta=pg[1], ray_precision="fp32",
                             root_precision="fp32")
            if name == "plain":
                m = hg.magnification(one.params, one.offsets, t_one)[0].cpu().numpy()
                ws = hg.workspace(sub.n_events, sub.n_epochs)
                r = rate(lambda: hg.magnification(sub.params, sub.offsets, t_sub, workspace=ws))
            else:
                m = hg.magnification_learned(one.params, one.offsets, t_one, model, n_r=n_r, n_theta=n_theta,
                                             gate_rel=gate_rel, gate_slack=gate_slack)[0].cpu().numpy()
                ws = hg.learned_workspace(sub.n_events, sub.n_epochs)
                r = rate(lambda: hg.magnification_learned(sub.params, sub.offsets, t_sub, model, workspace=ws,
                                                          n_r=n_r, n_theta=n_theta, gate_rel=gate_rel,
                                                          gate_slack=gate_slack, stats=False))
            rows.append({"grid": [n_r, n_theta], "epochs_per_s": r, **stats(m)})
            print(f"[bench] sweep {name} {n_r}x{n_theta}: {r:.3g} epochs/s, median err {rows[-1]['median']:.2e}",
                  file=sys.stderr, flush=True)
        out[name] = rows
    pick = {}
    for name in ("plain", "batched+learned"):
        ok = [r for r in out[name] if r["median"] <= 1e-4]
        pick[name] = max(ok, key=lambda r: r["epochs_per_s"]) if ok else None
    out["median_le_1e-4"] = pick
    return out


def timed_steps(fn, steps, warmup, label, after_warmup=None):
    import torch
    for k in range(warmup):
        fn()
        torch.cuda.synchronize()
        print(f"[bench] {label}: warmup step {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    if after_warmup:
        after_warmup()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for k in range(steps):
        out = fn()
        print(f"[bench] {label}: step {k + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def timed_graph(capture, steps, warmup, label, stream):
    """Capture one step into a HIP graph on stream (the handle's; after one eager warm-up of
    capture()), then replay: warmup untimed replays, steps timed replays bracketed by device
    synchronisation."""
    import torch
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        capture()
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        capture()
    for k in range(warmup):
        g.replay()
        torch.cuda.synchronize()
        print(f"[bench] {label}: warmup replay {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {label}: {steps} replays in {dt:.3f} s", file=sys.stderr, flush=True)
    return dt


def per_event_plain(h, w, t, n_events=128):
    """The plain path launched event by event (one call per event, no batching across
    events), on the first n_events events; epochs/s."""
    import torch
    sub = w.subset(range(min(n_events, w.n_events)))
    ts = torch.tensor(sub.t, device="cuda")
    ws = h.workspace(1, int(np.max(np.diff(sub.offsets))))
    calls = [(sub.params[i:i + 1], np.array([0, sub.offsets[i + 1] - sub.offsets[i]], np.int64),
              ts[sub.offsets[i]:sub.offsets[i + 1]]) for i in range(sub.n_events)]
    for p, o, tt in calls[:4]:
        h.magnification(p, o, tt, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, o, tt in calls:
        h.magnification(p, o, tt, workspace=ws)
    torch.cuda.synchronize()
    return sub.n_epochs / (time.perf_counter() - t0), sub.n_events


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=2048)
    ap.add_argument("--rays", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--roots", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the accuracy/throughput sweep over grids")
    ap.add_argument("--plain-only", action="store_true", help="time the plain path only (profiling runs)")
    ap.add_argument("--learned-only", action="store_true", help="time the batched+learned path only (profiling runs)")
    ap.add_argument("--grid", default=None, help="plain grid NRxNT instead of the autotuner's (profiling runs)")
    ap.add_argument("--learned", default=None,
                    help="learned grid and gate NRxNT:GATE:SLACK instead of the autotuner's (profiling runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the path has no multi-GPU leg); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe_mib:
        # one elementwise kernel that reads and writes copy_probe_mib MiB each, a few times
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "launches": 3}), flush=True)
        return
    from paper_2510_02639_amd import autotune, icrs, learned, workloads

    t_gen = time.perf_counter()
    w = workloads.metric_workload(args.events)
    print(f"[bench] workload {w.name}: {w.n_events} events, {w.n_epochs} epochs "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    t = torch.tensor(w.t, device="cuda")
    mag = torch.empty(w.n_epochs, dtype=torch.float64, device="cuda")
    status = torch.empty(w.n_epochs, dtype=torch.int32, device="cuda")

    # plain grid: the autotuner's smallest grid whose median error on a 1% calibration subset
    # is within 1e-4 of the grid-free disk quadrature (epochs where no caustic crosses the disk)
    t_tune = time.perf_counter()
    if args.grid:
        ptune = None
        grid = tuple(int(x) for x in args.grid.split("x"))
    else:
        ptune = autotune.tune(w, tol=1e-4, every=100, stat="median", roots=args.roots, reference="disk")
        grid = (ptune.n_r, ptune.n_theta)
    t_tune = time.perf_counter() - t_tune
    print(f"[bench] plain grid {grid[0]} x {grid[1]} (tuned in {t_tune:.1f} s)", file=sys.stderr, flush=True)
    hs = torch.cuda.Stream()   # the library's stream: eager calls and graph capture
    h = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=grid[0], n_theta=grid[1], ray_precision=args.rays,
                    root_precision=args.roots, stream=hs)
    ws = h.learned_workspace(w.n_events, w.n_epochs)

    # plain path, one eager call per step over the whole batch, profiled after the warm-up
    def start_profile():
        h.set_profiling(True)
        h.get_profile(reset=True)

    line = {"metric": METRIC}
    plain = {}
    if not args.learned_only:
        _, dt_plain = timed_steps(lambda: h.magnification(w.params, w.offsets, t, mag, status, ws), args.steps,
                                  args.warmup, "plain", start_profile)
        prof = h.get_profile()
        h.set_profiling(False)
        gm_plain = mag.cpu().numpy()
        st = status.cpu().numpy().astype(np.uint32)
        plain_value = w.n_epochs * args.steps / dt_plain
        # batched+plain: the same path prepared once and replayed as one captured graph
        h.prepare(w.params, w.offsets, w.n_epochs, workspace=ws)
        dt_bp = timed_graph(lambda: h.run(t, mag, status), args.steps, args.warmup, "batched+plain", hs)
        bp_equal = bool(np.array_equal(mag.cpu().numpy(), gm_plain))
        pe_rate, pe_events = per_event_plain(h, w, t)
        plain = {"value": plain_value, "ms_per_step": dt_plain * 1e3 / args.steps, "grid": list(grid),
                 "rays_per_s": prof["n_sector_passes"] * grid[0] * grid[1] / dt_plain,
                 "breakdown_ms_per_step": {k: prof[k] / args.steps for k in
                                           ("ms_centre", "ms_limb_sectors", "ms_rays", "ms_rays_main",
                                            "ms_finalize")},
                 "sectors_per_epoch": prof["n_sector_passes"] / max(prof["n_epochs"], 1),
                 "status_counts": {name: int(np.sum((st & bit) != 0)) for name, bit in
                                   [("root_nonconv", 1), ("img_count", 2), ("cap_overflow", 4), ("clip", 8),
                                    ("nan", 16)]},
                 "autotune": None if ptune is None else {
                     "target": "median rel err <= 1e-4 vs the grid-free disk quadrature (device, epochs where no "
                               "caustic crosses the disk at 16x96 and 24x144 nodes, agreeing to 1e-7)",
                     "calibration_epochs": ptune.n_calibration, "trusted": ptune.n_trusted,
                     "tried": ptune.errors, "seconds": t_tune}}
        line["batched+plain"] = {"value": w.n_epochs * args.steps / dt_bp, "ms_per_step": dt_bp * 1e3 / args.steps,
                                 "graph": True, "bitwise_equal_to_eager": bp_equal}
        line["plain_per_event"] = {"value": pe_rate, "events_timed": pe_events,
                                   "launch": "one icrs_magnification call per event"}

    value, dt_value = (plain.get("value"), None)
    if not args.plain_only:
        model = learned.BoundsModel.load()
        # learned grid and gate: the autotuner's fastest pair whose median error on the
        # calibration subset is within 1e-4 of the disk quadrature and whose p99 is no worse
        # than the plain path's at the plain grid
        t_lt = time.perf_counter()
        if args.learned:
            g, gate, slack = args.learned.split(":")
            nr, nt = (int(x) for x in g.split("x"))
            tune = autotune.LearnedTuneResult(nr, nt, float(gate), float(slack), tuple(grid), (None, None), [], 0, {})
        else:
            tune = autotune.tune_learned(w, model, plain_grid=grid, every=100)
        t_lt = time.perf_counter() - t_lt
        print(f"[bench] learned grid {tune.n_r} x {tune.n_theta}, gate {tune.gate_rel:g}/{tune.gate_slack:g} "
              f"(tuned in {t_lt:.1f} s)",
              file=sys.stderr, flush=True)
        kw = dict(n_r=tune.n_r, n_theta=tune.n_theta, gate_rel=tune.gate_rel, gate_slack=tune.gate_slack)
        mag_l = torch.empty_like(mag)
        status_l = torch.empty_like(status)
        # batched+learned (the headline): prepared once, one captured graph per step
        h.prepare(w.params, w.offsets, w.n_epochs, workspace=ws)
        dt_learned = timed_graph(lambda: h.run_learned(t, model, mag_l, status_l, **kw), args.steps, args.warmup,
                                 "batched+learned", hs)
        gm_learned = mag_l.cpu().numpy()
        value, dt_value = w.n_epochs * args.steps / dt_learned, dt_learned
        # statistics and the profiled learned main pass, from one more (eager, untimed) step
        h.set_profiling(True)
        h.get_profile(reset=True)
        _, _, lstats = h.magnification_learned(w.params, w.offsets, t, model, mag_l, status_l, ws, **kw)
        torch.cuda.synchronize()
        lprof = h.get_profile()
        h.set_profiling(False)
        eager_equal = bool(np.array_equal(mag_l.cpu().numpy(), gm_learned))
    else:
        dt_value = plain["ms_per_step"] * args.steps / 1e3

    peak = PEAK_TFLOPS[args.rays]

    def roofline(n_rays, ms, n_launch, n_r, n_theta, path, timed):
        achieved = n_rays * FLOPS_PER_RAY[2] / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": TRAFFIC.get((args.rays, w.n_events, path, n_r, n_theta)),
                "kernel": kernel_name(args.rays, n_theta),
                "flops_per_ray": FLOPS_PER_RAY[2], "rays_per_launch_avg": n_rays / max(n_launch, 1),
                "kernel_ms_per_launch_avg": ms / max(n_launch, 1), "path_timed": timed}

    if plain:
        plain["roofline"] = roofline(prof["n_main_rays"], prof["ms_rays_main"], prof["n_main_launches"], grid[0], grid[1],
                                     "plain", "plain (one main-pass launch per step)")
    line.update({
        "value": value, "unit": "epochs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt_value * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.rays == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_events": w.n_events, "n_epochs": w.n_epochs, "n_limb": w.n_limb,
                   "plain_grid": list(grid), "ray_precision": args.rays,
                   "root_precision": "fp32+fp64-polish" if args.roots == "fp32" else "fp64",
                   "path": "plain" if args.plain_only else "batched+learned", "rho": 1e-3,
                   "learned_grid": None if args.plain_only else [tune.n_r, tune.n_theta],
                   "graph": not args.plain_only},
    })
    if plain:
        line["plain"] = plain
    # the dominant kernel of the timed step: whichever main ray pass of the learned step takes
    # longer -- the learned boxes' or the plain path's on the epochs handed back (the plain
    # path's main pass when only that path runs)
    if args.plain_only:
        line["roofline"] = plain["roofline"]
    elif lprof["ms_rays_learned"] >= lprof["ms_rays_main"]:
        line["roofline"] = roofline(
            lprof["n_learned_rays"], lprof["ms_rays_learned"], lprof["n_learned_launches"], tune.n_r, tune.n_theta,
            "learned", "batched+learned: the learned boxes' main ray pass (one launch per step; profiled on one "
            "extra step)")
    else:
        line["roofline"] = roofline(
            lprof["n_main_rays"], lprof["ms_rays_main"], lprof["n_main_launches"], grid[0], grid[1], "fallback",
            "batched+learned: the plain main ray pass over the epochs the learned path hands back (one launch per "
            "step; profiled on one extra step)")
    if not args.plain_only:
        line["roofline"]["other_main_pass_ms"] = {"learned_boxes": lprof["ms_rays_learned"],
                                                  "plain_fallback": lprof["ms_rays_main"]}
    if not args.plain_only:
        line["learned"] = {"stats_per_step": lstats, "model": "paper_2510_02639_amd/data/bounds_mlp.npz",
                           "log_safety": model.log_safety, "grid": [tune.n_r, tune.n_theta],
                           "gate_rel": tune.gate_rel, "gate_slack": tune.gate_slack,
                           "graph_equal_to_eager": eager_equal,
                           "autotune": {"plain_error_median_p99": tune.plain_error, "tried": tune.errors,
                                        "calibration_epochs": tune.n_calibration, "rates": tune.rates,
                                        "seconds": t_lt}}
        if plain:
            d = np.abs(gm_learned / gm_plain - 1.0)
            line["learned"]["vs_plain_all_epochs"] = {
                "max": float(d.max()), "median": float(np.median(d)), "p99": float(np.quantile(d, 0.99)),
                "frac_above_1e-4": float(np.mean(d > 1e-4)), "plain_grid": list(grid),
                "learned_grid": [tune.n_r, tune.n_theta]}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        mags = {}
        if plain:
            mags["plain"] = gm_plain
        if not args.plain_only:
            mags["batched+learned"] = gm_learned
        wb = workloads.Workload(w.name, w.n_lens, w.params, w.offsets, w.t, w.n_limb, grid[0], grid[1], w.ray_precision,
                                w.root_precision)
        base, acc, (s_idx, s_ref) = cpu_baseline(wb, mags, args.cpu_seconds)
        line["cpu_baseline"] = base
        line["accuracy"] = acc
        hl = acc.get("batched+learned")
        if hl:
            line["accuracy_bar"] = {
                "target_rel_err": 1e-4, "reference": "grid-free source-disk quadrature (oracle), sampled epochs",
                "headline_median": hl["vs_disk_median"], "headline_p99": hl["vs_disk_p99"],
                "headline_max": hl["vs_disk_max"], "frac_le_1e-4": hl["vs_disk_frac_le_1e-4"],
                "met_by_median": hl["vs_disk_median"] <= 1e-4, "met_by_every_epoch": hl["vs_disk_max"] <= 1e-4}
        if not args.plain_only and not args.no_sweep and plain:
            line["accuracy_sweep"] = accuracy_sweep(w, model, tune.gate_rel, s_idx, s_ref, gate_slack=tune.gate_slack)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
