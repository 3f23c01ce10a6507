"""Throughput of the path's other rows on one GPU, one JSON line per measurement:

  config1   the plain FP64 path on the single binary event (s = 0.9, q = 0.1, rho = 1e-2,
            200 epochs across the central caustic, 64 x 256): epochs/s and the ray pass's
            FP64 roofline;
  config2   the planetary batch (2048 events, rho ~ logU[10^-3.5, 10^-2], 128 x 512, FP32
            rays) in one call: epochs/s, rays/s and the main pass's FP32 roofline;
  adjoint   forward + reverse-mode gradient on the differentiable-fit workload (512 binary
            events x 3000 epochs, rho = 1e-3; cotangent N(0,1), seed 40): epochs/s of the
            forward and of the VJP, and the VJP's ray rate;
  triple    the triple-lens workload (256 events x 2000 epochs, FP64 roots, FP32 rays);
  train     device training of the bounds network: rows/s of loss+gradient+AdamW steps;
  serve     the serving loop at 200 events/s for a few seconds (p50/p99 latency);
  hybrid    the hybrid light curve (Sec. 3.4, item iii) on a survey cadence (512 events x 8640
            epochs, 72 d at 12 min): the selected fraction, epochs/s of the hybrid curve and of
            the plain path on every epoch of the same batch;
  nll       the fit objective of App. B (marginalised NLL and its gradient through the
            reverse mode) on the cadence batch with the hybrid curve;
  fig2      the triple-lens gradient example of Fig. 2 (1000 epochs, 500 x 500, FP64):
            forward and Jacobian time;
  kernels   one eager plain step and one eager learned step of the metric workload at
            given grids (plain=NRxNT learned=NRxNT:GATE:SLACK), for counter and trace runs.

    python -m paper_2510_02639_amd.perf [config1 config2 adjoint triple train serve hybrid nll fig2 kernels]
        [plain=..] [learned=..]

Inputs are resident in HBM before each timed region; times are wall-clock around
synchronised device work.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from . import icrs, learned, serve, workloads

# algorithmic flop-equivalents per node (FMA = 2, a reciprocal or square root = 1) and the
# MI355X vector peaks they are held against
FLOPS_RAY_FP32 = {2: 35.0, 3: 48.0}     # FP32 map, squared distance, brightness
FLOPS_NODE_ADJOINT = {2: 85.0, 3: 122.0}  # FP64 map, d(d^2)/d(eps, a, w_c) and its accumulation
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}


def _roofline(units, flops_per_unit, seconds, peak_key):
    achieved = units * flops_per_unit / seconds / 1e12
    return {"bound": "alu" if peak_key != "bf16" else "mfma", "achieved": achieved, "peak": PEAK[peak_key],
            "unit": "TFLOP/s", "frac": achieved / PEAK[peak_key], "flops_per_unit": flops_per_unit}


def _timed(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / reps


def _plain(w, n_limb, n_r, n_theta, rays, roots, reps):
    h = icrs.Handle(n_lens=w.n_lens, n_limb=n_limb, n_r=n_r, n_theta=n_theta, ray_precision=rays,
                    root_precision=roots)
    t = torch.tensor(w.t, device="cuda")
    ws = h.workspace(w.n_events, w.n_epochs)
    h.magnification(w.params, w.offsets, t, workspace=ws)
    h.set_profiling(True)
    h.get_profile(reset=True)
    _, dt = _timed(lambda: h.magnification(w.params, w.offsets, t, workspace=ws), reps=reps)
    prof = h.get_profile()
    h.set_profiling(False)
    calls = reps + 1  # _timed's warm-up call is profiled too
    main = _roofline(prof["n_main_rays"] / calls, FLOPS_RAY_FP32[w.n_lens], prof["ms_rays_main"] / calls * 1e-3,
                     "fp32" if rays == "fp32" else "fp64")
    return {"n_events": w.n_events, "n_epochs": w.n_epochs, "grid": [n_r, n_theta], "rays": rays, "roots": roots,
            "epochs_per_s": w.n_epochs / dt, "ms_per_call": dt * 1e3,
            "rays_per_s": prof["n_main_rays"] / (prof["ms_rays_main"] * 1e-3),
            "breakdown_ms": {k: prof[k] / calls for k in ("ms_centre", "ms_limb_sectors", "ms_rays", "ms_rays_main",
                                                          "ms_finalize")},
            "sectors_per_epoch": prof["n_sector_passes"] / max(prof["n_epochs"], 1), "rays_roofline": main}


def config1():
    w = workloads.config1()
    return {"measure": "config1", "workload": w.name, **_plain(w, 64, 64, 256, "fp64", "fp64", reps=20)}


def config2():
    w = workloads.config2()
    return {"measure": "config2", "workload": w.name, **_plain(w, 128, 128, 512, "fp32", "fp32", reps=3)}


def adjoint():
    w = workloads.config4()
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    ws = h.workspace(w.n_events, w.n_epochs)
    _, dt_f = _timed(lambda: h.magnification(w.params, w.offsets, t, workspace=ws))
    sec, per, ns = h.get_sectors(w.n_epochs, ws)
    cot = torch.tensor(np.random.default_rng(40).normal(size=w.n_epochs), device="cuda")
    (grad, _, _), dt_b = _timed(lambda: h.magnification_vjp(w.params, w.offsets, t, sec, per, ns, cotangent=cot,
                                                            workspace=ws))
    rays = float(ns.sum().item()) * 128 * 512
    return {"measure": "adjoint", "workload": "binary-fit-rho1e-3", "n_events": w.n_events, "n_epochs": w.n_epochs,
            "grid": [128, 512], "forward_epochs_per_s": w.n_epochs / dt_f, "vjp_epochs_per_s": w.n_epochs / dt_b,
            "vjp_ms": dt_b * 1e3, "vjp_rays_per_s": rays / dt_b, "vjp_precision": "f64",
            "vjp_roofline": _roofline(rays, FLOPS_NODE_ADJOINT[2], dt_b, "fp64"),
            "grad_finite": bool(torch.isfinite(grad).all().item())}


def triple():
    w = workloads.config3()
    h = icrs.Handle(n_lens=3, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp64")
    t = torch.tensor(w.t, device="cuda")
    ws = h.workspace(w.n_events, w.n_epochs)
    h.set_profiling(True)
    h.get_profile(reset=True)
    _, dt = _timed(lambda: h.magnification(w.params, w.offsets, t, workspace=ws))
    prof = h.get_profile()
    h.set_profiling(False)
    per_call = {k: prof[k] / 4 for k in ("ms_centre", "ms_limb_sectors", "ms_rays", "ms_finalize")}
    main = _roofline(prof["n_main_rays"], FLOPS_RAY_FP32[3], prof["ms_rays_main"] * 1e-3, "fp32")
    main["kernel"] = "rays_kernel<3, 8, true, MapF32<3, 8>> (main pass)"
    return {"measure": "triple", "workload": "triple-rho1e-3", "n_events": w.n_events, "n_epochs": w.n_epochs,
            "grid": [128, 512], "epochs_per_s": w.n_epochs / dt, "ms_per_call": dt * 1e3, "breakdown_ms": per_call,
            "rays_roofline": main, "limb_points_per_s": w.n_epochs * 128 / (per_call["ms_limb_sectors"] * 1e-3),
            "sectors_per_epoch": prof["n_sector_passes"] / max(prof["n_epochs"], 1)}


def train():
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    w = workloads.binary_batch(50, 1024, n_epochs_fixed=100, name="bounds-training")
    x, y = learned.training_rows(h, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model, losses = learned.train(h, x, y, steps=1000, batch=16384)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pred_rows = 4 << 20
    xb = x[torch.randint(0, x.shape[0], (pred_rows,), device="cuda")]
    _, dt_inf = _timed(lambda: h.mlp_forward(model.packed, model.params, model.norm, xb))
    flops_row = 2 * (10 * 128 + 128 * 128 * 2 + 128 * 4)
    return {"measure": "train", "rows": int(x.shape[0]), "steps": 1000, "batch": 16384,
            "train_rows_per_s": 1000 * 16384 / dt, "final_loss": losses[-1][1],
            "inference_rows_per_s": pred_rows / dt_inf,
            "inference_tflops": pred_rows * flops_row / dt_inf / 1e12, "mfma_peak_bf16_tflops": 2500.0,
            "inference_roofline": _roofline(pred_rows, flops_row, dt_inf, "bf16")}


def serving(seconds=60.0, rate=200.0):
    """The serving loop for `seconds` of Poisson arrivals (200 events/s: ~12,000 events at
    60 s), each path with the grids and gate the autotuner picked on a calibration batch."""
    reqs = serve.make_requests(seconds, rate)
    out = {}
    for use in (True, False):
        srv = serve.tuned_server(4 << 30, use_learned=use)
        srv.run_batch(reqs[:4])
        srv.reset_stats()
        r = srv.serve([serve.Request(q.params, q.t, q.arrival) for q in reqs], verbose=True)
        out["learned" if use else "plain"] = r
        print(json.dumps({"serve": r}), flush=True)
    return {"measure": "serve", "rate_events_per_s": rate, "seconds": seconds, **out}


def hybrid(n_events=512):
    w = workloads.cadence_workload(n_events)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    ws = h.hybrid_workspace(w.n_events, w.n_epochs)
    mag = torch.empty(w.n_epochs, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_epochs, dtype=torch.int32, device="cuda")
    _, dt_h = _timed(lambda: h.magnification_hybrid(w.params, w.offsets, t, mag, st, ws))
    n_point = int(((st & icrs.ST_POINT) != 0).sum().item())
    # the plain path on every epoch, timed on every 8th event (same epoch mix)
    sub = w.subset(range(0, w.n_events, 8))
    ts = torch.tensor(sub.t, device="cuda")
    wsp = h.workspace(sub.n_events, sub.n_epochs)
    _, dt_p = _timed(lambda: h.magnification(sub.params, sub.offsets, ts, workspace=wsp), reps=2)
    return {"measure": "hybrid", "workload": w.name, "n_events": w.n_events, "n_epochs": w.n_epochs,
            "grid": [128, 512], "point_fraction": n_point / w.n_epochs, "hybrid_epochs_per_s": w.n_epochs / dt_h,
            "hybrid_ms": dt_h * 1e3, "plain_all_epochs_per_s": sub.n_epochs / dt_p,
            "selection": {"n_check": 16, "guard": 2.0, "tol": 1e-4, "vary_max": 0.1}}


def nll(n_events=512):
    w = workloads.cadence_workload(n_events)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    rng = np.random.default_rng(52)
    sigma = torch.tensor(rng.uniform(0.005, 0.02, w.n_epochs), device="cuda")
    m, _ = h.magnification_hybrid(w.params, w.offsets, t)
    flux = (m - 1.0) + 10.0 + torch.randn_like(m) * sigma
    prior = np.tile([1.0, 10.0, 0.5, 2.0], (w.n_events, 1))
    (v, g), dt = _timed(lambda: icrs.light_curve_nll_and_grad(h, w.params, w.offsets, t, flux, sigma, prior,
                                                             hybrid=True), reps=2)
    nll_only = lambda: h.marginal_nll(w.offsets, m, flux, sigma, prior)
    _, dt_n = _timed(nll_only)
    return {"measure": "nll", "workload": w.name, "n_events": w.n_events, "n_epochs": w.n_epochs,
            "objective_and_gradient_ms": dt * 1e3, "objective_and_gradient_epochs_per_s": w.n_epochs / dt,
            "likelihood_kernel_ms": dt_n * 1e3, "grad_finite": bool(torch.isfinite(g).all().item())}


def fig2():
    w = workloads.fig2_triple()
    h = icrs.Handle(n_lens=3, n_limb=128, n_r=w.n_r, n_theta=w.n_theta, ray_precision="fp64", root_precision="fp64")
    t = torch.tensor(w.t, device="cuda")
    ws = h.workspace(w.n_events, w.n_epochs)
    _, dt_f = _timed(lambda: h.magnification(w.params, w.offsets, t, workspace=ws))
    sec, per, ns = h.get_sectors(w.n_epochs, ws)
    _, dt_j = _timed(lambda: h.magnification_vjp(w.params, w.offsets, t, sec, per, ns, jac=True, workspace=ws))
    return {"measure": "fig2", "workload": w.name, "n_epochs": w.n_epochs, "grid": [w.n_r, w.n_theta],
            "forward_ms": dt_f * 1e3, "jacobian_ms": dt_j * 1e3, "jacobian_epochs_per_s": w.n_epochs / dt_j,
            "sectors_per_epoch": float(ns.float().mean().item()), "precision": "f64"}


def kernels(plain="256x1024", learned_cfg="192x768:0.01:0"):
    """One eager plain step and one eager learned step on the 2048-event metric workload at
    the given grids (for counter and trace runs: no autotuning, no graph, nothing else)."""
    w = workloads.metric_workload(2048)
    pr, pt = (int(x) for x in plain.split("x"))
    g, gate, slack = learned_cfg.split(":")
    lr, lt = (int(x) for x in g.split("x"))
    h = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=pr, n_theta=pt, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    ws = h.learned_workspace(w.n_events, w.n_epochs)
    mag = torch.empty(w.n_epochs, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_epochs, dtype=torch.int32, device="cuda")
    model = learned.BoundsModel.load()
    h.set_profiling(True)
    h.get_profile(reset=True)
    h.magnification(w.params, w.offsets, t, mag, st, ws)
    torch.cuda.synchronize()
    pp = h.get_profile(reset=True)
    h.magnification_learned(w.params, w.offsets, t, model, mag, st, ws, n_r=lr, n_theta=lt, gate_rel=float(gate),
                            gate_slack=float(slack), stats=False)
    torch.cuda.synchronize()
    lp = h.get_profile()
    h.set_profiling(False)
    return {"measure": "kernels", "workload": w.name, "plain_grid": [pr, pt], "learned": [lr, lt, float(gate),
            float(slack)], "plain_main_ms": pp["ms_rays_main"], "plain_main_rays": pp["n_main_rays"],
            "learned_main_ms": lp["ms_rays_learned"], "learned_main_rays": lp["n_learned_rays"]}


def main(argv):
    which = [a for a in argv if "=" not in a] or ["config1", "config2", "adjoint", "triple", "train", "serve",
                                                  "hybrid", "nll", "fig2"]
    opts = dict(a.split("=", 1) for a in argv if "=" in a)
    fns = {"config1": config1, "config2": config2, "adjoint": adjoint, "triple": triple, "train": train, "serve": serving, "hybrid": hybrid, "nll": nll,
           "fig2": fig2,
           "kernels": lambda: kernels(opts.get("plain", "256x1024"), opts.get("learned", "192x768:0.01:0"))}
    for k in which:
        print(json.dumps(fns[k]()), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
