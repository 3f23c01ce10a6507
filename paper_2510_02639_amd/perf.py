"""Throughput of the path's other rows on one GPU, one JSON line per measurement:

  adjoint   forward + reverse-mode gradient on the differentiable-fit workload (512 binary
            events x 3000 epochs, rho = 1e-3; cotangent N(0,1), seed 40): epochs/s of the
            forward and of the VJP, and the VJP's ray rate;
  triple    the triple-lens workload (256 events x 2000 epochs, FP64 roots, FP32 rays);
  train     device training of the bounds network: rows/s of loss+gradient+AdamW steps;
  serve     the serving loop at 200 events/s for a few seconds (p50/p99 latency).

    python -m paper_2510_02639_amd.perf [adjoint triple train serve]

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


def _timed(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / reps


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
    return {"measure": "triple", "workload": "triple-rho1e-3", "n_events": w.n_events, "n_epochs": w.n_epochs,
            "grid": [128, 512], "epochs_per_s": w.n_epochs / dt, "ms_per_call": dt * 1e3, "breakdown_ms": per_call,
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
            "inference_tflops": pred_rows * flops_row / dt_inf / 1e12, "mfma_peak_bf16_tflops": 2500.0}


def serving(seconds=6.0):
    reqs = serve.make_requests(seconds)
    out = {}
    for use in (True, False):
        srv = serve.Server(4 << 30, use_learned=use)
        srv.run_batch(reqs[:4])
        srv.reset_stats()
        r = srv.serve([serve.Request(q.params, q.t, q.arrival) for q in reqs])
        out["learned" if use else "plain"] = r
    return {"measure": "serve", "rate_events_per_s": 200.0, "seconds": seconds, **out}


def main(argv):
    which = argv or ["adjoint", "triple", "train", "serve"]
    fns = {"adjoint": adjoint, "triple": triple, "train": train, "serve": serving}
    for k in which:
        print(json.dumps(fns[k]()), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
