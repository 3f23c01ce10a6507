"""Serving loop: light-curve requests arriving at random, admitted by an HBM budget,
micro-batched through the batched ICRS path (learned bounds with plain fallback, or plain).

Not part of the paper.  Requests are whole events (parameters + epochs); arrivals are a
Poisson process (exponential gaps, default mean 5 ms = 200 events/s); each event has
N_e ~ U{100..5000} epochs placed like the planetary batch (seeded).  The loop runs in
wall-clock time: whenever the device is free it admits every request that has arrived,
oldest first, while the batch's workspace fits the budget, runs one call, and stamps each
request's completion.  Latency = completion - arrival.  The workspace is allocated once,
at the budget, and reused by every batch.

Grids and drift gate: by default the autotuner picks them, untimed, on a calibration batch of
the same event distribution (its own seed): the plain grid (the fallback's) as the smallest
whose median error is within 3e-5 of the converged path, the learned grid and gate as the
fastest no worse than plain at that grid (median and 99th percentile).

    python -m paper_2510_02639_amd.serve --seconds 60 [--plain] [--budget-gib 16] [--no-tune]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np
import torch

from . import autotune, icrs, learned, workloads


@dataclasses.dataclass
class Request:
    params: np.ndarray      # [11]
    t: np.ndarray           # epochs
    arrival: float          # seconds from the start
    done: float = -1.0
    status_bits: int = 0
    mag: np.ndarray = None  # filled when served


def make_requests(seconds=60.0, rate=200.0, seed=51, max_events=None):
    """Poisson arrivals over `seconds`; events drawn as in the planetary batch (rho = 1e-3)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(seconds * rate * 1.5) + 16)
    arr = np.cumsum(gaps)
    arr = arr[arr < seconds]
    if max_events is not None:
        arr = arr[:max_events]
    w = workloads.binary_batch(seed, arr.size, rho_fixed=1e-3, name="serving")
    return [Request(w.params[i], w.t[w.offsets[i]:w.offsets[i + 1]], float(arr[i])) for i in range(arr.size)]


class Server:
    def __init__(self, budget_bytes=16 << 30, use_learned=True, model=None, n_limb=128, n_r=128, n_theta=512,
                 learned_grid=None, gate_rel=1e-3, gate_slack=0.0):
        self.h = icrs.Handle(n_lens=2, n_limb=n_limb, n_r=n_r, n_theta=n_theta, ray_precision="fp32",
                             root_precision="fp32")
        self.use_learned = use_learned
        self.model = model if (model is not None or not use_learned) else learned.BoundsModel.load()
        self.learned_grid = learned_grid or (n_r, n_theta)
        self.gate = (float(gate_rel), float(gate_slack))
        self.budget = int(budget_bytes)
        self.ws = torch.empty(self.budget, dtype=torch.uint8, device="cuda")
        self.reset_stats()

    def reset_stats(self):
        self.stats = {"batches": 0, "fallback": 0, "learned": 0, "epochs": 0}

    def _bytes(self, n_events, n_epochs):
        f = icrs.lib().icrs_learned_workspace_bytes if self.use_learned else icrs.lib().icrs_workspace_bytes
        return f(self.h._h, n_events, n_epochs)

    def fits(self, n_events, n_epochs):
        return self._bytes(n_events, n_epochs) <= self.budget

    def run_batch(self, reqs):
        params = np.stack([r.params for r in reqs])
        counts = [r.t.size for r in reqs]
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        t = torch.tensor(np.concatenate([r.t for r in reqs]), device="cuda")
        n = t.numel()
        if self.use_learned:
            mag, status, st = self.h.magnification_learned(params, off, t, self.model, workspace=self.ws,
                                                           n_r=self.learned_grid[0], n_theta=self.learned_grid[1],
                                                           gate_rel=self.gate[0], gate_slack=self.gate[1])
            self.stats["fallback"] += st["n_fallback"]
            self.stats["learned"] += st["n_learned"]
        else:
            mag, status = self.h.magnification(params, off, t, workspace=self.ws)
        torch.cuda.synchronize()
        self.stats["batches"] += 1
        self.stats["epochs"] += n
        return mag, status, off

    def serve(self, requests, verbose=False):
        """Run the loop until every request is served; returns the summary."""
        pending = 0                       # index of the oldest request not yet admitted
        start = time.perf_counter()
        busy = 0.0
        batch_sizes = []
        while pending < len(requests):
            now = time.perf_counter() - start
            if requests[pending].arrival > now:
                time.sleep(min(requests[pending].arrival - now, 0.002))
                continue
            batch, n_ep = [], 0
            while (pending < len(requests) and requests[pending].arrival <= now
                   and self.fits(len(batch) + 1, n_ep + requests[pending].t.size)):
                batch.append(requests[pending])
                n_ep += requests[pending].t.size
                pending += 1
            if not batch:       # a single request larger than the budget
                raise RuntimeError("request exceeds the HBM budget")
            t0 = time.perf_counter()
            mag, status, off = self.run_batch(batch)
            t1 = time.perf_counter()
            busy += t1 - t0
            st = status.cpu().numpy()
            mg = mag.cpu().numpy()
            for i, r in enumerate(batch):
                r.done = t1 - start
                r.status_bits = int(np.bitwise_or.reduce(st[off[i]:off[i + 1]].astype(np.uint32)))
                r.mag = mg[off[i]:off[i + 1]]
            batch_sizes.append(len(batch))
            if verbose and len(batch_sizes) % 50 == 0:
                print(f"[serve] t={t1 - start:.1f}s batches={len(batch_sizes)}", flush=True)
        wall = time.perf_counter() - start
        lat = np.array([r.done - r.arrival for r in requests])
        epochs = sum(r.t.size for r in requests)
        return {"events": len(requests), "epochs": int(epochs), "wall_s": wall, "epochs_per_s": epochs / wall,
                "busy_frac": busy / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
                "batches": len(batch_sizes), "mean_batch_events": float(np.mean(batch_sizes)),
                "fallback_epochs": self.stats["fallback"], "learned_epochs": self.stats["learned"],
                "path": "learned" if self.use_learned else "plain", "plain_grid": [self.h.cfg.n_r, self.h.cfg.n_theta],
                "learned_grid": list(self.learned_grid) if self.use_learned else None,
                "gate": list(self.gate) if self.use_learned else None}


def tuned_server(budget_bytes, use_learned=True, n_calibration_events=256, seed=61, verbose=False):
    """A server whose grids and gate the autotuner picked on a calibration batch drawn like
    the requests (planetary events, rho = 1e-3) with its own seed."""
    cal = workloads.binary_batch(seed, n_calibration_events, rho_fixed=1e-3, name="serving-calibration")
    g = autotune.tune(cal, tol=3e-5, every=20, stat="median", verbose=verbose)
    kw = dict(n_r=g.n_r, n_theta=g.n_theta)
    if use_learned:
        model = learned.BoundsModel.load()
        lt = autotune.tune_learned(cal, model, plain_grid=(g.n_r, g.n_theta), every=20, verbose=verbose)
        kw.update(model=model, learned_grid=(lt.n_r, lt.n_theta), gate_rel=lt.gate_rel, gate_slack=lt.gate_slack)
    return Server(budget_bytes, use_learned=use_learned, **kw)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="fixed 128 x 512 grids and a 1e-3 gate")
    args = ap.parse_args()
    reqs = make_requests(args.seconds, args.rate)
    budget = int(args.budget_gib * (1 << 30))
    srv = (Server(budget, use_learned=not args.plain) if args.no_tune
           else tuned_server(budget, use_learned=not args.plain))
    srv.run_batch(reqs[:4])            # warm-up (kernel loading), not part of the run
    srv.reset_stats()
    print(json.dumps(srv.serve(reqs)), flush=True)


if __name__ == "__main__":
    main()
