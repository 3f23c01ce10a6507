"""Serving loop: light-curve requests arriving at random, admitted by an HBM budget,
micro-batched through the batched ICRS path (learned bounds with plain fallback, or plain).

Not part of the paper.  Requests are whole events (parameters + epochs); arrivals are a
Poisson process (exponential gaps, default mean 5 ms = 200 events/s); each event has
N_e ~ U{100..5000} epochs placed like the planetary batch (seeded).  The loop runs in
wall-clock time: whenever the device is free it admits every request that has arrived,
oldest first, while the batch's workspace fits the budget, runs one call, and stamps each
request's completion.  Latency = completion - arrival.  The workspace is allocated once,
at the budget, and reused by every batch.

    python -m paper_2510_02639_amd.serve --seconds 20 [--plain] [--budget-gib 16]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np
import torch

from . import icrs, learned, workloads


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
                 learned_grid=None):
        self.h = icrs.Handle(n_lens=2, n_limb=n_limb, n_r=n_r, n_theta=n_theta, ray_precision="fp32",
                             root_precision="fp32")
        self.use_learned = use_learned
        self.model = model if (model is not None or not use_learned) else learned.BoundsModel.load()
        self.learned_grid = learned_grid or (n_r, n_theta)
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
                                                           n_r=self.learned_grid[0], n_theta=self.learned_grid[1])
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
                "path": "learned" if self.use_learned else "plain"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--plain", action="store_true")
    args = ap.parse_args()
    reqs = make_requests(args.seconds, args.rate)
    srv = Server(int(args.budget_gib * (1 << 30)), use_learned=not args.plain)
    srv.run_batch(reqs[:4])            # warm-up (kernel loading), not part of the run
    srv.reset_stats()
    print(json.dumps(srv.serve(reqs)), flush=True)


if __name__ == "__main__":
    main()
