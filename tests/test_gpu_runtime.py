"""Batching runtime pieces on the GPU: the autotuner's grid choice and the serving loop."""
import numpy as np
import pytest
import torch

from paper_2510_02639_amd import autotune, icrs, learned, serve, workloads as W

pytestmark = pytest.mark.gpu


def test_autotuner_picks_the_cheapest_grid_meeting_its_tolerance():
    w = W.metric_workload(8)
    res = autotune.tune(w, tol=3e-4, every=40, n_r_ref=256, n_theta_ref=1024, stat="max", reference="grid",
                        candidates=[(32, 128), (64, 256), (128, 512), (256, 1024)])
    print(res, flush=True)
    assert res.n_trusted > 0
    tried = [(e[0], e[1]) for e in res.errors]
    costs = [a * b for a, b in tried]
    assert costs == sorted(costs)                       # tried cheapest first
    chosen = (res.n_r, res.n_theta)
    if res.errors[-1][2] <= res.tol:                    # stopped at the first grid within tolerance
        assert chosen == tried[-1]
        assert all(e[2] > res.tol for e in res.errors[:-1])
    assert res.ray_precision in ("fp32", "fp64") and all(v > 0 for v in res.timings.values())


def test_autotuner_against_the_disk_reference_stops_at_the_first_grid_within_tol():
    """Default mode: errors against the grid-free disk quadrature on the calibration epochs
    where no caustic crosses the disk; the chosen grid is the first (cheapest) whose median
    error is within tol, every cheaper one above it."""
    w = W.metric_workload(8)
    cands = [(32, 128), (64, 256), (128, 512), (256, 1024)]
    res = autotune.tune(w, tol=3e-4, every=20, candidates=cands)
    print(res.n_trusted, res.errors, flush=True)
    assert res.n_trusted >= 20
    med = [e[4] for e in res.errors]
    if med[-1] <= res.tol:
        assert (res.n_r, res.n_theta) == tuple(res.errors[-1][:2])
        assert all(m > res.tol for m in med[:-1])
    else:
        assert (res.n_r, res.n_theta) == (256, 1024) and len(med) == len(cands)


def test_serving_loop_serves_every_request_and_matches_direct_calls():
    reqs = serve.make_requests(seconds=1.5, rate=200.0, seed=52)
    srv = serve.Server(budget_bytes=1 << 30, use_learned=True)
    srv.run_batch(reqs[:2])
    srv.reset_stats()
    out = srv.serve(reqs)
    print(out, flush=True)
    assert out["events"] == len(reqs) and all(r.done > 0 for r in reqs)
    assert np.isfinite(out["p99_ms"]) and out["p50_ms"] <= out["p99_ms"]
    assert out["epochs_per_s"] > 0.5 * sum(r.t.size for r in reqs) / 1.5
    # a request's magnifications do not depend on the batch it was served in
    for r in (reqs[0], reqs[len(reqs) // 2], reqs[-1]):
        h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
        t = torch.tensor(r.t, device="cuda")
        m1, _, _ = h.magnification_learned(r.params[None], np.array([0, r.t.size]), t, srv.model)
        assert np.array_equal(m1.cpu().numpy(), r.mag)


def test_serving_budget_splits_batches():
    reqs = serve.make_requests(seconds=0.3, rate=400.0, seed=53)
    for r in reqs:
        r.arrival = 0.0                                  # everything waiting at once
    one = max(r.t.size for r in reqs)
    srv = serve.Server(budget_bytes=1 << 30, use_learned=False)
    budget = srv._bytes(1, one) * 2                      # room for about two requests
    srv2 = serve.Server(budget_bytes=budget, use_learned=False)
    out = srv2.serve(reqs)
    assert out["events"] == len(reqs)
    total = srv2._bytes(len(reqs), sum(r.t.size for r in reqs))
    assert out["batches"] >= total // budget and out["batches"] > 1


def test_served_plain_results_match_the_oracle():
    """Magnifications a plain server returns, on sampled epochs of sampled requests, against
    the oracle at the server's grid (FP32 rays: 3e-5)."""
    from oracle import oracle as O
    reqs = serve.make_requests(seconds=0.5, rate=200.0, seed=54)
    srv = serve.Server(budget_bytes=1 << 30, use_learned=False)
    out = srv.serve(reqs)
    assert out["events"] == len(reqs)
    rng = np.random.default_rng(54)
    worst = 0.0
    for r in (reqs[i] for i in rng.choice(len(reqs), size=min(6, len(reqs)), replace=False)):
        sel = np.sort(rng.choice(r.t.size, size=min(8, r.t.size), replace=False))
        ref = O.magnification(2, r.params, r.t[sel], n_limb=128, n_r=128, n_theta=512)["mag"]
        worst = max(worst, float(np.max(np.abs(r.mag[sel] / ref - 1.0))))
    print("served vs oracle max rel err", worst, flush=True)
    assert worst <= 3e-5
