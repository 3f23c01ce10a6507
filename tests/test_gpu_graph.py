"""The device-only path (icrs_prepare + icrs_run) equals the host-driven call and can be
captured into a HIP graph and replayed: every replay, with eager work and synchronisation
between replays, must reproduce the eager result bit for bit."""
import numpy as np
import pytest
import torch

from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu


def _planetary(n_events=8, per_event=12):
    big = W.binary_batch(2, 16, rho_fixed=1e-3)
    ts, off = [], [0]
    for i in range(n_events):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]]
        seg = seg[np.linspace(0, seg.size - 1, per_event).astype(int)]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    return W.Workload("planetary-graph", 2, big.params[:n_events], np.array(off, np.int64), np.concatenate(ts),
                      128, 128, 512, "fp32", "fp32")


@pytest.mark.parametrize("ray", ["fp32", "fp64"])
def test_graph_replay_matches_eager(ray):
    w = _planetary()
    s = torch.cuda.Stream()
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision=ray, root_precision="fp32",
                    stream=s)
    t = torch.tensor(w.t, device="cuda")
    with torch.cuda.stream(s):
        mag_ref, st_ref = h.magnification(w.params, w.offsets, t)
    s.synchronize()
    mag = torch.empty_like(mag_ref)
    st = torch.empty_like(st_ref)
    h.prepare(w.params, w.offsets, w.n_epochs)
    with torch.cuda.stream(s):
        h.run(t, mag, st)
    s.synchronize()
    assert torch.equal(mag, mag_ref) and torch.equal(st, st_ref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.run(t, mag, st)
    for _ in range(3):
        mag.fill_(-1.0)
        st.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(mag, mag_ref) and torch.equal(st, st_ref)


def test_learned_path_graph_replay_matches_eager():
    """The learned path keeps every list size on the device, so with no host statistics it
    can be captured: each replay reproduces the eager call bit for bit (magnifications and
    status words), with the routing across learned, gate-rejected and fallback epochs as in
    the eager call."""
    from paper_2510_02639_amd import learned
    w = W.metric_workload(24).sample_epochs(20)
    model = learned.BoundsModel.load()
    s = torch.cuda.Stream()
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32",
                    stream=s)
    t = torch.tensor(w.t, device="cuda")
    ws = h.learned_workspace(w.n_events, w.n_epochs)
    mag = torch.empty(w.n_epochs, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_epochs, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        _, _, stats = h.magnification_learned(w.params, w.offsets, t, model, mag, st, ws, n_r=64, n_theta=256,
                                              gate_rel=3e-3)
    s.synchronize()
    mag_ref, st_ref = mag.clone(), st.clone()
    assert stats["n_learned"] > 0 and stats["n_fallback"] > 0
    # the prepared form gives the same result eagerly, then inside a graph
    h.prepare(w.params, w.offsets, w.n_epochs, workspace=ws)
    with torch.cuda.stream(s):
        mag.fill_(-1.0)
        st2 = h.run_learned(t, model, mag, st, stats=True, n_r=64, n_theta=256, gate_rel=3e-3)
    s.synchronize()
    assert torch.equal(mag, mag_ref) and torch.equal(st, st_ref) and st2 == stats
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.run_learned(t, model, mag, st, n_r=64, n_theta=256, gate_rel=3e-3)
    for _ in range(3):
        mag.fill_(-1.0)
        st.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(mag, mag_ref) and torch.equal(st, st_ref)
