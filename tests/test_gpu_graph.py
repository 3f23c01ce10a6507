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
