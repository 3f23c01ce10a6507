"""The entry point that allocates nothing (icrs_magnification_noalloc, for callers that cannot
call hipMalloc) against icrs_magnification on the same inputs, through the C ABI: two calls
in a row on the library's per-GPU scratch, the second on a smaller batch, each bitwise equal
to the workspace form (the two share every kernel), and a batch beyond the scratch rejected
before launch."""
import numpy as np
import pytest
import torch

from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu


def _batch(n_events, per_event, seed):
    big = W.binary_batch(seed, n_events, rho_fixed=1e-3)
    return big.sample_epochs(max(1, int(np.max(np.diff(big.offsets))) // per_event))


def test_noalloc_matches_workspace_path_on_two_calls():
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    for w in (_batch(48, 60, 5), _batch(7, 25, 6)):          # the second call is smaller
        t = torch.tensor(w.t, device="cuda")
        assert h.workspace_bytes(w.n_events, w.n_epochs) <= icrs.NOALLOC_SCRATCH_BYTES
        ref_m, ref_s = h.magnification(w.params, w.offsets, t)
        m, s = h.magnification_noalloc(w.params, w.offsets, t)
        torch.cuda.synchronize()
        print(f"noalloc: {w.n_epochs} epochs, {w.n_events} events", flush=True)
        assert torch.all(torch.isfinite(m))
        assert torch.equal(m, ref_m) and torch.equal(s, ref_s)


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    w = W.config1()
    h = icrs.Handle(n_lens=2)
    n = 200_000                                   # ~140 MB of workspace > 64 MiB
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(icrs.IcrsError) as ei:
        h.magnification_noalloc(w.params, np.array([0, n], np.int64), t)
    assert ei.value.code == -2
