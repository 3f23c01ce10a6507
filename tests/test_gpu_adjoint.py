"""GPU adjoint (frozen-structure reverse mode) against the oracle's dual-number Jacobian and
against central differences of the GPU's own FP64 forward (uniform source, where the
quadrature is continuous in the parameters)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu


def _fit_subset(n_events=20, per_event=3, seed=4):
    """Events of the differentiable-fit workload (rho = 1e-3), a few epochs each."""
    big = W.binary_batch(seed, n_events, rho_fixed=1e-3, n_epochs_fixed=3000)
    ts, off = [], [0]
    for i in range(n_events):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]]
        seg = seg[np.linspace(0, seg.size - 1, per_event).astype(int)]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    return W.Workload("fit-subset", 2, big.params, np.array(off, np.int64), np.concatenate(ts), 128, 128, 512,
                      "fp64", "fp64")


def _oracle_frozen(w, n_r, n_theta):
    mags, jacs, secs, pers, nss = [], [], [], [], []
    for i in range(w.n_events):
        t = w.t[w.offsets[i]:w.offsets[i + 1]]
        r = O.magnification(w.n_lens, w.params[i], t, n_limb=w.n_limb, n_r=n_r, n_theta=n_theta)
        m, j = O.jacobian_given(w.n_lens, w.params[i], t, r["sectors"], r["periodic"], r["nsec"], n_r, n_theta)
        mags.append(m); jacs.append(j); secs.append(r["sectors"]); pers.append(r["periodic"]); nss.append(r["nsec"])
    return (np.concatenate(mags), np.concatenate(jacs), np.concatenate(secs), np.concatenate(pers),
            np.concatenate(nss))


def _gpu_vjp(w, sec, per, ns, cot, n_r, n_theta):
    h = icrs.Handle(n_lens=w.n_lens, n_limb=w.n_limb, n_r=n_r, n_theta=n_theta)
    t = torch.tensor(w.t, device="cuda")
    grad, jac, mag = h.magnification_vjp(w.params, w.offsets, t, torch.tensor(sec, device="cuda"),
                                         torch.tensor(per, device="cuda"), torch.tensor(ns, device="cuda"),
                                         cotangent=torch.tensor(cot, device="cuda"), jac=True, mag=True)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), jac.cpu().numpy(), mag.cpu().numpy()


def test_adjoint_matches_oracle_jacobian_binary():
    w = _fit_subset()
    om, oj, sec, per, ns = _oracle_frozen(w, 128, 512)
    cot = np.random.default_rng(40).normal(size=w.n_epochs)
    grad, jac, mag = _gpu_vjp(w, sec, per, ns, cot, 128, 512)
    assert np.allclose(mag, om, rtol=1e-10, atol=0)
    for k in range(8):
        scale = np.abs(oj[:, k]).max()
        err = np.abs(jac[:, k] - oj[:, k]).max() / scale
        print(f"param {k}: max |jac - oracle| / max|oracle| = {err:.2e}", flush=True)
        assert err <= 1e-6
    assert np.all(jac[:, 8:] == 0)
    # contraction with the cotangent, per event
    ev = np.repeat(np.arange(w.n_events), np.diff(w.offsets))
    ref = np.zeros((w.n_events, 11))
    np.add.at(ref, ev, cot[:, None] * oj)
    S = np.zeros((w.n_events, 11))
    np.add.at(S, ev, np.abs(cot[:, None] * oj))
    assert np.all(np.abs(grad - ref) <= 1e-6 * S + 1e-300)


def test_adjoint_matches_oracle_jacobian_triple():
    big = W.config3(n_events=2, n_epochs=2000)
    ts, off = [], [0]
    for i in range(2):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]][990:1010:5]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("triple-adj", 3, big.params, np.array(off, np.int64), np.concatenate(ts), 64, 64, 256, "fp64",
                   "fp64")
    om, oj, sec, per, ns = _oracle_frozen(w, 64, 256)
    cot = np.ones(w.n_epochs)
    grad, jac, mag = _gpu_vjp(w, sec, per, ns, cot, 64, 256)
    for k in [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10]:
        scale = np.abs(oj[:, k]).max()
        assert np.abs(jac[:, k] - oj[:, k]).max() <= 1e-6 * scale + 1e-12, k


def test_adjoint_against_gpu_central_differences_uniform_source():
    """Uniform source: the quadrature is continuous across chi flips, so central differences
    of the plain FP64 forward (same sectors) must match the adjoint to 1e-4 of
    S_p = sum_e |c_e dA_e/dp|.  Step 1e-8 relative: near caustic crossings the second
    derivatives are so large that 1e-6 steps carry ~1e-2 truncation error."""
    w = _fit_subset(n_events=6, per_event=4)
    w.params[:, 7] = 0.0
    om, oj, sec, per, ns = _oracle_frozen(w, 128, 512)
    cot = np.random.default_rng(41).normal(size=w.n_epochs)
    grad, jac, _ = _gpu_vjp(w, sec, per, ns, cot, 128, 512)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512)
    t = torch.tensor(w.t, device="cuda")
    args = [torch.tensor(x, device="cuda") for x in (sec, per, ns)]
    ev = np.repeat(np.arange(w.n_events), np.diff(w.offsets))
    worst = []
    for k in range(7):
        base = w.params[:, k]
        hs = 1e-8 * (np.abs(base) if k in (0, 1, 6) else np.maximum(np.abs(base), 1.0))
        pp, pm = w.params.copy(), w.params.copy()
        pp[:, k] += hs
        pm[:, k] -= hs
        mp, _ = h.magnification_given(pp, w.offsets, t, *args)
        mm, _ = h.magnification_given(pm, w.offsets, t, *args)
        fd_e = (mp.cpu().numpy() - mm.cpu().numpy()) / (2 * hs[ev])
        fd = np.zeros(w.n_events)
        np.add.at(fd, ev, cot * fd_e)
        S = np.zeros(w.n_events)
        np.add.at(S, ev, np.abs(cot * jac[:, k]))
        err = np.abs(grad[:, k] - fd) / S
        print(f"param {k}: max |g - fd| / S_p = {err.max():.2e}", flush=True)
        worst.append(err.max())
    assert max(worst) <= 1e-4, worst


def test_autograd_function_backward_equals_vjp():
    w = _fit_subset(n_events=3, per_event=2)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512)
    t = torch.tensor(w.t, device="cuda")
    params = torch.tensor(w.params, requires_grad=True)
    mag = icrs.ICRSFunction.apply(params, h, w.offsets, t)
    cot = torch.linspace(-1.0, 1.0, w.n_epochs, dtype=torch.float64, device="cuda")
    (mag * cot).sum().backward()
    sec, per, ns = h.get_sectors(w.n_epochs)
    grad, _, _ = h.magnification_vjp(w.params, w.offsets, t, sec, per, ns, cotangent=cot)
    assert torch.equal(params.grad, grad.cpu())
