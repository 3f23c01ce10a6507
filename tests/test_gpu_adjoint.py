"""GPU adjoint (frozen-structure reverse mode) against the oracle's dual-number Jacobian and
against central differences of the GPU's own FP64 forward."""
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


def test_adjoint_against_gpu_central_differences():
    """Central differences of the GPU's own FP64 forward on the same sectors, in a regime
    where they are meaningful: the config-1 lens (s=0.9, q=0.1, rho=1e-2) at epochs at
    least 1 d from every caustic crossing, 64 x 256 grids.  Near caustics at rho=1e-3 the
    quadrature's kinks (a node's chi flipping changes which stencil places a crossing) lie
    closer together than any step that survives rounding, so there the adjoint is held to
    the oracle's exact dual-number Jacobian instead (test above).  Parameters 0-6 use a
    uniform source (step 1e-7 relative); the limb-darkening coefficient, which moves no
    node across the limb, uses u = 0.5 and a 1e-6 step.  Bar: |g - fd| <= 1e-4 S_p with
    S_p = sum_e |c_e dA_e/dp|, and per epoch 1e-4 of the largest |dA/dp|."""
    t_np = np.array([-20.0, -10.0, -6.0, -1.5, 1.5, 8.0, 12.0, 24.0])
    n_r, n_theta = 64, 256
    cot = np.random.default_rng(41).normal(size=t_np.size)
    off = np.array([0, t_np.size], np.int64)
    t = torch.tensor(t_np, device="cuda")
    h = icrs.Handle(n_lens=2, n_limb=64, n_r=n_r, n_theta=n_theta)
    for u_ld, ks, hrel in ((0.0, range(7), 1e-7), (0.5, [7], 1e-6)):
        p = np.array([[0.9, 0.1, 0.05, 0.6, 0.0, 20.0, 1e-2, u_ld, 0.0, 0.0, 0.0]])
        r = O.magnification(2, p[0], t_np, n_limb=64, n_r=n_r, n_theta=n_theta)
        sec, per, ns = r["sectors"], r["periodic"], r["nsec"]
        args = [torch.tensor(x, device="cuda") for x in (sec, per, ns)]
        grad, jac, _ = h.magnification_vjp(p, off, t, *args, cotangent=torch.tensor(cot, device="cuda"), jac=True)
        grad, jac = grad.cpu().numpy()[0], jac.cpu().numpy()
        for k in ks:
            step = hrel * (abs(p[0, k]) if k in (0, 1, 6) else max(abs(p[0, k]), 1.0))
            pp, pm = p.copy(), p.copy()
            pp[0, k] += step
            pm[0, k] -= step
            mp, _ = h.magnification_given(pp, off, t, *args)
            mm, _ = h.magnification_given(pm, off, t, *args)
            fd_e = (mp.cpu().numpy() - mm.cpu().numpy()) / (2 * step)
            S = np.sum(np.abs(cot * jac[:, k]))
            err = abs(grad[k] - np.sum(cot * fd_e)) / S
            err_e = np.abs(jac[:, k] - fd_e).max() / np.abs(jac[:, k]).max()
            print(f"param {k}: |g - fd| / S_p = {err:.2e}, per-epoch {err_e:.2e}", flush=True)
            assert err <= 1e-4 and err_e <= 1e-4, k


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


def test_vjp_does_not_depend_on_workspace_contents():
    """The reverse-mode call on the forward's sectors, with a workspace prefilled with
    different byte patterns, gives bitwise identical gradients, Jacobian rows and
    magnifications (no stale accumulator or counter is read)."""
    w = _fit_subset(n_events=6, per_event=4)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=64, n_theta=256, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    mag, _ = h.magnification(w.params, w.offsets, t)
    sec, per, ns = h.get_sectors(w.n_epochs)
    cot = torch.tensor(np.random.default_rng(7).normal(size=w.n_epochs), device="cuda")
    nb = h.workspace_bytes(w.n_events, w.n_epochs)
    out = []
    for fill in (0x00, 0xFF, 0x3C):
        ws = torch.full((nb,), fill, dtype=torch.uint8, device="cuda")
        g, j, m = h.magnification_vjp(w.params, w.offsets, t, sec, per, ns, cotangent=cot, jac=True, mag=True,
                                      workspace=ws)
        torch.cuda.synchronize()
        out.append((g.cpu().numpy(), j.cpu().numpy(), m.cpu().numpy()))
    g0, j0, m0 = out[0]
    assert np.all(np.isfinite(g0)) and np.all(np.isfinite(j0))
    for g, j, m in out[1:]:
        assert np.array_equal(g, g0) and np.array_equal(j, j0) and np.array_equal(m, m0)
