"""Marginalised light-curve likelihood (App. B, eq. NLL) on the GPU against the oracle's
Woodbury-form reference: per-event NLL, posterior moments of the flux parameters and
dNLL/dA; and the fit objective (NLL and its gradient with respect to the event parameters
through the frozen-structure reverse mode) against the oracle's dNLL/dA contracted with the
oracle's Jacobian on the same sectors."""
import numpy as np
import pytest
import torch

from oracle import likelihood_ref as LR
from oracle import oracle as O
from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu


def _synthetic(n_events, sizes, seed=90):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mag = 1.0 + np.abs(rng.normal(0.0, 5.0, off[-1]))
    sigma = rng.uniform(0.01, 0.1, off[-1])
    prior = np.stack([rng.uniform(0.5, 2.0, n_events), rng.uniform(5.0, 20.0, n_events),
                      rng.uniform(0.1, 1.0, n_events), rng.uniform(0.5, 5.0, n_events)], axis=1)
    ev = np.repeat(np.arange(n_events), sizes)
    flux = (mag - 1.0) * prior[ev, 0] * 1.05 + prior[ev, 1] * 0.98 + rng.normal(0.0, 1.0, off[-1]) * sigma
    return off, mag, flux, sigma, prior


def test_nll_kernel_matches_oracle():
    sizes = [0, 1, 7, 300, 4999, 64, 257]                    # an empty event and a long one
    off, mag, flux, sigma, prior = _synthetic(len(sizes), sizes)
    h = icrs.Handle(n_lens=2)
    d = lambda a: torch.tensor(a, device="cuda")
    nll, beta, g = h.marginal_nll(off, d(mag), d(flux), d(sigma), prior, beta=True)
    torch.cuda.synchronize()
    onll, og, obeta = LR.light_curve_nll(mag, off, flux, sigma, prior)
    nll, beta, g = nll.cpu().numpy(), beta.cpu().numpy(), g.cpu().numpy()
    assert np.allclose(nll, onll, rtol=1e-10, atol=1e-9)
    assert np.allclose(beta, obeta, rtol=1e-9, atol=1e-14)
    assert np.allclose(g, og, rtol=1e-9, atol=1e-9 * np.abs(og).max())


def test_fit_objective_gradient_matches_oracle():
    """Events of the differentiable-fit workload (rho = 1e-3), a few epochs each, with fluxes
    made from a nearby model; gradient of sum NLL with respect to every parameter."""
    big = W.binary_batch(4, 6, rho_fixed=1e-3, n_epochs_fixed=3000)
    w = big.sample_epochs(300)
    h = icrs.Handle(n_lens=2, n_limb=64, n_r=64, n_theta=256)
    t = torch.tensor(w.t, device="cuda")
    p_true = w.params.copy()
    p_true[:, 2] *= 1.01
    m_true, _ = h.magnification(p_true, w.offsets, t)
    rng = np.random.default_rng(91)
    sigma = rng.uniform(0.005, 0.02, w.n_epochs)
    prior = np.tile([1.0, 10.0, 0.5, 2.0], (w.n_events, 1))
    flux = (m_true.cpu().numpy() - 1.0) * 1.0 + 10.0 + rng.normal(0, 1, w.n_epochs) * sigma
    nll, grad = icrs.light_curve_nll_and_grad(h, w.params, w.offsets, t, torch.tensor(flux, device="cuda"),
                                              torch.tensor(sigma, device="cuda"), prior)
    mag, _ = h.magnification(w.params, w.offsets, t)
    sec, per, ns = h.get_sectors(w.n_epochs)
    torch.cuda.synchronize()
    mag, sec, per, ns = mag.cpu().numpy(), sec.cpu().numpy(), per.cpu().numpy(), ns.cpu().numpy()
    onll, og, _ = LR.light_curve_nll(mag, w.offsets, flux, sigma, prior)
    assert np.allclose(nll.cpu().numpy(), onll, rtol=1e-10)
    gref = np.zeros((w.n_events, 11))
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        _, J = O.jacobian_given(2, w.params[i], w.t[sl], sec[sl], per[sl], ns[sl], 64, 256)
        gref[i] = og[sl] @ J
    grad = grad.cpu().numpy()
    scale = np.abs(gref).max(axis=0) + 1e-300
    err = np.abs(grad - gref) / scale
    print(f"fit objective: max rel gradient error {err.max():.2e}", flush=True)
    assert np.all(err[:, :8] <= 1e-6)
