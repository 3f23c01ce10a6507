"""Pins of the oracle's marginalised likelihood (App. B, eq. NLL), which evaluates the
Woodbury forms the appendix prints:

* the dense Gaussian: eq. NLL + n/2 ln 2 pi equals -log N(F | M mu, C + M Lambda M^T) from
  scipy's multivariate normal (a different computation: the full covariance, no lemma);
* the Bayesian identity itself: p(F) = integral over beta of N(F | M beta, C) N(beta | mu,
  Lambda), brute-force 2-D quadrature on a few points;
* limits: Lambda -> 0 gives the plain Gaussian NLL at beta = mu; Lambda -> infinity makes the
  posterior mean the weighted least-squares fit (numpy.linalg.lstsq);
* dNLL/dA against central differences of NLL.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import likelihood_ref as L

RNG = np.random.default_rng(71)


def _data(n, mu=(2.0, 10.0)):
    mag = 1.0 + np.abs(RNG.normal(0.0, 3.0, n))
    sigma = RNG.uniform(0.05, 0.3, n)
    flux = (mag - 1.0) * mu[0] * 1.1 + mu[1] * 0.97 + RNG.normal(0.0, 1.0, n) * sigma
    return mag, flux, sigma


@pytest.mark.parametrize("n", [1, 5, 40])
def test_nll_equals_dense_gaussian(n):
    mag, flux, sigma = _data(n)
    prior = np.array([2.0, 10.0, 0.7, 3.0])
    M = np.stack([mag - 1.0, np.ones(n)], axis=1)
    B = np.diag(sigma ** 2) + M @ np.diag(prior[2:] ** 2) @ M.T
    ref = -stats.multivariate_normal(mean=M @ prior[:2], cov=B).logpdf(flux) - 0.5 * n * np.log(2 * np.pi)
    assert L.marginal_nll(mag, flux, sigma, prior) == pytest.approx(ref, rel=1e-11, abs=1e-10)


def test_nll_equals_brute_force_marginal():
    mag, flux, sigma = _data(3)
    prior = np.array([2.0, 10.0, 0.5, 1.5])
    M = np.stack([mag - 1.0, np.ones(3)], axis=1)
    # integrate over beta on a grid of +-9 prior sigmas (the integrand is a Gaussian in beta)
    bs = np.linspace(prior[0] - 9 * prior[2], prior[0] + 9 * prior[2], 801)
    bb = np.linspace(prior[1] - 9 * prior[3], prior[1] + 9 * prior[3], 801)
    S, Bb = np.meshgrid(bs, bb, indexing="ij")
    pred = S[..., None] * M[:, 0] + Bb[..., None] * M[:, 1]
    like = np.prod(stats.norm.pdf(flux, loc=pred, scale=sigma), axis=-1)
    prior_pdf = stats.norm.pdf(S, prior[0], prior[2]) * stats.norm.pdf(Bb, prior[1], prior[3])
    p = np.trapezoid(np.trapezoid(like * prior_pdf, bb, axis=1), bs)
    ref = -np.log(p) - 0.5 * 3 * np.log(2 * np.pi)
    assert L.marginal_nll(mag, flux, sigma, prior) == pytest.approx(ref, rel=1e-8)


def test_tight_prior_gives_the_plain_gaussian():
    mag, flux, sigma = _data(12)
    prior = np.array([2.0, 10.0, 1e-9, 1e-9])
    r = flux - (mag - 1.0) * prior[0] - prior[1]
    ref = 0.5 * np.sum(r ** 2 / sigma ** 2) + 0.5 * np.sum(np.log(sigma ** 2))
    assert L.marginal_nll(mag, flux, sigma, prior) == pytest.approx(ref, rel=1e-9)


def test_broad_prior_posterior_is_weighted_least_squares():
    mag, flux, sigma = _data(30)
    a, A = L.posterior_beta(mag, flux, sigma, np.array([0.0, 0.0, 1e8, 1e8]))
    M = np.stack([mag - 1.0, np.ones(mag.size)], axis=1)
    ls, *_ = np.linalg.lstsq(M / sigma[:, None], flux / sigma, rcond=None)
    assert np.allclose(a, ls, rtol=1e-9)
    assert np.allclose(A, np.linalg.inv(M.T @ (M / sigma[:, None] ** 2)), rtol=1e-9)


def test_gradient_against_central_differences():
    mag, flux, sigma = _data(15)
    prior = np.array([2.0, 10.0, 0.7, 3.0])
    v, g = L.marginal_nll_grad(mag, flux, sigma, prior)
    for i in range(15):
        h = 1e-6 * mag[i]
        mp, mm = mag.copy(), mag.copy()
        mp[i] += h
        mm[i] -= h
        fd = (L.marginal_nll(mp, flux, sigma, prior) - L.marginal_nll(mm, flux, sigma, prior)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-8)
