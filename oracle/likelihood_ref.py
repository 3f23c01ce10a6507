"""Plain FP64 reference of the marginalised light-curve likelihood (App. B).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product path; it shares
no code with the HIP library.

App. B ("Application to Microlensing Modeling"): each data set j (here: one event) has
fluxes F = (A(t; theta) - 1) F_S + F_base, i.e. the design matrix M = [A - 1, 1] (n x 2)
and linear parameters beta = (F_S, F_base) with a Gaussian prior N(mu, Lambda),
Lambda = diag(sigma_FS^2, sigma_Fbase^2), and independent Gaussian noise C = diag(sigma_i^2).
Marginalising beta gives eq. NLL,
    NLL = 1/2 r^T (C + M Lambda M^T)^{-1} r + 1/2 ln |C + M Lambda M^T|,   r = F - M mu,
evaluated, as the appendix writes it, with the matrix inversion lemma
    (C + M Lambda M^T)^{-1} = C^{-1} - C^{-1} M (Lambda^{-1} + M^T C^{-1} M)^{-1} M^T C^{-1},
    ln |C + M Lambda M^T|   = ln |C| + ln |Lambda| + ln |Lambda^{-1} + M^T C^{-1} M|.
The posterior of beta is N(a, A) with A^{-1} = Lambda^{-1} + M^T C^{-1} M and
a = A (Lambda^{-1} mu + M^T C^{-1} F).  (eq. NLL leaves out the constant n/2 ln 2 pi of the
Gaussian; so does this reference.)

The derivative of NLL with respect to each magnification A_i is taken by automatic
differentiation of the same formula (PyTorch, CPU, float64).
"""
from __future__ import annotations

import numpy as np
import torch


def _nll_torch(mag, flux, sigma, prior):
    """eq. NLL of one data set in torch float64 (mag may require grad)."""
    mu = torch.as_tensor(prior[:2], dtype=torch.float64)
    lam = torch.as_tensor(np.asarray(prior[2:4]) ** 2, dtype=torch.float64)
    F = torch.as_tensor(flux, dtype=torch.float64)
    s2 = torch.as_tensor(sigma, dtype=torch.float64) ** 2
    M = torch.stack([mag - 1.0, torch.ones_like(mag)], dim=1)          # design matrix, n x 2
    r = F - M @ mu                                                      # residual about the prior mean
    Cinv_r = r / s2
    Cinv_M = M / s2[:, None]
    K = torch.diag(1.0 / lam) + M.T @ Cinv_M                            # Lambda^{-1} + M^T C^{-1} M
    # Woodbury: B^{-1} r = C^{-1} r - C^{-1} M K^{-1} M^T C^{-1} r
    Binv_r = Cinv_r - Cinv_M @ torch.linalg.solve(K, M.T @ Cinv_r)
    logdet = torch.sum(torch.log(s2)) + torch.sum(torch.log(lam)) + torch.logdet(K)
    return 0.5 * (r @ Binv_r) + 0.5 * logdet


def marginal_nll(mag, flux, sigma, prior):
    """eq. NLL for one data set: mag, flux, sigma [n]; prior = (mu_S, mu_B, sigma_S, sigma_B)."""
    return float(_nll_torch(torch.as_tensor(np.asarray(mag, np.float64)), flux, sigma, prior))


def marginal_nll_grad(mag, flux, sigma, prior):
    """(NLL, dNLL/dA_i [n]) for one data set."""
    m = torch.tensor(np.asarray(mag, np.float64), requires_grad=True)
    v = _nll_torch(m, flux, sigma, prior)
    v.backward()
    return float(v.detach()), m.grad.numpy().copy()


def posterior_beta(mag, flux, sigma, prior):
    """Mean a [2] and covariance A [2, 2] of the linear parameters (F_S, F_base)."""
    mag = np.asarray(mag, np.float64)
    M = np.stack([mag - 1.0, np.ones_like(mag)], axis=1)
    w = 1.0 / np.asarray(sigma, np.float64) ** 2
    mu = np.asarray(prior[:2], np.float64)
    lam = np.asarray(prior[2:4], np.float64) ** 2
    Ainv = np.diag(1.0 / lam) + M.T @ (M * w[:, None])
    A = np.linalg.inv(Ainv)
    a = A @ (mu / lam + M.T @ (w * np.asarray(flux, np.float64)))
    return a, A


def light_curve_nll(mag, offsets, flux, sigma, priors):
    """Per-event NLL, dNLL/dmag and posterior moments of a CSR batch of light curves."""
    n_ev = len(offsets) - 1
    nll = np.zeros(n_ev)
    g = np.zeros(len(mag))
    beta = np.zeros((n_ev, 5))
    for i in range(n_ev):
        sl = slice(offsets[i], offsets[i + 1])
        nll[i], g[sl] = marginal_nll_grad(mag[sl], flux[sl], sigma[sl], priors[i])
        a, A = posterior_beta(mag[sl], flux[sl], sigma[sl], priors[i])
        beta[i] = [a[0], a[1], A[0, 0], A[0, 1], A[1, 1]]
    return nll, g, beta
