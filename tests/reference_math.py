"""Independent references used to pin the oracle (tests only).

Nothing here calls the oracle or the HIP library.  Each function is a closed form, a
library routine or a brute-force computation of a quantity that the paper's method
approximates (microJAX, arXiv 2510.02639):

* single point-lens magnification A(u) = (u^2 + 2) / (u sqrt(u^2 + 4)) -- the N = 1 case of
  eq. amp_point, and its finite-source average over a uniform or limb-darkened disk (the
  integral that Sec. 2.2 says ICRS approximates);
* images by Newton's method on eq. lens_eq from a dense set of seeds (no polynomial);
* Cartesian inverse ray shooting over a fixed box (Sec. 1 mentions it as the classic
  alternative): no sectors, no crossings, just pixels.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def lens_map(eps, a, z):
    z = np.asarray(z, dtype=np.complex128)
    w = z.copy()
    for e, ak in zip(eps, a):
        w -= e / np.conj(z - ak)
    return w


def point_lens_mag(u):
    u = np.asarray(u, dtype=np.float64)
    return (u * u + 2.0) / (u * np.sqrt(u * u + 4.0))


def limb_darkened_I(x, u1):
    """Linear limb darkening normalised to unit flux over the unit disk."""
    x = np.asarray(x, dtype=np.float64)
    I0 = 3.0 / (np.pi * (3.0 - u1))
    return I0 * (1.0 - u1 * (1.0 - np.sqrt(np.clip(1.0 - x * x, 0.0, None))))


def uniform_disk_point_lens(u, rho):
    """Finite uniform source of radius rho at distance u from a unit point lens:
    (1/(pi rho^2)) * integral over the disk of A(|w|), written as an integral over the
    radius r = |w| of A(r) times the arc length of |w| = r inside the disk."""
    def arc(r):
        if u == 0.0:
            return 2.0 * np.pi * r if r < rho else 0.0
        c = (r * r + u * u - rho * rho) / (2.0 * r * u)
        if c <= -1.0:
            return 2.0 * np.pi * r
        if c >= 1.0:
            return 0.0
        return 2.0 * r * np.arccos(c)

    f = lambda r: point_lens_mag(r) * arc(r)
    lo, hi = abs(u - rho), u + rho
    total = 0.0
    if u < rho:
        total += integrate.quad(lambda r: point_lens_mag(r) * 2.0 * np.pi * r, 0.0, rho - u,
                                epsabs=0, epsrel=1e-13, limit=400)[0]
        lo = rho - u
    total += integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=400)[0]
    return total / (np.pi * rho * rho)


def ld_disk_point_lens(u, rho, u1):
    """Limb-darkened version: (1/rho^2) int_0^rho r' dr' int_0^2pi dphi I(r'/rho) A(|w_c + r' e^{i phi}|)."""
    def inner(rp):
        g = lambda ph: point_lens_mag(np.abs(u + rp * np.exp(1j * ph)))
        val = integrate.quad(g, 0.0, np.pi, epsabs=0, epsrel=1e-12, limit=400)[0] * 2.0
        return val * limb_darkened_I(rp / rho, u1) * rp

    return integrate.quad(inner, 0.0, rho, epsabs=0, epsrel=1e-11, limit=400)[0] / (rho * rho)


def newton_images(eps, a, w, extra_seeds=()):
    """All images of a point source at w by Newton's method on eq. lens_eq from a dense seed set."""
    eps = np.asarray(eps, dtype=np.float64)
    a = np.asarray(a, dtype=np.complex128)
    xs = np.linspace(-3.0, 3.0, 61)
    seeds = (xs[:, None] + 1j * xs[None, :]).ravel()
    rings = []
    for ak in a:
        for r in np.logspace(-7, 0, 36):
            rings.append(ak + r * np.exp(1j * np.linspace(0, 2 * np.pi, 24, endpoint=False)))
    z = np.concatenate([seeds, np.concatenate(rings) if rings else np.zeros(0), np.asarray(extra_seeds)])
    with np.errstate(all="ignore"):
        for _ in range(80):
            F = lens_map(eps, a, z) - w
            k = np.zeros_like(z)
            for e, ak in zip(eps, a):
                k += e / np.conj(z - ak) ** 2
            den = 1.0 - np.abs(k) ** 2
            dz = (k * np.conj(F) - F) / den
            dz = np.where(np.isfinite(dz), dz, 0.0)
            step = np.abs(dz)
            dz = np.where(step > 0.5, dz * 0.5 / np.maximum(step, 1e-300), dz)
            z = z + dz
        F = np.abs(lens_map(eps, a, z) - w)
    good = np.isfinite(F) & (F < 1e-11)
    out = []
    for zz in z[good]:
        if all(abs(zz - y) > 1e-8 * max(1.0, abs(zz)) for y in out):
            out.append(zz)
    return np.array(out)


def multiset_close(x, y, tol):
    """True when the complex multisets x and y match one-to-one within tol*max(1,|x|)."""
    x = list(np.asarray(x)); y = list(np.asarray(y))
    if len(x) != len(y):
        return False
    for v in x:
        d = [abs(v - u) for u in y]
        j = int(np.argmin(d))
        if d[j] > tol * max(1.0, abs(v)):
            return False
        y.pop(j)
    return True


def roots_match_conditioned(x, y, coef, c=1e4):
    """Match root multisets x and y of sum_j coef[j] z^j one-to-one, each pair within the
    first-order forward-error bound of a backward-stable solver:
    c * u * sum_j |b_j| |z|^j / |P'(z)| + 1e-13 max(1,|z|), u = 2^-53 (clustered roots
    near a low-mass lens are ill-conditioned for any method, LAPACK included)."""
    coef = np.asarray(coef, dtype=np.complex128)
    dcoef = coef[1:] * np.arange(1, coef.size)
    x = list(np.asarray(x)); y = list(np.asarray(y))
    if len(x) != len(y):
        return False
    for v in x:
        scale = np.sum(np.abs(coef) * abs(v) ** np.arange(coef.size))
        dp = abs(np.polyval(dcoef[::-1], v))
        tol = c * 2.0 ** -53 * scale / max(dp, 1e-300) + 1e-13 * max(1.0, abs(v))
        d = [abs(v - u) for u in y]
        j = int(np.argmin(d))
        if d[j] > tol:
            return False
        y.pop(j)
    return True


def brute_force_irs(eps, a, wc, rho, u1, half=2.0, npix=8192, center=0j, chunk=256):
    """Cartesian inverse ray shooting over the square |Re z - Re c|, |Im z - Im c| <= half:
    magnification = sum over pixels of I(d/rho) * pixel area / rho^2 (I normalised)."""
    h = 2.0 * half / npix
    xs = center.real - half + (np.arange(npix) + 0.5) * h
    ys = center.imag - half + (np.arange(npix) + 0.5) * h
    total = 0.0
    for r0 in range(0, npix, chunk):
        z = xs[None, :] + 1j * ys[r0:r0 + chunk, None]
        d = np.abs(lens_map(eps, a, z) - wc)
        m = d < rho
        if m.any():
            total += limb_darkened_I(d[m] / rho, u1).sum()
    return total * h * h / (rho * rho)
