"""Pins of the oracle's source-disk quadrature (the grid-free finite-source reference):
closed forms and 1-D / nested adaptive quadrature for a point lens, exact normalisation,
spectral convergence, and the point-source limit for a binary lens."""
import numpy as np

from oracle import oracle as O
from tests import reference_math as R


def _p(u0, rho, u1):
    return O.params(u0=u0, alpha=0.0, t0=0.0, tE=1.0, rho=rho, u1=u1)


def test_no_lens_gives_one():
    m, ch = O.disk_mag(0, _p(0.3, 0.05, 0.5), [0.0, 0.7])
    assert np.allclose(m, 1.0, rtol=0, atol=1e-14) and np.all(ch == 0)


def test_point_lens_uniform_disk_matches_1d_integral():
    for u, rho in ((0.5, 0.1), (0.2, 0.05), (1.0, 1e-2)):
        m, ch = O.disk_mag(1, _p(u, rho, 0.0), [0.0], n_x=48, n_phi=256)
        ref = R.uniform_disk_point_lens(u, rho)
        assert ch[0] == 0
        assert abs(m[0] / ref - 1) < 1e-9, (u, rho, m[0], ref)


def test_point_lens_limb_darkened_disk_matches_nested_quadrature():
    for u, rho, u1 in ((0.5, 0.1, 0.5), (0.3, 0.05, 0.7)):
        m, _ = O.disk_mag(1, _p(u, rho, u1), [0.0], n_x=48, n_phi=256)
        ref = R.ld_disk_point_lens(u, rho, u1)
        assert abs(m[0] / ref - 1) < 1e-8, (u, rho, u1, m[0], ref)


def test_spectral_convergence_and_point_source_limit_binary():
    p = O.params(s=0.9, q=0.1, u0=0.05, alpha=0.6, t0=0.0, tE=20.0, rho=1e-3, u1=0.5)
    t = np.array([-20.0, -10.0, 8.0, 24.0])           # far from the caustic crossings
    m1, ch = O.disk_mag(2, p, t, n_x=16, n_phi=64)
    m2, _ = O.disk_mag(2, p, t, n_x=32, n_phi=128)
    assert np.all(ch == 0)
    assert np.max(np.abs(m1 / m2 - 1)) < 1e-12
    eps, a = O.frame(2, p)
    aps = np.array([O.point_mag(eps, a, O.source_center(p, tt))[0] for tt in t])
    # finite-source corrections at rho = 1e-3 are O(rho^2) away from caustics
    assert np.max(np.abs(m2 / aps - 1)) < 1e-4


def test_count_changes_flag_a_disk_on_a_caustic():
    p = O.params(s=0.9, q=0.1, u0=0.05, alpha=0.6, t0=0.0, tE=20.0, rho=1e-2, u1=0.5)
    _, ch = O.disk_mag(2, p, [-0.17, 3.08], n_x=16, n_phi=64)   # where the centre crosses the caustic
    assert np.all(ch > 0)
