"""Pins of the oracle's clip certificate and retry step (O12; the paper's safety margin of
Sec. 3.2 comes with no coverage check, so this step is a reading of this project).

The retry step widens every sector whose inside rays touch an edge on exactly the touched
sides, by half the sector's extent, merges the list again and recomputes.  Pinned by its
observable properties: only flagged sides move, outward, by half the extent; periodic
sectors keep their full ring; the merged list still covers every widened sector; and on a
point lens whose first sectors are cut short (8 limb points for a ring image), zero retries
leave the clip bit and a large error while two retries clear it and reach the exact
finite-source magnification (a 1-D quadrature of the point-lens magnification over the
disk, independent of the oracle) within the grid's error.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import reference_math as R

TWO_PI = 2.0 * np.pi


@pytest.mark.parametrize("clip", range(16))
def test_widen_moves_exactly_the_flagged_sides(clip):
    r_lo, r_hi, t_lo, t_hi = 1.0, 1.4, -0.5, 0.3
    (out,), per = O.retry_sectors([[r_lo, r_hi, t_lo, t_hi]], [0], [clip])
    assert not per[0]
    er, et = r_hi - r_lo, t_hi - t_lo
    want = [r_lo - 0.5 * er if clip & 1 else r_lo, r_hi + 0.5 * er if clip & 2 else r_hi,
            t_lo - 0.5 * et if clip & 4 else t_lo, t_hi + 0.5 * et if clip & 8 else t_hi]
    assert np.allclose(out, want, rtol=0, atol=1e-15), (clip, out, want)
    # every side that moved moved outward: the new sector contains the old one
    assert out[0] <= r_lo and out[1] >= r_hi and out[2] <= t_lo and out[3] >= t_hi


def test_widen_floors_r_at_zero_and_keeps_a_periodic_ring():
    (out,), per = O.retry_sectors([[0.1, 0.5, -np.pi, np.pi]], [1], [15])
    assert per[0] and out[0] == 0.0 and out[1] == pytest.approx(0.7) and out[2] == -np.pi and out[3] == np.pi


def test_widen_across_the_branch_cut_and_to_a_full_ring():
    (out,), per = O.retry_sectors([[1.0, 1.1, 2.9, 3.1]], [0], [8])
    assert not per[0]
    assert -np.pi <= out[2] < np.pi and out[3] - out[2] == pytest.approx(0.3)
    assert np.isclose((out[2] - 2.9 + np.pi) % TWO_PI - np.pi, 0.0)
    (out,), per = O.retry_sectors([[1.0, 1.1, -2.0, 2.0]], [0], [12])   # 4 + 2 + 2 >= 2 pi
    assert per[0] and out[2] == -np.pi and out[3] == np.pi


def _inside(pt, s, per):
    r, th = pt
    if not (s[0] <= r <= s[1]):
        return False
    if per:
        return True
    return any(s[2] <= th + k * TWO_PI <= s[3] for k in (-1, 0, 1))


def test_retry_merge_covers_every_widened_sector():
    rng = np.random.default_rng(12)
    for trial in range(300):
        n = int(rng.integers(1, 7))
        sec, per, clips = [], [], []
        for _ in range(n):
            r0 = rng.uniform(0.2, 2.0)
            t0 = rng.uniform(-np.pi, np.pi)
            sec.append([r0, r0 + rng.uniform(0.01, 0.3), t0, t0 + rng.uniform(0.01, 1.0)])
            per.append(int(rng.uniform() < 0.1))
            clips.append(int(rng.integers(0, 16)))
        out, oper = O.retry_sectors(sec, per, clips)
        assert 1 <= out.shape[0] <= n
        # sorted by (theta_lo, r_lo) and pairwise disjoint (the merge ran to its fixpoint)
        keys = [(o[2], o[0]) for o in out]
        assert keys == sorted(keys)
        # points of every widened input sector lie in some output sector
        for s, p, c in zip(sec, per, clips):
            (w,), (wp,) = O.retry_sectors([s], [p], [c])
            for _ in range(20):
                r = rng.uniform(w[0], w[1])
                th = rng.uniform(w[2], w[3]) if not wp else rng.uniform(-np.pi, np.pi)
                assert any(_inside((r, th), o, op) for o, op in zip(out, oper)), (trial, s, c, out)


def test_clip_retry_end_to_end_on_a_ring_image():
    """Point lens, uniform source of rho = 0.1 over the lens (u = 0.3 rho): the image is a
    ring, and 8 limb points give sectors that cut it short."""
    rho, u = 0.1, 0.03
    p = O.params(s=1.0, q=1.0, u0=u, alpha=0.0, t0=0.0, tE=1.0, rho=rho, u1=0.0)
    exact = R.uniform_disk_point_lens(u, rho)
    r0 = O.magnification(1, p, np.array([0.0]), n_limb=8, n_r=128, n_theta=512, max_retries=0)
    assert r0["status"][0] & 8, "the first sectors must clip"
    assert abs(r0["mag"][0] / exact - 1) > 0.05
    r2 = O.magnification(1, p, np.array([0.0]), n_limb=8, n_r=128, n_theta=512, max_retries=2)
    assert not r2["status"][0] & 8
    assert abs(r2["mag"][0] / exact - 1) < 1e-4
    # the final sectors hold every inside ray away from their edges
    eps, a = O.frame(1, p)
    wc = O.source_center(p, 0.0)
    for k in range(r2["nsec"][0]):
        _, clip = O.sector_flux(eps, a, wc, rho, 0.0, 128, 512, r2["sectors"][0, k], bool(r2["periodic"][0, k]))
        assert clip == 0
