"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same inputs.

Tolerances: 1e-6 relative on magnifications from the FP64 ray loop; sector bounds within
1e-12 (they are min/max of the same FP64 image points, up to last-bit differences of the
device hypot/atan2); centre images 1e-9.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-6


def _run(w, ray="fp64", root="fp64", n_r=None, n_theta=None, n_limb=None, retries=2):
    h = icrs.Handle(n_lens=w.n_lens, n_limb=n_limb or w.n_limb, n_r=n_r or w.n_r, n_theta=n_theta or w.n_theta,
                    ray_precision=ray, root_precision=root, max_retries=retries)
    t = torch.tensor(w.t, device="cuda")
    mag, st = h.magnification(w.params, w.offsets, t)
    sec, per, ns = h.get_sectors(w.n_epochs)
    torch.cuda.synchronize()
    return (mag.cpu().numpy(), st.cpu().numpy().astype(np.uint32), sec.cpu().numpy(), per.cpu().numpy(),
            ns.cpu().numpy(), h)


def _oracle(w, n_r=None, n_theta=None, n_limb=None, retries=2):
    out = dict(mag=[], status=[], sectors=[], periodic=[], nsec=[], a_ps=[])
    for i in range(w.n_events):
        t = w.t[w.offsets[i]:w.offsets[i + 1]]
        if t.size == 0:
            continue
        r = O.magnification(w.n_lens, w.params[i], t, n_limb=n_limb or w.n_limb, n_r=n_r or w.n_r,
                            n_theta=n_theta or w.n_theta, max_retries=retries)
        for k in out:
            out[k].append(r[k])
    return {k: np.concatenate(v) for k, v in out.items()}


def _report(name, rel):
    print(f"{name}: n={rel.size} max rel {np.max(rel):.3e} median {np.median(rel):.3e}", flush=True)


def _check_every_epoch(w, mag, sec, per, ns, ref, tol, name, n_r=None, n_theta=None, min_same=0.9):
    """Value check of every epoch.  Where the device and the oracle chose the same sector
    count, the device's magnification is compared with the oracle's end-to-end result;
    where they did not (image-limb points on the other side of a bin edge after last-bit
    differences of the two root paths), it is compared with the oracle's quadrature on the
    device's own final sectors on the same grid, so no epoch goes unchecked.  Returns the
    per-epoch relative errors."""
    n_r = n_r or w.n_r
    n_theta = n_theta or w.n_theta
    same = ns == ref["nsec"]
    rel = np.abs(mag / ref["mag"] - 1)
    ev_of = np.repeat(np.arange(w.n_events), np.diff(w.offsets))
    for e in np.nonzero(~same)[0]:
        om, _ = O.magnification_given(w.n_lens, w.params[ev_of[e]], w.t[e:e + 1], sec[e:e + 1], per[e:e + 1],
                                      ns[e:e + 1], n_r, n_theta)
        rel[e] = abs(mag[e] / om[0] - 1)
    print(f"{name}: sector-count agreement {same.mean():.3f} ({np.count_nonzero(~same)} epochs checked on the "
          f"device's own sectors)", flush=True)
    _report(name, rel)
    assert same.mean() >= min_same
    assert np.all(rel <= tol), np.nonzero(rel > tol)
    return rel


def test_config1_end_to_end_fp64():
    w = W.config1()
    mag, st, sec, per, ns, _ = _run(w)
    ref = _oracle(w)
    assert np.array_equal(ns, ref["nsec"]), np.nonzero(ns != ref["nsec"])
    rel = np.abs(mag / ref["mag"] - 1)
    _report("config1 fp64", rel)
    assert np.all(rel <= FP64_TOL)
    assert np.array_equal(st, ref["status"])


def test_config1_sectors_match_oracle():
    w = W.config1()
    _, _, sec, per, ns, _ = _run(w)
    ref = _oracle(w)
    for e in range(w.n_epochs):
        k = ns[e]
        assert np.array_equal(per[e, :k], ref["periodic"][e, :k])
        assert np.allclose(sec[e, :k], ref["sectors"][e, :k], rtol=1e-12, atol=1e-12), e


@pytest.mark.parametrize("n_r,n_theta", [(64, 256), (48, 768)])
def test_given_grid_fp64_matches_oracle_quadrature(n_r, n_theta):
    """Given-grid mode isolates the ray kernel: the oracle's own sectors in, same rule out
    (FP64 map; 4 and 12 column chunks per lane)."""
    w = W.config1()
    ref = _oracle(w)
    h = icrs.Handle(n_lens=2, n_limb=64, n_r=n_r, n_theta=n_theta)
    t = torch.tensor(w.t, device="cuda")
    mag, st = h.magnification_given(w.params, w.offsets, t, torch.tensor(ref["sectors"], device="cuda"),
                                    torch.tensor(ref["periodic"], device="cuda"),
                                    torch.tensor(ref["nsec"], device="cuda"))
    torch.cuda.synchronize()
    omag, ost = O.magnification_given(2, w.params[0], w.t, ref["sectors"], ref["periodic"], ref["nsec"], n_r,
                                      n_theta)
    rel = np.abs(mag.cpu().numpy() / omag - 1)
    _report("given fp64", rel)
    assert np.all(rel <= FP64_TOL)
    assert np.array_equal(st.cpu().numpy().astype(np.uint32), ost)


def test_point_images_and_point_magnification():
    w = W.config1()
    h = icrs.Handle(n_lens=2)
    img, nimg, aps = h.point_images(w.params, w.offsets, torch.tensor(w.t, device="cuda"))
    torch.cuda.synchronize()
    img, nimg, aps = img.cpu().numpy(), nimg.cpu().numpy(), aps.cpu().numpy()
    eps, a = O.frame(2, w.params[0])
    for e in range(w.n_epochs):
        wc = O.source_center(w.params[0], w.t[e])
        A, mu = O.point_mag(eps, a, wc)
        ref_img, _ = O.images(eps, a, wc)
        assert nimg[e] == ref_img.size
        assert abs(aps[e] / A - 1) < 1e-9
        got = img[e, :nimg[e], 0] + 1j * img[e, :nimg[e], 1]
        for z in ref_img:
            assert np.min(np.abs(got - z)) < 1e-9


# planetary binaries and source positions where two spurious polynomial roots drift under
# Newton's method onto a true image (the same cases as the oracle's pins)
_SPURIOUS_ROOT_CASES = [
    (1.0793728902057527, 0.001167028363938295, complex(-0.008990128174860168, -0.010468223600270318)),
    (1.089884594939463, 0.0004575128863159917, complex(-0.021429513775496872, 0.01119651425329449)),
    (0.9083764282993901, 0.007207658833706398, complex(0.1583932445640939, 0.002727332799449043)),
]


@pytest.mark.parametrize("roots", ["fp32", "fp64"])
def test_spurious_roots_are_not_kept_as_second_images(roots):
    """The device's validated images at those positions (trajectory along the real axis
    through each, alpha = 0) equal the oracle's three, with no image-count flag."""
    params = np.stack([O.params(s=s, q=q, u0=w.imag, alpha=0.0, t0=0.0, tE=1.0, rho=1e-3, u1=0.5)
                       for s, q, w in _SPURIOUS_ROOT_CASES])
    t = np.array([w.real for _, _, w in _SPURIOUS_ROOT_CASES])
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision=roots)
    img, nimg, _ = h.point_images(params, np.arange(4, dtype=np.int64), torch.tensor(t, device="cuda"))
    torch.cuda.synchronize()
    img, nimg = img.cpu().numpy(), nimg.cpu().numpy()
    for e, (s, q, w) in enumerate(_SPURIOUS_ROOT_CASES):
        eps, a = O.frame(2, params[e])
        assert abs(O.source_center(params[e], t[e]) - w) < 1e-15
        ref, st = O.images(eps, a, w)
        assert st == 0 and ref.size == 3
        got = img[e, :nimg[e], 0] + 1j * img[e, :nimg[e], 1]
        assert nimg[e] == 3, got
        for z in ref:
            assert np.min(np.abs(got - z)) < 1e-9


# a planetary binary (s = 0.768, q = 1.4e-5) and source points just inside its planetary
# caustic, limb points of benchmark-workload epochs (the same points as the oracle's pins):
# five images, three or four of them within a few 1e-3 of each other next to the planet.  At
# the last point two images 2e-5 apart straddle the critical curve: a cold solve's cluster
# roots land 3e-5 off, both polished onto one image under a fixed 8-step Newton cap, and the
# step-test-only continuation then divided by an exactly zero P(z) and returned NaN roots.
_PLANETARY_CLUSTER_S_Q = (0.7680762680197694, 1.3738029330516958e-05)
_PLANETARY_CLUSTER_POINTS = [complex(-0.5342693897421594, -0.00689307926796158),
                             complex(-0.5339617226949848, -0.0073322717253918885),
                             complex(-0.5337469782160287, -0.007306817365788684),
                             complex(-0.5351270736998957, -0.0062434861140690575),
                             complex(-0.5336263835786164, -0.007107361116016892),
                             complex(-0.5325874217950066, -0.00622251111559628)]


@pytest.mark.parametrize("roots", ["fp32", "fp64"])
def test_images_of_a_root_cluster_next_to_a_planet(roots):
    """Device images at those points (each taken as the source centre of a cold solve) equal
    the oracle's five, each within 1e-9, with no status bit."""
    s, q = _PLANETARY_CLUSTER_S_Q
    pts = _PLANETARY_CLUSTER_POINTS
    params = np.stack([O.params(s=s, q=q, u0=w.imag, alpha=0.0, t0=0.0, tE=1.0, rho=1e-3, u1=0.5) for w in pts])
    t = np.array([w.real for w in pts])
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision=roots)
    img, nimg, aps = h.point_images(params, np.arange(len(pts) + 1, dtype=np.int64), torch.tensor(t, device="cuda"))
    torch.cuda.synchronize()
    img, nimg, aps = img.cpu().numpy(), nimg.cpu().numpy(), aps.cpu().numpy()
    for e, w in enumerate(pts):
        eps, a = O.frame(2, params[e])
        assert abs(O.source_center(params[e], t[e]) - w) < 1e-15
        ref, st = O.images(eps, a, w)
        assert st == 0 and ref.size == 5
        got = img[e, :nimg[e], 0] + 1j * img[e, :nimg[e], 1]
        print(f"point {e}: device {nimg[e]} images, oracle {ref.size}", flush=True)
        assert nimg[e] == 5 and np.all(np.isfinite(got)), got
        for z in ref:
            assert np.min(np.abs(got - z)) < 1e-9
        A, _ = O.point_mag(eps, a, w)
        assert abs(aps[e] / A - 1) < 1e-9


def test_ragged_binary_batch_fp64():
    """Uneven events (one empty), planetary mass ratios, FP64 roots and rays at 64 x 256."""
    big = W.binary_batch(2, 8)
    sub = big.subset([0, 1, 2, 3, 4, 5])
    ts, off = [], [0]
    for i in range(sub.n_events):
        seg = sub.t[sub.offsets[i]:sub.offsets[i + 1]]
        take = [0, 7, 3, 11, 1, 5][i]
        seg = seg[:: max(1, seg.size // max(take, 1))][:take]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("ragged", 2, sub.params, np.array(off, np.int64), np.concatenate(ts), 64, 64, 256, "fp64", "fp64")
    mag, st, sec, per, ns, _ = _run(w)
    ref = _oracle(w)
    _check_every_epoch(w, mag, sec, per, ns, ref, FP64_TOL, "ragged fp64", min_same=0.95)


def test_triple_fp64_small():
    big = W.config3(n_events=3, n_epochs=2000)
    ts, off = [], [0]
    for i in range(3):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]][980:1020:4]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("triple-small", 3, big.params, np.array(off, np.int64), np.concatenate(ts), 64, 64, 256,
                   "fp64", "fp64")
    mag, st, sec, per, ns, _ = _run(w)
    ref = _oracle(w)
    _check_every_epoch(w, mag, sec, per, ns, ref, FP64_TOL, "triple fp64")


def test_run_to_run_bitwise_determinism():
    w = W.config1()
    a = _run(w)[0]
    b = _run(w)[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("ray", ["fp32", "fp64"])
def test_results_do_not_depend_on_workspace_contents(ray):
    """Planetary events at rho = 1e-3 (FP32 roots): the same call on a workspace prefilled
    with different byte patterns gives bitwise identical magnifications, status words and
    final sectors, so no kernel reads workspace memory it has not written in the call."""
    w = _planetary_subset(n_events=8, per_event=12, rho=1e-3)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision=ray, root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    nb = h.workspace_bytes(w.n_events, w.n_epochs)
    out = []
    for fill in (0x00, 0xFF, 0x3C, 0x00):
        ws = torch.full((nb,), fill, dtype=torch.uint8, device="cuda")
        mag, st = h.magnification(w.params, w.offsets, t, workspace=ws)
        sec, per, ns = h.get_sectors(w.n_epochs, ws)
        torch.cuda.synchronize()
        ns = ns.cpu().numpy()
        sec = sec.cpu().numpy()
        out.append((mag.cpu().numpy(), st.cpu().numpy(), ns, [sec[e, :ns[e]] for e in range(w.n_epochs)]))
    m0, s0, n0, sec0 = out[0]
    assert np.all(np.isfinite(m0))
    for m, st, ns, sec in out[1:]:
        assert np.array_equal(m, m0) and np.array_equal(st, s0) and np.array_equal(ns, n0)
        assert all(np.array_equal(a, b, equal_nan=True) for a, b in zip(sec, sec0))


def test_triple_results_do_not_depend_on_workspace_contents():
    """The triple-lens workload's configuration (FP64 roots, FP32 rays, 128 x 512) on a few
    epochs around each event's peak, with differently prefilled workspaces."""
    big = W.config3(n_events=3, n_epochs=2000)
    ts, off = [], [0]
    for i in range(3):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]][990:1010:4]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    h = icrs.Handle(n_lens=3, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp64")
    t = torch.tensor(np.concatenate(ts), device="cuda")
    offsets = np.array(off, np.int64)
    nb = h.workspace_bytes(3, t.numel())
    out = []
    for fill in (0x00, 0xFF, 0x3C):
        ws = torch.full((nb,), fill, dtype=torch.uint8, device="cuda")
        mag, st = h.magnification(big.params, offsets, t, workspace=ws)
        torch.cuda.synchronize()
        out.append((mag.cpu().numpy(), st.cpu().numpy()))
    assert np.all(np.isfinite(out[0][0]))
    for m, st in out[1:]:
        assert np.array_equal(m, out[0][0]) and np.array_equal(st, out[0][1])


def test_invalid_arguments_are_rejected_before_launch():
    w = W.config1()
    h = icrs.Handle(n_lens=2)
    t = torch.tensor(w.t, device="cuda")
    bad = w.params.copy()
    bad[0, 1] = -0.1                        # q <= 0
    with pytest.raises(icrs.IcrsError) as ei:
        h.magnification(bad, w.offsets, t)
    assert ei.value.code == -1
    with pytest.raises(icrs.IcrsError):
        h.magnification(w.params, np.array([0, 199]), t)   # offsets do not cover n_epochs
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(icrs.IcrsError) as ei:
        h.magnification(w.params, w.offsets, t, workspace=small)
    assert ei.value.code == -2


FP32_TOL = 3e-5


def _planetary_subset(n_events=6, per_event=6, rho=None, seed=2):
    big = W.binary_batch(seed, 24, rho_fixed=rho)
    ts, off = [], [0]
    for i in range(n_events):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]]
        seg = seg[np.linspace(0, seg.size - 1, per_event).astype(int)]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    return W.Workload("planetary-subset", 2, big.params[:n_events], np.array(off, np.int64), np.concatenate(ts),
                      128, 128, 512, "fp32", "fp32")


@pytest.mark.parametrize("n_r,n_theta", [(32, 128), (24, 96), (128, 512), (64, 256), (48, 320), (48, 768),
                                         (40, 704), (32, 1024)])
def test_fp32_rays_given_grid_planetary(n_r, n_theta):
    """FP32 ray loop (anchor-relative) on the oracle's own sectors: 3e-5 of the FP64 oracle.
    The grids cover every kernel shape: 2 (with a partial chunk at 96), 4, 8 (with a partial
    chunk at 320), 12 (with a partial chunk at 704) and 16 column chunks per lane."""
    w = _planetary_subset(rho=1e-3)
    ref = _oracle(w)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=n_r, n_theta=n_theta, ray_precision="fp32", root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    mag, st = h.magnification_given(w.params, w.offsets, t, torch.tensor(ref["sectors"], device="cuda"),
                                    torch.tensor(ref["periodic"], device="cuda"),
                                    torch.tensor(ref["nsec"], device="cuda"))
    torch.cuda.synchronize()
    om = []
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        om.append(O.magnification_given(2, w.params[i], w.t[sl], ref["sectors"][sl], ref["periodic"][sl],
                                        ref["nsec"][sl], n_r, n_theta)[0])
    om = np.concatenate(om)
    rel = np.abs(mag.cpu().numpy() / om - 1)
    _report(f"given fp32 planetary {n_r}x{n_theta}", rel)
    assert np.all(rel <= FP32_TOL)


@pytest.mark.parametrize("delta_c", [0.05, 0.3, 0.6])
@pytest.mark.parametrize("n_r,n_theta", [(32, 128), (64, 256), (48, 320), (128, 1024)])
def test_fp32_edge_rule_branch_at_other_delta_c(n_r, n_theta, delta_c):
    """The limb-darkened edge rule jumps at delta_c (App. A.2), and the FP32 path takes the
    branch of a crossing within its rounding of delta_c from FP64 stencil distances.  With the
    jump moved to 0.05, 0.3 or 0.6 every epoch still matches the oracle's quadrature on the
    same sectors and delta_c to the FP32 bar (a branch flip costs ~0.2 of a node's weight,
    up to 4e-4 of a poorly resolved image at the coarse grids).  The grids cover the 2-, 4-,
    8- (with a partial chunk) and 16-chunk kernels."""
    w = _planetary_subset(n_events=8, per_event=8, rho=1e-3)
    ref = _oracle(w)
    t = torch.tensor(w.t, device="cuda")
    args = [torch.tensor(ref[k], device="cuda") for k in ("sectors", "periodic", "nsec")]
    om = []
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        om.append(O.magnification_given(2, w.params[i], w.t[sl], ref["sectors"][sl], ref["periodic"][sl],
                                        ref["nsec"][sl], n_r, n_theta, delta_c=delta_c)[0])
    om = np.concatenate(om)
    for rays, tol in (("fp64", FP64_TOL), ("fp32", FP32_TOL)):
        h = icrs.Handle(n_lens=2, n_limb=128, n_r=n_r, n_theta=n_theta, ray_precision=rays, root_precision="fp32",
                        delta_c=delta_c)
        mag, st = h.magnification_given(w.params, w.offsets, t, *args)
        torch.cuda.synchronize()
        rel = np.abs(mag.cpu().numpy() / om - 1)
        _report(f"given {rays} planetary {n_r}x{n_theta} delta_c={delta_c}", rel)
        assert np.all(rel <= tol)


def test_fp32_end_to_end_planetary():
    """Config-2 shape: FP32 EA + FP64 polish, FP32 rays, 128 limb points, 128 x 512."""
    w = _planetary_subset()
    mag, st, sec, per, ns, _ = _run(w, ray="fp32", root="fp32")
    ref = _oracle(w)
    _check_every_epoch(w, mag, sec, per, ns, ref, FP32_TOL, "e2e fp32 planetary", min_same=0.95)


def test_fp32_rays_fall_back_to_fp64_next_to_a_planet():
    """A sector that contains the low-mass lens: FP32 rounding near the planet exceeds the
    budget, the sector goes to the FP64 pass, and the epoch stays within 3e-5 (planetary
    event drawn by the rho = 1e-3 batch generator; epochs around its planetary-image epoch)."""
    p = np.array([1.53866678e+00, 1.13826451e-04, 2.06074577e-01, 3.35158414e+00, 0.0, 20.0, 1e-3,
                  4.97966683e-01, 0.0, 0.0, 0.0])
    t = -17.391698122749006 + np.linspace(-0.02, 0.02, 9)
    w = W.Workload("planet-sector", 2, p[None, :], np.array([0, t.size], np.int64), t, 128, 128, 512, "fp32", "fp32")
    mag, st, sec, per, ns, _ = _run(w, ray="fp32", root="fp32")
    ref = _oracle(w)
    rel = np.abs(mag / ref["mag"] - 1)
    _report("fp32 near planet", rel)
    assert np.all(ns == ref["nsec"])
    assert np.all(rel <= FP32_TOL)


def test_triple_fp32_rays_config3_grid():
    """The triple-lens workload as configured: FP64 roots, FP32 rays, 128 limb points,
    128 x 512 grids; given-grid parity with the oracle at the FP32 bar."""
    big = W.config3(n_events=3, n_epochs=2000)
    ts, off = [], [0]
    for i in range(3):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]][985:1015:6]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("triple-fp32", 3, big.params, np.array(off, np.int64), np.concatenate(ts), 128, 128, 512,
                   "fp32", "fp64")
    ref = _oracle(w)
    h = icrs.Handle(n_lens=3, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp64")
    t = torch.tensor(w.t, device="cuda")
    args = [torch.tensor(ref[k], device="cuda") for k in ("sectors", "periodic", "nsec")]
    mag, _ = h.magnification_given(w.params, w.offsets, t, *args)
    rel = np.abs(mag.cpu().numpy() / ref["mag"] - 1)
    _report("triple fp32 given grid", rel)
    assert np.all(rel <= FP32_TOL)


@pytest.mark.parametrize("n_r,n_theta", [(32, 128), (64, 512)])
@pytest.mark.parametrize("delta_c", [0.1, 0.3])
def test_triple_fp32_edge_rule_branch(n_r, n_theta, delta_c):
    """The triple lens's FP32 ray loop (its own kernel instantiation) with the FP64 retake of
    crossings next to delta_c: given-grid parity with the oracle's quadrature on the same
    sectors and delta_c, at a coarse and at the configured column count."""
    big = W.config3(n_events=3, n_epochs=2000)
    ts, off = [], [0]
    for i in range(3):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]][980:1020:4]
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("triple-fp32", 3, big.params, np.array(off, np.int64), np.concatenate(ts), 128, 128, 512,
                   "fp32", "fp64")
    ref = _oracle(w)
    h = icrs.Handle(n_lens=3, n_limb=128, n_r=n_r, n_theta=n_theta, ray_precision="fp32", root_precision="fp64",
                    delta_c=delta_c)
    t = torch.tensor(w.t, device="cuda")
    args = [torch.tensor(ref[k], device="cuda") for k in ("sectors", "periodic", "nsec")]
    mag, _ = h.magnification_given(w.params, w.offsets, t, *args)
    om = []
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        om.append(O.magnification_given(3, w.params[i], w.t[sl], ref["sectors"][sl], ref["periodic"][sl],
                                        ref["nsec"][sl], n_r, n_theta, delta_c=delta_c)[0])
    rel = np.abs(mag.cpu().numpy() / np.concatenate(om) - 1)
    _report(f"triple fp32 given {n_r}x{n_theta} delta_c={delta_c}", rel)
    assert np.all(rel <= FP32_TOL)


def test_fp32_rays_on_poorly_resolved_near_caustic_images():
    """Epochs of the 2048-event benchmark workload where an image covers only a few hundred
    to a few thousand nodes of its 128 x 512 box, next to a caustic (magnification 10-30).
    There a node whose FP32 distance falls on the other side of rho than its FP64 distance
    moves the magnification by up to 4e-4 under the limb-darkened edge rule; the FP32 loop
    decides such nodes in FP64 and must stay within the FP32 bar on the oracle's sectors."""
    big = W.metric_workload(2048)
    epochs = [902185, 2408231, 4723974, 365802, 2649306, 4664374, 367163, 2857995]
    ev = np.searchsorted(big.offsets, epochs, side="right") - 1
    t = big.t[epochs]
    w = W.Workload("near-caustic-fp32", 2, big.params[ev], np.arange(len(epochs) + 1, dtype=np.int64), t, 128, 128,
                   512, "fp32", "fp32")
    ref = _oracle(w)
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    args = [torch.tensor(ref[k], device="cuda") for k in ("sectors", "periodic", "nsec")]
    mag, _ = h.magnification_given(w.params, w.offsets, torch.tensor(t, device="cuda"), *args)
    rel = np.abs(mag.cpu().numpy() / ref["mag"] - 1)
    _report("fp32 near-caustic images", rel)
    assert np.all(ref["mag"] > 10)
    assert np.all(rel <= FP32_TOL)


# epochs of the 2048-event workload (event 2035, q = 1.4e-5) where one limb point lies inside
# the planetary caustic while the source centre does not: warm-started from the centre's
# roots, two Ehrlich-Aberth iterates settled in the root cluster next to the planet on one
# root, one of the five images went missing and the epoch carried a false image-count flag
# (the last one: a cold solve's pair of cluster roots 3e-5 off, rejected by a fixed 8-step
# polish, then NaN roots from the continuation dividing by an exactly zero P(z))
_LOST_ROOT_EPOCHS = np.array([5083418, 5083483, 5083637, 5083769, 5083922, 5084692, 5085325])


def test_full_benchmark_workload_sampled_against_oracle():
    """The whole 2048-event binary workload (about 5.2 M epochs, FP32 roots and rays,
    128 limb points, 128 x 512) in the configuration the benchmark times: one handle, one
    preallocated workspace, output buffers passed in.  Every output is finite, epochs whose
    limb points lost an image or a root are rare, a second call is bitwise identical, and a
    seeded sample of epochs (the first and last epoch of the batch and a few flagged ones
    among them, and the epochs where a warm-started limb solve once lost an image) matches
    the oracle run end to end on each epoch alone: the image-count flag epoch by epoch, and
    every magnification at the FP32 bar (on the oracle's sectors where the sector counts
    agree, else on the device's own)."""
    w = W.metric_workload(2048)
    h = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=w.n_r, n_theta=w.n_theta, ray_precision="fp32",
                    root_precision="fp32")
    t = torch.tensor(w.t, device="cuda")
    mag = torch.empty(w.n_epochs, dtype=torch.float64, device="cuda")
    status = torch.empty(w.n_epochs, dtype=torch.int32, device="cuda")
    ws = h.learned_workspace(w.n_events, w.n_epochs)
    h.magnification(w.params, w.offsets, t, mag, status, ws)
    first = mag.clone()
    sec_all, per_all, ns_all = h.get_sectors(w.n_epochs, ws)
    h.magnification(w.params, w.offsets, t, mag, status, ws)
    torch.cuda.synchronize()
    assert torch.equal(first, mag)
    m, st = mag.cpu().numpy(), status.cpu().numpy().astype(np.uint32)
    bits = {name: int(np.count_nonzero(st & v)) for name, v in
            (("root_nonconv", icrs.ST_ROOT_NONCONV), ("img_count", icrs.ST_IMG_COUNT),
             ("cap_overflow", icrs.ST_CAP_OVERFLOW), ("clip", icrs.ST_CLIP), ("nan", icrs.ST_NAN))}
    print(f"full workload: {w.n_epochs} epochs, status bits {bits}", flush=True)
    assert np.all(np.isfinite(m)) and np.all(m > 0) and bits["nan"] == 0
    flagged = np.nonzero(st & (icrs.ST_IMG_COUNT | icrs.ST_ROOT_NONCONV | icrs.ST_IMG_RECHECK))[0]
    assert flagged.size <= 64 and bits["img_count"] <= 64   # every flagged epoch is checked below
    assert not np.any(st & icrs.ST_IMG_RECHECK)

    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, w.n_epochs - 1], rng.choice(w.n_epochs, 46, replace=False), flagged,
                                    _LOST_ROOT_EPOCHS]))
    ev = np.searchsorted(w.offsets, idx, side="right") - 1
    sub = W.Workload("full-sample", 2, w.params[ev], np.arange(idx.size + 1, dtype=np.int64), w.t[idx], w.n_limb,
                     w.n_r, w.n_theta, "fp32", "fp32")
    ref = _oracle(sub)
    di = torch.tensor(idx, device="cuda")
    sec, per, ns = sec_all[di].cpu().numpy(), per_all[di].cpu().numpy(), ns_all[di].cpu().numpy()
    for e in np.intersect1d(idx, flagged):
        k = np.searchsorted(idx, e)
        print(f"flagged epoch {e}: status {st[e]} (oracle {ref['status'][k]}), sectors {ns[k]} (oracle "
              f"{ref['nsec'][k]})", flush=True)
    # the image-count flag is the oracle's, epoch by epoch
    assert np.array_equal(st[idx] & icrs.ST_IMG_COUNT, ref["status"] & icrs.ST_IMG_COUNT)
    _check_every_epoch(sub, m[idx], sec, per, ns, ref, FP32_TOL, "full workload, sampled epochs")


def test_repeated_calls_are_bitwise_identical_and_images_validated():
    """Planetary events at rho = 1e-3 with FP32 roots (the configuration in which earlier
    builds returned run-dependent results): twelve eager calls and twelve prepare/run calls,
    with FP32 and with FP64 rays, all give bitwise identical magnifications and status words;
    no kept image ever fails the final substitution check; and the centre images equal the
    oracle's on every epoch (same count, each within 1e-9)."""
    w = _planetary_subset(n_events=8, per_event=12, rho=1e-3)
    t = torch.tensor(w.t, device="cuda")
    for ray in ("fp32", "fp64"):
        h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision=ray, root_precision="fp32")
        ref_m, ref_s = (x.clone() for x in h.magnification(w.params, w.offsets, t))
        for _ in range(11):
            m, s = h.magnification(w.params, w.offsets, t)
            assert torch.equal(m, ref_m) and torch.equal(s, ref_s)
        ws = h.prepare(w.params, w.offsets, w.n_epochs)
        m = torch.empty_like(ref_m)
        s = torch.empty_like(ref_s)
        for _ in range(12):
            m.fill_(-1.0)
            s.fill_(-1)
            h.run(t, m, s)
            torch.cuda.synchronize()
            assert torch.equal(m, ref_m) and torch.equal(s, ref_s)
        st = ref_s.cpu().numpy().astype(np.uint32)
        assert not np.any(st & (icrs.ST_IMG_RECHECK | icrs.ST_NAN))
    h = icrs.Handle(n_lens=2, n_limb=128, n_r=128, n_theta=512, ray_precision="fp32", root_precision="fp32")
    img, nimg, aps = h.point_images(w.params, w.offsets, t)
    torch.cuda.synchronize()
    img, nimg = img.cpu().numpy(), nimg.cpu().numpy()
    for i in range(w.n_events):
        eps, a = O.frame(2, w.params[i])
        for e in range(w.offsets[i], w.offsets[i + 1]):
            ref, _ = O.images(eps, a, O.source_center(w.params[i], w.t[e]))
            got = img[e, :nimg[e], 0] + 1j * img[e, :nimg[e], 1]
            assert nimg[e] == ref.size, (e, got, ref)
            for z in ref:
                assert np.min(np.abs(got - z)) < 1e-9
            # every kept image satisfies the lens equation
            wc = O.source_center(w.params[i], w.t[e])
            for z in got:
                assert abs(z - np.sum(eps / np.conj(z - a)) - wc) < 1e-9


def test_out_of_range_sector_counts_give_nan_and_a_status_bit():
    """icrs_magnification_given and the reverse mode take the sector counts from device memory;
    a count outside 0..10 shoots no rays and marks that epoch (NaN, ICRS_ST_BAD_SECTORS), and
    the other epochs are unchanged."""
    w = W.config1()
    ref = _oracle(w)
    h = icrs.Handle(n_lens=2, n_limb=64, n_r=64, n_theta=256)
    t = torch.tensor(w.t, device="cuda")
    sec = torch.tensor(ref["sectors"], device="cuda")
    per = torch.tensor(ref["periodic"], device="cuda")
    ns_ok = torch.tensor(ref["nsec"], device="cuda")
    good, _ = h.magnification_given(w.params, w.offsets, t, sec, per, ns_ok)
    ns_bad = ns_ok.clone()
    bad_idx = [3, 50, 120]
    ns_bad[3], ns_bad[50], ns_bad[120] = 11, -1, 1 << 20
    m, s = h.magnification_given(w.params, w.offsets, t, sec, per, ns_bad)
    _, J, M = h.magnification_vjp(w.params, w.offsets, t, sec, per, ns_bad, jac=True, mag=True)
    torch.cuda.synchronize()
    m, s, good = m.cpu().numpy(), s.cpu().numpy().astype(np.uint32), good.cpu().numpy()
    J, M = J.cpu().numpy(), M.cpu().numpy()
    mask = np.zeros(w.n_epochs, bool)
    mask[bad_idx] = True
    assert np.all(np.isnan(m[mask])) and np.all(s[mask] & icrs.ST_BAD_SECTORS)
    assert np.array_equal(m[~mask], good[~mask]) and not np.any(s[~mask] & icrs.ST_BAD_SECTORS)
    assert np.all(np.isnan(J[mask])) and np.all(np.isnan(M[mask]))
    assert np.all(np.isfinite(J[~mask])) and np.all(np.abs(M[~mask] / good[~mask] - 1) <= FP64_TOL)


def test_triple_config3_end_to_end_fp32_rays():
    """The triple-lens workload's configuration end to end (FP64 roots, FP32 rays, 128 limb
    points, 128 x 512 grids) on epochs around each of four events' peaks and on their first
    epochs, every epoch value-checked at the FP32 bar."""
    big = W.config3(n_events=4, n_epochs=2000)
    ts, off = [], [0]
    for i in range(4):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]]
        seg = np.concatenate([seg[:2], seg[980:1020:5]])
        ts.append(seg)
        off.append(off[-1] + seg.size)
    w = W.Workload("triple-config3", 3, big.params, np.array(off, np.int64), np.concatenate(ts), 128, 128, 512,
                   "fp32", "fp64")
    mag, st, sec, per, ns, _ = _run(w, ray="fp32", root="fp64")
    ref = _oracle(w)
    assert np.all(np.isfinite(mag))
    _check_every_epoch(w, mag, sec, per, ns, ref, FP32_TOL, "triple config3 e2e")
