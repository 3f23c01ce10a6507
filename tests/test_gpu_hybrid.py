"""Hybrid light curve on the GPU (Sec. 3.4, item iii: finite-source treatment only on the
selected epochs, eq. amp_point elsewhere) and its gradient (Sec. 3.5), through the C ABI,
against the oracle: the same epochs selected, point epochs equal to the oracle's A_ps,
extended epochs equal to the oracle's full method (on the device's own sectors where the
sector counts differ), the point-source Jacobian equal to the oracle's dz*/db route, and the
hybrid reverse mode equal to the oracle's rows contracted with the cotangent."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_02639_amd import icrs, workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-6


def _cadence_subset(n_events=6, n_epochs=120, seed=2, rho=1e-3):
    """Planetary events on a regular cadence across the whole event (most epochs far from
    the caustics), plus the clustered epochs next to the caustic crossings."""
    big = W.binary_batch(seed, n_events, rho_fixed=rho)
    ts, off = [], [0]
    for i in range(n_events):
        seg = big.t[big.offsets[i]:big.offsets[i + 1]]
        reg = np.linspace(-30.0, 30.0, n_epochs)
        t = np.sort(np.concatenate([reg, seg[:: max(1, seg.size // 20)]]))
        ts.append(t)
        off.append(off[-1] + t.size)
    return W.Workload("cadence", 2, big.params[:n_events], np.array(off, np.int64), np.concatenate(ts), 64, 64, 256,
                      "fp64", "fp64")


def _run_hybrid(w, h):
    t = torch.tensor(w.t, device="cuda")
    mag, st = h.magnification_hybrid(w.params, w.offsets, t)
    sec, per, ns = h.get_sectors(w.n_epochs, h._hyb_ws)
    torch.cuda.synchronize()
    return (mag.cpu().numpy(), st.cpu().numpy().astype(np.uint32), sec.cpu().numpy(), per.cpu().numpy(),
            ns.cpu().numpy())


@pytest.mark.parametrize("ray,root", [("fp64", "fp64"), ("fp32", "fp32")])
def test_hybrid_matches_oracle(ray, root):
    w = _cadence_subset()
    h = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=w.n_r, n_theta=w.n_theta, ray_precision=ray, root_precision=root)
    mag, st, sec, per, ns = _run_hybrid(w, h)
    point = (st & icrs.ST_POINT) != 0
    tol = FP64_TOL if ray == "fp64" else 3e-5
    n_checked = 0
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        t = w.t[sl]
        ext, aps = O.hybrid_select(2, w.params[i], t)
        assert np.array_equal(~point[sl], ext), (i, np.nonzero(~point[sl] != ext))
        # point epochs: eq. amp_point at the centre
        assert np.all(np.abs(mag[sl][~ext] / aps[~ext] - 1) <= 1e-9)
        # extended epochs: the full method, on the oracle's sectors or on the device's own
        if np.any(ext):
            te = t[ext]
            r = O.magnification(2, w.params[i], te, n_limb=w.n_limb, n_r=w.n_r, n_theta=w.n_theta)
            me, se, pe, ne = mag[sl][ext], sec[sl][ext], per[sl][ext], ns[sl][ext]
            for k in range(te.size):
                if ne[k] == r["nsec"][k]:
                    ref = r["mag"][k]
                else:
                    ref = O.magnification_given(2, w.params[i], te[k:k + 1], se[k:k + 1], pe[k:k + 1], ne[k:k + 1],
                                                w.n_r, w.n_theta)[0][0]
                assert abs(me[k] / ref - 1) <= tol, (i, k, me[k], ref)
                n_checked += 1
    print(f"hybrid {ray}: {w.n_epochs} epochs, {int(point.sum())} point, {n_checked} extended checked", flush=True)
    assert 0.3 * w.n_epochs < point.sum() < w.n_epochs and n_checked > 20


@pytest.mark.parametrize("n_lens", [2, 3])
def test_point_jacobian_matches_oracle_root_derivative(n_lens):
    if n_lens == 2:
        w = _cadence_subset(n_events=4, n_epochs=40)
    else:
        big = W.config3(n_events=3, n_epochs=2000)
        w = big.sample_epochs(50)
    h = icrs.Handle(n_lens=n_lens, n_limb=64, n_r=64, n_theta=256)
    a, J, st = h.point_jacobian(w.params, w.offsets, torch.tensor(w.t, device="cuda"))
    torch.cuda.synchronize()
    a, J, st = a.cpu().numpy(), J.cpu().numpy(), st.cpu().numpy()
    for i in range(w.n_events):
        sl = slice(w.offsets[i], w.offsets[i + 1])
        oa, oj, ost = O.point_jacobian(n_lens, w.params[i], w.t[sl])
        ok = (ost == 0) & (st[sl] == 0)
        assert ok.mean() > 0.9
        assert np.all(np.abs(a[sl][ok] / oa[ok] - 1) <= 1e-9)
        scale = np.abs(oj[ok]).max(axis=0) + 1e-300
        err = np.abs(J[sl][ok] - oj[ok]) / scale
        assert np.all(err <= FP64_TOL), err.max(axis=0)


def test_hybrid_reverse_mode_and_autograd():
    """Point rows from the images, extended rows on the forward's frozen sectors (the
    oracle's dual-number Jacobian on the same sectors), contracted per event; the autograd
    Function's backward returns the same gradient."""
    w = _cadence_subset(n_events=6, n_epochs=40)
    h = icrs.Handle(n_lens=2, n_limb=w.n_limb, n_r=w.n_r, n_theta=w.n_theta)
    t = torch.tensor(w.t, device="cuda")
    mag, st = h.magnification_hybrid(w.params, w.offsets, t)
    sec, per, ns = h.get_sectors(w.n_epochs, h._hyb_ws)
    cot = np.random.default_rng(41).normal(size=w.n_epochs)
    grad, J = h.hybrid_vjp(w.params, w.offsets, t, st, sec, per, ns, cotangent=torch.tensor(cot, device="cuda"),
                           jac=True)
    torch.cuda.synchronize()
    st_np, J, grad = st.cpu().numpy().astype(np.uint32), J.cpu().numpy(), grad.cpu().numpy()
    secn, pern, nsn = sec.cpu().numpy(), per.cpu().numpy(), ns.cpu().numpy()
    point = (st_np & icrs.ST_POINT) != 0
    assert point.any() and (~point).any()
    ref = np.zeros_like(J)
    for i in range(w.n_events):
        sl = np.arange(w.offsets[i], w.offsets[i + 1])
        _, pj, _ = O.point_jacobian(2, w.params[i], w.t[sl])
        _, gj = O.jacobian_given(2, w.params[i], w.t[sl], secn[sl], pern[sl], nsn[sl], w.n_r, w.n_theta)
        ref[sl] = np.where(point[sl][:, None], pj, gj)
    scale = np.abs(ref).max(axis=0) + 1e-300
    assert np.all(np.abs(J - ref) / scale <= FP64_TOL)
    ev = np.repeat(np.arange(w.n_events), np.diff(w.offsets))
    gref = np.zeros((w.n_events, 11))
    np.add.at(gref, ev, cot[:, None] * ref)
    assert np.allclose(grad, gref, rtol=1e-8, atol=1e-10 * np.abs(gref).max())
    params = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    m = icrs.HybridFunction.apply(params, h, w.offsets, t)
    m.backward(torch.tensor(cot, device="cuda"))
    assert np.allclose(params.grad.numpy(), grad, rtol=1e-12, atol=0)
