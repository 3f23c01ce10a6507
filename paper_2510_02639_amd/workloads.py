"""Seeded synthetic workloads shaped like the paper's (shared by tests and the benchmark).

Holds no step of the ICRS method: it only draws event parameters and epoch times.  To put
epochs around caustic crossings it traces binary-lens caustics (critical curve
sum_k eps_k/(z - a_k)^2 = e^{i phi}, mapped to the source plane) with numpy; that geometry
places inputs and is not used to compute any magnification.

Parameter rows: [s, q, u0, alpha, t0, tE, rho, u_ld, q3, r3, psi] (float64).  Offsets are
CSR int64 [n_events + 1]; epochs t float64 [n_epochs], sorted within each event.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_PARAMS = 11


@dataclass
class Workload:
    name: str
    n_lens: int
    params: np.ndarray    # [n_events, 11]
    offsets: np.ndarray   # [n_events + 1]
    t: np.ndarray         # [n_epochs]
    n_limb: int
    n_r: int
    n_theta: int
    ray_precision: str
    root_precision: str

    @property
    def n_events(self):
        return self.params.shape[0]

    @property
    def n_epochs(self):
        return self.t.size

    def subset(self, events):
        """Events `events` (indices) with all their epochs."""
        events = np.asarray(events)
        p = self.params[events]
        ts, off = [], [0]
        for i in events:
            seg = self.t[self.offsets[i]:self.offsets[i + 1]]
            ts.append(seg)
            off.append(off[-1] + seg.size)
        return Workload(self.name + "-sub", self.n_lens, p, np.array(off, np.int64),
                        np.concatenate(ts) if ts else np.zeros(0), self.n_limb, self.n_r, self.n_theta,
                        self.ray_precision, self.root_precision)

    def sample_epochs(self, every):
        """Every `every`-th epoch of each event (at least one per event)."""
        ts, off = [], [0]
        for i in range(self.n_events):
            seg = self.t[self.offsets[i]:self.offsets[i + 1]][::every]
            ts.append(seg)
            off.append(off[-1] + seg.size)
        return Workload(self.name + f"-every{every}", self.n_lens, self.params.copy(), np.array(off, np.int64),
                        np.concatenate(ts), self.n_limb, self.n_r, self.n_theta, self.ray_precision,
                        self.root_precision)


def _row(s, q, u0, alpha, t0, tE, rho, u1, q3=0.0, r3=0.0, psi=0.0):
    return np.array([s, q, u0, alpha, t0, tE, rho, u1, q3, r3, psi], dtype=np.float64)


def config1() -> Workload:
    """Binary, plain FP64: s=0.9, q=0.1, u0=0.05, alpha=0.6, t0=0, tE=20 d, 200 epochs uniform
    in [-1.5 tE, 1.5 tE], rho=1e-2, u=0.5, 64 limb points, 64 x 256 grids."""
    p = _row(0.9, 0.1, 0.05, 0.6, 0.0, 20.0, 1e-2, 0.5)[None, :]
    t = np.linspace(-30.0, 30.0, 200)
    return Workload("binary-fp64-200", 2, p, np.array([0, 200], np.int64), t, 64, 64, 256, "fp64", "fp64")


# --- binary caustics (input placement only) ----------------------------------------------

def _binary_frame(s, q):
    eps = np.array([1.0 / (1.0 + q), q / (1.0 + q)])
    a = np.array([-q * s / (1.0 + q), s / (1.0 + q)], dtype=np.complex128)
    return eps, a


def binary_caustics(s, q, n_phi=1024):
    """Caustic points [n_lenses, n_phi, 4] of binary lenses, branches tracked along phi."""
    import itertools
    s = np.atleast_1d(np.asarray(s, float))
    q = np.atleast_1d(np.asarray(q, float))
    nl = s.size
    eps1, eps2 = 1.0 / (1.0 + q), q / (1.0 + q)
    a1, a2 = -q * s / (1.0 + q), s / (1.0 + q)
    phi = np.linspace(0.0, 2.0 * np.pi, n_phi, endpoint=False)
    # eps1 (z-a2)^2 + eps2 (z-a1)^2 - e^{i phi} (z-a1)^2 (z-a2)^2 = 0, descending powers
    p1 = np.stack([np.ones(nl), -2 * a1, a1 * a1], -1)
    p2 = np.stack([np.ones(nl), -2 * a2, a2 * a2], -1)
    quart = np.zeros((nl, 5))
    for i in range(3):
        for j in range(3):
            quart[:, i + j] += p1[:, i] * p2[:, j]
    base = np.zeros((nl, 5))
    base[:, 2:] = eps1[:, None] * p2 + eps2[:, None] * p1
    coef = base[:, None, :] - np.exp(1j * phi)[None, :, None] * quart[:, None, :]
    def eig_roots(c):                              # c: [m, 5] descending
        comp = np.zeros((c.shape[0], 4, 4), dtype=np.complex128)
        comp[:, 0, :] = -c[:, 1:] / c[:, :1]
        comp[:, 1, 0] = comp[:, 2, 1] = comp[:, 3, 2] = 1.0
        return np.linalg.eigvals(comp)

    perms = np.array(list(itertools.permutations(range(4))))   # [24, 4]
    z = np.empty((nl, n_phi, 4), dtype=np.complex128)
    z[:, 0] = eig_roots(coef[:, 0])
    dcoef = coef[..., :4] * np.array([4.0, 3.0, 2.0, 1.0])
    for k in range(1, n_phi):
        c, dc = coef[:, k], dcoef[:, k]
        zk = z[:, k - 1].copy()
        for _ in range(4):                           # Newton from the previous phi's roots
            pv = (((c[:, :1] * zk + c[:, 1:2]) * zk + c[:, 2:3]) * zk + c[:, 3:4]) * zk + c[:, 4:5]
            dv = ((dc[:, :1] * zk + dc[:, 1:2]) * zk + dc[:, 2:3]) * zk + dc[:, 3:4]
            zk = zk - pv / dv
        gap = np.abs(zk[:, :, None] - zk[:, None, :]) + np.eye(4) * 1e300
        bad = ~np.isfinite(zk).all(1) | (gap.min(axis=(1, 2)) < 1e-7)
        if bad.any():                                # two tracks met: re-solve and match
            fresh = eig_roots(c[bad])
            prev = z[bad, k - 1]
            cost = np.abs(fresh[:, perms] - prev[:, None, :]).sum(-1)
            zk[bad] = np.take_along_axis(fresh, perms[np.argmin(cost, axis=1)], axis=1)
        z[:, k] = zk
    w = z - eps1[:, None, None] / np.conj(z - a1[:, None, None]) - eps2[:, None, None] / np.conj(z - a2[:, None, None])
    return w


def caustic_crossings(caustic, u0, alpha, tau_max=2.0):
    """Along-track positions tau where the trajectory w(tau) = (tau + i u0) e^{i alpha}
    crosses the caustic polyline; also the tau of closest approach."""
    rot = np.exp(-1j * alpha)
    c = caustic * rot                       # trajectory frame: the path is Im = u0
    y = c.imag - u0
    x = c.real
    taus = []
    n_phi = c.shape[0]
    for b in range(c.shape[1]):
        y0, y1 = y[:, b], np.roll(y[:, b], -1)
        x0, x1 = x[:, b], np.roll(x[:, b], -1)
        idx = np.nonzero((y0 == 0) | (np.sign(y0) != np.sign(y1)))[0]
        for k in idx:
            if abs(c[(k + 1) % n_phi, b] - c[k, b]) > 0.05:   # branch swap at the seam, not a crossing
                continue
            f = y0[k] / (y0[k] - y1[k]) if y0[k] != y1[k] else 0.0
            tx = x0[k] + f * (x1[k] - x0[k])
            if abs(tx) <= tau_max:
                taus.append(tx)
    j = np.argmin(np.abs(y).ravel())
    closest = x.ravel()[j]
    return np.unique(np.round(np.array(taus), 12)), float(np.clip(closest, -tau_max, tau_max))


def _clustered_epochs(rng, taus, closest, n_e, rho, tE, t0=0.0):
    centres = taus if taus.size else np.array([closest])
    k = centres.size
    per = np.full(k, n_e // k)
    per[: n_e - per.sum()] += 1
    parts = [rng.uniform(c - 3 * rho, c + 3 * rho, size=m) for c, m in zip(centres, per)]
    tau = np.sort(np.concatenate(parts))
    return t0 + tau * tE


def binary_batch(seed=2, n_events=2048, rho_fixed=None, n_epochs_fixed=None, name="binary-batch") -> Workload:
    """Planetary-regime binary events: log10 q ~ U[-5,-2], ln s ~ U[ln 0.5, ln 2], u0 ~ U[0,0.3],
    alpha ~ U[0,2 pi), log10 rho ~ U[-3.5,-2] (or fixed), u ~ U[0.3,0.7], N_e ~ U{100..5000}
    (or fixed); t0 = 0, tE = 20 d; epochs uniform within +-3 rho tE of each caustic crossing
    (closest approach when the path misses the caustics).  128 limb points, 128 x 512 grids,
    FP32 rays, FP32 roots with FP64 polish."""
    rng = np.random.default_rng(seed)
    rows, counts = [], []
    for _ in range(n_events):
        lq = rng.uniform(-5.0, -2.0)
        s = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        u0 = rng.uniform(0.0, 0.3)
        alpha = rng.uniform(0.0, 2.0 * np.pi)
        lr = rng.uniform(-3.5, -2.0)
        u1 = rng.uniform(0.3, 0.7)
        n_e = int(rng.integers(100, 5001))
        rho = 10 ** lr if rho_fixed is None else rho_fixed
        if n_epochs_fixed is not None:
            n_e = n_epochs_fixed
        rows.append(_row(s, 10 ** lq, u0, alpha, 0.0, 20.0, rho, u1))
        counts.append(n_e)
    params = np.stack(rows)
    caus = binary_caustics(params[:, 0], params[:, 1], n_phi=1024)
    ts = []
    for i in range(n_events):
        taus, closest = caustic_crossings(caus[i], params[i, 2], params[i, 3])
        ts.append(_clustered_epochs(rng, taus, closest, counts[i], params[i, 6], params[i, 5]))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return Workload(name, 2, params, off, np.concatenate(ts), 128, 128, 512, "fp32", "fp32")


def config2(n_events=2048) -> Workload:
    return binary_batch(2, n_events, name="binary-planetary-batch")


def metric_workload(n_events=2048) -> Workload:
    """The benchmark workload: config-2 draws (seed 2) with rho fixed at 1e-3."""
    return binary_batch(2, n_events, rho_fixed=1e-3, name="binary-planetary-rho1e-3")


def config4(n_events=512) -> Workload:
    """Differentiable-fit workload: config-2 draws (seed 4) with rho = 1e-3, 3000 epochs each."""
    return binary_batch(4, n_events, rho_fixed=1e-3, n_epochs_fixed=3000, name="binary-fit-rho1e-3")


def config3(n_events=256, n_epochs=2000, seed=3) -> Workload:
    """Triple lens: m1 = 1, m2, m3 ~ logU[1e-4, 1e-2]; companions at |z| ~ U[0.7, 1.4],
    arg ~ U[0, 2 pi) from the primary; u0 ~ U[0, 0.2], alpha ~ U[0, 2 pi), t0 = 0, tE = 20 d;
    epochs uniform in [-1.5 tE, 1.5 tE]; rho = 1e-3, u = 0.5; 128 limb points, 128 x 512.
    Expressed in the Fig. 3 parameters: the frame is turned so that M2 lies on the +x axis
    (s = |z2|, q = m2, q3 = m3, M3 at r3 e^{i psi} from the M1-M2 midpoint); the trajectory
    angle is drawn in that frame."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n_events):
        m2 = 10 ** rng.uniform(-4, -2)
        m3 = 10 ** rng.uniform(-4, -2)
        z2 = rng.uniform(0.7, 1.4) * np.exp(1j * rng.uniform(0, 2 * np.pi))
        z3 = rng.uniform(0.7, 1.4) * np.exp(1j * rng.uniform(0, 2 * np.pi))
        u0 = rng.uniform(0.0, 0.2)
        alpha = rng.uniform(0.0, 2 * np.pi)
        s = abs(z2)
        z3r = z3 * np.exp(-1j * np.angle(z2)) - s / 2
        rows.append(_row(s, m2, u0, alpha, 0.0, 20.0, 1e-3, 0.5, m3, abs(z3r), float(np.angle(z3r))))
    params = np.stack(rows)
    t = np.tile(np.linspace(-30.0, 30.0, n_epochs), n_events)
    off = np.arange(0, n_events * n_epochs + 1, n_epochs, dtype=np.int64)
    return Workload("triple-batch", 3, params, off, t, 128, 128, 512, "fp32", "fp64")


def fig2_triple(n_epochs=1000, rho=1e-2) -> Workload:
    """The triple-lens gradient example of Sec. 3.5 / Fig. 2: (t0, tE, u0, q, s, alpha, q3,
    r3, psi) = (0, 10 d, 0, 0.5, 1.1, 60 deg, 0.03, 1.24, 76 deg), uniform source, 500 x 500
    grids.  The caption gives no rho and no time range: rho = 1e-2 and t in [-1.5 tE, 1.5 tE]
    are taken."""
    p = _row(1.1, 0.5, 0.0, np.deg2rad(60.0), 0.0, 10.0, rho, 0.0, 0.03, 1.24, np.deg2rad(76.0))[None, :]
    t = np.linspace(-15.0, 15.0, n_epochs)
    return Workload("triple-fig2", 3, p, np.array([0, n_epochs], np.int64), t, 128, 500, 500, "fp64", "fp64")


def cadence_workload(n_events=512, seed=5, rho=1e-3, days=72.0, cadence_min=12.0) -> Workload:
    """Light curves on a survey cadence (Sec. 5.1: 72 days at a 12-minute cadence, 8640 epochs
    per event), planetary-regime binaries drawn as in the benchmark batch (rho fixed), each
    event's window centred on t0 = 0 with tE = 20 d.  Most epochs lie far from the caustics:
    the workload of the hybrid light curve (Sec. 3.4, item iii)."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n_events):
        lq = rng.uniform(-5.0, -2.0)
        s = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        u0 = rng.uniform(0.0, 0.3)
        alpha = rng.uniform(0.0, 2.0 * np.pi)
        u1 = rng.uniform(0.3, 0.7)
        rows.append(_row(s, 10 ** lq, u0, alpha, 0.0, 20.0, rho, u1))
    n_e = int(round(days * 24 * 60 / cadence_min))
    t1 = np.arange(n_e) * (cadence_min / (24 * 60)) - days / 2
    t = np.tile(t1, n_events)
    off = np.arange(0, n_events * n_e + 1, n_e, dtype=np.int64)
    return Workload("binary-cadence-72d-12min", 2, np.stack(rows), off, t, 128, 128, 512, "fp32", "fp32")


def fig4_sources(rho, n_sources=24, seed=44, s=1.0, q=0.1, u1=0.0) -> Workload:
    """The accuracy protocol of Sec. 4.1 / Fig. 4: source centres drawn uniformly inside a
    circle of radius rho around a randomly chosen point of the caustic of the q = 0.1, s = 1
    binary (one resonant caustic, so every source lies within rho of it); uniform source.
    One event per source with a single epoch: t0 = 0, tE = 1, alpha = 0 put the centre at
    w_c = t + i u0."""
    rng = np.random.default_rng(seed)
    caus = binary_caustics(s, q, n_phi=4096)[0].reshape(-1)
    rows, ts = [], []
    for _ in range(n_sources):
        c = caus[rng.integers(caus.size)]
        r = rho * np.sqrt(rng.uniform())
        w = c + r * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi))
        rows.append(_row(s, q, w.imag, 0.0, 0.0, 1.0, rho, u1))
        ts.append(w.real)
    off = np.arange(n_sources + 1, dtype=np.int64)
    return Workload(f"fig4-rho{rho:g}", 2, np.stack(rows), off, np.array(ts), 256, 1000, 1000, "fp64", "fp64")
