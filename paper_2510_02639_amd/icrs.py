"""Python binding of the ICRS C ABI (``include/icrs.h``): argument marshalling only.

Every step of the computation runs in the HIP library ``libicrs.so``; this module only
packs host arrays, takes device pointers from torch tensors and calls the C entry points
of the same names.  It raises if the library is missing -- there is no fallback.

Event parameters: float64 [n_events, 11] = [s, q, u0, alpha, t0, tE, rho, u_ld, q3, r3, psi]
(host); epoch offsets int64 [n_events + 1] (host); epochs t float64 [n_epochs] (device).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicrs.so")

ICRS_ABI_VERSION = 1
ICRS_N_PARAMS = 11
ICRS_MAX_SECTORS = 10
ICRS_FP64, ICRS_FP32 = 0, 1
ST_ROOT_NONCONV, ST_IMG_COUNT, ST_CAP_OVERFLOW, ST_CLIP, ST_NAN, ST_GIVEN = 1, 2, 4, 8, 16, 64
_STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "HIP runtime error", -4: "unsupported"}


class IcrsError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {_STATUS.get(code, code)} ({code})")
        self.code = code


class icrs_profile(ctypes.Structure):
    _fields_ = [("ms_centre", ctypes.c_double), ("ms_limb_sectors", ctypes.c_double), ("ms_rays", ctypes.c_double),
                ("ms_finalize", ctypes.c_double), ("n_calls", ctypes.c_int64), ("n_rays_launches", ctypes.c_int64),
                ("n_sector_passes", ctypes.c_int64), ("n_epochs", ctypes.c_int64), ("ms_rays_main", ctypes.c_double),
                ("n_main_launches", ctypes.c_int64), ("n_main_sectors", ctypes.c_int64),
                ("n_main_rays", ctypes.c_int64), ("ms_rays_learned", ctypes.c_double),
                ("n_learned_launches", ctypes.c_int64), ("n_learned_sectors", ctypes.c_int64),
                ("n_learned_rays", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class icrs_learned_config(ctypes.Structure):
    _fields_ = [("n_check", ctypes.c_int32), ("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("log_safety", ctypes.c_double), ("prune_ratio", ctypes.c_double),
                ("vary_max", ctypes.c_double), ("gate_rel", ctypes.c_double), ("margin_frac", ctypes.c_double),
                ("gate_slack", ctypes.c_double)]


class icrs_learned_stats(ctypes.Structure):
    _fields_ = [("n_epochs", ctypes.c_int64), ("n_learned", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("n_gate_rejected", ctypes.c_int64), ("n_pruned_images", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class icrs_hybrid_config(ctypes.Structure):
    _fields_ = [("n_check", ctypes.c_int32), ("reserved", ctypes.c_int32), ("guard", ctypes.c_double),
                ("tol", ctypes.c_double), ("vary_max", ctypes.c_double)]


class icrs_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("n_lens", ctypes.c_int32), ("n_limb", ctypes.c_int32),
                ("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("ray_precision", ctypes.c_int32),
                ("root_precision", ctypes.c_int32), ("max_retries", ctypes.c_int32), ("delta_c", ctypes.c_double)]


_lib = None


def lib():
    """Load libicrs.so (built in-tree by ``__graft_entry__.build()``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    L.icrs_default_config.argtypes = [ctypes.POINTER(icrs_config)]
    L.icrs_create.argtypes = [ctypes.POINTER(icrs_config), vp, ctypes.POINTER(vp)]
    L.icrs_create.restype = ctypes.c_int
    L.icrs_destroy.argtypes = [vp]
    L.icrs_workspace_bytes.argtypes = [vp, i64, i64]
    L.icrs_workspace_bytes.restype = sz
    L.icrs_magnification.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, sz]
    L.icrs_magnification.restype = ctypes.c_int
    L.icrs_magnification_given.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, sz]
    L.icrs_magnification_given.restype = ctypes.c_int
    L.icrs_get_sectors.argtypes = [vp, vp, i64, vp, vp, vp]
    L.icrs_get_sectors.restype = ctypes.c_int
    L.icrs_point_images.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, sz]
    L.icrs_point_images.restype = ctypes.c_int
    L.icrs_magnification_vjp.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz]
    L.icrs_magnification_vjp.restype = ctypes.c_int
    L.icrs_magnification_noalloc.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp]
    L.icrs_magnification_noalloc.restype = ctypes.c_int
    L.icrs_prepare.argtypes = [vp, i64, vp, vp, i64, vp, sz]
    L.icrs_prepare.restype = ctypes.c_int
    L.icrs_run.argtypes = [vp, vp, vp, vp, vp, sz]
    L.icrs_run.restype = ctypes.c_int
    L.icrs_set_profiling.argtypes = [vp, ctypes.c_int]
    L.icrs_set_profiling.restype = ctypes.c_int
    L.icrs_get_profile.argtypes = [vp, ctypes.POINTER(icrs_profile), ctypes.c_int]
    L.icrs_get_profile.restype = ctypes.c_int
    f32 = ctypes.c_float
    L.icrs_mlp_pack.argtypes = [vp, vp, vp]
    L.icrs_mlp_pack.restype = ctypes.c_int
    L.icrs_mlp_forward.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    L.icrs_mlp_forward.restype = ctypes.c_int
    L.icrs_mlp_workspace_bytes.argtypes = [i64]
    L.icrs_mlp_workspace_bytes.restype = sz
    L.icrs_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, sz]
    L.icrs_mlp_loss_grad.restype = ctypes.c_int
    L.icrs_mlp_adamw.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, f32, vp]
    L.icrs_mlp_adamw.restype = ctypes.c_int
    L.icrs_image_bounds.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, sz]
    L.icrs_image_bounds.restype = ctypes.c_int
    L.icrs_default_learned_config.argtypes = [ctypes.POINTER(icrs_learned_config)]
    L.icrs_learned_workspace_bytes.argtypes = [vp, i64, i64]
    L.icrs_learned_workspace_bytes.restype = sz
    L.icrs_magnification_learned.argtypes = [vp, i64, vp, vp, i64, vp, ctypes.POINTER(icrs_learned_config), vp, vp,
                                             vp, vp, vp, ctypes.POINTER(icrs_learned_stats), vp, sz]
    L.icrs_magnification_learned.restype = ctypes.c_int
    L.icrs_run_learned.argtypes = [vp, vp, ctypes.POINTER(icrs_learned_config), vp, vp, vp, vp, vp,
                                   ctypes.POINTER(icrs_learned_stats), vp, sz]
    L.icrs_run_learned.restype = ctypes.c_int
    L.icrs_default_hybrid_config.argtypes = [ctypes.POINTER(icrs_hybrid_config)]
    L.icrs_hybrid_workspace_bytes.argtypes = [vp, i64, i64]
    L.icrs_hybrid_workspace_bytes.restype = sz
    L.icrs_magnification_hybrid.argtypes = [vp, i64, vp, vp, i64, vp, ctypes.POINTER(icrs_hybrid_config), vp, vp,
                                            vp, sz]
    L.icrs_magnification_hybrid.restype = ctypes.c_int
    L.icrs_point_jacobian.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, sz]
    L.icrs_point_jacobian.restype = ctypes.c_int
    L.icrs_disk_magnification.argtypes = [vp, i64, vp, vp, i64, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, sz]
    L.icrs_disk_magnification.restype = ctypes.c_int
    L.icrs_hybrid_vjp.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz]
    L.icrs_hybrid_vjp.restype = ctypes.c_int
    L.icrs_marginal_nll_workspace_bytes.argtypes = [i64]
    L.icrs_marginal_nll_workspace_bytes.restype = sz
    L.icrs_marginal_nll.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, sz]
    L.icrs_marginal_nll.restype = ctypes.c_int
    L.icrs_status_string.argtypes = [ctypes.c_int]
    L.icrs_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


EXPORTED = ["icrs_default_config", "icrs_create", "icrs_destroy", "icrs_workspace_bytes", "icrs_magnification",
            "icrs_magnification_noalloc",
            "icrs_magnification_given", "icrs_magnification_vjp", "icrs_get_sectors", "icrs_point_images",
            "icrs_prepare", "icrs_run", "icrs_set_profiling",
            "icrs_get_profile", "icrs_mlp_pack", "icrs_mlp_forward", "icrs_mlp_workspace_bytes",
            "icrs_mlp_loss_grad", "icrs_mlp_adamw", "icrs_image_bounds", "icrs_default_learned_config",
            "icrs_learned_workspace_bytes", "icrs_magnification_learned", "icrs_run_learned",
            "icrs_default_hybrid_config", "icrs_hybrid_workspace_bytes", "icrs_magnification_hybrid",
            "icrs_point_jacobian", "icrs_hybrid_vjp", "icrs_marginal_nll_workspace_bytes", "icrs_marginal_nll",
            "icrs_disk_magnification", "icrs_status_string"]
ST_LEARNED, ST_FALLBACK, ST_IMG_RECHECK, ST_BAD_SECTORS, ST_POINT = 128, 256, 512, 1024, 2048
ICRS_MAX_EPOCHS = 1 << 27
NOALLOC_SCRATCH_BYTES = 64 << 20
MLP_PARAM_FLOATS, MLP_PACKED_HALFS, MLP_NORM_FLOATS = 39312, 75776, 32


def _check(code, where):
    if code != 0:
        raise IcrsError(code, where)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def _host_events(params, offsets):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, ICRS_N_PARAMS))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1))
    return p, o


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous CUDA tensor of {dtype}")
    return t


class Handle:
    """One icrs_handle bound to the current torch stream of the current device."""

    def __init__(self, n_lens=2, n_limb=64, n_r=64, n_theta=256, ray_precision="fp64", root_precision="fp64",
                 max_retries=2, delta_c=0.1, stream=None):
        L = lib()
        cfg = icrs_config()
        L.icrs_default_config(ctypes.byref(cfg))
        cfg.n_lens, cfg.n_limb, cfg.n_r, cfg.n_theta = n_lens, n_limb, n_r, n_theta
        cfg.ray_precision = ICRS_FP32 if ray_precision == "fp32" else ICRS_FP64
        cfg.root_precision = ICRS_FP32 if root_precision == "fp32" else ICRS_FP64
        cfg.max_retries, cfg.delta_c = max_retries, delta_c
        self.cfg = cfg
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p()
        _check(L.icrs_create(ctypes.byref(cfg), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)), "icrs_create")
        self._h = h
        self._ws = None

    def close(self):
        if self._h:
            lib().icrs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on=True):
        _check(lib().icrs_set_profiling(self._h, int(bool(on))), "icrs_set_profiling")

    def get_profile(self, reset=False):
        out = icrs_profile()
        _check(lib().icrs_get_profile(self._h, ctypes.byref(out), int(bool(reset))), "icrs_get_profile")
        return out.as_dict()

    def workspace_bytes(self, n_events, n_epochs):
        return int(lib().icrs_workspace_bytes(self._h, int(n_events), int(n_epochs)))

    def workspace(self, n_events, n_epochs):
        nb = self.workspace_bytes(n_events, n_epochs)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
            assert self._ws.data_ptr() % 256 == 0
        return self._ws

    def magnification(self, params, offsets, t, mag=None, status=None, workspace=None):
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        mag = torch.empty(n, dtype=torch.float64, device=t.device) if mag is None else mag
        status = torch.empty(n, dtype=torch.int32, device=t.device) if status is None else status
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        code = lib().icrs_magnification(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(mag), _ptr(status),
                                        _ptr(ws), ws.numel())
        _check(code, "icrs_magnification")
        return mag, status

    def magnification_noalloc(self, params, offsets, t, mag=None, status=None):
        """icrs_magnification_noalloc: the plain path on the library's own per-GPU scratch (no
        workspace; the outputs are the caller's)."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        mag = torch.empty(n, dtype=torch.float64, device=t.device) if mag is None else mag
        status = torch.empty(n, dtype=torch.int32, device=t.device) if status is None else status
        _check(lib().icrs_magnification_noalloc(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(mag),
                                                _ptr(status)), "icrs_magnification_noalloc")
        return mag, status

    def prepare(self, params, offsets, n_epochs, workspace=None):
        """Upload a batch once (icrs_prepare); run() then needs no host work (capturable)."""
        p, o = _host_events(params, offsets)
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n_epochs)
        _check(lib().icrs_prepare(self._h, p.shape[0], _ptr(p), _ptr(o), int(n_epochs), _ptr(ws), ws.numel()),
               "icrs_prepare")
        self._prep_ws = ws
        return ws

    def run(self, t, mag, status):
        """icrs_run on the prepared batch: device work only, safe inside stream capture."""
        ws = self._prep_ws
        _check(lib().icrs_run(self._h, _ptr(t), _ptr(mag), _ptr(status), _ptr(ws), ws.numel()), "icrs_run")

    def magnification_given(self, params, offsets, t, sectors, periodic, nsec, workspace=None):
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        sectors = _dev(sectors, torch.float64)
        periodic = _dev(periodic, torch.uint8)
        nsec = _dev(nsec, torch.int32)
        assert sectors.numel() == n * ICRS_MAX_SECTORS * 4 and periodic.numel() == n * ICRS_MAX_SECTORS
        mag = torch.empty(n, dtype=torch.float64, device=t.device)
        status = torch.empty(n, dtype=torch.int32, device=t.device)
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        code = lib().icrs_magnification_given(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(sectors),
                                              _ptr(periodic), _ptr(nsec), _ptr(mag), _ptr(status), _ptr(ws),
                                              ws.numel())
        _check(code, "icrs_magnification_given")
        return mag, status

    def magnification_vjp(self, params, offsets, t, sectors, periodic, nsec, cotangent=None, jac=False, mag=False,
                          workspace=None):
        """Frozen-structure derivatives on the given sectors: returns (grad [V, 11] or None,
        jac [E, 11] or None, mag [E] or None), all CUDA float64."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        sectors = _dev(sectors, torch.float64)
        periodic = _dev(periodic, torch.uint8)
        nsec = _dev(nsec, torch.int32)
        grad = None
        if cotangent is not None:
            cotangent = _dev(cotangent, torch.float64)
            grad = torch.empty((p.shape[0], ICRS_N_PARAMS), dtype=torch.float64, device=t.device)
        J = torch.empty((n, ICRS_N_PARAMS), dtype=torch.float64, device=t.device) if jac else None
        M = torch.empty(n, dtype=torch.float64, device=t.device) if mag else None
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        code = lib().icrs_magnification_vjp(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(sectors),
                                            _ptr(periodic), _ptr(nsec), _ptr(cotangent), _ptr(grad), _ptr(J),
                                            _ptr(M), _ptr(ws), ws.numel())
        _check(code, "icrs_magnification_vjp")
        return grad, J, M

    # ---- hybrid light curve (Sec. 3.4 item iii) and point-source gradient ------------------
    def hybrid_workspace(self, n_events, n_epochs):
        n = lib().icrs_hybrid_workspace_bytes(self._h, n_events, n_epochs)
        return torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")

    def magnification_hybrid(self, params, offsets, t, mag=None, status=None, workspace=None, n_check=16, guard=2.0,
                             tol=1e-4, vary_max=0.1):
        """Hybrid light curve: the plain path on the epochs the selection rule marks, the
        point-source magnification (status ST_POINT) elsewhere.  Returns (mag, status)."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        hc = icrs_hybrid_config()
        lib().icrs_default_hybrid_config(ctypes.byref(hc))
        hc.n_check, hc.guard, hc.tol, hc.vary_max = n_check, guard, tol, vary_max
        mag = torch.empty(n, dtype=torch.float64, device=t.device) if mag is None else mag
        status = torch.empty(n, dtype=torch.int32, device=t.device) if status is None else status
        ws = workspace if workspace is not None else self.hybrid_workspace(p.shape[0], n)
        self._hyb_ws = ws
        _check(lib().icrs_magnification_hybrid(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), ctypes.byref(hc),
                                               _ptr(mag), _ptr(status), _ptr(ws), ws.numel()),
               "icrs_magnification_hybrid")
        return mag, status

    def point_jacobian(self, params, offsets, t, workspace=None):
        """(a_ps [E], jac [E, 11], status [E]) of every epoch's source centre, CUDA."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        a = torch.empty(n, dtype=torch.float64, device=t.device)
        J = torch.empty((n, ICRS_N_PARAMS), dtype=torch.float64, device=t.device)
        st = torch.empty(n, dtype=torch.int32, device=t.device)
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        _check(lib().icrs_point_jacobian(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(a), _ptr(J),
                                         _ptr(st), _ptr(ws), ws.numel()), "icrs_point_jacobian")
        return a, J, st

    def disk_magnification(self, params, offsets, t, n_x=16, n_phi=96, workspace=None):
        """Grid-free reference (mag [E], count_changes [E] int32), CUDA: the brightness-weighted
        mean of the point-source magnification over the source disk; valid where
        count_changes == 0 (no caustic crosses the disk)."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        mag = torch.empty(n, dtype=torch.float64, device=t.device)
        ch = torch.empty(n, dtype=torch.int32, device=t.device)
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        _check(lib().icrs_disk_magnification(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), int(n_x), int(n_phi),
                                             _ptr(mag), _ptr(ch), _ptr(ws), ws.numel()), "icrs_disk_magnification")
        return mag, ch

    def hybrid_vjp(self, params, offsets, t, status, sectors, periodic, nsec, cotangent=None, jac=False,
                   workspace=None):
        """Reverse mode of the hybrid curve: (grad [V, 11] or None, jac [E, 11] or None)."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        grad = None
        if cotangent is not None:
            cotangent = _dev(cotangent, torch.float64)
            grad = torch.empty((p.shape[0], ICRS_N_PARAMS), dtype=torch.float64, device=t.device)
        J = torch.empty((n, ICRS_N_PARAMS), dtype=torch.float64, device=t.device) if jac else None
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        _check(lib().icrs_hybrid_vjp(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(_dev(status, torch.int32)),
                                     _ptr(_dev(sectors, torch.float64)), _ptr(_dev(periodic, torch.uint8)),
                                     _ptr(_dev(nsec, torch.int32)), _ptr(cotangent), _ptr(grad), _ptr(J), _ptr(ws),
                                     ws.numel()), "icrs_hybrid_vjp")
        return grad, J

    # ---- marginalised likelihood (App. B) --------------------------------------------------
    def marginal_nll(self, offsets, mag, flux, sigma, prior, beta=False, grad=True):
        """eq. NLL per event; returns (nll [V], beta [V, 5] or None, dnll/dmag [E] or None)."""
        o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1))
        pr = np.ascontiguousarray(np.asarray(prior, dtype=np.float64).reshape(-1, 4))
        mag = _dev(mag, torch.float64)
        n_ev = o.size - 1
        nll = torch.empty(n_ev, dtype=torch.float64, device=mag.device)
        b = torch.empty((n_ev, 5), dtype=torch.float64, device=mag.device) if beta else None
        g = torch.empty(mag.numel(), dtype=torch.float64, device=mag.device) if grad else None
        nb = lib().icrs_marginal_nll_workspace_bytes(n_ev)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=mag.device)
        _check(lib().icrs_marginal_nll(self._h, n_ev, _ptr(o), mag.numel(), _ptr(mag), _ptr(_dev(flux, torch.float64)),
                                       _ptr(_dev(sigma, torch.float64)), _ptr(pr), _ptr(nll), _ptr(b), _ptr(g),
                                       _ptr(ws), ws.numel()), "icrs_marginal_nll")
        return nll, b, g

    # ---- learned-bounds path ----------------------------------------------------------------
    def learned_workspace(self, n_events, n_epochs):
        n = lib().icrs_learned_workspace_bytes(self._h, n_events, n_epochs)
        return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")

    def image_bounds(self, params, offsets, t, workspace=None):
        """Training data: (features [E, MI, 10] f32, targets [E, MI, 4] f32, n_images [E] i32,
        flags [E] u32 as int32), all CUDA."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        mi = self.cfg.n_lens ** 2 + 1
        feat = torch.empty((n, mi, 10), dtype=torch.float32, device=t.device)
        tgt = torch.empty((n, mi, 4), dtype=torch.float32, device=t.device)
        nimg = torch.empty(n, dtype=torch.int32, device=t.device)
        flags = torch.empty(n, dtype=torch.int32, device=t.device)
        ws = workspace if workspace is not None else self.learned_workspace(p.shape[0], n)
        _check(lib().icrs_image_bounds(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(feat), _ptr(tgt),
                                       _ptr(nimg), _ptr(flags), _ptr(ws), ws.numel()), "icrs_image_bounds")
        return feat, tgt, nimg, flags

    def magnification_learned(self, params, offsets, t, model, mag=None, status=None, workspace=None,
                              n_check=16, n_r=None, n_theta=None, prune_ratio=1e-6, vary_max=0.1, gate_rel=1e-3,
                              margin_frac=0.02, stats=True, gate_slack=0.0):
        """Learned-bounds path; model: a learned.BoundsModel.  Returns (mag, status, stats dict);
        with stats=False the call enqueues device work only (no host wait, capturable) and the
        dict is None."""
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        lc = self._learned_config(model, n_check, n_r, n_theta, prune_ratio, vary_max, gate_rel, margin_frac,
                                  gate_slack)
        mag = mag if mag is not None else torch.empty(n, dtype=torch.float64, device=t.device)
        status = status if status is not None else torch.empty(n, dtype=torch.int32, device=t.device)
        ws = workspace if workspace is not None else self.learned_workspace(p.shape[0], n)
        st = icrs_learned_stats() if stats else None
        _check(lib().icrs_magnification_learned(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), ctypes.byref(lc),
                                                _ptr(model.packed), _ptr(model.params), _ptr(model.norm),
                                                _ptr(mag), _ptr(status), ctypes.byref(st) if stats else None,
                                                _ptr(ws), ws.numel()),
               "icrs_magnification_learned")
        return mag, status, (st.as_dict() if stats else None)

    def _learned_config(self, model, n_check=16, n_r=None, n_theta=None, prune_ratio=1e-6, vary_max=0.1,
                        gate_rel=1e-3, margin_frac=0.02, gate_slack=0.0):
        lc = icrs_learned_config()
        lib().icrs_default_learned_config(ctypes.byref(lc))
        lc.n_check = n_check
        lc.n_r = n_r if n_r is not None else self.cfg.n_r
        lc.n_theta = n_theta if n_theta is not None else self.cfg.n_theta
        lc.log_safety = model.log_safety
        lc.prune_ratio, lc.vary_max, lc.gate_rel = prune_ratio, vary_max, gate_rel
        lc.margin_frac = margin_frac
        lc.gate_slack = gate_slack
        return lc

    def run_learned(self, t, model, mag, status, stats=False, **kw):
        """icrs_run_learned on the batch uploaded by prepare() (whose workspace must be a
        learned workspace): device work only when stats=False, safe inside stream capture."""
        ws = self._prep_ws
        lc = self._learned_config(model, **kw)
        st = icrs_learned_stats() if stats else None
        _check(lib().icrs_run_learned(self._h, _ptr(_dev(t, torch.float64)), ctypes.byref(lc), _ptr(model.packed),
                                      _ptr(model.params), _ptr(model.norm), _ptr(mag), _ptr(status),
                                      ctypes.byref(st) if stats else None, _ptr(ws), ws.numel()),
               "icrs_run_learned")
        return st.as_dict() if stats else None

    # ---- learned-bounds network (blob layouts in include/icrs.h) -------------------------
    def mlp_pack(self, params, packed):
        _check(lib().icrs_mlp_pack(self._h, _ptr(_dev(params, torch.float32)), _ptr(_dev(packed, torch.int16))),
               "icrs_mlp_pack")

    def mlp_forward(self, packed, params, norm, x, y=None):
        x = _dev(x, torch.float32)
        n = x.shape[0]
        y = y if y is not None else torch.empty((n, 4), dtype=torch.float32, device=x.device)
        _check(lib().icrs_mlp_forward(self._h, _ptr(_dev(packed, torch.int16)), _ptr(_dev(params, torch.float32)),
                                      _ptr(_dev(norm, torch.float32)), n, _ptr(x), _ptr(_dev(y, torch.float32))),
               "icrs_mlp_forward")
        return y

    def mlp_loss_grad(self, packed, params, norm, x, target, workspace=None, grad=None, loss=None):
        x = _dev(x, torch.float32)
        n = x.shape[0]
        nb = lib().icrs_mlp_workspace_bytes(n)
        ws = workspace if workspace is not None else torch.empty(nb, dtype=torch.uint8, device=x.device)
        grad = grad if grad is not None else torch.empty(MLP_PARAM_FLOATS, dtype=torch.float32, device=x.device)
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().icrs_mlp_loss_grad(self._h, _ptr(_dev(packed, torch.int16)), _ptr(_dev(params, torch.float32)),
                                        _ptr(_dev(norm, torch.float32)), n, _ptr(x),
                                        _ptr(_dev(target, torch.float32)), _ptr(grad), _ptr(loss), _ptr(ws),
                                        ws.numel()), "icrs_mlp_loss_grad")
        return grad, loss

    def mlp_adamw(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0,
                  packed=None):
        _check(lib().icrs_mlp_adamw(self._h, _ptr(_dev(params, torch.float32)), _ptr(_dev(grad, torch.float32)),
                                    _ptr(_dev(m, torch.float32)), _ptr(_dev(v, torch.float32)), int(step), lr,
                                    beta1, beta2, eps, weight_decay,
                                    _ptr(_dev(packed, torch.int16)) if packed is not None else None),
               "icrs_mlp_adamw")

    def get_sectors(self, n_epochs, workspace=None):
        ws = workspace if workspace is not None else self._ws
        sec = torch.empty((n_epochs, ICRS_MAX_SECTORS, 4), dtype=torch.float64, device="cuda")
        per = torch.empty((n_epochs, ICRS_MAX_SECTORS), dtype=torch.uint8, device="cuda")
        ns = torch.empty(n_epochs, dtype=torch.int32, device="cuda")
        _check(lib().icrs_get_sectors(self._h, _ptr(ws), n_epochs, _ptr(sec), _ptr(per), _ptr(ns)), "icrs_get_sectors")
        return sec, per, ns

    def point_images(self, params, offsets, t, workspace=None):
        p, o = _host_events(params, offsets)
        t = _dev(t, torch.float64)
        n = t.numel()
        img = torch.empty((n, 10, 2), dtype=torch.float64, device=t.device)
        nimg = torch.empty(n, dtype=torch.int32, device=t.device)
        aps = torch.empty(n, dtype=torch.float64, device=t.device)
        ws = workspace if workspace is not None else self.workspace(p.shape[0], n)
        code = lib().icrs_point_images(self._h, p.shape[0], _ptr(p), _ptr(o), n, _ptr(t), _ptr(img), _ptr(nimg),
                                       _ptr(aps), _ptr(ws), ws.numel())
        _check(code, "icrs_point_images")
        return img, nimg, aps


class ICRSFunction(torch.autograd.Function):
    """mag = ICRSFunction.apply(params, handle, offsets, t): plain ICRS light curves with a
    reverse-mode gradient for params (CPU float64 [n_events, 11]).  The backward pass keeps
    the forward's sectors and differentiates on that frozen structure with the library's
    adjoint (FP64 rays recomputed, nothing stored per ray)."""

    @staticmethod
    def forward(ctx, params, handle, offsets, t):
        p = params.detach().cpu().numpy()
        mag, status = handle.magnification(p, offsets, t)
        ctx.frozen = handle.get_sectors(t.numel())
        ctx.handle, ctx.offsets, ctx.t = handle, offsets, t
        ctx.save_for_backward(params)
        ctx.status = status
        return mag

    @staticmethod
    def backward(ctx, grad_mag):
        (params,) = ctx.saved_tensors
        sec, per, ns = ctx.frozen
        grad, _, _ = ctx.handle.magnification_vjp(params.detach().cpu().numpy(), ctx.offsets, ctx.t, sec, per, ns,
                                                  cotangent=grad_mag.contiguous().to(torch.float64))
        return grad.to(params.device), None, None, None


class HybridFunction(torch.autograd.Function):
    """mag = HybridFunction.apply(params, handle, offsets, t): hybrid light curves (the full
    method on the selected epochs, the point-source magnification elsewhere) with a
    reverse-mode gradient for params (CPU float64 [n_events, 11]): point epochs through their
    images, the others on the forward's frozen sectors."""

    @staticmethod
    def forward(ctx, params, handle, offsets, t):
        p = params.detach().cpu().numpy()
        mag, status = handle.magnification_hybrid(p, offsets, t)
        ctx.frozen = handle.get_sectors(t.numel(), handle._hyb_ws)
        ctx.handle, ctx.offsets, ctx.t, ctx.status = handle, offsets, t, status
        ctx.save_for_backward(params)
        return mag

    @staticmethod
    def backward(ctx, grad_mag):
        (params,) = ctx.saved_tensors
        sec, per, ns = ctx.frozen
        grad, _ = ctx.handle.hybrid_vjp(params.detach().cpu().numpy(), ctx.offsets, ctx.t, ctx.status, sec, per, ns,
                                        cotangent=grad_mag.contiguous().to(torch.float64))
        return grad.to(params.device), None, None, None


def light_curve_nll_and_grad(handle, params, offsets, t, flux, sigma, prior, hybrid=False):
    """Fit objective of App. B: total eq. NLL over the events and its gradient with respect
    to the event parameters [V, 11] (dNLL/dmag from the likelihood kernel, contracted by the
    frozen-structure reverse mode of the plain or hybrid path).  Returns (nll [V], grad)."""
    p, o = _host_events(params, offsets)
    if hybrid:
        mag, status = handle.magnification_hybrid(p, o, t)
        sec, per, ns = handle.get_sectors(t.numel(), handle._hyb_ws)
    else:
        mag, status = handle.magnification(p, o, t)
        sec, per, ns = handle.get_sectors(t.numel())
    nll, _, g = handle.marginal_nll(o, mag, flux, sigma, prior)
    if hybrid:
        grad, _ = handle.hybrid_vjp(p, o, t, status, sec, per, ns, cotangent=g)
    else:
        grad, _, _ = handle.magnification_vjp(p, o, t, sec, per, ns, cotangent=g)
    return nll, grad
