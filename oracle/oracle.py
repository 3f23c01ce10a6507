"""ctypes wrapper of the FP64 CPU oracle (``icrs_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with the HIP
library.  Every function mirrors one step of the paper's method (microJAX, arXiv
2510.02639); the C++ source cites the passages.

Parameter vector of an event (doubles): [s, q, u0, alpha, t0, tE, rho, u1, q3, r3, psi].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "icrs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

N_PARAMS = 11
ST_ROOT_NONCONV, ST_IMG_COUNT, ST_CAP_OVERFLOW, ST_CLIP, ST_NAN, ST_GIVEN = 1, 2, 4, 8, 16, 64
ST_POINT = 2048


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, OpenMP over epochs)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i, u8, u32, i32, i64 = (ctypes.c_double, ctypes.c_int, ctypes.c_uint8, ctypes.c_uint32,
                                    ctypes.c_int32, ctypes.c_int64)
        P = ctypes.POINTER
        L.orc_num_threads.restype = i
        L.orc_set_num_threads.argtypes = [i]
        L.orc_frame.argtypes = [i, P(d), P(d), P(d)]
        L.orc_source_center.argtypes = [P(d), d, P(d)]
        L.orc_lens_map.argtypes = [i, P(d), P(d), P(d), P(d)]
        L.orc_lens_poly.argtypes = [i, P(d), P(d), P(d), P(d)]
        L.orc_lens_poly.restype = i
        L.orc_ea_roots.argtypes = [i, P(d), P(d), P(i)]
        L.orc_ea_roots.restype = i
        L.orc_ea_continue.argtypes = [i, P(d), P(d), i]
        L.orc_ea_continue.restype = i
        L.orc_polish.argtypes = [i, P(d), P(d), P(d), P(d)]
        L.orc_polish.restype = d
        L.orc_images.argtypes = [i, P(d), P(d), P(d), P(d), P(u32)]
        L.orc_images.restype = i
        L.orc_point_mag.argtypes = [i, P(d), P(d), P(d), P(i), P(d)]
        L.orc_point_mag.restype = d
        L.orc_brightness.argtypes = [d, d]
        L.orc_brightness.restype = d
        L.orc_edge_factor.argtypes = [d, d, d]
        L.orc_edge_factor.restype = d
        L.orc_crossing_t.argtypes = [P(d), i, d]
        L.orc_crossing_t.restype = d
        L.orc_build_sectors.argtypes = [i, P(d), P(d), d, i, P(d), P(i), P(u32)]
        L.orc_build_sectors.restype = i
        L.orc_sector_flux.argtypes = [i, P(d), P(d), P(d), d, d, d, i, i, P(d), i, P(i)]
        L.orc_retry_sectors.argtypes = [i, P(d), P(i), P(i), P(d), P(i)]
        L.orc_retry_sectors.restype = i
        L.orc_sector_flux.restype = d
        L.orc_magnification.argtypes = [i, P(d), i64, P(d), i, i, i, d, i, i, P(d), P(u32), P(d), P(u8),
                                        P(i32), P(d)]
        L.orc_magnification_given.argtypes = [i, P(d), i64, P(d), i, i, d, i, P(d), P(u8), P(i32), P(d),
                                              P(u32)]
        L.orc_jacobian_given.argtypes = [i, P(d), i64, P(d), i, i, d, i, P(d), P(u8), P(i32), P(d), P(d)]
        L.orc_magnification_frozen.argtypes = [i, P(d), P(d), i64, P(d), i, i, d, i, P(d), P(u8), P(i32), P(d)]
        L.orc_disk_mag.argtypes = [i, P(d), i64, P(d), i, i, P(d), P(i32)]
        L.orc_point_jacobian.argtypes = [i, P(d), i64, P(d), P(d), P(d), P(u32)]
        L.orc_hybrid_select.argtypes = [i, P(d), i64, P(d), i, d, d, d, P(i32), P(d)]
        L.orc_hybrid.argtypes = [i, P(d), i64, P(d), i, d, d, d, i, i, i, d, i, P(d), P(u32)]
        _lib = L
    return _lib


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Thread count of the oracle's later parallel regions."""
    lib().orc_set_num_threads(int(n))


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _dbl(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def params(s=1.0, q=1.0, u0=0.0, alpha=0.0, t0=0.0, tE=1.0, rho=1e-2, u1=0.0, q3=0.0, r3=0.0, psi=0.0):
    return np.array([s, q, u0, alpha, t0, tE, rho, u1, q3, r3, psi], dtype=np.float64)


def frame(n_lens, p):
    """Fractional masses eps[n] and complex positions a[n] of the lens (Sec. 2.1, Fig. 3)."""
    p = _dbl(p)
    eps = np.zeros(max(n_lens, 1))
    a = np.zeros(2 * max(n_lens, 1))
    lib().orc_frame(n_lens, _p(p), _p(eps), _p(a))
    return eps[:n_lens].copy(), (a[0::2] + 1j * a[1::2])[:n_lens].copy()


def _lens_arrays(eps, a):
    eps = _dbl(eps)
    a = np.asarray(a, dtype=np.complex128)
    ab = _dbl(np.stack([a.real, a.imag], axis=-1).reshape(-1)) if a.size else np.zeros(2)
    return (eps if eps.size else np.zeros(1)), ab


def source_center(p, t):
    p = _dbl(p)
    out = np.zeros(2)
    lib().orc_source_center(_p(p), float(t), _p(out))
    return complex(out[0], out[1])


def lens_map(eps, a, z):
    e, ab = _lens_arrays(eps, a)
    zz = _dbl([complex(z).real, complex(z).imag])
    out = np.zeros(2)
    lib().orc_lens_map(len(np.atleast_1d(eps)) if np.size(eps) else 0, _p(e), _p(ab), _p(zz), _p(out))
    return complex(out[0], out[1])


def lens_poly(eps, a, w):
    """Coefficients b_0..b_n (ascending powers) of eq. lens_eq_z."""
    n = int(np.size(eps))
    e, ab = _lens_arrays(eps, a)
    ww = _dbl([complex(w).real, complex(w).imag])
    out = np.zeros(2 * (n * n + 2))
    deg = lib().orc_lens_poly(n, _p(e), _p(ab), _p(ww), _p(out))
    c = out[0::2] + 1j * out[1::2]
    return c[: deg + 1]


def ea_roots(coef):
    """Ehrlich-Aberth roots of sum_j coef[j] z^j; returns (roots, converged, iterations)."""
    coef = np.asarray(coef, dtype=np.complex128)
    deg = coef.size - 1
    cb = _dbl(np.stack([coef.real, coef.imag], -1).reshape(-1))
    out = np.zeros(2 * deg)
    it = ctypes.c_int(0)
    ok = lib().orc_ea_roots(deg, _p(cb), _p(out), ctypes.byref(it))
    return out[0::2] + 1j * out[1::2], bool(ok), it.value


def ea_continue(coef, z0, cap=100):
    """Ehrlich-Aberth continued from the estimates z0 with the step test only (no
    rounding-noise stop), at most cap iterations; returns (roots, converged)."""
    coef = np.asarray(coef, dtype=np.complex128)
    deg = coef.size - 1
    cb = _dbl(np.stack([coef.real, coef.imag], -1).reshape(-1))
    z0 = np.asarray(z0, dtype=np.complex128)
    zz = _dbl(np.stack([z0.real, z0.imag], -1).reshape(-1))
    ok = lib().orc_ea_continue(deg, _p(cb), _p(zz), int(cap))
    return zz[0::2] + 1j * zz[1::2], bool(ok)


def polish(eps, a, w, z):
    """The validation's Newton polish of one candidate z; returns (z, |F|)."""
    n = int(np.size(eps))
    e, ab = _lens_arrays(eps, a)
    ww = _dbl([complex(w).real, complex(w).imag])
    zz = _dbl([complex(z).real, complex(z).imag])
    f = lib().orc_polish(n, _p(e), _p(ab), _p(ww), _p(zz))
    return complex(zz[0], zz[1]), float(f)


def images(eps, a, w):
    """Validated images of a point source at w; returns (images, status bits)."""
    n = int(np.size(eps))
    e, ab = _lens_arrays(eps, a)
    ww = _dbl([complex(w).real, complex(w).imag])
    out = np.zeros(2 * 12)
    st = ctypes.c_uint32(0)
    k = lib().orc_images(n, _p(e), _p(ab), _p(ww), _p(out), ctypes.byref(st))
    return (out[0::2] + 1j * out[1::2])[:k].copy(), st.value


def point_mag(eps, a, w):
    """eq. amp_point; returns (A, signed magnifications 1/det J per image)."""
    n = int(np.size(eps))
    e, ab = _lens_arrays(eps, a)
    ww = _dbl([complex(w).real, complex(w).imag])
    mu = np.zeros(12)
    k = ctypes.c_int(0)
    A = lib().orc_point_mag(n, _p(e), _p(ab), _p(ww), ctypes.byref(k), _p(mu))
    return A, mu[: k.value].copy()


def brightness(x, u1):
    return lib().orc_brightness(float(x), float(u1))


def edge_factor(delta, u1, delta_c=0.1):
    return lib().orc_edge_factor(float(delta), float(u1), float(delta_c))


def crossing_t(d4, cubic, rho):
    d4 = _dbl(d4)
    return lib().orc_crossing_t(_p(d4), int(cubic), float(rho))


def build_sectors(r, th, rho, cap):
    r, th = _dbl(r), _dbl(th)
    sec = np.zeros((64, 4))
    per = np.zeros(64, dtype=np.int32)
    st = ctypes.c_uint32(0)
    k = lib().orc_build_sectors(r.size, _p(r), _p(th), float(rho), int(cap), _p(sec), _p(per, ctypes.c_int),
                                ctypes.byref(st))
    return sec[:k].copy(), per[:k].astype(bool), st.value


def retry_sectors(sectors, periodic, clips):
    """O12 retry step: widen each flagged sector on its flagged sides, merge, sort."""
    sec = _dbl(sectors).reshape(-1, 4)
    per = np.ascontiguousarray(periodic, dtype=np.int32).reshape(-1)
    cl = np.ascontiguousarray(clips, dtype=np.int32).reshape(-1)
    out = np.zeros((max(sec.shape[0], 1), 4))
    operi = np.zeros(max(sec.shape[0], 1), dtype=np.int32)
    k = lib().orc_retry_sectors(sec.shape[0], _p(sec), _p(per, ctypes.c_int), _p(cl, ctypes.c_int), _p(out),
                                _p(operi, ctypes.c_int))
    return out[:k].copy(), operi[:k].astype(bool)


def sector_flux(eps, a, wc, rho, u1, nr, nth, sector, periodic=False, delta_c=0.1):
    """Un-normalised flux of one sector (App. A); returns (flux, clip bits)."""
    n = int(np.size(eps))
    e, ab = _lens_arrays(eps, a)
    wcb = _dbl([complex(wc).real, complex(wc).imag])
    s4 = _dbl(sector)
    clip = ctypes.c_int(0)
    f = lib().orc_sector_flux(n, _p(e), _p(ab), _p(wcb), float(rho), float(u1), float(delta_c), int(nr), int(nth),
                              _p(s4), int(bool(periodic)), ctypes.byref(clip))
    return f, clip.value


def magnification(n_lens, p, t, n_limb=64, n_r=64, n_theta=256, delta_c=0.1, max_retries=2, kmax=10):
    """Light curve of one event; returns dict(mag, status, sectors, periodic, nsec, a_ps)."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    mag = np.zeros(n)
    st = np.zeros(n, dtype=np.uint32)
    sec = np.zeros((n, kmax, 4))
    per = np.zeros((n, kmax), dtype=np.uint8)
    nsec = np.zeros(n, dtype=np.int32)
    aps = np.zeros(n)
    lib().orc_magnification(n_lens, _p(p), n, _p(t), n_limb, n_r, n_theta, delta_c, max_retries, kmax, _p(mag),
                            _p(st, ctypes.c_uint32), _p(sec), _p(per, ctypes.c_uint8), _p(nsec, ctypes.c_int32),
                            _p(aps))
    return dict(mag=mag, status=st, sectors=sec, periodic=per, nsec=nsec, a_ps=aps)


def magnification_given(n_lens, p, t, sectors, periodic, nsec, n_r=64, n_theta=256, delta_c=0.1):
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    sectors = _dbl(sectors)
    kmax = sectors.shape[1]
    periodic = np.ascontiguousarray(periodic, dtype=np.uint8)
    nsec = np.ascontiguousarray(nsec, dtype=np.int32)
    mag = np.zeros(n)
    st = np.zeros(n, dtype=np.uint32)
    lib().orc_magnification_given(n_lens, _p(p), n, _p(t), n_r, n_theta, delta_c, kmax, _p(sectors),
                                  _p(periodic, ctypes.c_uint8), _p(nsec, ctypes.c_int32), _p(mag),
                                  _p(st, ctypes.c_uint32))
    return mag, st


def jacobian_given(n_lens, p, t, sectors, periodic, nsec, n_r=64, n_theta=256, delta_c=0.1):
    """Magnifications and d mag / d params [n_epochs, 11] on given sectors, frozen structure."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    sectors = _dbl(sectors)
    kmax = sectors.shape[1]
    periodic = np.ascontiguousarray(periodic, dtype=np.uint8)
    nsec = np.ascontiguousarray(nsec, dtype=np.int32)
    mag = np.zeros(n)
    jac = np.zeros((n, N_PARAMS))
    lib().orc_jacobian_given(n_lens, _p(p), n, _p(t), n_r, n_theta, delta_c, kmax, _p(sectors),
                             _p(periodic, ctypes.c_uint8), _p(nsec, ctypes.c_int32), _p(mag), _p(jac))
    return mag, jac


def magnification_frozen(n_lens, p_eval, p_ref, t, sectors, periodic, nsec, n_r=64, n_theta=256, delta_c=0.1):
    """Magnification at p_eval with every decision (chi, edge branches) taken at p_ref."""
    pe, pr = _dbl(p_eval), _dbl(p_ref)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    sectors = _dbl(sectors)
    kmax = sectors.shape[1]
    periodic = np.ascontiguousarray(periodic, dtype=np.uint8)
    nsec = np.ascontiguousarray(nsec, dtype=np.int32)
    mag = np.zeros(n)
    lib().orc_magnification_frozen(n_lens, _p(pe), _p(pr), n, _p(t), n_r, n_theta, delta_c, kmax, _p(sectors),
                                   _p(periodic, ctypes.c_uint8), _p(nsec, ctypes.c_int32), _p(mag))
    return mag


def disk_mag(n_lens, p, t, n_x=32, n_phi=128):
    """Brightness-weighted mean of eq. amp_point over the source disk (no image-plane grid;
    valid where no caustic crosses the disk).  Returns (mag, count_changes) per epoch;
    count_changes > 0 marks epochs where the reference does not apply."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    mag = np.zeros(n)
    ch = np.zeros(n, dtype=np.int32)
    lib().orc_disk_mag(n_lens, _p(p), n, _p(t), n_x, n_phi, _p(mag), ch.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return mag, ch



def point_jacobian(n_lens, p, t):
    """Point-source magnification of each epoch's source centre and dA/dparams [E, 11],
    through the root derivative dz*/db of Sec. 3.5; returns (a_ps, jac, status)."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    a = np.zeros(n)
    jac = np.zeros((n, N_PARAMS))
    st = np.zeros(n, dtype=np.uint32)
    lib().orc_point_jacobian(n_lens, _p(p), n, _p(t), _p(a), _p(jac), _p(st, ctypes.c_uint32))
    return a, jac, st


def hybrid_select(n_lens, p, t, n_check=16, guard=2.0, tol=1e-4, vary_max=0.1):
    """Epochs that need the finite-source computation (Sec. 3.4, item iii; selection rule
    O15); returns (extended bool [E], a_ps [E])."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    ext = np.zeros(n, dtype=np.int32)
    a = np.zeros(n)
    lib().orc_hybrid_select(n_lens, _p(p), n, _p(t), int(n_check), float(guard), float(tol), float(vary_max),
                            _p(ext, ctypes.c_int32), _p(a))
    return ext.astype(bool), a


def hybrid(n_lens, p, t, n_check=16, guard=2.0, tol=1e-4, vary_max=0.1, n_limb=64, n_r=64, n_theta=256,
           delta_c=0.1, max_retries=2):
    """Hybrid light curve: the full method on the selected epochs, A_ps elsewhere (status
    ST_POINT); returns (mag, status)."""
    p = _dbl(p)
    t = _dbl(np.atleast_1d(t))
    n = t.size
    mag = np.zeros(n)
    st = np.zeros(n, dtype=np.uint32)
    lib().orc_hybrid(n_lens, _p(p), n, _p(t), int(n_check), float(guard), float(tol), float(vary_max), n_limb, n_r,
                     n_theta, delta_c, max_retries, _p(mag), _p(st, ctypes.c_uint32))
    return mag, st
