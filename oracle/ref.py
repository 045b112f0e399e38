"""ctypes binding of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the CPU-baseline leg of the benchmark import
this module.  It loads oracle/libtwk_ref.so (built by oracle/build.py) and
exposes numpy-friendly wrappers.  Nothing here touches the GPU library.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtwk_ref.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)

FLAG_POINT = 1 << 0
FLAG_CAP = 1 << 1
FLAG_ANOMALY = 1 << 2
FLAG_SLOPE = 1 << 3
FLAG_NONFINITE = 1 << 4
FLAG_NEARDEGEN = 1 << 5


class Cfg(C.Structure):
    _fields_ = [("tol", C.c_double), ("n0", C.c_int32), ("nnew", C.c_int32),
                ("cap", C.c_int32), ("grow", C.c_int32), ("slope", C.c_int32),
                ("kgap", C.c_double), ("cross_flip", C.c_int32),
                ("cross_tol", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.twk_ref_coeffs.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
        L.twk_ref_coeffs_conventional.argtypes = L.twk_ref_coeffs.argtypes
        L.twk_ref_roots.argtypes = [_dp, _dp]
        L.twk_ref_images.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                     _dp, _dp, _dp, _ip, _up]
        L.twk_ref_point_mag.argtypes = [C.c_double, C.c_double, C.c_int64, _dp, _dp,
                                        _dp, _ip, _up]
        L.twk_ref_limb_derivs.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_double, _dp, _dp, _dp, _ip]
        L.twk_ref_cfg_default.argtypes = [C.POINTER(Cfg), C.c_double]
        L.twk_ref_cfg_default.restype = None
        L.twk_ref_finite_mag.argtypes = [C.c_double, C.c_double, C.c_int64, _dp, _dp,
                                         C.c_double, C.c_double, C.POINTER(Cfg),
                                         _dp, _dp, _ip, _up]
        L.twk_ref_finite_trace.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.POINTER(Cfg), _dp, _dp, _ip, _up,
                                           _dp, C.c_int32]
        L.twk_ref_trajectory.argtypes = [C.c_double, C.c_double, C.c_int64, _dp, _dp, _dp]
        L.twk_ref_cross_piece.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int32,
                                          C.c_double, C.c_int32, _dp, _dp, _dp]
        L.twk_ref_ld_combine.argtypes = [C.c_double, C.c_int32, _dp, _dp]
        L.twk_ref_ps_adequate.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_double, _ip, _dp]
        L.twk_ref_features.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.POINTER(C.c_float), _dp, _ip]
        for name in ("twk_ref_coeffs", "twk_ref_coeffs_conventional", "twk_ref_roots",
                     "twk_ref_images", "twk_ref_point_mag", "twk_ref_limb_derivs",
                     "twk_ref_finite_mag", "twk_ref_finite_trace", "twk_ref_trajectory",
                     "twk_ref_ld_combine", "twk_ref_ps_adequate", "twk_ref_features",
                     "twk_ref_cross_piece"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _check(rc):
    if rc < 0:
        raise RuntimeError(f"oracle call failed with status {rc}")
    return rc


def coeffs(s, q, zeta, conventional=False):
    out = np.zeros(12)
    f = lib().twk_ref_coeffs_conventional if conventional else lib().twk_ref_coeffs
    _check(f(s, q, float(np.real(zeta)), float(np.imag(zeta)), _d(out)))
    return out[0::2] + 1j * out[1::2]


def roots(c):
    c = np.asarray(c, dtype=np.complex128)
    c12 = np.empty(12)
    c12[0::2] = c.real
    c12[1::2] = c.imag
    out = np.zeros(10)
    it = _check(lib().twk_ref_roots(_d(c12), _d(out)))
    return out[0::2] + 1j * out[1::2], it


def images(s, q, zeta):
    img = np.zeros(10)
    res = np.zeros(10)
    jac = np.zeros(5)
    n = C.c_int32()
    fl = C.c_uint32()
    _check(lib().twk_ref_images(s, q, float(np.real(zeta)), float(np.imag(zeta)), _d(img),
                                _d(res), _d(jac), C.byref(n), C.byref(fl)))
    return dict(z=img[0::2] + 1j * img[1::2], R=res[0::2] + 1j * res[1::2], J=jac,
                n=n.value, flags=fl.value)


def point_mag(s, q, zx, zy):
    zx = np.ascontiguousarray(zx, dtype=np.float64)
    zy = np.ascontiguousarray(zy, dtype=np.float64)
    n = zx.size
    mag = np.zeros(n)
    nimg = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint32)
    _check(lib().twk_ref_point_mag(s, q, n, _d(zx), _d(zy), _d(mag),
                                   nimg.ctypes.data_as(_ip), fl.ctypes.data_as(_up)))
    return mag, nimg, fl


def limb_derivs(s, q, zc, rho, theta):
    img = np.zeros(10)
    dz = np.zeros(10)
    w = np.zeros(5)
    n = C.c_int32()
    _check(lib().twk_ref_limb_derivs(s, q, float(np.real(zc)), float(np.imag(zc)), rho, theta,
                                     _d(img), _d(dz), _d(w), C.byref(n)))
    return img[0::2] + 1j * img[1::2], dz[0::2] + 1j * dz[1::2], w, n.value


def cfg(tol, **kw):
    c = Cfg()
    lib().twk_ref_cfg_default(C.byref(c), tol)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


# The tight configuration: a much tighter tolerance than the GPU's 1e-4
# gate, more initial samples, geometric growth of the sample count and a
# large cap, so that the oracle's own error is negligible against the gate.
TIGHT_TOL = 1e-6


def tight_cfg():
    return cfg(TIGHT_TOL, n0=256, nnew=64, cap=1 << 17, grow=4)


def finite_mag(s, q, zx, zy, rho, tol, config=None):
    zx = np.ascontiguousarray(np.atleast_1d(zx), dtype=np.float64)
    zy = np.ascontiguousarray(np.atleast_1d(zy), dtype=np.float64)
    n = zx.size
    mag = np.zeros(n)
    err = np.zeros(n)
    ns = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint32)
    cp = C.byref(config) if config is not None else None
    _check(lib().twk_ref_finite_mag(s, q, n, _d(zx), _d(zy), rho, tol, cp, _d(mag), _d(err),
                                    ns.ctypes.data_as(_ip), fl.ctypes.data_as(_up)))
    return mag, err, ns, fl


def finite_trace(s, q, zeta, rho, config, max_out=1 << 17):
    th = np.zeros(max_out)
    mag = C.c_double()
    err = C.c_double()
    ns = C.c_int32()
    fl = C.c_uint32()
    _check(lib().twk_ref_finite_trace(s, q, float(np.real(zeta)), float(np.imag(zeta)), rho,
                                      C.byref(config), C.byref(mag), C.byref(err), C.byref(ns),
                                      C.byref(fl), _d(th), max_out))
    return mag.value, err.value, ns.value, fl.value, th[:min(ns.value, max_out)]


def cross_piece(zp, zm, dp, dm, wp, wm, kind, dth, flip=0):
    """Chord + cross-caustic correction and errors of an interval in which a
    pair is created (kind > 0) or destroyed (kind < 0): (dA, E, E2)."""
    def c2(z):
        return np.array([np.real(z), np.imag(z)], dtype=np.float64)
    a, b, cp, cm = c2(zp), c2(zm), c2(dp), c2(dm)
    dA, E, E2 = C.c_double(), C.c_double(), C.c_double()
    _check(lib().twk_ref_cross_piece(_d(a), _d(b), _d(cp), _d(cm), wp, wm, kind, dth, flip,
                                     C.byref(dA), C.byref(E), C.byref(E2)))
    return dA.value, E.value, E2.value


def trajectory(u0, alpha, tau):
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    zx = np.zeros_like(tau)
    zy = np.zeros_like(tau)
    _check(lib().twk_ref_trajectory(u0, alpha, tau.size, _d(tau), _d(zx), _d(zy)))
    return zx, zy


def ld_combine(gamma, mu_k):
    mu_k = np.ascontiguousarray(mu_k, dtype=np.float64)
    out = C.c_double()
    _check(lib().twk_ref_ld_combine(gamma, mu_k.size, _d(mu_k), C.byref(out)))
    return out.value


def ps_adequate(s, q, zeta, rho, tol):
    ok = C.c_int32()
    mu = C.c_double()
    _check(lib().twk_ref_ps_adequate(s, q, float(np.real(zeta)), float(np.imag(zeta)), rho, tol,
                                     C.byref(ok), C.byref(mu)))
    return bool(ok.value), mu.value


def features(s, q, zeta, rho, tol):
    """The eight float32 features of one epoch, mu_ps and the adequacy flag."""
    f = np.zeros(8, dtype=np.float32)
    ok = C.c_int32()
    mu = C.c_double()
    _check(lib().twk_ref_features(s, q, float(np.real(zeta)), float(np.imag(zeta)), rho, tol,
                                  f.ctypes.data_as(C.POINTER(C.c_float)), C.byref(mu),
                                  C.byref(ok)))
    return f, mu.value, bool(ok.value)
