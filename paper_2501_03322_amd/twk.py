"""ctypes binding of libtwk.so (C ABI in include/twk.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Torch tensors supply device memory and the stream.
The binding refuses to run when the library is missing: there is no CPU
fallback.
"""
import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# TWK_LIB may name another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("TWK_LIB") or os.path.join(HERE, "libtwk.so")

OK, EINVAL, EDEVICE, ENOMEM, ENOMLP = 0, -1, -2, -3, -4
MODE_FP64 = 0
MODE_MIXED = 1 << 0
MODE_MLP = 1 << 2
MODE_ALL_FS = 1 << 3
MODE_ROUNDS = 1 << 4
MODE_CONVENTIONAL = 1 << 5
COEF_REFINED, COEF_CONVENTIONAL = 0, 1

FLAG_POINT = 1 << 0
FLAG_CAP = 1 << 1
FLAG_ANOMALY = 1 << 2
FLAG_SLOPE = 1 << 3
FLAG_NONFINITE = 1 << 4
FLAG_NEARDEGEN = 1 << 5

EXPORTS = ("twk_create", "twk_destroy", "twk_sync", "twk_last_hip_error", "twk_strerror",
           "twk_point_mag", "twk_coefficients", "twk_finite_mag", "twk_finite_mag_each", "twk_finite_mag_noalloc",
           "twk_lightcurves",
           "twk_last_stats",
           "twk_enable_timing", "twk_kernel_times", "twk_mag_map", "twk_features",
           "twk_mlp_set", "twk_mlp_get", "twk_mlp_save", "twk_mlp_load", "twk_mlp_infer",
           "twk_mlp_grad", "twk_mlp_train", "twk_get_tuning", "twk_set_tuning", "twk_autotune")

MLP_NPARAM = 34450
MLP_GRAD_MAX_ROWS = 65536


class TrainCfg(C.Structure):
    """twk_train_cfg."""
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("lr_end", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("huber_delta", C.c_float), ("init", C.c_int32),
                ("seed", C.c_uint64)]



class Tuning(C.Structure):
    """twk_tuning."""
    _fields_ = [("waves_per_cu", C.c_int32), ("lds_cap", C.c_int32), ("budget_shift", C.c_float),
                ("graphs", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = C.c_void_p


class TwkError(RuntimeError):
    def __init__(self, status, what, hip=0):
        self.status = status
        super().__init__(f"{what} failed: {status} ({strerror(status)}), hip error {hip}")


def load():
    """Load libtwk.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2501_03322_amd/build.py "
                          "(there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    L.twk_create.argtypes = [C.POINTER(_vp), C.c_int, _vp]
    L.twk_destroy.argtypes = [_vp]
    L.twk_sync.argtypes = [_vp]
    L.twk_last_hip_error.argtypes = [_vp]
    L.twk_strerror.argtypes = [C.c_int]
    L.twk_strerror.restype = C.c_char_p
    L.twk_point_mag.argtypes = [_vp, C.c_double, C.c_double, C.c_int64, _vp, _vp, _vp, _vp, _vp]
    L.twk_coefficients.argtypes = [_vp, C.c_double, C.c_double, C.c_int64, _vp, _vp, C.c_int32, _vp]
    L.twk_finite_mag.argtypes = [_vp, C.c_double, C.c_double, C.c_int64, _vp, _vp, C.c_double,
                                 C.c_double, C.c_uint32, _vp, _vp, _vp, _vp]
    L.twk_finite_mag_noalloc.argtypes = L.twk_finite_mag.argtypes
    L.twk_finite_mag_each.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_double,
                                      C.c_uint32, _vp, _vp, _vp, _vp]
    L.twk_lightcurves.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int64, _vp,
                                  C.c_int32, C.c_double, C.c_uint32, _vp, _vp, _vp, _vp]
    L.twk_mag_map.argtypes = [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_uint32,
                              _vp, _vp, _vp, _vp]
    L.twk_last_stats.argtypes = [_vp, C.POINTER(C.c_int64)]
    L.twk_enable_timing.argtypes = [_vp, C.c_int]
    L.twk_kernel_times.argtypes = [_vp, C.POINTER(C.c_double)]
    L.twk_features.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_int64, _vp,
                               C.c_double, _vp, _vp, _vp]
    L.twk_mlp_set.argtypes = [_vp, C.POINTER(C.c_float), C.c_int64]
    L.twk_mlp_get.argtypes = [_vp, C.POINTER(C.c_float), C.c_int64]
    L.twk_mlp_save.argtypes = [_vp, C.c_char_p]
    L.twk_mlp_load.argtypes = [_vp, C.c_char_p]
    L.twk_mlp_infer.argtypes = [_vp, C.c_int64, _vp, _vp]
    L.twk_mlp_grad.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.c_float, _vp,
                               C.POINTER(C.c_double)]
    L.twk_mlp_train.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.POINTER(TrainCfg),
                                C.POINTER(C.c_float)]
    L.twk_get_tuning.argtypes = [_vp, C.POINTER(Tuning)]
    L.twk_set_tuning.argtypes = [_vp, C.POINTER(Tuning)]
    L.twk_autotune.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int64, _vp,
                               C.c_int32, C.c_double, C.c_uint32, C.c_int32, C.POINTER(Tuning)]
    for f in EXPORTS:
        if f != "twk_strerror":
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


def strerror(status):
    return load().twk_strerror(status).decode()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("arrays must be device tensors")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous")
    return t.data_ptr()


def _dev(x, device, dtype=torch.float64):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(x, dtype=dtype, device=device).contiguous()


class Context:
    """A library context bound to one device and one stream."""

    def __init__(self, device=0, stream=None):
        self.lib = load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _vp()
        rc = self.lib.twk_create(C.byref(h), device, _vp(stream.cuda_stream))
        if rc:
            raise TwkError(rc, "twk_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.twk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise TwkError(rc, what, self.lib.twk_last_hip_error(self.h))

    def sync(self):
        self._check(self.lib.twk_sync(self.h), "twk_sync")

    def stats(self):
        out = (C.c_int64 * 8)()
        self._check(self.lib.twk_last_stats(self.h, out), "twk_last_stats")
        return dict(fs_tasks=out[0], spilled=out[1], samples=out[2], waves=out[3],
                    sweeps32=out[4], sweeps64=out[5], intervals=out[6], launches=out[7])

    def enable_timing(self, on=True):
        self._check(self.lib.twk_enable_timing(self.h, 1 if on else 0), "twk_enable_timing")

    def kernel_times(self):
        out = (C.c_double * 5)()
        self._check(self.lib.twk_kernel_times(self.h, out), "twk_kernel_times")
        return dict(ps_ms=out[0], mlp_ms=out[1], fs_ms=out[2], rest_ms=out[3], total_ms=out[4])

    def point_mag(self, s, q, zx, zy):
        zx = _dev(zx, self.device)
        zy = _dev(zy, self.device)
        n = zx.numel()
        mag = torch.empty(n, dtype=torch.float64, device=self.device)
        nimg = torch.empty(n, dtype=torch.int32, device=self.device)
        fl = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(self.lib.twk_point_mag(self.h, s, q, n, _ptr(zx), _ptr(zy), _ptr(mag),
                                           _ptr(nimg), _ptr(fl)), "twk_point_mag")
        return mag, nimg, fl

    def coefficients(self, s, q, zx, zy, form=COEF_REFINED):
        """Quintic coefficients c0..c5 of each source position ([n, 6] complex
        tensor on the device), refined or conventional form."""
        zx = _dev(zx, self.device)
        zy = _dev(zy, self.device)
        n = zx.numel()
        out = torch.empty((n, 12), dtype=torch.float64, device=self.device)
        self._check(self.lib.twk_coefficients(self.h, s, q, n, _ptr(zx), _ptr(zy), form, _ptr(out)),
                    "twk_coefficients")
        return torch.view_as_complex(out.view(n, 6, 2))

    def finite_mag(self, s, q, zx, zy, rho, tol, mode=MODE_FP64, out=None):
        zx = _dev(zx, self.device)
        zy = _dev(zy, self.device)
        n = zx.numel()
        if out is None:
            out = self.alloc_out(n)
        mag, err, ns, fl = out
        self._check(self.lib.twk_finite_mag(self.h, s, q, n, _ptr(zx), _ptr(zy), rho, tol, mode,
                                            _ptr(mag), _ptr(err), _ptr(ns), _ptr(fl)),
                    "twk_finite_mag")
        return out

    def finite_mag_noalloc(self, s, q, zx, zy, rho, tol, mode=MODE_FP64, out=None):
        """twk_finite_mag without any allocation by the library (its scratch
        is a fixed device array): at most 65536 sources per call."""
        zx = _dev(zx, self.device)
        zy = _dev(zy, self.device)
        n = zx.numel()
        if out is None:
            out = self.alloc_out(n)
        mag, err, ns, fl = out
        self._check(self.lib.twk_finite_mag_noalloc(self.h, s, q, n, _ptr(zx), _ptr(zy), rho, tol,
                                                    mode, _ptr(mag), _ptr(err), _ptr(ns), _ptr(fl)),
                    "twk_finite_mag_noalloc")
        return out

    def finite_mag_each(self, s, q, zx, zy, rho, tol, mode=MODE_FP64, out=None):
        """Per-element lens and source: s, q, zx, zy, rho of equal length."""
        s, q, zx, zy, rho = (_dev(a, self.device) for a in (s, q, zx, zy, rho))
        n = zx.numel()
        if not all(a.numel() == n for a in (s, q, zy, rho)):
            raise ValueError("s, q, zx, zy and rho must have the same length")
        if out is None:
            out = self.alloc_out(n)
        mag, err, ns, fl = out
        self._check(self.lib.twk_finite_mag_each(self.h, n, _ptr(s), _ptr(q), _ptr(zx), _ptr(zy),
                                                 _ptr(rho), tol, mode, _ptr(mag), _ptr(err),
                                                 _ptr(ns), _ptr(fl)),
                    "twk_finite_mag_each")
        return out

    def alloc_out(self, n):
        return (torch.empty(n, dtype=torch.float64, device=self.device),
                torch.empty(n, dtype=torch.float64, device=self.device),
                torch.empty(n, dtype=torch.int32, device=self.device),
                torch.empty(n, dtype=torch.int32, device=self.device))

    def lightcurves(self, s, q, u0, alpha, rho, tau, tol, mode=MODE_FP64, gamma=None,
                    n_annuli=1, out=None):
        s, q, u0, alpha, rho = (_dev(a, self.device) for a in (s, q, u0, alpha, rho))
        tau = _dev(tau, self.device)
        g = None if gamma is None else _dev(gamma, self.device)
        nsets, nep = s.numel(), tau.numel()
        if out is None:
            out = self.alloc_out(nsets * nep)
        mag, err, ns, fl = out
        self._check(self.lib.twk_lightcurves(self.h, nsets, _ptr(s), _ptr(q), _ptr(u0), _ptr(alpha),
                                             _ptr(rho), _ptr(g), nep, _ptr(tau), n_annuli, tol, mode,
                                             _ptr(mag), _ptr(err), _ptr(ns), _ptr(fl)),
                    "twk_lightcurves")
        return out

    def mag_map(self, s, q, rho, centre, width, height, nx, ny, tol, mode=MODE_FP64, out=None):
        if out is None:
            out = self.alloc_out(nx * ny)
        mag, err, ns, fl = out
        self._check(self.lib.twk_mag_map(self.h, s, q, rho, centre[0], centre[1], width, height, nx,
                                         ny, tol, mode, _ptr(mag), _ptr(err), _ptr(ns), _ptr(fl)),
                    "twk_mag_map")
        return out

    # ------------------------------------------------------------ learned part
    def features(self, s, q, u0, alpha, rho, tau, tol):
        """Per-epoch features [nsets*nepochs, 8] (float32), mu_ps, adequacy."""
        s, q, u0, alpha, rho = (_dev(a, self.device) for a in (s, q, u0, alpha, rho))
        tau = _dev(tau, self.device)
        n = s.numel() * tau.numel()
        feat = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        mu = torch.empty(n, dtype=torch.float64, device=self.device)
        ok = torch.empty(n, dtype=torch.int32, device=self.device)
        self._check(self.lib.twk_features(self.h, s.numel(), _ptr(s), _ptr(q), _ptr(u0),
                                          _ptr(alpha), _ptr(rho), tau.numel(), _ptr(tau), tol,
                                          _ptr(feat), _ptr(mu), _ptr(ok)), "twk_features")
        return feat, mu, ok

    def mlp_set(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.twk_mlp_set(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size),
                    "twk_mlp_set")

    def mlp_get(self):
        import numpy as np
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(self.lib.twk_mlp_get(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size),
                    "twk_mlp_get")
        return p

    def mlp_save(self, path):
        self._check(self.lib.twk_mlp_save(self.h, os.fsencode(path)), "twk_mlp_save")

    def mlp_load(self, path):
        self._check(self.lib.twk_mlp_load(self.h, os.fsencode(path)), "twk_mlp_load")

    def mlp_infer(self, feat, out=None):
        feat = _dev(feat, self.device, torch.float32)
        n = feat.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        self._check(self.lib.twk_mlp_infer(self.h, n, _ptr(feat), _ptr(out)), "twk_mlp_infer")
        return out

    def mlp_grad(self, feat, y_budget, y_fs, huber_delta=1.0):
        feat = _dev(feat, self.device, torch.float32)
        yb = _dev(y_budget, self.device, torch.float32)
        yf = _dev(y_fs, self.device, torch.float32)
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=self.device)
        loss = C.c_double()
        self._check(self.lib.twk_mlp_grad(self.h, feat.shape[0], _ptr(feat), _ptr(yb), _ptr(yf),
                                          huber_delta, _ptr(g), C.byref(loss)), "twk_mlp_grad")
        return loss.value, g

    def mlp_train(self, feat, y_budget, y_fs, epochs=8, batch=4096, lr=2e-3, lr_end=1e-4,
                  huber_delta=1.0, init=True, seed=1):
        import numpy as np
        feat = _dev(feat, self.device, torch.float32)
        yb = _dev(y_budget, self.device, torch.float32)
        yf = _dev(y_fs, self.device, torch.float32)
        cfg = TrainCfg(epochs=epochs, batch=batch, lr=lr, lr_end=lr_end, beta1=0.9, beta2=0.999,
                       eps=1e-8, huber_delta=huber_delta, init=1 if init else 0, seed=seed)
        hist = np.zeros(epochs, dtype=np.float32)
        self._check(self.lib.twk_mlp_train(self.h, feat.shape[0], _ptr(feat), _ptr(yb), _ptr(yf),
                                           C.byref(cfg), hist.ctypes.data_as(C.POINTER(C.c_float))),
                    "twk_mlp_train")
        return hist

    # ------------------------------------------------------------ tuning
    def get_tuning(self):
        t = Tuning()
        self._check(self.lib.twk_get_tuning(self.h, C.byref(t)), "twk_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, v)
        self._check(self.lib.twk_set_tuning(self.h, C.byref(t)), "twk_set_tuning")
        return t

    def autotune(self, s, q, u0, alpha, rho, tau, tol, mode=MODE_FP64, gamma=None, n_annuli=1,
                 trials=2):
        s, q, u0, alpha, rho = (_dev(a, self.device) for a in (s, q, u0, alpha, rho))
        tau = _dev(tau, self.device)
        g = None if gamma is None else _dev(gamma, self.device)
        best = Tuning()
        self._check(self.lib.twk_autotune(self.h, s.numel(), _ptr(s), _ptr(q), _ptr(u0), _ptr(alpha),
                                          _ptr(rho), _ptr(g), tau.numel(), _ptr(tau), n_annuli, tol,
                                          mode, trials, C.byref(best)), "twk_autotune")
        return best
