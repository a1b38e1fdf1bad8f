"""Python binding of libsaltbf (the C ABI in include/saltbf.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch provides device memory (tensor data
pointers) and streams (the current stream is passed to every call).  If the
library is not built, every entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsaltbf.so")

SB_OK, SB_PENDING, SB_CANCELLED, SB_FIT_DIVERGED = 0, 1, 2, 3
SB_ERR_ARG, SB_ERR_RANGE, SB_ERR_DEVICE, SB_ERR_NOMEM = -1, -2, -3, -4
SB_ERR_BUDGET, SB_ERR_STATE, SB_ERR_NOTFOUND = -5, -6, -7
SB_OBS_BROADCAST, SB_OUT_CHI2, SB_PERSISTENT = 1, 2, 4
SB_QUAD_TRAPEZOID, SB_QUAD_MIDPOINT = 0, 1
SB_FREE_T0, SB_FREE_X0, SB_FREE_X1, SB_FREE_C, SB_FREE_ALL = 1, 2, 4, 8, 15
SB_SOLVER_LM, SB_SOLVER_LBFGSB = 0, 1
SB_MAGSYS_AB = 0
SB_PRIOR_FIXED, SB_PRIOR_UNIFORM, SB_PRIOR_LOG_UNIFORM = 0, 1, 2
SB_MAX_BANDS, SB_MAX_BAND_POINTS, SB_N_PARAMS = 64, 2048, 5
SB_FIT_NOALLOC_MAX = 8192
SB_PROBE_FMA_F32, SB_PROBE_LDS_READ, SB_PROBE_COPY = 0, 1, 2
PROBE_THREADS = 256

EXPORTED = (
    "sb_config_default", "sb_create", "sb_destroy", "sb_add_band", "sb_band_grid", "sb_bandflux",
    "sb_bandflux_vjp", "sb_device_check", "sb_fit_submit", "sb_fit_poll", "sb_fit_wait", "sb_fit_cancel",
    "sb_stats", "sb_status_string", "sb_last_error", "sb_fit_batch", "sb_fit_batch_noalloc",
    "sb_read_band_file", "sb_add_band_file", "sb_band_zeropoint", "sb_band_zeropoint_ab",
    "sb_nested_sampling", "sb_philox4x64_10", "sb_peak_probe",
)

_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_phase", ctypes.c_int32), ("n_wave", ctypes.c_int32),
                ("phase0", ctypes.c_double), ("dphase", ctypes.c_double),
                ("wave0", ctypes.c_double), ("dwave", ctypes.c_double),
                ("m0", ctypes.c_void_p), ("m1", ctypes.c_void_p),
                ("cl_degree", ctypes.c_int32), ("cl_coef", ctypes.c_void_p),
                ("cl_wave_b", ctypes.c_double), ("cl_wave_v", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("max_spacing", ctypes.c_double), ("max_obs_per_fit", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("iters_per_tick", ctypes.c_int32), ("fit_iters", ctypes.c_int32),
                ("lm_lambda0", ctypes.c_double), ("quad_rule", ctypes.c_int32),
                ("lds_limit_bytes", ctypes.c_int64), ("solver", ctypes.c_int32), ("lbfgs_m", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_sn", ctypes.c_int32), ("n_obs", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("z", ctypes.c_void_p), ("t0", ctypes.c_void_p), ("x0", ctypes.c_void_p),
                ("x1", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("band", ctypes.c_void_p), ("sn_offsets", ctypes.c_void_p),
                ("data", ctypes.c_void_p), ("inv_sigma2", ctypes.c_void_p)]


class FitRequest(ctypes.Structure):
    _fields_ = [("n_obs", ctypes.c_int32), ("t", ctypes.c_void_p), ("band", ctypes.c_void_p),
                ("data", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("z", ctypes.c_float), ("t0", ctypes.c_float), ("x0", ctypes.c_float),
                ("x1", ctypes.c_float), ("c", ctypes.c_float), ("free_mask", ctypes.c_uint32),
                ("has_bounds", ctypes.c_int32), ("lower", ctypes.c_float * 4), ("upper", ctypes.c_float * 4)]


class FitResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("z", ctypes.c_float), ("t0", ctypes.c_float),
                ("x0", ctypes.c_float), ("x1", ctypes.c_float), ("c", ctypes.c_float),
                ("chi2", ctypes.c_float), ("iters", ctypes.c_int32), ("n_accept", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FitBatchDesc(ctypes.Structure):
    _fields_ = [("n_fit", ctypes.c_int32), ("n_obs", ctypes.c_int32),
                ("z", ctypes.c_void_p), ("t0", ctypes.c_void_p), ("x0", ctypes.c_void_p),
                ("x1", ctypes.c_void_p), ("c", ctypes.c_void_p), ("free_mask", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("band", ctypes.c_void_p), ("fit_offsets", ctypes.c_void_p),
                ("data", ctypes.c_void_p), ("inv_sigma2", ctypes.c_void_p),
                ("lower", ctypes.c_void_p), ("upper", ctypes.c_void_p)]


class FitOut(ctypes.Structure):
    """sb_fit_out: one batch fit's result (8 x 4 bytes; a device array of these is a float32/int32 view)."""
    _fields_ = [("t0", ctypes.c_float), ("x0", ctypes.c_float), ("x1", ctypes.c_float), ("c", ctypes.c_float),
                ("chi2", ctypes.c_float), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("n_accept", ctypes.c_int32)]


FIT_OUT_WORDS = 8


class Prior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class NsConfig(ctypes.Structure):
    _fields_ = [("prior", Prior * 5), ("n_live", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("max_iter", ctypes.c_int64), ("max_evals", ctypes.c_int64), ("dlogz", ctypes.c_double),
                ("enlarge", ctypes.c_double), ("seed", ctypes.c_uint64), ("log_norm", ctypes.c_double)]


class NsSummary(ctypes.Structure):
    _fields_ = [("logz", ctypes.c_double), ("logz_err", ctypes.c_double), ("information", ctypes.c_double),
                ("n_iter", ctypes.c_int64), ("n_eval", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("stopped_on_evals", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("rejected", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("queue_depth", ctypes.c_int32), ("active_slots", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("busy_seconds", ctypes.c_double), ("slot_ticks", ctypes.c_int64),
                ("latency_hist", ctypes.c_int64 * 24)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["latency_hist"] = list(self.latency_hist)
        return d


class SaltBFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None


def lib():
    """The loaded libsaltbf.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime under the same soname as the system one; importing
        # torch first makes the library bind to that runtime, so the process holds only one.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, st = ctypes.c_void_p, ctypes.c_int32
        L.sb_config_default.argtypes = [ctypes.POINTER(Config)]
        L.sb_config_default.restype = None
        L.sb_create.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(Config), ctypes.c_int, ctypes.POINTER(vp)]
        L.sb_create.restype = st
        L.sb_destroy.argtypes = [vp]
        L.sb_destroy.restype = st
        L.sb_add_band.argtypes = [vp, _f64p, _f64p, ctypes.c_int32, _i32p]
        L.sb_add_band.restype = st
        L.sb_band_grid.argtypes = [_f64p, _f64p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                   _f32p, _f32p, _i32p]
        L.sb_band_grid.restype = st
        L.sb_bandflux.argtypes = [vp, ctypes.POINTER(Batch), vp, vp]
        L.sb_bandflux.restype = st
        L.sb_bandflux_vjp.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, vp, vp, vp, vp]
        L.sb_bandflux_vjp.restype = st
        L.sb_device_check.argtypes = [vp, vp]
        L.sb_device_check.restype = st
        L.sb_fit_submit.argtypes = [vp, ctypes.POINTER(FitRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.sb_fit_submit.restype = st
        L.sb_fit_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(FitResult)]
        L.sb_fit_poll.restype = st
        L.sb_fit_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(FitResult)]
        L.sb_fit_wait.restype = st
        L.sb_fit_cancel.argtypes = [vp, ctypes.c_uint64]
        L.sb_fit_cancel.restype = st
        L.sb_fit_batch.argtypes = [vp, ctypes.POINTER(FitBatchDesc), vp, vp]
        L.sb_fit_batch.restype = st
        L.sb_fit_batch_noalloc.argtypes = [vp, ctypes.POINTER(FitBatchDesc), vp, vp]
        L.sb_fit_batch_noalloc.restype = st
        L.sb_read_band_file.argtypes = [ctypes.c_char_p, _f64p, _f64p, ctypes.c_int32, _i32p]
        L.sb_read_band_file.restype = st
        L.sb_add_band_file.argtypes = [vp, ctypes.c_char_p, _i32p]
        L.sb_add_band_file.restype = st
        L.sb_band_zeropoint.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _f64p]
        L.sb_band_zeropoint.restype = st
        L.sb_band_zeropoint_ab.argtypes = [_f64p, _f64p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _f64p]
        L.sb_band_zeropoint_ab.restype = st
        L.sb_nested_sampling.argtypes = [vp, ctypes.POINTER(NsConfig), ctypes.c_int32, vp, vp, vp, vp, _f64p, _f64p,
                                         _f64p, ctypes.POINTER(ctypes.c_int64), _f64p, _f64p, _f64p,
                                         ctypes.POINTER(NsSummary), vp]
        L.sb_nested_sampling.restype = st
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.sb_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.sb_philox4x64_10.restype = None
        L.sb_peak_probe.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, vp, vp, _f64p, vp]
        L.sb_peak_probe.restype = st
        L.sb_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.sb_stats.restype = st
        L.sb_status_string.argtypes = [st]
        L.sb_status_string.restype = ctypes.c_char_p
        L.sb_last_error.argtypes = []
        L.sb_last_error.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def _check(status, what):
    if status < 0:
        L = lib()
        raise SaltBFError(status, f"{what}: {L.sb_status_string(status).decode()}: {L.sb_last_error().decode()}")
    return status


def default_config(**over) -> Config:
    cfg = Config()
    lib().sb_config_default(ctypes.byref(cfg))
    for k, v in over.items():
        setattr(cfg, k, v)
    return cfg


def band_grid(wave, trans, max_spacing=5.0, rule=0):
    """Host-only quadrature grid of a band as the library builds it: (lam_k, W_k) float32.
    rule: SB_QUAD_TRAPEZOID (0) or SB_QUAD_MIDPOINT (1)."""
    w = np.ascontiguousarray(wave, np.float64)
    t = np.ascontiguousarray(trans, np.float64)
    lam = np.zeros(SB_MAX_BAND_POINTS, np.float32)
    W = np.zeros(SB_MAX_BAND_POINTS, np.float32)
    n = ctypes.c_int32(0)
    _check(lib().sb_band_grid(w.ctypes.data_as(_f64p), t.ctypes.data_as(_f64p), len(w), float(max_spacing),
                              int(rule), SB_MAX_BAND_POINTS, lam.ctypes.data_as(_f32p), W.ctypes.data_as(_f32p),
                              ctypes.byref(n)), "sb_band_grid")
    return lam[: n.value].copy(), W[: n.value].copy()


def read_band_file(path):
    """Rows (wave, trans) of a two-column bandpass text file, as the library reads it (host only)."""
    p = os.fsencode(path)
    n = ctypes.c_int32(0)
    st = lib().sb_read_band_file(p, None, None, 0, ctypes.byref(n))
    if st < 0 and n.value == 0:
        _check(st, "sb_read_band_file")
    w = np.zeros(max(1, n.value))
    t = np.zeros(max(1, n.value))
    _check(lib().sb_read_band_file(p, w.ctypes.data_as(_f64p), t.ctypes.data_as(_f64p), n.value, ctypes.byref(n)),
           "sb_read_band_file")
    return w[: n.value].copy(), t[: n.value].copy()


def band_zeropoint_ab(wave, trans, max_spacing=5.0, rule=0):
    """AB zero-point flux of band samples with the library's quadrature (host only)."""
    w = np.ascontiguousarray(wave, np.float64)
    t = np.ascontiguousarray(trans, np.float64)
    zp = ctypes.c_double(0.0)
    _check(lib().sb_band_zeropoint_ab(w.ctypes.data_as(_f64p), t.ctypes.data_as(_f64p), len(w), float(max_spacing),
                                      int(rule), ctypes.byref(zp)), "sb_band_zeropoint_ab")
    return zp.value


def philox4x64_10(ctr, key):
    """One block of the library's draws generator (host only)."""
    c = (ctypes.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib().sb_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def peak_probe(kind, n, iters=1, src=None, dst=None, stream=None):
    """One launch of a peak-rate probe (SB_PROBE_*) on the current device; returns its FLOPs or bytes.
    FMA_F32 and LDS_READ: n workgroups, dst a float32 CUDA tensor of n * 256 elements; COPY: n bytes
    from src to dst (CUDA tensors of at least n bytes)."""
    if kind in (SB_PROBE_FMA_F32, SB_PROBE_LDS_READ):
        _dev(dst, __import__("torch").float32, "dst")
        if dst.numel() < n * PROBE_THREADS:
            raise ValueError("dst must hold n * 256 floats")
    elif kind == SB_PROBE_COPY:
        for x, name in ((src, "src"), (dst, "dst")):
            if x is None or not x.is_cuda or not x.is_contiguous() or x.numel() * x.element_size() < n:
                raise ValueError(f"{name} must be a contiguous CUDA tensor of at least n bytes")
    work = ctypes.c_double(0.0)
    _check(lib().sb_peak_probe(int(kind), int(n), int(iters), _ptr(src), _ptr(dst), ctypes.byref(work),
                               _stream(stream)), "sb_peak_probe")
    return work.value


def _dev(x, dtype, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _grad_buffer(grad, n_sn, device):
    """The gradient output [n_sn, 5] of an adjoint call: a new tensor, or the caller's, which must be a
    contiguous float32 device tensor of n_sn * 5 elements (the kernel writes that many floats)."""
    import torch
    if grad is None:
        return torch.empty((n_sn, SB_N_PARAMS), dtype=torch.float32, device=device)
    _dev(grad, torch.float32, "grad")
    if grad.numel() != n_sn * SB_N_PARAMS:
        raise ValueError("grad must have n_sn * 5 elements")
    return grad


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class PreparedCall:
    """A library call whose arguments were validated and marshalled once.  Calling it launches the
    kernel again on the same buffers and stream (the caller may update the buffers in place)."""
    __slots__ = ("_fn", "_name", "_args", "_keep", "outputs")

    def __init__(self, fn, name, args, keep, outputs):
        self._fn, self._name, self._args, self._keep, self.outputs = fn, name, args, keep, outputs

    def __call__(self):
        st = self._fn(*self._args)
        if st < 0:
            _check(st, self._name)


class Context:
    """A library context: the model surfaces and the registered bands on one GPU."""

    def __init__(self, m0, m1, phase0, dphase, wave0, dwave, cl_coef, cl_wave_b, cl_wave_v,
                 config: Optional[Config] = None, device: int = 0, **config_over):
        m0 = np.ascontiguousarray(m0, np.float32)
        m1 = np.ascontiguousarray(m1, np.float32)
        if m0.shape != m1.shape or m0.ndim != 2:
            raise ValueError("m0 and m1 must be 2-D arrays of one shape")
        cl = np.ascontiguousarray(cl_coef, np.float64)
        d = ModelDesc(m0.shape[0], m0.shape[1], phase0, dphase, wave0, dwave,
                      m0.ctypes.data, m1.ctypes.data, len(cl), cl.ctypes.data, cl_wave_b, cl_wave_v)
        cfg = config if config is not None else default_config(**config_over)
        h = ctypes.c_void_p()
        _check(lib().sb_create(ctypes.byref(d), ctypes.byref(cfg), device, ctypes.byref(h)), "sb_create")
        self._h = h
        self.config = cfg
        self.device = device
        self.n_bands = 0

    @classmethod
    def from_model(cls, model, bands: Sequence = (), **kw):
        """Build from an object with m0, m1, phase0, dphase, wave0, dwave, cl_coef, cl_wave_b, cl_wave_v
        attributes and register `bands` (objects with .wave and .trans)."""
        ctx = cls(model.m0, model.m1, model.phase0, model.dphase, model.wave0, model.dwave,
                  model.cl_coef, model.cl_wave_b, model.cl_wave_v, **kw)
        for b in bands:
            ctx.add_band(b.wave, b.trans)
        return ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().sb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_band(self, wave, trans) -> int:
        w = np.ascontiguousarray(wave, np.float64)
        t = np.ascontiguousarray(trans, np.float64)
        bid = ctypes.c_int32(-1)
        _check(lib().sb_add_band(self._h, w.ctypes.data_as(_f64p), t.ctypes.data_as(_f64p), len(w),
                                 ctypes.byref(bid)), "sb_add_band")
        self.n_bands += 1
        return bid.value

    def add_band_file(self, path) -> int:
        """Register the bandpass in a two-column text file (sb_add_band_file)."""
        bid = ctypes.c_int32(-1)
        _check(lib().sb_add_band_file(self._h, os.fsencode(path), ctypes.byref(bid)), "sb_add_band_file")
        self.n_bands += 1
        return bid.value

    def zeropoint(self, band_id, magsys=SB_MAGSYS_AB) -> float:
        """The band's zero-point flux (AB): m = -2.5 log10(f / zeropoint)."""
        zp = ctypes.c_double(0.0)
        _check(lib().sb_band_zeropoint(self._h, band_id, magsys, ctypes.byref(zp)), "sb_band_zeropoint")
        return zp.value

    # ------------------------------------------------------------------ compute
    def _batch(self, z, t0, x0, x1, c, t, band, sn_offsets, broadcast, data, inv_sigma2, chi2):
        import torch
        for n, v in (("z", z), ("t0", t0), ("x0", x0), ("x1", x1), ("c", c), ("t", t)):
            _dev(v, torch.float32, n)
        _dev(band, torch.int32, "band")
        n_sn, n_obs = z.numel(), t.numel()
        for n, v in (("t0", t0), ("x0", x0), ("x1", x1), ("c", c)):
            if v.numel() != n_sn:
                raise ValueError(f"{n} must have n_sn elements")
        if band.numel() != n_obs:
            raise ValueError("band must have n_obs elements")
        if not broadcast:
            _dev(sn_offsets, torch.int32, "sn_offsets")
            if sn_offsets.numel() != n_sn + 1:
                raise ValueError("sn_offsets must have n_sn + 1 elements")
        if chi2:
            _dev(data, torch.float32, "data")
            _dev(inv_sigma2, torch.float32, "inv_sigma2")
            if data.numel() != n_obs or inv_sigma2.numel() != n_obs:
                raise ValueError("data / inv_sigma2 must have n_obs elements")
        if broadcast not in (False, True, "persistent"):
            raise ValueError('broadcast must be False, True or "persistent"')
        flags = ((SB_OBS_BROADCAST if broadcast else 0) | (SB_PERSISTENT if broadcast == "persistent" else 0)
                 | (SB_OUT_CHI2 if chi2 else 0))
        return Batch(n_sn, n_obs, flags, _ptr(z), _ptr(t0), _ptr(x0), _ptr(x1), _ptr(c), _ptr(t), _ptr(band),
                     None if broadcast else _ptr(sn_offsets), _ptr(data) if chi2 else None,
                     _ptr(inv_sigma2) if chi2 else None)

    def bandflux(self, z, t0, x0, x1, c, t, band, sn_offsets=None, *, broadcast=False, data=None,
                 inv_sigma2=None, chi2=False, out=None, stream=None):
        """Fluxes [n_obs] ([n_sn, n_obs] with broadcast), or chi2 [n_sn] with chi2=True.  broadcast:
        False (CSR batch), True (one observation table for all samples, a workgroup per sample) or
        "persistent" (the same sweep as a persistent launch; bitwise the same results)."""
        import torch
        b = self._batch(z, t0, x0, x1, c, t, band, sn_offsets, broadcast, data, inv_sigma2, chi2)
        shape = (b.n_sn,) if chi2 else ((b.n_sn, b.n_obs) if broadcast else (b.n_obs,))
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=z.device)
        else:
            _dev(out, torch.float32, "out")
            if tuple(out.shape) != shape:
                raise ValueError(f"out must have shape {shape}")
        _check(lib().sb_bandflux(self._h, ctypes.byref(b), _ptr(out), _stream(stream)), "sb_bandflux")
        return out

    def bandflux_vjp(self, z, t0, x0, x1, c, t, band, sn_offsets=None, cotangent=None, *, broadcast=False,
                     data=None, inv_sigma2=None, chi2=False, want_flux=False, want_jac=False, grad=None,
                     stream=None):
        """Adjoint: returns dict(grad [n_sn, 5] (z, t0, x0, x1, c), flux?, jac?, chi2?)."""
        import torch
        b = self._batch(z, t0, x0, x1, c, t, band, sn_offsets, broadcast, data, inv_sigma2, chi2)
        dev = z.device
        grad = _grad_buffer(grad, b.n_sn, dev)
        nrow = b.n_sn * b.n_obs if broadcast else b.n_obs
        flux = torch.empty(nrow, dtype=torch.float32, device=dev) if want_flux else None
        jac = torch.empty((nrow, SB_N_PARAMS), dtype=torch.float32, device=dev) if want_jac else None
        c2 = torch.empty(b.n_sn, dtype=torch.float32, device=dev) if chi2 else None
        if not chi2:
            _dev(cotangent, torch.float32, "cotangent")
            if cotangent.numel() != nrow:
                raise ValueError("cotangent has the wrong size")
        _check(lib().sb_bandflux_vjp(self._h, ctypes.byref(b), None if chi2 else _ptr(cotangent), _ptr(grad),
                                     _ptr(flux), _ptr(jac), _ptr(c2), _stream(stream)), "sb_bandflux_vjp")
        return {"grad": grad, "flux": flux, "jac": jac, "chi2": c2}

    # ------------------------------------------------------------------ prepared calls
    def prepare_bandflux(self, z, t0, x0, x1, c, t, band, sn_offsets=None, *, broadcast=False, data=None,
                         inv_sigma2=None, chi2=False, out=None, stream=None) -> "PreparedCall":
        """Validate the arguments and build the call once; the returned object launches sb_bandflux on
        the same buffers each time it is called (for loops that re-evaluate buffers updated in place)."""
        import torch
        b = self._batch(z, t0, x0, x1, c, t, band, sn_offsets, broadcast, data, inv_sigma2, chi2)
        shape = (b.n_sn,) if chi2 else ((b.n_sn, b.n_obs) if broadcast else (b.n_obs,))
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=z.device)
        _dev(out, torch.float32, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out must have shape {shape}")
        keep = (z, t0, x0, x1, c, t, band, sn_offsets, data, inv_sigma2, out)
        return PreparedCall(lib().sb_bandflux, "sb_bandflux",
                            (self._h, ctypes.byref(b), _ptr(out), _stream(stream)), (b, keep), {"out": out})

    def prepare_bandflux_vjp(self, z, t0, x0, x1, c, t, band, sn_offsets=None, cotangent=None, *, broadcast=False,
                             data=None, inv_sigma2=None, chi2=False, want_flux=False, want_jac=False, grad=None,
                             stream=None) -> "PreparedCall":
        """As prepare_bandflux, for sb_bandflux_vjp; the result buffers are in .outputs."""
        import torch
        b = self._batch(z, t0, x0, x1, c, t, band, sn_offsets, broadcast, data, inv_sigma2, chi2)
        dev = z.device
        grad = _grad_buffer(grad, b.n_sn, dev)
        nrow = b.n_sn * b.n_obs if broadcast else b.n_obs
        flux = torch.empty(nrow, dtype=torch.float32, device=dev) if want_flux else None
        jac = torch.empty((nrow, SB_N_PARAMS), dtype=torch.float32, device=dev) if want_jac else None
        c2 = torch.empty(b.n_sn, dtype=torch.float32, device=dev) if chi2 else None
        if not chi2:
            _dev(cotangent, torch.float32, "cotangent")
            if cotangent.numel() != nrow:
                raise ValueError("cotangent has the wrong size")
        keep = (z, t0, x0, x1, c, t, band, sn_offsets, data, inv_sigma2, cotangent)
        outs = {"grad": grad, "flux": flux, "jac": jac, "chi2": c2}
        args = (self._h, ctypes.byref(b), None if chi2 else _ptr(cotangent), _ptr(grad), _ptr(flux), _ptr(jac),
                _ptr(c2), _stream(stream))
        return PreparedCall(lib().sb_bandflux_vjp, "sb_bandflux_vjp", args, (b, keep), outs)

    def device_check(self, stream=None):
        """Synchronise the stream and raise if the device flagged a range error."""
        _check(lib().sb_device_check(self._h, _stream(stream)), "sb_device_check")

    # ------------------------------------------------------------------ serving
    def fit_submit(self, t, band, data, sigma, z, t0, x0, x1, c, free_mask=0, lower=None, upper=None) -> int:
        """Queue one fit; free_mask: an OR of SB_FREE_* (0: all four parameters free); lower/upper:
        bounds of (t0, x0, x1, c) for the L-BFGS-B solver (None: unbounded)."""
        t = np.ascontiguousarray(t, np.float32)
        band = np.ascontiguousarray(band, np.int32)
        data = np.ascontiguousarray(data, np.float32)
        sigma = np.ascontiguousarray(sigma, np.float32)
        has = lower is not None or upper is not None
        lo = np.full(4, -np.inf, np.float32) if lower is None else np.float32(lower)
        hi = np.full(4, np.inf, np.float32) if upper is None else np.float32(upper)
        r = FitRequest(len(t), t.ctypes.data, band.ctypes.data, data.ctypes.data, sigma.ctypes.data,
                       z, t0, x0, x1, c, free_mask, int(has), (ctypes.c_float * 4)(*lo.tolist()),
                       (ctypes.c_float * 4)(*hi.tolist()))
        tk = ctypes.c_uint64(0)
        _check(lib().sb_fit_submit(self._h, ctypes.byref(r), ctypes.byref(tk)), "sb_fit_submit")
        return tk.value

    def fit_poll(self, ticket):
        res = FitResult()
        st = _check(lib().sb_fit_poll(self._h, ticket, ctypes.byref(res)), "sb_fit_poll")
        return None if st == SB_PENDING else res

    def fit_wait(self, ticket, timeout_s=10.0):
        res = FitResult()
        st = _check(lib().sb_fit_wait(self._h, ticket, timeout_s, ctypes.byref(res)), "sb_fit_wait")
        return None if st == SB_PENDING else res

    def fit_cancel(self, ticket):
        _check(lib().sb_fit_cancel(self._h, ticket), "sb_fit_cancel")

    # ------------------------------------------------------------------ batch fits
    def _fit_batch_desc(self, z, t0, x0, x1, c, t, band, fit_offsets, data, inv_sigma2, free_mask, lower=None,
                        upper=None):
        import torch
        for n, v in (("z", z), ("t0", t0), ("x0", x0), ("x1", x1), ("c", c), ("t", t), ("data", data),
                     ("inv_sigma2", inv_sigma2)):
            _dev(v, torch.float32, n)
        _dev(band, torch.int32, "band")
        _dev(fit_offsets, torch.int32, "fit_offsets")
        n_fit, n_obs = z.numel(), t.numel()
        for n, v in (("t0", t0), ("x0", x0), ("x1", x1), ("c", c)):
            if v.numel() != n_fit:
                raise ValueError(f"{n} must have n_fit elements")
        for n, v in (("band", band), ("data", data), ("inv_sigma2", inv_sigma2)):
            if v.numel() != n_obs:
                raise ValueError(f"{n} must have n_obs elements")
        if fit_offsets.numel() != n_fit + 1:
            raise ValueError("fit_offsets must have n_fit + 1 elements")
        if free_mask is not None:
            _dev(free_mask, torch.int32, "free_mask")
            if free_mask.numel() != n_fit:
                raise ValueError("free_mask must have n_fit elements")
        for n, v in (("lower", lower), ("upper", upper)):
            if v is not None:
                _dev(v, torch.float32, n)
                if v.numel() != 4 * n_fit:
                    raise ValueError(f"{n} must have n_fit * 4 elements")
        return FitBatchDesc(n_fit, n_obs, _ptr(z), _ptr(t0), _ptr(x0), _ptr(x1), _ptr(c), _ptr(free_mask),
                            _ptr(t), _ptr(band), _ptr(fit_offsets), _ptr(data), _ptr(inv_sigma2), _ptr(lower),
                            _ptr(upper))

    @staticmethod
    def _fit_out_buffer(out, n_fit, device):
        import torch
        if out is None:
            return torch.empty((n_fit, FIT_OUT_WORDS), dtype=torch.int32, device=device)
        _dev(out, torch.int32, "out")
        if out.numel() != n_fit * FIT_OUT_WORDS:
            raise ValueError("out must hold n_fit sb_fit_out records (8 int32 words each)")
        return out

    def fit_batch(self, z, t0, x0, x1, c, t, band, fit_offsets, data, inv_sigma2, free_mask=None, lower=None,
                  upper=None, out=None, stream=None):
        """Fits every light curve of a device-resident batch (sb_fit_batch).  Returns the raw result
        records as an int32 tensor [n_fit, 8]; fit_results() unpacks them."""
        d = self._fit_batch_desc(z, t0, x0, x1, c, t, band, fit_offsets, data, inv_sigma2, free_mask, lower, upper)
        out = self._fit_out_buffer(out, d.n_fit, z.device)
        _check(lib().sb_fit_batch(self._h, ctypes.byref(d), _ptr(out), _stream(stream)), "sb_fit_batch")
        return out

    def fit_batch_noalloc(self, z, t0, x0, x1, c, t, band, fit_offsets, data, inv_sigma2, free_mask=None,
                          lower=None, upper=None, out=None, stream=None):
        """As fit_batch, through sb_fit_batch_noalloc (fixed per-device state array, no allocation in
        the library; at most SB_FIT_NOALLOC_MAX fits; calls overlapping on one GPU race)."""
        d = self._fit_batch_desc(z, t0, x0, x1, c, t, band, fit_offsets, data, inv_sigma2, free_mask, lower, upper)
        out = self._fit_out_buffer(out, d.n_fit, z.device)
        _check(lib().sb_fit_batch_noalloc(self._h, ctypes.byref(d), _ptr(out), _stream(stream)),
               "sb_fit_batch_noalloc")
        return out

    # ------------------------------------------------------------------ nested sampling
    def nested_sampling(self, priors, t, band, data, inv_sigma2, n_live=400, batch=4096, max_iter=100000,
                        max_evals=50_000_000, dlogz=0.01, enlarge=1.5, seed=1, log_norm=0.0, stream=None):
        """Nested sampling of one light curve's posterior (sb_nested_sampling).  priors: five (kind, a, b)
        for z, t0, x0, x1, c; t, band, data, inv_sigma2: the device observation table.  Returns a dict
        with logz, logz_err, information, n_iter, n_eval, n_batches, dead_* and live_* arrays."""
        import torch
        _dev(t, torch.float32, "t")
        _dev(band, torch.int32, "band")
        _dev(data, torch.float32, "data")
        _dev(inv_sigma2, torch.float32, "inv_sigma2")
        n_obs = t.numel()
        if band.numel() != n_obs or data.numel() != n_obs or inv_sigma2.numel() != n_obs:
            raise ValueError("the observation arrays must have one length")
        cfg = NsConfig()
        for d, (kind, a, b) in enumerate(priors):
            cfg.prior[d] = Prior(int(kind), float(a), float(b))
        cfg.n_live, cfg.batch, cfg.max_iter, cfg.max_evals = n_live, batch, max_iter, max_evals
        cfg.dlogz, cfg.enlarge, cfg.seed, cfg.log_norm = dlogz, enlarge, seed, log_norm
        dth = np.zeros((max_iter, 5))
        dl = np.zeros(max_iter)
        dw = np.zeros(max_iter)
        dd = np.zeros(max_iter, np.int64)
        lth = np.zeros((n_live, 5))
        ll = np.zeros(n_live)
        lw = np.zeros(n_live)
        summ = NsSummary()
        f64 = lambda a: a.ctypes.data_as(_f64p)
        _check(lib().sb_nested_sampling(self._h, ctypes.byref(cfg), n_obs, _ptr(t), _ptr(band), _ptr(data),
                                        _ptr(inv_sigma2), f64(dth), f64(dl), f64(dw),
                                        dd.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), f64(lth), f64(ll), f64(lw),
                                        ctypes.byref(summ), _stream(stream)), "sb_nested_sampling")
        n = summ.n_iter
        return {"logz": summ.logz, "logz_err": summ.logz_err, "information": summ.information, "n_iter": n,
                "n_eval": summ.n_eval, "n_batches": summ.n_batches, "stopped_on_evals": bool(summ.stopped_on_evals),
                "dead_theta": dth[:n], "dead_logl": dl[:n], "dead_logw": dw[:n], "dead_draw": dd[:n],
                "live_theta": lth, "live_logl": ll, "live_logw": lw}

    def stats(self):
        s = Stats()
        _check(lib().sb_stats(self._h, ctypes.byref(s)), "sb_stats")
        return s.as_dict()


def fit_results(out):
    """Unpack sb_fit_out records ([n_fit, 8] int32 tensor or array) into a dict of numpy arrays."""
    a = np.ascontiguousarray(out.cpu().numpy() if hasattr(out, "cpu") else out, dtype=np.int32).reshape(-1, 8)
    f = a.view(np.float32)
    return {"t0": f[:, 0].copy(), "x0": f[:, 1].copy(), "x1": f[:, 2].copy(), "c": f[:, 3].copy(),
            "chi2": f[:, 4].copy(), "status": a[:, 5].copy(), "iters": a[:, 6].copy(), "n_accept": a[:, 7].copy()}


def _saltbandflux_function():
    import torch

    class SaltBandflux(torch.autograd.Function):
        """flux = bandflux(z, t0, x0, x1, c; observations); backward through the hand-written adjoint."""

        @staticmethod
        def forward(fctx, lib_ctx, z, t0, x0, x1, c, t, band, sn_offsets):
            fctx.lib_ctx = lib_ctx
            fctx.save_for_backward(z, t0, x0, x1, c, t, band, sn_offsets)
            return lib_ctx.bandflux(z, t0, x0, x1, c, t, band, sn_offsets)

        @staticmethod
        def backward(fctx, gflux):
            z, t0, x0, x1, c, t, band, off = fctx.saved_tensors
            g = fctx.lib_ctx.bandflux_vjp(z, t0, x0, x1, c, t, band, off, gflux.contiguous())["grad"]
            return (None, g[:, 0], g[:, 1], g[:, 2], g[:, 3], g[:, 4], None, None, None)

    return SaltBandflux


_SBF = None


def salt_bandflux(lib_ctx: Context, z, t0, x0, x1, c, t, band, sn_offsets):
    """Differentiable bandflux (torch.autograd) over the library's forward and adjoint kernels."""
    global _SBF
    if _SBF is None:
        _SBF = _saltbandflux_function()
    return _SBF.apply(lib_ctx, z, t0, x0, x1, c, t, band, sn_offsets)
