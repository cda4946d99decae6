"""Python binding of libmwf (ctypes): argument marshalling only.

Every step of the filter runs in the HIP kernels of libmwf.so; PyTorch provides
device memory and streams. There is no fallback: if the library is missing or
cannot be loaded, every entry point raises.
"""
import ctypes
import os

import numpy as np

WF_OK, WF_EINVAL, WF_ENOMEM, WF_EDEVICE, WF_EUNSUPPORTED, WF_EBUSY, WF_ENOTREADY = 0, -1, -2, -3, -4, -5, -6
WF_F64, WF_F32, WF_BF16X3, WF_BF16X6 = 0, 1, 2, 3
WF_FLAG_TIMING, WF_FLAG_CHI2 = 1, 2

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmwf.so")

# (name, restype, argtypes) of every function declared in include/mwf.h
_c = ctypes
_SIGS = [
    ("wf_plan", _c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p,
                           _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("wf_solve", _c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32,
                            _c.c_void_p, _c.c_void_p]),
    ("wf_solve_batch", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_solve_batch_static", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                         _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("sht_map2alm", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("sht_alm2map", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("wf_footprint", _c.c_int, [_c.c_int32, _c.c_int32, _c.c_int32, _c.c_int32, _c.POINTER(_c.c_size_t)]),
    ("wf_plan_info", _c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64)]),
    ("wf_pixel_angles", _c.c_int, [_c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_autotune", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.POINTER(_c.c_int32),
                               _c.POINTER(_c.c_int32)]),
    ("wf_group_create", _c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_group_solve", _c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                  _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_group_autotune", _c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    ("wf_group_destroy", None, [_c.c_void_p]),
    ("wf_server_create", _c.c_int, [_c.POINTER(_c.c_void_p), _c.c_size_t, _c.c_int32]),
    ("wf_server_submit", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                    _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_int32, _c.POINTER(_c.c_uint64)]),
    ("wf_server_poll", _c.c_int, [_c.c_void_p, _c.c_uint64, _c.c_void_p, _c.POINTER(_c.c_double)]),
    ("wf_server_query", _c.c_int, [_c.c_void_p, _c.c_void_p]),
    ("wf_server_destroy", None, [_c.c_void_p]),
    ("wf_chi2", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int32, _c.c_void_p]),
    ("wf_constrained_batch", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                        _c.c_void_p, _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_solve_banded", _c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                   _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("wf_adaptive_defaults", None, [_c.c_void_p]),
    ("wf_adaptive_levels", _c.c_int, [_c.c_int32, _c.c_void_p, _c.c_double, _c.c_double, _c.c_void_p, _c.c_int32,
                                      _c.c_void_p, _c.c_void_p, _c.POINTER(_c.c_int32)]),
    ("wf_solve_adaptive", _c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32,
                                     _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.POINTER(_c.c_int32),
                                     _c.POINTER(_c.c_int32), _c.c_void_p, _c.c_void_p]),
    ("wf_pol_plan", _c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int32, _c.c_int32, _c.c_void_p, _c.c_void_p,
                               _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("wf_pol_solve_batch", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                      _c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p]),
    ("sht_pol_map2alm", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("sht_pol_alm2map", _c.c_int, [_c.c_void_p, _c.c_int32, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    ("wf_pol_plan_info", _c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                    _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64)]),
    ("wf_pol_sync", _c.c_int, [_c.c_void_p]),
    ("wf_pol_destroy", None, [_c.c_void_p]),
    ("wf_sync", _c.c_int, [_c.c_void_p]),
    ("wf_destroy", None, [_c.c_void_p]),
    ("wf_strerror", _c.c_char_p, [_c.c_int]),
    ("wf_last_error", _c.c_char_p, []),
]

_lib = None


class WFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def lib():
    """Load libmwf.so (once). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmwf.so not built ({LIB_PATH}); run python -m paper_1211_0585_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != WF_OK:
        L = lib()
        raise WFError(rc, f"{L.wf_strerror(rc).decode()}: {L.wf_last_error().decode()}")


class wf_plan_opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class wf_stats(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int32), ("timed", ctypes.c_int32),
                ("ms_ring", ctypes.c_double), ("ms_analysis", ctypes.c_double),
                ("ms_synthesis", ctypes.c_double), ("n_ring", ctypes.c_int32),
                ("n_analysis", ctypes.c_int32), ("n_synthesis", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("chi2_last", ctypes.c_double)]


class wf_adaptive_opts(ctypes.Structure):
    _fields_ = [("l_iter0", ctypes.c_int32), ("l_pad", ctypes.c_int32), ("full_band", ctypes.c_int32),
                ("max_level_sweeps", ctypes.c_int32), ("plateau_tol", ctypes.c_double),
                ("stop_tol", ctypes.c_double)]


def adaptive_opts(**kw):
    """wf_adaptive_defaults with the given fields replaced."""
    o = wf_adaptive_opts()
    lib().wf_adaptive_defaults(ctypes.byref(o))
    for k, v in kw.items():
        if k not in dict(wf_adaptive_opts._fields_):
            raise TypeError(f"unknown adaptive option {k}")
        setattr(o, k, v)
    return o


def adaptive_levels(lmax, cl, tau, omega, **kw):
    """Level table of the adaptive schedule (host only): list of (lambda, band limit)."""
    cl = np.ascontiguousarray(cl, dtype=np.float64)
    if cl.size != lmax + 1:
        raise ValueError("cl must have lmax+1 entries")
    cap = 64
    lam = np.empty(cap)
    lm = np.empty(cap, dtype=np.int32)
    n = ctypes.c_int32()
    o = adaptive_opts(**kw)
    _check(lib().wf_adaptive_levels(lmax, cl.ctypes.data, tau, omega, ctypes.byref(o), cap, lam.ctypes.data,
                                    lm.ctypes.data, ctypes.byref(n)))
    return [(float(lam[j]), int(lm[j])) for j in range(n.value)]


def footprint(nside, lmax, dtype=WF_F64, nmaps=1):
    out = ctypes.c_size_t(0)
    _check(lib().wf_footprint(nside, lmax, dtype, nmaps, ctypes.byref(out)))
    return out.value


def pixel_angles(nside):
    """(theta, phi) of every pixel centre in RING order, from the library's geometry."""
    npix = 12 * nside * nside
    th = np.empty(npix)
    ph = np.empty(npix)
    _check(lib().wf_pixel_angles(nside, th.ctypes.data, ph.ctypes.data))
    return th, ph


def n_alm(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A planned (nside, lmax, C_l, N^-1, mask) problem; owns device tables and buffers."""

    def __init__(self, nside, lmax, cl, ninv, mask=None, dtype=WF_F64, max_batch=1, stream=None,
                 flags=0, tune_cache=None):
        L = lib()
        cl = np.ascontiguousarray(cl, dtype=np.float64)
        ninv = np.ascontiguousarray(ninv, dtype=np.float64)
        npix = 12 * nside * nside
        if cl.size != lmax + 1:
            raise ValueError("cl must have lmax+1 entries")
        if ninv.size != npix:
            raise ValueError("ninv must have npix entries")
        mptr = None
        if mask is not None:
            mask = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
            if mask.size != npix:
                raise ValueError("mask must have npix entries")
            mptr = mask.ctypes.data
        opts = wf_plan_opts(dtype, max_batch, flags,
                            None if tune_cache is None else os.fsencode(tune_cache))
        h = ctypes.c_void_p()
        sh = _stream_handle(stream)
        _check(L.wf_plan(ctypes.byref(h), nside, lmax, cl.ctypes.data, ninv.ctypes.data, mptr,
                         ctypes.byref(opts), sh))
        self._h = h
        self.nside, self.lmax, self.dtype, self.max_batch = nside, lmax, dtype, max_batch
        a, b, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        u1, u2 = ctypes.c_int64(), ctypes.c_int64()
        _check(L.wf_plan_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t), ctypes.byref(u1),
                              ctypes.byref(u2)))
        self.npix, self.nalm, self.tau = a.value, b.value, t.value
        self.units_all, self.units_active = u1.value, u2.value
        self.last_stats = None

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan has been closed")
        return self._h

    def _types(self):
        import torch
        if self.dtype == WF_F64:
            return torch.float64, torch.complex128
        return torch.float32, torch.complex64

    def solve(self, d, lambdas, s_wf=None, s_alm=None, stream=None, want_alm=True, static=False):
        """Run the messenger iteration; d is [npix] or [nmaps, npix]. Returns (s_wf, s_alm).
        static=True runs wf_solve_batch_static (work buffers in the per-device static
        workspace; pass preallocated s_wf / s_alm to allocate nothing at all)."""
        import torch
        rt, ct = self._types()
        nmaps = 1 if d.dim() == 1 else d.shape[0]
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        if s_wf is None:
            s_wf = torch.empty_like(d)
        if s_alm is None and want_alm:
            shape = (self.nalm,) if d.dim() == 1 else (nmaps, self.nalm)
            s_alm = torch.empty(shape, dtype=ct, device=d.device)
        aptr = _dev_ptr(s_alm, ct, nmaps * self.nalm, "s_alm") if s_alm is not None else None
        st = wf_stats()
        fn = lib().wf_solve_batch_static if static else lib().wf_solve_batch
        _check(fn(self.handle, nmaps, _dev_ptr(d, rt, nmaps * self.npix, "d"),
                                    _dev_ptr(s_wf, rt, nmaps * self.npix, "s_wf"), aptr,
                                    lam.ctypes.data, lam.size, _stream_handle(stream), ctypes.byref(st)))
        self.last_stats = st
        return s_wf, s_alm

    def constrained(self, d, xi, eta, lambdas, s_cr=None, s_alm=None, stream=None, want_alm=True):
        """Constrained realisations s_rand + WF(d - s_rand - n_rand) from unit draws xi
        (packed alm, complex) and eta (per pixel); d, eta: [npix] or [nmaps, npix]."""
        import torch
        rt, ct = self._types()
        nmaps = 1 if d.dim() == 1 else d.shape[0]
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        if s_cr is None:
            s_cr = torch.empty_like(d)
        if s_alm is None and want_alm:
            shape = (self.nalm,) if d.dim() == 1 else (nmaps, self.nalm)
            s_alm = torch.empty(shape, dtype=ct, device=d.device)
        aptr = _dev_ptr(s_alm, ct, nmaps * self.nalm, "s_alm") if s_alm is not None else None
        st = wf_stats()
        _check(lib().wf_constrained_batch(self.handle, nmaps, _dev_ptr(d, rt, nmaps * self.npix, "d"),
                                          _dev_ptr(xi, ct, nmaps * self.nalm, "xi"),
                                          _dev_ptr(eta, rt, nmaps * self.npix, "eta"),
                                          _dev_ptr(s_cr, rt, nmaps * self.npix, "s_cr"), aptr, lam.ctypes.data,
                                          lam.size, _stream_handle(stream), ctypes.byref(st)))
        self.last_stats = st
        return s_cr, s_alm

    def solve_banded(self, d, lambdas, lmax_sht, s_wf=None, s_alm=None, stream=None, want_alm=True):
        """One map, sweep k at band limit lmax_sht[k] (non-decreasing). Returns (s_wf, s_alm)."""
        import torch
        rt, ct = self._types()
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        lm = np.ascontiguousarray(lmax_sht, dtype=np.int32)
        if lm.size != lam.size:
            raise ValueError("need one band limit per lambda")
        if s_wf is None:
            s_wf = torch.empty_like(d)
        if s_alm is None and want_alm:
            s_alm = torch.empty((self.nalm,), dtype=ct, device=d.device)
        aptr = _dev_ptr(s_alm, ct, self.nalm, "s_alm") if s_alm is not None else None
        st = wf_stats()
        _check(lib().wf_solve_banded(self.handle, _dev_ptr(d, rt, self.npix, "d"), _dev_ptr(s_wf, rt, self.npix, "s_wf"),
                                     aptr, lam.ctypes.data, lm.ctypes.data, lam.size, _stream_handle(stream),
                                     ctypes.byref(st)))
        self.last_stats = st
        return s_wf, s_alm

    def solve_adaptive(self, d, max_sweeps, s_wf=None, s_alm=None, stream=None, want_alm=True, **opts):
        """One map under the adaptive schedule (keyword options of wf_adaptive_opts).

        Returns (s_wf, s_alm, info) with info = dict(lambdas, lmax_sht, chi2, converged)."""
        import torch
        rt, ct = self._types()
        if s_wf is None:
            s_wf = torch.empty_like(d)
        if s_alm is None and want_alm:
            s_alm = torch.empty((self.nalm,), dtype=ct, device=d.device)
        aptr = _dev_ptr(s_alm, ct, self.nalm, "s_alm") if s_alm is not None else None
        o = adaptive_opts(**opts)
        lam = np.empty(max_sweeps)
        lm = np.empty(max_sweeps, dtype=np.int32)
        chi = np.empty(max_sweeps)
        n, conv = ctypes.c_int32(), ctypes.c_int32()
        st = wf_stats()
        _check(lib().wf_solve_adaptive(self.handle, _dev_ptr(d, rt, self.npix, "d"),
                                       _dev_ptr(s_wf, rt, self.npix, "s_wf"), aptr, ctypes.byref(o), max_sweeps,
                                       lam.ctypes.data, lm.ctypes.data, chi.ctypes.data, ctypes.byref(n),
                                       ctypes.byref(conv), _stream_handle(stream), ctypes.byref(st)))
        self.last_stats = st
        k = n.value
        info = {"lambdas": lam[:k].copy(), "lmax_sht": lm[:k].copy(), "chi2": chi[:k].copy(),
                "converged": bool(conv.value)}
        return s_wf, s_alm, info

    def chi2(self, nmaps, nsweeps):
        """chi^2 after every sweep of the last solve (plan flag WF_FLAG_CHI2): [nmaps, nsweeps]."""
        out = np.empty((nmaps, nsweeps))
        _check(lib().wf_chi2(self.handle, nmaps, nsweeps, out.ctypes.data))
        return out

    def map2alm(self, maps, alm=None, stream=None):
        import torch
        rt, ct = self._types()
        nmaps = 1 if maps.dim() == 1 else maps.shape[0]
        if alm is None:
            shape = (self.nalm,) if maps.dim() == 1 else (nmaps, self.nalm)
            alm = torch.empty(shape, dtype=ct, device=maps.device)
        _check(lib().sht_map2alm(self.handle, nmaps, _dev_ptr(maps, rt, nmaps * self.npix, "map"),
                                 _dev_ptr(alm, ct, nmaps * self.nalm, "alm"), _stream_handle(stream)))
        return alm

    def alm2map(self, alm, maps=None, stream=None):
        import torch
        rt, ct = self._types()
        nmaps = 1 if alm.dim() == 1 else alm.shape[0]
        if maps is None:
            shape = (self.npix,) if alm.dim() == 1 else (nmaps, self.npix)
            maps = torch.empty(shape, dtype=rt, device=alm.device)
        _check(lib().sht_alm2map(self.handle, nmaps, _dev_ptr(alm, ct, nmaps * self.nalm, "alm"),
                                 _dev_ptr(maps, rt, nmaps * self.npix, "map"), _stream_handle(stream)))
        return maps

    def autotune(self, nmaps=None, stream=None):
        """Pick the fastest matrix-core launch shape at nmaps maps; returns (ana_ct, syn_nct)."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().wf_autotune(self.handle, nmaps or self.max_batch, _stream_handle(stream),
                                 ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def sync(self):
        _check(lib().wf_sync(self.handle))

    def close(self):
        if self._h is not None:
            lib().wf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class PolPlan:
    """A polarised (T, Q, U) problem: spectra cl4 [4, lmax+1] (TT, EE, BB, TE), noise
    precision ninv6 [6, npix] (TT, QQ, UU, TQ, TU, QU), mask bytes (bit 0 T observed,
    bit 1 Q/U observed). Maps are [nmaps, 3, npix], alm [nmaps, 3, N_lm] (FP64)."""

    def __init__(self, nside, lmax, cl4, ninv6, mask=None, max_batch=1, stream=None, flags=0):
        L = lib()
        cl4 = np.ascontiguousarray(cl4, dtype=np.float64)
        ninv6 = np.ascontiguousarray(ninv6, dtype=np.float64)
        npix = 12 * nside * nside
        if cl4.shape != (4, lmax + 1):
            raise ValueError("cl4 must have shape (4, lmax+1)")
        if ninv6.shape != (6, npix):
            raise ValueError("ninv6 must have shape (6, npix)")
        mptr = None
        if mask is not None:
            mask = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
            if mask.size != npix:
                raise ValueError("mask must have npix entries")
            mptr = mask.ctypes.data
        opts = wf_plan_opts(WF_F64, max_batch, flags, None)
        h = ctypes.c_void_p()
        _check(L.wf_pol_plan(ctypes.byref(h), nside, lmax, cl4.ctypes.data, ninv6.ctypes.data, mptr,
                             ctypes.byref(opts), _stream_handle(stream)))
        self._h = h
        self.nside, self.lmax, self.max_batch = nside, lmax, max_batch
        a, b, t, u = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check(L.wf_pol_plan_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t), ctypes.byref(u)))
        self.npix, self.nalm, self.tau, self.units_active = a.value, b.value, t.value, u.value
        self.last_stats = None

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan has been closed")
        return self._h

    def solve(self, d, lambdas, s_wf=None, s_alm=None, stream=None, want_alm=True):
        """d: [3, npix] or [nmaps, 3, npix] float64 on the device. Returns (s_wf, s_alm)."""
        import torch
        nmaps = 1 if d.dim() == 2 else d.shape[0]
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        if s_wf is None:
            s_wf = torch.empty_like(d)
        if s_alm is None and want_alm:
            shape = (3, self.nalm) if d.dim() == 2 else (nmaps, 3, self.nalm)
            s_alm = torch.empty(shape, dtype=torch.complex128, device=d.device)
        aptr = _dev_ptr(s_alm, torch.complex128, nmaps * 3 * self.nalm, "s_alm") if s_alm is not None else None
        st = wf_stats()
        _check(lib().wf_pol_solve_batch(self.handle, nmaps, _dev_ptr(d, torch.float64, nmaps * 3 * self.npix, "d"),
                                        _dev_ptr(s_wf, torch.float64, nmaps * 3 * self.npix, "s_wf"), aptr,
                                        lam.ctypes.data, lam.size, _stream_handle(stream), ctypes.byref(st)))
        self.last_stats = st
        return s_wf, s_alm

    def map2alm(self, maps, alm=None, stream=None):
        import torch
        nmaps = 1 if maps.dim() == 2 else maps.shape[0]
        if alm is None:
            shape = (3, self.nalm) if maps.dim() == 2 else (nmaps, 3, self.nalm)
            alm = torch.empty(shape, dtype=torch.complex128, device=maps.device)
        _check(lib().sht_pol_map2alm(self.handle, nmaps, _dev_ptr(maps, torch.float64, nmaps * 3 * self.npix, "map"),
                                     _dev_ptr(alm, torch.complex128, nmaps * 3 * self.nalm, "alm"),
                                     _stream_handle(stream)))
        return alm

    def alm2map(self, alm, maps=None, stream=None):
        import torch
        nmaps = 1 if alm.dim() == 2 else alm.shape[0]
        if maps is None:
            shape = (3, self.npix) if alm.dim() == 2 else (nmaps, 3, self.npix)
            maps = torch.empty(shape, dtype=torch.float64, device=alm.device)
        _check(lib().sht_pol_alm2map(self.handle, nmaps, _dev_ptr(alm, torch.complex128, nmaps * 3 * self.nalm, "alm"),
                                     _dev_ptr(maps, torch.float64, nmaps * 3 * self.npix, "map"),
                                     _stream_handle(stream)))
        return maps

    def sync(self):
        _check(lib().wf_pol_sync(self.handle))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().wf_pol_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p.value if isinstance(p, ctypes.c_void_p) else p
    return arr


class Group:
    """Several matrix-core plans stepped together, one launch per phase (wf_group_*).

    plans: list of Plan (same dtype); nmaps: maps per plan. The group borrows the
    plans, which must stay open while it is used.
    """

    def __init__(self, plans, nmaps):
        if len(plans) != len(nmaps) or not plans:
            raise ValueError("need one nmaps entry per plan")
        self.plans, self.nmaps = list(plans), [int(n) for n in nmaps]
        hp = _ptr_array([p.handle for p in self.plans])
        nm = (ctypes.c_int32 * len(nmaps))(*self.nmaps)
        h = ctypes.c_void_p()
        _check(lib().wf_group_create(ctypes.byref(h), len(plans), hp, nm))
        self._h = h
        self.last_stats = None

    def _bufs(self, ds, s_wf, s_alm, want_alm):
        import torch
        if len(ds) != len(self.plans):
            raise ValueError("need one data tensor per plan")
        s_wf = s_wf or [torch.empty_like(d) for d in ds]
        if s_alm is None and want_alm:
            s_alm = [torch.empty((n, p.nalm), dtype=torch.complex64, device=d.device)
                     for p, n, d in zip(self.plans, self.nmaps, ds)]
        pd, pw, pa = [], [], []
        for i, (p, n) in enumerate(zip(self.plans, self.nmaps)):
            pd.append(_dev_ptr(ds[i], torch.float32, n * p.npix, f"d[{i}]"))
            pw.append(_dev_ptr(s_wf[i], torch.float32, n * p.npix, f"s_wf[{i}]"))
            if s_alm is not None:
                pa.append(_dev_ptr(s_alm[i], torch.complex64, n * p.nalm, f"s_alm[{i}]"))
        return s_wf, s_alm, _ptr_array(pd), _ptr_array(pw), (_ptr_array(pa) if s_alm is not None else None)

    def solve(self, ds, lambdas, s_wf=None, s_alm=None, stream=None, want_alm=True):
        """ds[i]: float32 [nmaps_i, npix_i] data of plan i. Returns (s_wf list, s_alm list)."""
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        s_wf, s_alm, pd, pw, pa = self._bufs(ds, s_wf, s_alm, want_alm)
        st = wf_stats()
        _check(lib().wf_group_solve(self._h, pd, pw, pa, lam.ctypes.data, lam.size, _stream_handle(stream),
                                    ctypes.byref(st)))
        self.last_stats = st
        return s_wf, s_alm

    def autotune(self, ds, stream=None):
        """Time every launch shape on data ds and keep the fastest; returns (ana_ct, syn_nct)."""
        _, _, pd, pw, _ = self._bufs(ds, None, None, False)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().wf_group_autotune(self._h, pd, pw, _stream_handle(stream), ctypes.byref(a),
                                       ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self._h is not None:
            lib().wf_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class wf_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "steps", "map_sweeps", "peak_slots", "lanes_created", "lanes_evicted",
        "bytes_in_use", "peak_bytes", "slots_in_use", "pending", "lanes")]


class Server:
    """Continuous-batching request loop (wf_server_*): submit solves, poll results.

    Inputs are host arrays; results come back as host float64 maps with the
    submit-to-result latency measured inside the library.
    """

    def __init__(self, hbm_budget=64 << 30, max_slots=64):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a HIP device")
        torch.cuda.init()
        h = ctypes.c_void_p()
        _check(lib().wf_server_create(ctypes.byref(h), int(hbm_budget), int(max_slots)))
        self._h = h
        self._npix = {}

    def submit(self, nside, lmax, cl, ninv, d, lambdas, mask=None, dtype=WF_F32):
        npix = 12 * nside * nside
        cl = np.ascontiguousarray(cl, dtype=np.float64)
        ninv = np.ascontiguousarray(ninv, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        if cl.size != lmax + 1 or ninv.size != npix or d.size != npix:
            raise ValueError("cl needs lmax+1 entries, ninv and d npix entries")
        mptr = None
        if mask is not None:
            mask = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
            if mask.size != npix:
                raise ValueError("mask must have npix entries")
            mptr = mask.ctypes.data
        t = ctypes.c_uint64()
        _check(lib().wf_server_submit(self._h, nside, lmax, cl.ctypes.data, ninv.ctypes.data, mptr, d.ctypes.data,
                                      lam.ctypes.data, lam.size, dtype, ctypes.byref(t)))
        self._npix[t.value] = npix
        return t.value

    def poll(self, ticket):
        """None while running; (s_wf float64 [npix], latency seconds) once finished."""
        out = np.empty(self._npix[ticket])
        lat = ctypes.c_double()
        rc = lib().wf_server_poll(self._h, ticket, out.ctypes.data, ctypes.byref(lat))
        if rc == WF_ENOTREADY:
            return None
        del self._npix[ticket]
        _check(rc)
        return out, lat.value

    def wait(self, ticket, timeout=120.0, interval=2e-4):
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not finished after {timeout} s")
            time.sleep(interval)

    def stats(self):
        st = wf_server_stats()
        _check(lib().wf_server_query(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in wf_server_stats._fields_}

    def close(self):
        if self._h is not None:
            lib().wf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
