"""Directional scale-discretised wavelet transform on the sphere for MI355X.

Thin Python binding over the C-ABI library libs2w.so (declared in
include/s2w.h).  Every step of the transform runs in the library's HIP
kernels; this module only marshals pointers, sizes and streams.  PyTorch
provides device memory and the current stream.

The library must be built (``python -m paper_2402_01282_amd._build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libs2w.so")

S2W_FP64 = 0
S2W_MIXED = 1
S2W_PLAN_TUNE = 1
S2W_PLAN_GRAPH = 2
S2W_PLAN_NO_WORKSPACE = 4
S2W_PLAN_PERSISTENT = 8
S2W_PLAN_PRECOMPUTE = 16
S2W_PLAN_WIGNER = 32
S2W_SCRATCH_BYTES = 64 << 20
S2W_OK, S2W_EINVAL, S2W_ENOMEM, S2W_EHIP, S2W_EUNSUPPORTED, S2W_ESTATE = 0, -1, -2, -3, -4, -5

_STATUS = {0: "S2W_OK", -1: "S2W_EINVAL", -2: "S2W_ENOMEM", -3: "S2W_EHIP",
           -4: "S2W_EUNSUPPORTED", -5: "S2W_ESTATE"}


class S2WError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -m paper_2402_01282_amd._build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sigs = {
        "s2w_plan_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint],
        "s2w_plan_create_spin": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint],
        "s2w_spin_sht_forward": [vp, vp, vp, vp],
        "s2w_spin_sht_inverse": [vp, vp, vp, vp],
        "s2w_spin_analysis": [vp, vp, vp, vp, vp],
        "s2w_spin_synthesis": [vp, vp, vp, vp, vp],
        "s2w_plan_destroy": [vp],
        "s2w_plan_layout": [vp, ip, ip, ip, ip, i64p, ip],
        "s2w_analysis": [vp, vp, vp, vp, vp],
        "s2w_synthesis": [vp, vp, vp, vp, vp],
        "s2w_analysis_adjoint": [vp, vp, vp, vp, vp],
        "s2w_synthesis_adjoint": [vp, vp, vp, vp, vp],
        "s2w_analysis_lm": [vp, vp, vp, vp, vp],
        "s2w_analysis_noalloc": [vp, vp, vp, vp, vp],
        "s2w_sht_forward": [vp, vp, vp, vp],
        "s2w_wigner_forward": [vp, vp, vp, vp],
        "s2w_wigner_inverse": [vp, vp, vp, vp],
        "s2w_sht_inverse": [vp, vp, vp, vp],
        "s2w_plan_profile": [vp, ctypes.c_int],
        "s2w_plan_profile_read": [vp, ctypes.c_int, ctypes.c_char_p, dp, i64p, dp, dp, dp, ip, i64p],
        "s2w_host_scales": [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip, ip, ip, ip],
        "s2w_host_filters": [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp],
        "s2w_host_theta_matrix": [ctypes.c_int, ctypes.c_int, dp],
        "s2w_host_wigner_d": [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp],
        "s2w_host_laguerre_rule": [ctypes.c_int, ctypes.c_double, dp, dp],
        "b3w_plan_create": [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_uint],
        "b3w_plan_destroy": [vp],
        "b3w_plan_layout": [vp, ip, ip, ip, ip, ip, i64p, dp],
        "b3w_analysis": [vp, vp, vp, vp, vp],
        "b3w_synthesis": [vp, vp, vp, vp, vp],
        "b3w_analysis_adjoint": [vp, vp, vp, vp, vp],
        "b3w_synthesis_adjoint": [vp, vp, vp, vp, vp],
        "b3w_sl_forward": [vp, vp, vp, vp],
        "b3w_wl_forward": [vp, vp, vp, vp],
        "b3w_wl_inverse": [vp, vp, vp, vp],
        "b3w_sl_inverse": [vp, vp, vp, vp],
        "b3w_plan_profile": [vp, ctypes.c_int],
        "b3w_plan_profile_read": [vp, ctypes.c_int, ctypes.c_char_p, dp, i64p, dp, dp, dp, ip, i64p],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.s2w_last_error.argtypes = []
    lib.s2w_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()

# every symbol the header declares (checked by the tests)
EXPORTS = ["s2w_plan_create", "s2w_plan_destroy", "s2w_plan_layout", "s2w_analysis", "s2w_synthesis",
           "s2w_analysis_lm", "s2w_analysis_noalloc", "s2w_analysis_adjoint", "s2w_synthesis_adjoint", "s2w_sht_forward", "s2w_sht_inverse",
           "s2w_wigner_forward", "s2w_wigner_inverse",
           "s2w_plan_create_spin", "s2w_spin_sht_forward", "s2w_spin_sht_inverse", "s2w_spin_analysis",
           "s2w_spin_synthesis",
           "s2w_plan_profile", "s2w_plan_profile_read",
           "s2w_last_error", "s2w_host_scales", "s2w_host_filters", "s2w_host_theta_matrix",
           "s2w_host_wigner_d", "s2w_host_laguerre_rule",
           "b3w_plan_create", "b3w_plan_destroy", "b3w_plan_layout", "b3w_analysis", "b3w_synthesis",
           "b3w_analysis_adjoint", "b3w_synthesis_adjoint", "b3w_sl_forward", "b3w_sl_inverse", "b3w_wl_forward", "b3w_wl_inverse", "b3w_plan_profile", "b3w_plan_profile_read"]


def lib():
    return _lib


def _check(st: int):
    if st != 0:
        raise S2WError(st, _lib.s2w_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------- host helpers

def host_scales(L, N, lam=2.0, J0=0):
    ns = ctypes.c_int()
    Lk = (ctypes.c_int * 70)()
    Nk = (ctypes.c_int * 70)()
    Lp = ctypes.c_int()
    _check(_lib.s2w_host_scales(L, N, lam, J0, ctypes.byref(ns), Lk, Nk, ctypes.byref(Lp)))
    return list(Lk[:ns.value]), list(Nk[:ns.value]), Lp.value


def host_filters(L, N, lam=2.0, J0=0):
    Lk, _, _ = host_scales(L, N, lam, J0)
    psi = np.zeros(len(Lk) * L * (2 * N - 1) * 2)
    phi = np.zeros(L)
    _check(_lib.s2w_host_filters(L, N, lam, J0, _dptr(psi), _dptr(phi)))
    return psi.view(np.complex128).reshape(len(Lk), L, 2 * N - 1), phi


def host_theta_matrix(L, sigma):
    T = np.zeros(L * L)
    _check(_lib.s2w_host_theta_matrix(L, sigma, _dptr(T)))
    return T.reshape(L, L)


def host_wigner_d(L, m, n):
    out = np.zeros(L * L)
    _check(_lib.s2w_host_wigner_d(L, m, n, _dptr(out)))
    return out.reshape(L, L)


def host_laguerre_rule(P, tau=1.0):
    """Radial nodes r_k and weights W_k of the ball's Laguerre rule."""
    r = np.zeros(P)
    w = np.zeros(P)
    _check(_lib.s2w_host_laguerre_rule(P, float(tau), _dptr(r), _dptr(w)))
    return r, w


# --------------------------------------------------------------- GPU plans

def _require(t, what, dtype, shape, device):
    """Raise ValueError unless t is a contiguous tensor of dtype and shape on cuda:device.

    Every tensor handed to the library is checked here first: the kernels index it by
    the plan's sizes, so a short, mistyped or strided buffer would be read or written
    out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{what}: expected a tensor on cuda:{device}, got {t.device}")
    return t


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A transform plan (filters, tables, workspace) for (L, N, lambda, J0, batch).

    Maps are torch float64 tensors [B, L, 2L-1] on the plan's device; wavelet
    coefficients are returned as one packed tensor plus per-scale views.
    """

    def __init__(self, L, N, lam=2.0, J0=0, batch=1, precision=S2W_FP64, device=0, flags=0):
        import torch
        self._torch = torch
        self.L, self.N, self.lam, self.J0, self.batch = L, N, float(lam), J0, batch
        self.precision = precision
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.s2w_plan_create(ctypes.byref(h), L, N, float(lam), J0, batch, precision, device, int(flags)))
        self._h = h
        ns, j0 = ctypes.c_int(), ctypes.c_int()
        Lk = (ctypes.c_int * 70)()
        Nk = (ctypes.c_int * 70)()
        off = (ctypes.c_int64 * 71)()
        Lp = ctypes.c_int()
        _check(_lib.s2w_plan_layout(h, ctypes.byref(ns), ctypes.byref(j0), Lk, Nk, off, ctypes.byref(Lp)))
        self.nscales = ns.value
        self.Lk = list(Lk[:ns.value])
        self.Nk = list(Nk[:ns.value])
        self.wav_offset = list(off[:ns.value + 1])
        self.Lphi = Lp.value
        self.wav_dtype = torch.float64 if precision == S2W_FP64 else torch.float32

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.s2w_plan_destroy(h)
            self._h = None

    # shapes ------------------------------------------------------------
    @property
    def map_shape(self):
        return (self.batch, self.L, 2 * self.L - 1)

    @property
    def scal_shape(self):
        return (self.batch, self.Lphi, 2 * self.Lphi - 1)

    def scale_shape(self, k):
        return (self.batch, 2 * self.Nk[k] - 1, self.Lk[k], 2 * self.Lk[k] - 1)

    def wav_views(self, packed):
        return [packed[self.wav_offset[k]:self.wav_offset[k + 1]].view(self.scale_shape(k))
                for k in range(self.nscales)]

    def _dev(self):
        return self._torch.device("cuda", self.device)

    def empty_wav(self):
        return self._torch.empty(self.wav_offset[-1], dtype=self.wav_dtype, device=self._dev())

    def _check_map(self, t, what="f"):
        return _require(t, what, self._torch.float64, self.map_shape, self.device)

    def _check_wav(self, t, what="wav"):
        return _require(t, what, self.wav_dtype, (self.wav_offset[-1],), self.device)

    def _check_scal(self, t, what="scal"):
        return _require(t, what, self._torch.float64, self.scal_shape, self.device)

    def _check_flm(self, t, what="flm"):
        """flm as a contiguous float64 [B, L, 2L-1, 2] (re, im) tensor."""
        return _require(t, what, self._torch.float64, self.map_shape + (2,), self.device)

    def _out(self, t, shape, dtype, what):
        torch = self._torch
        if t is None:
            return torch.empty(shape, dtype=dtype, device=self._dev())
        return _require(t, what, dtype, shape, self.device)

    def _p(self, t):
        return ctypes.c_void_p(t.data_ptr())

    # transforms --------------------------------------------------------
    def analysis(self, f, wav=None, scal=None):
        torch = self._torch
        self._check_map(f)
        wav = self._out(wav, (self.wav_offset[-1],), self.wav_dtype, "wav")
        scal = self._out(scal, self.scal_shape, torch.float64, "scal")
        _check(_lib.s2w_analysis(self._h, self._p(f), self._p(wav), self._p(scal),
                                 _stream_ptr(torch, self.device)))
        return wav, scal

    def analysis_noalloc(self, f, wav, scal):
        """s2w_analysis with the workspace in the library's static device scratch (no
        allocation in the call; outputs must be given)."""
        torch = self._torch
        self._check_map(f)
        self._check_wav(wav)
        self._check_scal(scal)
        _check(_lib.s2w_analysis_noalloc(self._h, self._p(f), self._p(wav), self._p(scal),
                                         _stream_ptr(torch, self.device)))
        return wav, scal

    def analysis_lm(self, flm, wav=None, scal=None):
        """Analysis from harmonic coefficients flm [B, L, 2L-1] (complex, real maps)."""
        torch = self._torch
        if tuple(flm.shape) != self.map_shape or not flm.is_complex():
            raise ValueError(f"flm: expected complex coefficients of shape {self.map_shape}")
        x = self._check_flm(torch.view_as_real(flm.to(torch.complex128)).contiguous())
        wav = self._out(wav, (self.wav_offset[-1],), self.wav_dtype, "wav")
        scal = self._out(scal, self.scal_shape, torch.float64, "scal")
        _check(_lib.s2w_analysis_lm(self._h, self._p(x), self._p(wav), self._p(scal),
                                    _stream_ptr(torch, self.device)))
        return wav, scal

    def synthesis(self, wav, scal, f=None):
        torch = self._torch
        self._check_wav(wav)
        self._check_scal(scal)
        f = self._out(f, self.map_shape, torch.float64, "f")
        _check(_lib.s2w_synthesis(self._h, self._p(wav), self._p(scal), self._p(f),
                                  _stream_ptr(torch, self.device)))
        return f

    def analysis_adjoint(self, gwav, gscal, gf=None):
        torch = self._torch
        self._check_wav(gwav, "gwav")
        self._check_scal(gscal, "gscal")
        gf = self._out(gf, self.map_shape, torch.float64, "gf")
        _check(_lib.s2w_analysis_adjoint(self._h, self._p(gwav), self._p(gscal), self._p(gf),
                                         _stream_ptr(torch, self.device)))
        return gf

    def synthesis_adjoint(self, gf, gwav=None, gscal=None):
        """Transpose of synthesis: map cotangent gf -> (gwav, gscal)."""
        torch = self._torch
        self._check_map(gf, "gf")
        gwav = self._out(gwav, (self.wav_offset[-1],), self.wav_dtype, "gwav")
        gscal = self._out(gscal, self.scal_shape, torch.float64, "gscal")
        _check(_lib.s2w_synthesis_adjoint(self._h, self._p(gf), self._p(gwav), self._p(gscal),
                                          _stream_ptr(torch, self.device)))
        return gwav, gscal

    # kernel timing ------------------------------------------------------
    def profile(self, capacity):
        """Record HIP events around every kernel launch (capacity pairs); 0 stops."""
        _check(_lib.s2w_plan_profile(self._h, int(capacity)))

    def profile_read(self):
        """{kernel name: (total ms, launches, flop, flop64, dense)} since profiling started
        (algorithmic work as counted by the library, see include/s2w.h)."""
        return _profile_read(_lib.s2w_plan_profile_read, self._h)

    @property
    def so3_shape(self):
        """Samples of a function on SO(3) at the plan's band limits: [B, 2N-1, L, 2L-1]."""
        return (self.batch, 2 * self.N - 1, self.L, 2 * self.L - 1)

    def wigner_forward(self, f):
        """Wigner coefficients [B, 2N-1, L, 2L-1] (complex128, "nlm") of real SO(3) samples
        (plan made with S2W_PLAN_WIGNER)."""
        torch = self._torch
        _require(f, "f", torch.float64, self.so3_shape, self.device)
        out = torch.empty(self.so3_shape + (2,), dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_wigner_forward(self._h, self._p(f), self._p(out), _stream_ptr(torch, self.device)))
        return torch.view_as_complex(out)

    def wigner_inverse(self, flmn):
        """Real SO(3) samples [B, 2N-1, L, 2L-1] from Wigner coefficients of a real function."""
        torch = self._torch
        if tuple(flmn.shape) != self.so3_shape or not flmn.is_complex():
            raise ValueError(f"flmn: expected complex coefficients of shape {self.so3_shape}")
        x = _require(torch.view_as_real(flmn.to(device=self._dev(), dtype=torch.complex128)).contiguous(),
                     "flmn", torch.float64, self.so3_shape + (2,), self.device)
        f = torch.empty(self.so3_shape, dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_wigner_inverse(self._h, self._p(x), self._p(f), _stream_ptr(torch, self.device)))
        return f

    def sht_forward(self, f):
        torch = self._torch
        self._check_map(f)
        flm = torch.empty((self.batch, self.L, 2 * self.L - 1, 2), dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_sht_forward(self._h, self._p(f), self._p(flm), _stream_ptr(torch, self.device)))
        return torch.view_as_complex(flm)

    def sht_inverse(self, flm):
        torch = self._torch
        if tuple(flm.shape) != self.map_shape or not flm.is_complex():
            raise ValueError(f"flm: expected complex coefficients of shape {self.map_shape}")
        x = self._check_flm(torch.view_as_real(flm.to(torch.complex128)).contiguous())
        f = torch.empty(self.map_shape, dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_sht_inverse(self._h, self._p(x), self._p(f), _stream_ptr(torch, self.device)))
        return f


class SpinPlan(Plan):
    """Plan for complex spin-s maps (s2w_plan_create_spin).

    Maps are planar float64 tensors [B, 2, L, 2L-1] (real part, imaginary part); spin-s
    harmonic coefficients complex [B, L, 2L-1]; wavelet coefficients one packed tensor
    whose per-scale views are [B, 2, 2N_k-1, L_k, 2L_k-1] (Re, Im); scaling coefficients
    [B, 2, L_phi, 2L_phi-1].
    """

    def __init__(self, L, N, spin, lam=2.0, J0=0, batch=1, precision=S2W_FP64, device=0, flags=0):
        import torch
        self._torch = torch
        self.L, self.N, self.spin, self.lam, self.J0, self.batch = L, N, int(spin), float(lam), J0, batch
        self.precision = precision
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.s2w_plan_create_spin(ctypes.byref(h), L, N, float(lam), J0, int(spin), batch, precision,
                                         device, int(flags)))
        self._h = h
        ns, j0 = ctypes.c_int(), ctypes.c_int()
        Lk = (ctypes.c_int * 70)()
        Nk = (ctypes.c_int * 70)()
        off = (ctypes.c_int64 * 71)()
        Lp = ctypes.c_int()
        _check(_lib.s2w_plan_layout(h, ctypes.byref(ns), ctypes.byref(j0), Lk, Nk, off, ctypes.byref(Lp)))
        self.nscales = ns.value
        self.Lk = list(Lk[:ns.value])
        self.Nk = list(Nk[:ns.value])
        self.wav_offset = list(off[:ns.value + 1])
        self.Lphi = Lp.value
        self.wav_dtype = torch.float64 if precision == S2W_FP64 else torch.float32

    @property
    def map_shape(self):
        return (self.batch, 2, self.L, 2 * self.L - 1)

    @property
    def scal_shape(self):
        return (self.batch, 2, self.Lphi, 2 * self.Lphi - 1)

    def scale_shape(self, k):
        return (self.batch, 2, 2 * self.Nk[k] - 1, self.Lk[k], 2 * self.Lk[k] - 1)

    def analysis(self, f, wav=None, scal=None):
        torch = self._torch
        self._check_map(f)
        wav = self._out(wav, (self.wav_offset[-1],), self.wav_dtype, "wav")
        scal = self._out(scal, self.scal_shape, torch.float64, "scal")
        _check(_lib.s2w_spin_analysis(self._h, self._p(f), self._p(wav), self._p(scal),
                                      _stream_ptr(torch, self.device)))
        return wav, scal

    def synthesis(self, wav, scal, f=None):
        torch = self._torch
        self._check_wav(wav)
        self._check_scal(scal)
        f = self._out(f, self.map_shape, torch.float64, "f")
        _check(_lib.s2w_spin_synthesis(self._h, self._p(wav), self._p(scal), self._p(f),
                                       _stream_ptr(torch, self.device)))
        return f

    def sht_forward(self, f):
        torch = self._torch
        self._check_map(f)
        flm = torch.empty((self.batch, self.L, 2 * self.L - 1, 2), dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_spin_sht_forward(self._h, self._p(f), self._p(flm), _stream_ptr(torch, self.device)))
        return torch.view_as_complex(flm)

    def sht_inverse(self, flm):
        torch = self._torch
        shape = (self.batch, self.L, 2 * self.L - 1)
        if tuple(flm.shape) != shape or not flm.is_complex():
            raise ValueError(f"flm: expected complex coefficients of shape {shape}")
        x = _require(torch.view_as_real(flm.to(torch.complex128)).contiguous(), "flm", torch.float64,
                     shape + (2,), self.device)
        f = torch.empty(self.map_shape, dtype=torch.float64, device=self._dev())
        _check(_lib.s2w_spin_sht_inverse(self._h, self._p(x), self._p(f), _stream_ptr(torch, self.device)))
        return f

    def _unsupported(self, *a, **k):
        raise S2WError(S2W_ESTATE, "spin plans run analysis, synthesis, sht_forward and sht_inverse only")

    analysis_lm = analysis_noalloc = analysis_adjoint = synthesis_adjoint = _unsupported
    wigner_forward = wigner_inverse = _unsupported


def _profile_read(fn, h):
    """{kernel name: (total ms, launches, flop, flop64, dense)} and the dropped-launch count."""
    mx = 64
    names = ctypes.create_string_buffer(32 * mx)
    ms = (ctypes.c_double * mx)()
    cnt = (ctypes.c_int64 * mx)()
    fl = (ctypes.c_double * mx)()
    f64 = (ctypes.c_double * mx)()
    dn = (ctypes.c_double * mx)()
    k = ctypes.c_int()
    dropped = ctypes.c_int64()
    _check(fn(h, mx, names, ms, cnt, fl, f64, dn, ctypes.byref(k), ctypes.byref(dropped)))
    out = {}
    for i in range(k.value):
        name = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
        out[name] = (ms[i], cnt[i], fl[i], f64[i], dn[i])
    return out, dropped.value


class BallPlan:
    """Ball wavelet plan for (L, N, P, lambda, nu, J0, J0', tau, batch).

    Maps and scaling coefficients are float64 tensors [B, P, L, 2L-1] on the radial
    nodes (``nodes``); wavelet coefficients are one packed tensor with a view per
    (radial scale i, angular scale k) of shape [B, P_i, 2N_k-1, L_k, 2L_k-1].
    """

    def __init__(self, L, N, P, lam=2.0, nu=2.0, J0=0, J0p=0, tau=1.0, batch=1, precision=S2W_FP64, device=0,
                 flags=0):
        import torch
        self._torch = torch
        self.L, self.N, self.P, self.lam, self.nu = L, N, P, float(lam), float(nu)
        self.J0, self.J0p, self.tau, self.batch, self.precision, self.device = J0, J0p, float(tau), batch, precision, device
        h = ctypes.c_void_p()
        _check(_lib.b3w_plan_create(ctypes.byref(h), L, N, P, float(lam), float(nu), J0, J0p, float(tau), batch,
                                    precision, device, int(flags)))
        self._h = h
        na, nr = ctypes.c_int(), ctypes.c_int()
        _check(_lib.b3w_plan_layout(h, ctypes.byref(na), ctypes.byref(nr), None, None, None, None, None))
        Lk = (ctypes.c_int * na.value)()
        Nk = (ctypes.c_int * na.value)()
        Pk = (ctypes.c_int * nr.value)()
        off = (ctypes.c_int64 * (na.value * nr.value + 1))()
        nodes = np.zeros(P)
        _check(_lib.b3w_plan_layout(h, ctypes.byref(na), ctypes.byref(nr), Lk, Nk, Pk, off, _dptr(nodes)))
        self.nang, self.nrad = na.value, nr.value
        self.Lk, self.Nk, self.Pk = list(Lk), list(Nk), list(Pk)
        self.wav_offset = list(off)
        self.nodes = nodes
        self.wav_dtype = torch.float64 if precision == S2W_FP64 else torch.float32

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.b3w_plan_destroy(h)
            self._h = None

    @property
    def map_shape(self):
        return (self.batch, self.P, self.L, 2 * self.L - 1)

    def block_shape(self, i, k):
        return (self.batch, self.Pk[i], 2 * self.Nk[k] - 1, self.Lk[k], 2 * self.Lk[k] - 1)

    def wav_views(self, packed):
        """{(i, k): view of block (radial scale i, angular scale k)}."""
        out = {}
        for i in range(self.nrad):
            for k in range(self.nang):
                o = self.wav_offset[i * self.nang + k]
                shp = self.block_shape(i, k)
                out[(i, k)] = packed[o:o + int(np.prod(shp))].view(shp)
        return out

    def _dev(self):
        return self._torch.device("cuda", self.device)

    def empty_wav(self):
        return self._torch.empty(self.wav_offset[-1], dtype=self.wav_dtype, device=self._dev())

    def _map(self, t, what):
        return _require(t, what, self._torch.float64, self.map_shape, self.device)

    def _wav(self, t, what):
        return _require(t, what, self.wav_dtype, (self.wav_offset[-1],), self.device)

    def _out(self, t, shape, dtype, what):
        if t is None:
            return self._torch.empty(shape, dtype=dtype, device=self._dev())
        return _require(t, what, dtype, shape, self.device)

    def analysis(self, f, wav=None, scal=None):
        torch = self._torch
        self._map(f, "f")
        wav = self._out(wav, (self.wav_offset[-1],), self.wav_dtype, "wav")
        scal = self._out(scal, self.map_shape, torch.float64, "scal")
        _check(_lib.b3w_analysis(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(wav.data_ptr()),
                                 ctypes.c_void_p(scal.data_ptr()), _stream_ptr(torch, self.device)))
        return wav, scal

    def synthesis(self, wav, scal, f=None):
        torch = self._torch
        self._wav(wav, "wav")
        self._map(scal, "scal")
        f = self._out(f, self.map_shape, torch.float64, "f")
        _check(_lib.b3w_synthesis(self._h, ctypes.c_void_p(wav.data_ptr()), ctypes.c_void_p(scal.data_ptr()),
                                  ctypes.c_void_p(f.data_ptr()), _stream_ptr(torch, self.device)))
        return f

    def analysis_adjoint(self, gwav, gscal, gf=None):
        """Transpose of analysis: (gwav, gscal) -> gf."""
        torch = self._torch
        self._wav(gwav, "gwav")
        self._map(gscal, "gscal")
        gf = self._out(gf, self.map_shape, torch.float64, "gf")
        _check(_lib.b3w_analysis_adjoint(self._h, ctypes.c_void_p(gwav.data_ptr()), ctypes.c_void_p(gscal.data_ptr()),
                                         ctypes.c_void_p(gf.data_ptr()), _stream_ptr(torch, self.device)))
        return gf

    def synthesis_adjoint(self, gf, gwav=None, gscal=None):
        """Transpose of synthesis: gf -> (gwav, gscal)."""
        torch = self._torch
        self._map(gf, "gf")
        gwav = self._out(gwav, (self.wav_offset[-1],), self.wav_dtype, "gwav")
        gscal = self._out(gscal, self.map_shape, torch.float64, "gscal")
        _check(_lib.b3w_synthesis_adjoint(self._h, ctypes.c_void_p(gf.data_ptr()), ctypes.c_void_p(gwav.data_ptr()),
                                          ctypes.c_void_p(gscal.data_ptr()), _stream_ptr(torch, self.device)))
        return gwav, gscal

    def sl_forward(self, f):
        """Spherical-Laguerre coefficients f_lmp [B, P, L, 2L-1] (complex128) of maps on the nodes."""
        torch = self._torch
        self._map(f, "f")
        flmp = torch.empty(self.map_shape + (2,), dtype=torch.float64, device=self._dev())
        _check(_lib.b3w_sl_forward(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(flmp.data_ptr()),
                                   _stream_ptr(torch, self.device)))
        return torch.view_as_complex(flmp)

    def sl_inverse(self, flmp):
        """Maps on the radial nodes from real-map spherical-Laguerre coefficients [B, P, L, 2L-1]."""
        torch = self._torch
        if tuple(flmp.shape) != self.map_shape or not flmp.is_complex():
            raise ValueError(f"flmp: expected complex coefficients of shape {self.map_shape}")
        x = torch.view_as_real(flmp.to(device=self._dev(), dtype=torch.complex128)).contiguous()
        _require(x, "flmp", torch.float64, self.map_shape + (2,), self.device)
        f = torch.empty(self.map_shape, dtype=torch.float64, device=self._dev())
        _check(_lib.b3w_sl_inverse(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                   _stream_ptr(torch, self.device)))
        return f

    @property
    def wl_shape(self):
        """Samples on the radial nodes x SO(3): [B, P, 2N-1, L, 2L-1]."""
        return (self.batch, self.P, 2 * self.N - 1, self.L, 2 * self.L - 1)

    def wl_forward(self, f):
        """Wigner-Laguerre coefficients [B, P, 2N-1, L, 2L-1] (complex128) of real samples
        (ball plan made with S2W_PLAN_WIGNER)."""
        torch = self._torch
        _require(f, "f", torch.float64, self.wl_shape, self.device)
        out = torch.empty(self.wl_shape + (2,), dtype=torch.float64, device=self._dev())
        _check(_lib.b3w_wl_forward(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(torch, self.device)))
        return torch.view_as_complex(out)

    def wl_inverse(self, flmnp):
        """Real samples on the radial nodes x SO(3) from Wigner-Laguerre coefficients."""
        torch = self._torch
        if tuple(flmnp.shape) != self.wl_shape or not flmnp.is_complex():
            raise ValueError(f"flmnp: expected complex coefficients of shape {self.wl_shape}")
        x = _require(torch.view_as_real(flmnp.to(device=self._dev(), dtype=torch.complex128)).contiguous(),
                     "flmnp", torch.float64, self.wl_shape + (2,), self.device)
        f = torch.empty(self.wl_shape, dtype=torch.float64, device=self._dev())
        _check(_lib.b3w_wl_inverse(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                   _stream_ptr(torch, self.device)))
        return f

    def profile(self, capacity):
        _check(_lib.b3w_plan_profile(self._h, int(capacity)))

    def profile_read(self):
        return _profile_read(_lib.b3w_plan_profile_read, self._h)


def _autograd():
    import torch

    class WaveletAnalysis(torch.autograd.Function):
        """W = A f with the hand-written adjoint A^T in backward (Wigner d recomputed)."""

        @staticmethod
        def forward(ctx, f, plan):
            wav, scal = plan.analysis(f.contiguous())
            ctx.plan = plan
            return wav, scal

        @staticmethod
        def backward(ctx, gwav, gscal):
            plan = ctx.plan
            if gwav is None:
                gwav = torch.zeros(plan.wav_offset[-1], dtype=plan.wav_dtype, device=plan._dev())
            if gscal is None:
                gscal = torch.zeros(plan.scal_shape, dtype=torch.float64, device=plan._dev())
            gf = plan.analysis_adjoint(gwav.contiguous(), gscal.contiguous())
            return gf, None

    return WaveletAnalysis


def analysis(f, plan):
    """Differentiable wavelet analysis: returns (packed wavelet coefficients, scaling coefficients)."""
    return _autograd().apply(f, plan)
