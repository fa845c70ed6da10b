"""Host-side checks of the C ABI and the binding (CPU only, no device work).

* A handle that is not a live plan is looked up, never dereferenced: destroying it
  or querying its layout returns S2W_ESTATE (a bogus address would otherwise be read).
* Every tensor the binding hands to the library is checked against the plan's
  sizes, dtype, contiguity and device before any call, so that a mistyped, short or
  strided buffer raises ValueError instead of reaching a kernel."""
import ctypes

import pytest
import torch

import paper_2402_01282_amd as s2w

S2W_ESTATE = -5


@pytest.mark.parametrize("fn", ["s2w_plan_destroy", "b3w_plan_destroy"])
def test_destroy_of_a_handle_that_is_not_live(fn):
    bogus = ctypes.c_void_p(0x10)           # never a plan; reading it would fault
    assert getattr(s2w.lib(), fn)(bogus) == S2W_ESTATE
    assert b"not a live" in s2w.lib().s2w_last_error()


def test_entry_points_reject_a_handle_that_is_not_live():
    lib = s2w.lib()
    bogus = ctypes.c_void_p(0x20)
    n = ctypes.c_int()
    assert lib.s2w_plan_layout(bogus, ctypes.byref(n), None, None, None, None, None) == S2W_ESTATE
    p = ctypes.c_void_p(0x1000)
    for name in ("s2w_analysis", "s2w_synthesis", "s2w_analysis_lm", "s2w_analysis_adjoint",
                 "s2w_synthesis_adjoint", "b3w_analysis", "b3w_synthesis", "b3w_analysis_adjoint",
                 "b3w_synthesis_adjoint"):
        assert getattr(lib, name)(bogus, p, p, p, None) == S2W_ESTATE, name
    assert lib.b3w_plan_layout(bogus, None, None, None, None, None, None, None) == S2W_ESTATE


def test_null_handle_is_an_argument_error():
    lib = s2w.lib()
    assert lib.s2w_plan_destroy(None) == 0            # NULL is accepted by destroy
    p = ctypes.c_void_p(0x1000)
    assert lib.s2w_analysis(None, p, p, p, None) == -1


def _fake_plan(prec=s2w.S2W_FP64):
    """A Plan with the sizes of (L=8, N=3, batch 2) and no library handle: the
    binding's checks run before any library call, so a failing check never reaches it."""
    p = object.__new__(s2w.Plan)
    p._torch = torch
    p.L, p.N, p.batch, p.device = 8, 3, 2, 0
    p.Lphi = 1
    p.nscales = 2
    p.Lk, p.Nk = [4, 8], [3, 3]
    p.wav_offset = [0, 2 * 5 * 4 * 7, 2 * 5 * 4 * 7 + 2 * 5 * 8 * 15]
    p.precision = prec
    p.wav_dtype = torch.float64 if prec == s2w.S2W_FP64 else torch.float32
    p._h = ctypes.c_void_p(0)
    return p


def test_binding_rejects_wrong_dtype_shape_and_layout():
    """Each check on its own (the plan's checkers), then through the transform methods,
    where the first failing argument raises before the library is called."""
    p = _fake_plan()
    nw = p.wav_offset[-1]
    with pytest.raises(ValueError, match="wav: expected dtype"):
        p._check_wav(torch.zeros(nw, dtype=torch.float32))
    with pytest.raises(ValueError, match="wav: expected shape"):
        p._check_wav(torch.zeros(nw - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="scal: expected shape"):
        p._check_scal(torch.zeros((2, 1, 2), dtype=torch.float64))
    with pytest.raises(ValueError, match="gscal: expected dtype"):
        p._check_scal(torch.zeros(p.scal_shape, dtype=torch.float32), "gscal")
    with pytest.raises(ValueError, match="f: expected shape"):
        p._check_map(torch.zeros((2, 8, 14), dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        p._check_map(torch.zeros((2, 15, 8), dtype=torch.float64).transpose(1, 2))
    with pytest.raises(ValueError, match="cuda:0"):
        p._check_map(torch.zeros(p.map_shape, dtype=torch.float64))
    with pytest.raises(ValueError, match="flm"):
        p._check_flm(torch.zeros(p.map_shape, dtype=torch.float64))
    # through the methods
    with pytest.raises(ValueError, match="wav: expected dtype"):
        p.synthesis(torch.zeros(nw, dtype=torch.float32), torch.zeros(p.scal_shape))
    with pytest.raises(ValueError, match="gwav: expected shape"):
        p.analysis_adjoint(torch.zeros(nw + 3, dtype=torch.float64), torch.zeros(p.scal_shape))
    with pytest.raises(ValueError, match="gf: expected dtype"):
        p.synthesis_adjoint(torch.zeros(p.map_shape, dtype=torch.float32))
    with pytest.raises(ValueError, match="f: expected shape"):
        p.analysis(torch.zeros((2, 8, 14), dtype=torch.float64))
    with pytest.raises(ValueError, match="flm"):
        p.sht_inverse(torch.zeros((2, 8, 14), dtype=torch.complex128))
    with pytest.raises(ValueError, match="flm"):
        p.analysis_lm(torch.zeros(p.map_shape, dtype=torch.float64))


def test_mixed_plan_takes_fp32_coefficients_only():
    q = _fake_plan(s2w.S2W_MIXED)
    nw = q.wav_offset[-1]
    with pytest.raises(ValueError, match="wav: expected dtype torch.float32"):
        q.synthesis(torch.zeros(nw, dtype=torch.float64), torch.zeros(q.scal_shape, dtype=torch.float64))
    with pytest.raises(ValueError, match="gwav: expected dtype torch.float32"):
        q.analysis_adjoint(torch.zeros(nw, dtype=torch.float64), torch.zeros(q.scal_shape, dtype=torch.float64))
