"""Complex spin-s maps on the GPU (s2w_plan_create_spin and the s2w_spin_* calls) against
the oracle's spin-s transforms, element by element.

Bars: FP64 plans 1e-11 relative L2 per result and per wavelet scale, and max |error| within
1e-10 of the reference rms; mixed plans 1e-6 relative L2 per scale and 2e-5 of the rms per
element (single-precision coefficients)."""
import numpy as np
import pytest

import synthetic as S
from _gpuutil import elementwise, fmt, rel
from oracle import mw, wavelets

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _planar(fs):
    """complex maps [B, L, 2L-1] -> planar float64 [B, 2, L, 2L-1]"""
    return np.ascontiguousarray(np.stack([fs.real, fs.imag], axis=1))


def _cel(got, ref, theta_axis):
    """elementwise() for complex arrays (real and imaginary parts stacked)."""
    return elementwise(np.stack([got.real, got.imag]), np.stack([ref.real, ref.imag]), theta_axis + 1)


def _maps(L, s, B, seed):
    flms = np.stack([S.spin_flm(L, s, S.stream_key(seed, b)) for b in range(B)])
    fs = np.stack([mw.spin_sht_inverse(flms[b], L, s) for b in range(B)])
    return flms, fs


@pytest.mark.parametrize("L,s,B", [(2, 1, 1), (16, 1, 2), (33, -2, 1), (64, 3, 2), (100, 0, 1), (128, 2, 2),
                                   (32, 10, 1), (17, -16, 1)])
def test_spin_sht_parity(L, s, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[spin sht L={L} s={s} B={B}]", flush=True)
    plan = s2w.SpinPlan(L, 1, s, batch=B, device=0)
    flms, fs = _maps(L, s, B, 90)
    got = plan.sht_forward(torch.from_numpy(_planar(fs)).cuda()).cpu().numpy()
    back = plan.sht_inverse(torch.from_numpy(flms).cuda()).cpu().numpy()
    for b in range(B):
        want = mw.spin_sht_forward(fs[b], L, s)
        assert rel(got[b], want) < 1e-11, (b, rel(got[b], want))
        assert rel(got[b], flms[b]) < 1e-11
        e = _cel(got[b], want, 0)
        assert e["all"] < 1e-10, fmt(e)
        fb = back[b, 0] + 1j * back[b, 1]
        assert rel(fb, fs[b]) < 1e-11, (b, rel(fb, fs[b]))


def _check_wavelets(plan, P, fs, s, B, tol, etol, tag):
    import paper_2402_01282_amd as s2w  # noqa: F401
    torch = _torch()
    wav, scal = plan.analysis(torch.from_numpy(_planar(fs)).cuda())
    views = [v.double().cpu().numpy() for v in plan.wav_views(wav)]
    sc = scal.cpu().numpy()
    worst = 0.0
    for b in range(B):
        rw, rs = wavelets.analysis_spin(fs[b], P, s)
        for k, v in enumerate(views):
            got = v[b, 0] + 1j * v[b, 1]
            r = rel(got, rw[k])
            worst = max(worst, r)
            e = _cel(got, rw[k], 1)
            assert r < tol and e["all"] < etol, (tag, b, k, r, fmt(e))
        gs = sc[b, 0] + 1j * sc[b, 1]
        assert rel(gs, rs) < tol, (tag, b, rel(gs, rs))
    print(f"  {tag}: worst per-scale rel {worst:.1e}", flush=True)
    # synthesis of the oracle's coefficients (map 0; the others zero)
    rw, rs = wavelets.analysis_spin(fs[0], P, s)
    wav_in = torch.zeros_like(wav)
    for k, v in enumerate(plan.wav_views(wav_in)):
        v[0, 0].copy_(torch.from_numpy(np.ascontiguousarray(rw[k].real)))
        v[0, 1].copy_(torch.from_numpy(np.ascontiguousarray(rw[k].imag)))
    scal_in = torch.zeros_like(scal)
    scal_in[0, 0].copy_(torch.from_numpy(np.ascontiguousarray(rs.real)))
    scal_in[0, 1].copy_(torch.from_numpy(np.ascontiguousarray(rs.imag)))
    g = plan.synthesis(wav_in, scal_in).cpu().numpy()
    want = wavelets.synthesis_spin(rw, rs, P, s)
    assert rel(g[0, 0] + 1j * g[0, 1], want) < tol, (tag, rel(g[0, 0] + 1j * g[0, 1], want))
    assert np.abs(g[1:]).max(initial=0.0) == 0.0
    # round trip on the plan's own coefficients
    back = plan.synthesis(wav, scal).cpu().numpy()
    for b in range(B):
        assert rel(back[b, 0] + 1j * back[b, 1], fs[b]) < tol


@pytest.mark.parametrize("L,N,J0,s,B", [(8, 3, 0, 1, 1), (16, 3, 0, -2, 2), (48, 2, 0, 0, 1), (64, 4, 1, 3, 2),
                                        (65, 5, 0, -1, 1), (128, 4, 0, 2, 1)])
def test_spin_wavelets_fp64(L, N, J0, s, B):
    import paper_2402_01282_amd as s2w
    print(f"[spin wavelets fp64 L={L} N={N} J0={J0} s={s} B={B}]", flush=True)
    plan = s2w.SpinPlan(L, N, s, 2.0, J0, batch=B, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    _, fs = _maps(L, s, B, 91)
    _check_wavelets(plan, P, fs, s, B, 1e-11, 1e-10, "fp64")


@pytest.mark.parametrize("L,N,s,B,flags", [(64, 4, 2, 2, 0), (96, 3, -1, 3, 1), (128, 8, 1, 4, 1 | 8)])
def test_spin_wavelets_mixed(L, N, s, B, flags):
    import paper_2402_01282_amd as s2w
    print(f"[spin wavelets mixed L={L} N={N} s={s} B={B} flags={flags}]", flush=True)
    plan = s2w.SpinPlan(L, N, s, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=flags)
    P = wavelets.Plan(L, N, 2.0, 0)
    _, fs = _maps(L, s, B, 92)
    _check_wavelets(plan, P, fs, s, B, 1e-6, 2e-5, "mixed")


def test_spin_plans_refuse_real_calls():
    torch = _torch()
    import paper_2402_01282_amd as s2w
    sp = s2w.SpinPlan(16, 2, 1, device=0)
    rp = s2w.Plan(16, 2, device=0)
    f = torch.zeros((1, 16, 31), dtype=torch.float64, device="cuda")
    wav = torch.zeros(sp.wav_offset[-1], dtype=torch.float64, device="cuda")
    scal = torch.zeros((2, sp.Lphi, 2 * sp.Lphi - 1), dtype=torch.float64, device="cuda")
    lib = s2w.lib()
    p = lambda t: s2w.ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.s2w_analysis(sp._h, p(f), p(wav), p(scal), None) == s2w.S2W_ESTATE
    assert lib.s2w_analysis_noalloc(sp._h, p(f), p(wav), p(scal), None) == s2w.S2W_ESTATE
    assert lib.s2w_spin_analysis(rp._h, p(f), p(wav), p(scal), None) == s2w.S2W_ESTATE
    torch.cuda.synchronize()


def test_spin_wavelets_mixed_L512():
    """A larger case: L = 512, N = 4, spin 2, mixed, two maps (two 64-column groups of the
    matrix-core contractions: 4 real maps x 2 scales x 8 columns)."""
    import paper_2402_01282_amd as s2w
    print("[spin wavelets mixed L=512 N=4 s=2 B=2]", flush=True)
    L, N, s, B = 512, 4, 2, 2
    plan = s2w.SpinPlan(L, N, s, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=s2w.S2W_PLAN_TUNE)
    P = wavelets.Plan(L, N, 2.0, 0)
    _, fs = _maps(L, s, B, 93)
    _check_wavelets(plan, P, fs, s, B, 1e-6, 2e-5, "mixed L=512")


@pytest.mark.parametrize("L,N,s,B,flags", [(64, 3, 1, 8, "precompute"), (128, 4, -2, 4, "precompute+tune"),
                                           (96, 2, 2, 8, "tune+persistent")])
def test_spin_plan_flags(L, N, s, B, flags):
    """Spin plans with precompute tables, tuning and the persistent list: the same results
    as the plain spin plan to the mixed bar, and against the oracle for the last map."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[spin flags {flags} L={L} N={N} s={s} B={B}]", flush=True)
    fl = 0
    if "precompute" in flags:
        fl |= s2w.S2W_PLAN_PRECOMPUTE
    if "tune" in flags:
        fl |= s2w.S2W_PLAN_TUNE
    if "persistent" in flags:
        fl |= s2w.S2W_PLAN_PERSISTENT
    plan = s2w.SpinPlan(L, N, s, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=fl)
    ref = s2w.SpinPlan(L, N, s, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0)
    _, fs = _maps(L, s, B, 94)
    f = torch.from_numpy(_planar(fs)).cuda()
    w1, s1 = plan.analysis(f)
    w1, s1 = w1.clone(), s1.clone()
    w2, s2 = ref.analysis(f)
    assert rel(w1.double().cpu().numpy(), w2.double().cpu().numpy()) < 1e-6
    g1 = plan.synthesis(w1, s1).clone()
    g2 = ref.synthesis(w1, s1)
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) < 1e-6
    P = wavelets.Plan(L, N, 2.0, 0)
    _check_wavelets(plan, P, fs, s, B, 1e-6, 2e-5, f"mixed {flags}")
