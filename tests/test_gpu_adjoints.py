"""Transposes (gradients) and the harmonic-input analysis through the C ABI, against the
oracle's literal transposes: s2w_synthesis_adjoint, s2w_analysis_adjoint in the mixed
precision split, s2w_analysis_lm, b3w_analysis_adjoint, b3w_synthesis_adjoint; and the
live-handle check of a destroyed plan on the device."""
import ctypes

import numpy as np
import pytest

import synthetic as S
from oracle import ball, mw, wavelets
from _gpuutil import elementwise, fmt, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _maps(L, B, seed):
    return np.stack([np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(seed, b)), L)) for b in range(B)])


@pytest.mark.parametrize("prec,L,N,J0,B", [(0, 16, 3, 0, 2), (0, 64, 8, 0, 2), (0, 33, 4, 1, 3),
                                           (1, 32, 3, 0, 3), (1, 64, 8, 0, 32), (1, 130, 4, 1, 20)])
def test_synthesis_adjoint_against_oracle(prec, L, N, J0, B):
    """gwav, gscal of random (not band-limited) map cotangents against the oracle's
    transpose of the synthesis; dot test <S(w, s), g> = <w, S^T g> on the device."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[synthesis adjoint prec={prec} L={L} N={N} J0={J0} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    plan = s2w.Plan(L, N, 2.0, J0, batch=B, precision=prec, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L * 10 + B)
    g = rng.normal(size=plan.map_shape)
    gw, gs = plan.synthesis_adjoint(torch.from_numpy(g).cuda())
    views = plan.wav_views(gw)
    for b in sorted({0, B - 1}):
        rw, rs = wavelets.synthesis_adjoint(g[b], P)
        es = [rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(rw)]
        print(f"  map {b}: per-scale rel err " + " ".join(f"{e:.1e}" for e in es)
              + f"; scaling {rel(gs[b].cpu().numpy(), rs):.1e}", flush=True)
        assert max(es) < tol
        assert rel(gs[b].cpu().numpy(), rs) < tol
    # dot test with random coefficients
    w = torch.from_numpy(rng.normal(size=plan.wav_offset[-1])).to(plan.wav_dtype).cuda()
    s = torch.from_numpy(rng.normal(size=plan.scal_shape)).cuda()
    Sw = plan.synthesis(w, s)
    lhs = torch.sum(Sw * torch.from_numpy(g).cuda()).item()
    rhs = (torch.dot(w.double(), gw.double()) + torch.sum(s * gs)).item()
    assert abs(lhs - rhs) < (1e-12 if prec == 0 else 3e-6) * abs(lhs)


@pytest.mark.parametrize("L,N,J0,B", [(32, 3, 0, 3), (64, 8, 0, 32), (130, 4, 1, 20)])
def test_mixed_analysis_adjoint_against_oracle(L, N, J0, B):
    """Mixed plans run the transpose of the analysis in their forward precision split
    (FP32 matrix-core DFTs and theta sum, FP64 recursion and sums): within 1e-6 of the
    oracle's transpose of the same cotangents, per map."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[mixed analysis adjoint L={L} N={N} J0={J0} B={B}]", flush=True)
    plan = s2w.Plan(L, N, 2.0, J0, batch=B, precision=s2w.S2W_MIXED, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L + B)
    gw = torch.from_numpy(rng.normal(size=plan.wav_offset[-1])).float().cuda()
    gs = torch.from_numpy(rng.normal(size=plan.scal_shape)).cuda()
    gf = plan.analysis_adjoint(gw, gs).cpu().numpy()
    views = plan.wav_views(gw)
    for b in sorted({0, B - 1}):
        ref = wavelets.analysis_adjoint([v[b].double().cpu().numpy() for v in views], gs[b].cpu().numpy(), P)
        e = rel(gf[b], ref)
        st = elementwise(gf[b], ref, 0)
        print(f"  map {b}: rel err {e:.1e}; max/rms {fmt(st)}", flush=True)
        assert e < 1e-6
        assert st["all"] < 1e-5


@pytest.mark.parametrize("prec,L,N,J0,B", [(0, 32, 3, 0, 2), (0, 64, 4, 1, 1), (1, 64, 8, 0, 32)])
def test_analysis_lm_against_oracle(prec, L, N, J0, B):
    """s2w_analysis_lm on the seeded coefficients against the oracle's analysis_lm, and
    equal to s2w_analysis of their inverse SHT."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[analysis_lm prec={prec} L={L} N={N} J0={J0} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    plan = s2w.Plan(L, N, 2.0, J0, batch=B, precision=prec, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(60, b)) for b in range(B)])
    w1, s1 = plan.analysis_lm(torch.from_numpy(flm).cuda())
    w1, s1 = w1.clone(), s1.clone()
    views = plan.wav_views(w1)
    for b in sorted({0, B - 1}):
        rw, rs = wavelets.analysis_lm(flm[b], P)
        es = [rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(rw)]
        assert max(es) < tol, es
        assert rel(s1[b].cpu().numpy(), rs) < tol
    p64 = s2w.Plan(L, N, 2.0, J0, batch=B, device=0)
    f = p64.sht_inverse(torch.from_numpy(flm).cuda())
    w2, s2 = plan.analysis(f)
    assert (torch.linalg.norm((w1 - w2).double()) / torch.linalg.norm(w1.double())).item() < tol


@pytest.mark.parametrize("prec,L,N,P,B", [(0, 8, 3, 6, 2), (0, 16, 2, 8, 1), (1, 16, 3, 8, 4)])
def test_ball_adjoints_against_oracle(prec, L, N, P, B):
    """b3w_analysis_adjoint and b3w_synthesis_adjoint on random cotangents against the
    oracle's transposes of the ball maps."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[ball adjoints prec={prec} L={L} N={N} P={P} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    bp = s2w.BallPlan(L, N, P, batch=B, precision=prec, device=0)
    BP = ball.BallPlan(L, N, P)
    rng = np.random.default_rng(L + P + B)
    gw = torch.from_numpy(rng.normal(size=bp.wav_offset[-1])).to(bp.wav_dtype).cuda()
    gs = torch.from_numpy(rng.normal(size=bp.map_shape)).cuda()
    gf = bp.analysis_adjoint(gw, gs).cpu().numpy()
    views = bp.wav_views(gw)
    x = rng.normal(size=bp.map_shape)
    aw, as_ = bp.synthesis_adjoint(torch.from_numpy(x).cuda())
    aviews = bp.wav_views(aw)
    for b in sorted({0, B - 1}):
        ref = ball.analysis_adjoint({k: v[b].double().cpu().numpy() for k, v in views.items()},
                                    gs[b].cpu().numpy(), BP)
        e = rel(gf[b], ref)
        print(f"  map {b}: analysis adjoint rel err {e:.1e}", flush=True)
        assert e < tol
        rw, rs = ball.synthesis_adjoint(x[b], BP)
        es = [rel(aviews[k][b].double().cpu().numpy(), rw[k]) for k in rw]
        print(f"  map {b}: synthesis adjoint rel err max {max(es):.1e}, scaling {rel(as_[b].cpu().numpy(), rs):.1e}",
              flush=True)
        assert max(es) < tol
        assert rel(as_[b].cpu().numpy(), rs) < tol


def test_destroyed_plan_is_not_live():
    """Destroy, then destroy again and query: S2W_ESTATE, with nothing read from the
    released plan."""
    _torch()
    import paper_2402_01282_amd as s2w
    lib = s2w.lib()
    h = ctypes.c_void_p()
    assert lib.s2w_plan_create(ctypes.byref(h), 16, 3, 2.0, 0, 1, 0, 0, 0) == 0
    assert lib.s2w_plan_destroy(h) == 0
    assert lib.s2w_plan_destroy(h) == -5
    n = ctypes.c_int()
    assert lib.s2w_plan_layout(h, ctypes.byref(n), None, None, None, None, None) == -5
    hb = ctypes.c_void_p()
    assert lib.b3w_plan_create(ctypes.byref(hb), 8, 3, 4, 2.0, 2.0, 0, 0, 1.0, 1, 0, 0, 0) == 0
    assert lib.b3w_plan_destroy(hb) == 0
    assert lib.b3w_plan_destroy(hb) == -5
