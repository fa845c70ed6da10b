"""Parity at the headline configuration L=1024, N=8, lambda=2, J0=0 (eleven wavelet
scales, L_j = 2, 4, ..., 512, 1024, 1024), element by element against the oracle.

* Mixed form, batch 64 (the measured workload, tuned, with and without precompute
  mode) of independently seeded Gaussian fields: every scale and the scaling coefficients of maps 0 and 63 against the
  oracle's analysis; the synthesis of the oracle's coefficients of maps 0 and 63 (the
  other 62 maps zero, so every column group of the theta contraction is full) against
  the input maps, which the exact transform reconstructs; round trip of every map.
* FP64 form, one map: every scale against the oracle, the synthesis of the oracle's
  coefficients, the round trip.
* Gradient of sum_j sum (W^j)^2 (config 4) against the oracle's transpose of the
  analysis, FP64 at one map and mixed at 16 maps.

Each comparison reports the relative L2 error and max |error| / rms(reference) over all
samples, the 4 theta rows next to each pole, and the theta rows of the last wave of the
16-wave theta tiles (theta >= 960), printed per scale."""
import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets
from _gpuutil import elementwise, fmt, rel

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

L, N, LAM, J0 = 1024, 8, 2.0, 0


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def oracle_plan():
    return wavelets.Plan(L, N, LAM, J0)


def _check_scales(plan, wav, scal, b, flm_b, P, tol_l2, tol_el):
    """All scales and the scaling coefficients of map b against the oracle."""
    views = plan.wav_views(wav)
    wr, sr = wavelets.analysis_lm(flm_b, P)
    worst = 0.0
    for k, w in enumerate(wr):
        got = views[k][b].double().cpu().numpy()
        e = rel(got, w)
        st = elementwise(got, w, 1, 960 if P.Lj[k] == L else None)
        print(f"  map {b} scale {k} (L_j={P.Lj[k]}): rel {e:.1e}; max/rms {fmt(st)}", flush=True)
        assert e < tol_l2, (b, k, e)
        assert st["all"] < tol_el, (b, k, st)
        worst = max(worst, e)
    es = rel(scal[b].cpu().numpy(), sr)
    print(f"  map {b} scaling: rel {es:.1e}", flush=True)
    assert es < tol_l2
    return wr, sr, worst


def _check_synthesis(plan, wr_by_map, sr_by_map, f, tol_l2, tol_el):
    """Synthesis of the oracle's coefficients for the given maps (others zero) against
    the input maps; untouched maps stay zero."""
    torch = _torch()
    packed = torch.zeros(plan.wav_offset[-1], dtype=plan.wav_dtype, device="cuda")
    pv = plan.wav_views(packed)
    sc = torch.zeros(plan.scal_shape, dtype=torch.float64, device="cuda")
    for b, wr in wr_by_map.items():
        for k, w in enumerate(wr):
            pv[k][b].copy_(torch.from_numpy(w).to(plan.wav_dtype))
        sc[b].copy_(torch.from_numpy(sr_by_map[b]))
    g = plan.synthesis(packed, sc)
    for b in wr_by_map:
        ref = f[b].cpu().numpy()
        got = g[b].cpu().numpy()
        e = rel(got, ref)
        st = elementwise(got, ref, 0, 960)
        print(f"  map {b} synthesis of the oracle's coefficients: rel {e:.1e}; max/rms {fmt(st)}", flush=True)
        assert e < tol_l2
        assert st["all"] < tol_el
    others = [b for b in range(plan.batch) if b not in wr_by_map]
    if others:
        assert torch.count_nonzero(g[others]).item() == 0


@pytest.mark.parametrize("precompute", [False, True])
def test_mixed_headline_B64_all_scales(oracle_plan, precompute):
    """The measured plans: tuned, with and without precompute mode (folded SHT and
    synthesis tables)."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    B = 64
    print(f"[headline mixed L=1024 N=8 B=64 precompute={precompute}]", flush=True)
    flm = [S.sphere_flm(L, S.stream_key(4, b)) for b in range(B)]
    p1 = s2w.Plan(L, N, LAM, J0, batch=1, device=0)
    f = torch.empty((B, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    for b in range(B):
        f[b].copy_(p1.sht_inverse(torch.from_numpy(flm[b][None].copy()).cuda())[0])
    del p1
    flags = s2w.S2W_PLAN_TUNE | (s2w.S2W_PLAN_PRECOMPUTE if precompute else 0)
    plan = s2w.Plan(L, N, LAM, J0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=flags)
    wav, scal = plan.analysis(f)
    f2 = plan.synthesis(wav, scal)
    errs = [(torch.linalg.norm(f2[b] - f[b]) / torch.linalg.norm(f[b])).item() for b in range(B)]
    print(f"  round trip: max rel {max(errs):.2e}, mean {np.mean(errs):.2e}", flush=True)
    assert max(errs) < 1e-6
    wrs, srs = {}, {}
    for b in (0, B - 1):
        wrs[b], srs[b], _ = _check_scales(plan, wav, scal, b, flm[b], oracle_plan, 1e-6, 1e-5)
    _check_synthesis(plan, wrs, srs, f, 1e-6, 1e-5)


def test_fp64_headline_all_scales(oracle_plan):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print("[headline FP64 L=1024 N=8 B=1]", flush=True)
    flm = S.sphere_flm(L, S.stream_key(4, 0))
    plan = s2w.Plan(L, N, LAM, J0, batch=1, device=0)
    f = plan.sht_inverse(torch.from_numpy(flm[None].copy()).cuda())
    assert rel(f[0].cpu().numpy(), np.real(mw.sht_inverse(flm, L))) < 1e-12
    wav, scal = plan.analysis_lm(torch.from_numpy(flm[None].copy()).cuda())
    wav, scal = wav.clone(), scal.clone()
    wr, sr, _ = _check_scales(plan, wav, scal, 0, flm, oracle_plan, 1e-12, 1e-11)
    w2, s2 = plan.analysis(f)
    assert (torch.linalg.norm(w2 - wav) / torch.linalg.norm(wav)).item() < 1e-12
    _check_synthesis(plan, {0: wr}, {0: sr}, f, 1e-12, 1e-11)
    f2 = plan.synthesis(w2, s2)
    assert rel(f2[0].cpu().numpy(), f[0].cpu().numpy()) < 1e-12


@pytest.mark.parametrize("prec,B", [(0, 1), (1, 16)])
def test_headline_gradient_against_oracle_adjoint(oracle_plan, prec, B):
    """Gradient of sum_j sum (W^j)^2 through the autograd Function (the hand-written
    transpose behind it): against the oracle's transpose of the same cotangents 2 W, and
    (mixed) against the exact FP64 gradient, for the first and last map."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[headline gradient prec={prec} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    flm = [S.sphere_flm(L, S.stream_key(44, b)) for b in range(B)]
    p1 = s2w.Plan(L, N, LAM, J0, batch=1, device=0)
    f = torch.empty((B, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    for b in range(B):
        f[b].copy_(p1.sht_inverse(torch.from_numpy(flm[b][None].copy()).cuda())[0])
    plan = p1 if (prec == 0 and B == 1) else s2w.Plan(L, N, LAM, J0, batch=B, precision=prec, device=0)
    x = f.clone().requires_grad_(True)
    wav, scal = s2w.analysis(x, plan)
    (wav.double() ** 2).sum().backward()
    got = x.grad.cpu().numpy()
    views = plan.wav_views(wav.detach())
    P = oracle_plan
    for b in sorted({0, B - 1}):
        gw = [2.0 * v[b].double().cpu().numpy() for v in views]
        ref = wavelets.analysis_adjoint(gw, np.zeros(plan.scal_shape[1:]), P)
        e = rel(got[b], ref)
        st = elementwise(got[b], ref, 0, 960)
        print(f"  map {b}: gradient vs oracle transpose rel {e:.1e}; max/rms {fmt(st)}", flush=True)
        assert e < tol
        if prec == 1 and b == 0:
            wex, sex = wavelets.analysis_lm(flm[b], P)
            exact = wavelets.analysis_adjoint([2.0 * w for w in wex], np.zeros_like(sex), P)
            e2 = rel(got[b], exact)
            print(f"  map {b}: gradient vs exact FP64 gradient rel {e2:.1e}", flush=True)
            assert e2 < 1e-6
