"""Precompute mode (S2W_PLAN_PRECOMPUTE; Section 4.2, precomputed components): Wigner d
tabulated in device memory for grids of band limit <= 512 and read by the FP64 vector
contractions.  Against the oracle and against the recursion form of the same plan."""
import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec,L,N,J0,B", [(0, 64, 4, 0, 1), (0, 200, 5, 1, 2), (0, 256, 4, 2, 1), (1, 130, 3, 0, 1),
                                           (0, 600, 3, 0, 1)])
def test_precompute_against_oracle(prec, L, N, J0, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[precompute prec={prec} L={L} N={N} J0={J0} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    pre = s2w.Plan(L, N, 2.0, J0, batch=B, precision=prec, device=0, flags=s2w.S2W_PLAN_PRECOMPUTE)
    rec = s2w.Plan(L, N, 2.0, J0, batch=B, precision=prec, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(14, b)) for b in range(B)])
    f = np.stack([np.real(mw.sht_inverse(flm[b], L)) for b in range(B)])
    ft = torch.from_numpy(f).cuda()
    wp, sp = pre.analysis(ft)
    wp, sp = wp.clone(), sp.clone()
    wr, sr = rec.analysis(ft)
    d = (torch.linalg.norm((wp - wr).double()) / torch.linalg.norm(wr.double())).item()
    print(f"  precompute vs recursion rel diff {d:.1e}", flush=True)
    assert d < (1e-13 if prec == 0 else 1e-6)
    views = pre.wav_views(wp)
    for b in sorted({0, B - 1}):
        ow, os_ = wavelets.analysis_lm(flm[b], P)
        es = [_rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(ow)]
        print(f"  map {b} per-scale rel err " + " ".join(f"{e:.1e}" for e in es), flush=True)
        assert max(es) < tol
        assert _rel(sp[b].cpu().numpy(), os_) < tol
    f2 = pre.synthesis(wp, sp).cpu().numpy()
    assert _rel(f2, f) < tol
    # the transpose reads the same tables: dot test on random arrays
    g = torch.from_numpy(np.random.default_rng(L).normal(size=pre.map_shape)).cuda()
    yw = torch.from_numpy(np.random.default_rng(L + 1).normal(size=pre.wav_offset[-1])).to(pre.wav_dtype).cuda()
    ys = torch.from_numpy(np.random.default_rng(L + 2).normal(size=pre.scal_shape)).cuda()
    Aw, As = pre.analysis(g)
    lhs = (torch.dot(Aw.double(), yw.double()) + torch.sum(As * ys)).item()
    rhs = torch.sum(g * pre.analysis_adjoint(yw, ys)).item()
    assert abs(lhs - rhs) < (1e-12 if prec == 0 else 3e-6) * abs(lhs)


@pytest.mark.parametrize("L,N,J0,B", [(64, 4, 0, 4), (128, 3, 1, 8), (256, 4, 0, 16), (1000, 3, 0, 2)])
def test_mixed_precompute_synthesis(L, N, J0, B):
    """Mixed plans in precompute mode: the synthesis contracts through the folded table
    (d T_sigma in three BF16 parts).  Random coefficients (every entry nonzero) against the
    recursion form of the same plan and against the oracle's synthesis, element by element."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    from _gpuutil import elementwise, fmt
    print(f"[mixed precompute synthesis L={L} N={N} J0={J0} B={B}]", flush=True)
    pre = s2w.Plan(L, N, 2.0, J0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=s2w.S2W_PLAN_PRECOMPUTE)
    rec = s2w.Plan(L, N, 2.0, J0, batch=B, precision=s2w.S2W_MIXED, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L + B)
    wav = torch.from_numpy(rng.normal(size=pre.wav_offset[-1]).astype(np.float32)).cuda()
    scal = torch.from_numpy(rng.normal(size=pre.scal_shape)).cuda()
    fp = pre.synthesis(wav, scal).clone()
    fr = rec.synthesis(wav, scal)
    d = (torch.linalg.norm(fp - fr) / torch.linalg.norm(fr)).item()
    print(f"  precompute vs recursion rel diff {d:.1e}", flush=True)
    assert d < 1e-6
    views = pre.wav_views(wav)
    fpn = fp.cpu().numpy()
    for b in sorted({0, B - 1}):
        ref = wavelets.synthesis([v[b].double().cpu().numpy() for v in views], scal[b].cpu().numpy(), P)
        r = _rel(fpn[b], ref)
        e = elementwise(fpn[b], ref, 0)
        print(f"  map {b}: rel {r:.1e} {fmt(e)}", flush=True)
        assert r < 1e-6 and e["all"] < 2e-5
    # analysis (from 8 maps on, its forward SHT runs through the folded FP64 table)
    flm = np.stack([S.sphere_flm(L, S.stream_key(15, b)) for b in range(B)])
    f = torch.from_numpy(np.stack([np.real(mw.sht_inverse(flm[b], L)) for b in range(B)])).cuda()
    wa, sa = pre.analysis(f)
    wa, sa = wa.clone(), sa.clone()
    wb, sb = rec.analysis(f)
    da = (torch.linalg.norm((wa - wb).double()) / torch.linalg.norm(wb.double())).item()
    print(f"  analysis precompute vs recursion rel diff {da:.1e}", flush=True)
    assert da < 1e-6
    va = pre.wav_views(wa)
    ow, os_ = wavelets.analysis_lm(flm[B - 1], P)
    es = [_rel(va[k][B - 1].double().cpu().numpy(), w) for k, w in enumerate(ow)]
    assert max(es) < 1e-6 and _rel(sa[B - 1].cpu().numpy(), os_) < 1e-6, es


@pytest.mark.parametrize("L,B", [(64, 8), (256, 8), (1000, 8)])
def test_fp64_batched_precompute_sht(L, B):
    """Batched plans in precompute mode: the SHTs through the FP64 tables (forward: d T_sigma
    folded; inverse: d) keep FP64 accuracy (both transforms and the analysis against the
    oracle)."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[fp64 batched precompute sht L={L} B={B}]", flush=True)
    N = 3
    pre = s2w.Plan(L, N, 2.0, 0, batch=B, device=0, flags=s2w.S2W_PLAN_PRECOMPUTE)
    P = wavelets.Plan(L, N, 2.0, 0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(16, b)) for b in range(B)])
    f = np.stack([np.real(mw.sht_inverse(flm[b], L)) for b in range(B)])
    ft = torch.from_numpy(f).cuda()
    got = pre.sht_forward(ft).cpu().numpy()
    back = pre.sht_inverse(torch.from_numpy(flm).cuda()).cpu().numpy()
    for b in (0, B - 1):
        assert _rel(got[b], flm[b]) < 1e-12, (b, _rel(got[b], flm[b]))
        assert _rel(back[b], f[b]) < 1e-12, (b, _rel(back[b], f[b]))
    wav, scal = pre.analysis(ft)
    views = pre.wav_views(wav)
    ow, os_ = wavelets.analysis_lm(flm[B - 1], P)
    es = [_rel(views[k][B - 1].cpu().numpy(), w) for k, w in enumerate(ow)]
    print("  per-scale rel err " + " ".join(f"{e:.1e}" for e in es), flush=True)
    assert max(es) < 1e-11
    assert _rel(pre.synthesis(wav, scal).cpu().numpy(), f) < 1e-11
