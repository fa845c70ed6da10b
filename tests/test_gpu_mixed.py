"""Mixed-precision batched form (S2W_MIXED): FP64 Wigner-d recursion, FP32
matrix-core contractions and DFTs, FP64 scale sums.  Gate: <= 1e-6 relative L2
error against the FP64 oracle for every wavelet scale and for every result."""
import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _plan(L, N, J0, B):
    import paper_2402_01282_amd as s2w
    return s2w.Plan(L, N, 2.0, J0, batch=B, precision=s2w.S2W_MIXED, device=0)


@pytest.mark.parametrize("L,N,J0,B", [(8, 3, 0, 2), (32, 3, 0, 32), (64, 8, 0, 32), (33, 4, 1, 5), (128, 4, 2, 64),
                                     (64, 4, 0, 1), (130, 3, 1, 1), (96, 5, 0, 2)])
def test_mixed_analysis_and_synthesis(L, N, J0, B):
    torch = _torch()
    print(f"[mixed L={L} N={N} J0={J0} B={B}]", flush=True)
    plan = _plan(L, N, J0, B)
    P = wavelets.Plan(L, N, 2.0, J0)
    maps = np.stack([np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(3, b)), L)) for b in range(B)])
    ft = torch.from_numpy(maps).cuda()
    wav, scal = plan.analysis(ft)
    assert wav.dtype == torch.float32
    views = plan.wav_views(wav)
    for b in sorted({0, B - 1}):
        wr, sr = wavelets.analysis(maps[b], P)
        for k, w in enumerate(wr):
            e = _rel(views[k][b].double().cpu().numpy(), w)
            assert e < TOL, (b, k, e)
        assert _rel(scal[b].cpu().numpy(), sr) < TOL
        # synthesis of the oracle's coefficients (rounded to FP32 on input)
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    assert _rel(f2, maps) < TOL
    # synthesis parity on the oracle's own coefficients for one map (others zero)
    wr, sr = wavelets.analysis(maps[0], P)
    packed = torch.zeros(plan.wav_offset[-1], dtype=torch.float32, device="cuda")
    pv = plan.wav_views(packed)
    sc = torch.zeros(plan.scal_shape, dtype=torch.float64, device="cuda")
    for k, w in enumerate(wr):
        pv[k][0].copy_(torch.from_numpy(w).float())
    sc[0].copy_(torch.from_numpy(sr))
    g = plan.synthesis(packed, sc)[0].cpu().numpy()
    assert _rel(g, wavelets.synthesis(wr, sr, P)) < TOL


def test_mixed_L512_N4_B64_all_scales():
    """64 maps at L=512, N=4, lambda=2, all scales.  Round trip for every
    map; every scale against the oracle for two maps of the batch."""
    torch = _torch()
    print("[mixed L=512 N=4 B=64]", flush=True)
    L, N, J0, B = 512, 4, 0, 64
    plan = _plan(L, N, J0, B)
    P = wavelets.Plan(L, N, 2.0, J0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(3, b)) for b in range(B)])
    import paper_2402_01282_amd as s2w
    p64 = s2w.Plan(L, N, 2.0, J0, batch=B, device=0)
    f = p64.sht_inverse(torch.from_numpy(flm).cuda())
    wav, scal = plan.analysis(f)
    f2 = plan.synthesis(wav, scal)
    errs = [(torch.linalg.norm(f2[b] - f[b]) / torch.linalg.norm(f[b])).item() for b in range(B)]
    print(f"  round trip rel err: max {max(errs):.2e} mean {np.mean(errs):.2e}", flush=True)
    assert max(errs) < TOL
    views = plan.wav_views(wav)
    for b in (0, 37):
        wr, sr = wavelets.analysis_lm(flm[b], P)
        es = [_rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(wr)]
        print(f"  map {b} per-scale rel err: " + " ".join(f"{x:.1e}" for x in es), flush=True)
        assert max(es) < TOL
        assert _rel(scal[b].cpu().numpy(), sr) < TOL


def test_mixed_ragged_L1000_N3():
    """L=1000 (above 960: the 16-wave theta contraction, whose last wave holds 40 samples),
    N=3, three maps: every scale of the analysis against the oracle for two maps; the
    synthesis of the oracle's coefficients against the input map (the transform
    reconstructs exactly, so that map is the synthesis' exact value); the round trip."""
    torch = _torch()
    print("[mixed L=1000 N=3 B=3]", flush=True)
    L, N, J0, B = 1000, 3, 0, 3
    import paper_2402_01282_amd as s2w
    plan = _plan(L, N, J0, B)
    P = wavelets.Plan(L, N, 2.0, J0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(5, b)) for b in range(B)])
    p64 = s2w.Plan(L, N, 2.0, J0, batch=B, device=0)
    f = p64.sht_inverse(torch.from_numpy(flm).cuda())
    wav, scal = plan.analysis(f)
    views = plan.wav_views(wav)
    packed = torch.zeros(plan.wav_offset[-1], dtype=torch.float32, device="cuda")
    pv = plan.wav_views(packed)
    sc = torch.zeros(plan.scal_shape, dtype=torch.float64, device="cuda")
    for b in (0, B - 1):
        wr, sr = wavelets.analysis_lm(flm[b], P)
        es = [_rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(wr)]
        print(f"  map {b} per-scale rel err: " + " ".join(f"{x:.1e}" for x in es), flush=True)
        assert max(es) < TOL
        assert _rel(scal[b].cpu().numpy(), sr) < TOL
        for k, w in enumerate(wr):
            pv[k][b].copy_(torch.from_numpy(w).float())
        sc[b].copy_(torch.from_numpy(sr))
    g = plan.synthesis(packed, sc)
    for b in (0, B - 1):
        e = (torch.linalg.norm(g[b] - f[b]) / torch.linalg.norm(f[b])).item()
        print(f"  map {b} synthesis of the oracle's coefficients rel err {e:.2e}", flush=True)
        assert e < TOL
    assert torch.count_nonzero(g[1]).item() == 0
    f2 = plan.synthesis(wav, scal)
    errs = [(torch.linalg.norm(f2[b] - f[b]) / torch.linalg.norm(f[b])).item() for b in range(B)]
    print(f"  round trip rel err: max {max(errs):.2e}", flush=True)
    assert max(errs) < TOL


@pytest.mark.parametrize("L,N,B", [(128, 4, 1), (128, 4, 8), (256, 3, 2)])
def test_mixed_routes_agree(L, N, B):
    """The autotuned plan (matrix-core or FP64 vector contractions per degree group, chosen
    by timing) and the untuned plan (batch heuristic) give the same coefficients and
    round trip to the precision of the mixed form."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[mixed routes L={L} N={N} B={B}]", flush=True)
    maps = np.stack([np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(8, b)), L)) for b in range(B)])
    f = torch.from_numpy(maps).cuda()
    outs = []
    for flags in (0, s2w.S2W_PLAN_TUNE):
        plan = _plan_flags(L, N, 0, B, flags)
        wav, scal = plan.analysis(f)
        f2 = plan.synthesis(wav, scal)
        outs.append((wav.double().cpu().numpy(), f2.cpu().numpy()))
        assert _rel(f2.cpu().numpy(), maps) < TOL
    assert _rel(outs[1][0], outs[0][0]) < TOL
    assert _rel(outs[1][1], outs[0][1]) < TOL


def _plan_flags(L, N, J0, B, flags):
    import paper_2402_01282_amd as s2w
    return s2w.Plan(L, N, 2.0, J0, batch=B, precision=s2w.S2W_MIXED, device=0, flags=flags)


@pytest.mark.parametrize("L,N,B", [(256, 4, 16), (1000, 3, 4)])
def test_mixed_persistent_matches_per_group(L, N, B):
    """S2W_PLAN_PERSISTENT: the analysis l-contraction of every matrix-core degree group in one
    launch over the cost-sorted work list gives the same coefficients as one launch per group
    (the same per-unit arithmetic, so equal to rounding), and the oracle's on one map."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[mixed persistent L={L} N={N} B={B}]", flush=True)
    flm = np.stack([S.sphere_flm(L, S.stream_key(9, b)) for b in range(B)])
    p64 = s2w.Plan(L, N, 2.0, 0, batch=B, device=0)
    f = p64.sht_inverse(torch.from_numpy(flm).cuda())
    w0, s0 = _plan_flags(L, N, 0, B, 0).analysis(f)
    plan = _plan_flags(L, N, 0, B, s2w.S2W_PLAN_PERSISTENT)
    w1, s1 = plan.analysis(f)
    d = (torch.linalg.norm((w1 - w0).double()) / torch.linalg.norm(w0.double())).item()
    print(f"  persistent vs per-group rel diff {d:.1e}", flush=True)
    assert d < 1e-7
    P = wavelets.Plan(L, N, 2.0, 0)
    wr, _ = wavelets.analysis_lm(flm[B - 1], P)
    views = plan.wav_views(w1)
    es = [_rel(views[k][B - 1].double().cpu().numpy(), w) for k, w in enumerate(wr)]
    print("  per-scale rel err " + " ".join(f"{x:.1e}" for x in es), flush=True)
    assert max(es) < TOL
    f2 = plan.synthesis(w1, s1)
    assert (torch.linalg.norm(f2 - f) / torch.linalg.norm(f)).item() < TOL
