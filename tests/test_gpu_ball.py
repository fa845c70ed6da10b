"""Ball wavelet transform (b3w_* entry points) against the FP64 ball oracle."""
import numpy as np
import pytest

import synthetic as S
from oracle import ball

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _maps(L, P, BP, B, seed):
    flmp = [S.ball_flmp(L, P, S.stream_key(seed, b)) for b in range(B)]
    return flmp, np.stack([ball.sl_inverse(x, BP) for x in flmp])


@pytest.mark.parametrize("L,N,P,J0,J0p,tau,B", [(8, 3, 8, 0, 0, 1.0, 2), (12, 4, 10, 1, 1, 0.7, 1),
                                               (16, 2, 20, 0, 2, 1.3, 1), (9, 1, 5, 0, 0, 1.0, 3)])
def test_ball_fp64_against_oracle(L, N, P, J0, J0p, tau, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[ball L={L} N={N} P={P} J0={J0} J0p={J0p} tau={tau} B={B}]", flush=True)
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, J0, J0p, tau)
    plan = s2w.BallPlan(L, N, P, 2.0, 2.0, J0, J0p, tau, batch=B, device=0)
    np.testing.assert_allclose(plan.nodes, BP.rad.r, rtol=1e-13)
    assert plan.Pk == BP.Pj and plan.Lk == BP.ang.Lj
    _, f = _maps(L, P, BP, B, 5)
    ft = torch.from_numpy(f).cuda()
    wav, scal = plan.analysis(ft)
    views = plan.wav_views(wav)
    for b in range(B):
        wr, sr = ball.analysis(f[b], BP)
        assert _rel(scal[b].cpu().numpy(), sr) < 1e-12
        for key, w in wr.items():
            e = _rel(views[key][b].cpu().numpy(), w)
            assert e < 1e-12, (b, key, e)
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    assert _rel(f2, f) < 1e-12
    # synthesis of the oracle's own coefficients (map 0; the others zero)
    wr, sr = ball.analysis(f[0], BP)
    packed = torch.zeros_like(wav)
    pv = plan.wav_views(packed)
    for key, w in wr.items():
        pv[key][0].copy_(torch.from_numpy(w))
    sc = torch.zeros_like(scal)
    sc[0].copy_(torch.from_numpy(sr))
    g = plan.synthesis(packed, sc)[0].cpu().numpy()
    assert _rel(g, ball.synthesis(wr, sr, BP)) < 1e-12


@pytest.mark.parametrize("prec_tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_ball_L128_P128_N4_B4(prec_tol):
    """L = P = 128, N = 4, lambda = nu = 2, batch 4: round trip of every map, and
    sampled (radial scale, angular scale, shell) blocks of map 0 against the oracle."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    prec, tol = prec_tol
    print(f"[ball L=128 P=128 N=4 B=4 {prec}]", flush=True)
    L, N, P, B = 128, 4, 128, 4
    BP = ball.BallPlan(L, N, P)
    plan = s2w.BallPlan(L, N, P, batch=B, device=0,
                        precision=s2w.S2W_MIXED if prec == "mixed" else s2w.S2W_FP64)
    flmp, f = _maps(L, P, BP, B, 5)
    ft = torch.from_numpy(f).cuda()
    wav, scal = plan.analysis(ft)
    f2 = plan.synthesis(wav, scal)
    errs = [(torch.linalg.norm(f2[b] - ft[b]) / torch.linalg.norm(ft[b])).item() for b in range(B)]
    print(f"  round trip rel err: max {max(errs):.2e}", flush=True)
    assert max(errs) < tol
    views = plan.wav_views(wav)
    nr, na = len(BP.rscales), len(BP.ang.scales)
    for (i, k, s) in [(nr - 1, na - 1, 0), (nr - 1, na - 1, BP.Pj[nr - 1] - 1), (nr - 2, na - 2, 7),
                      (3, na - 1, 2), (nr - 1, 4, 100)]:
        g = ball._shell_coeffs(flmp[0], BP, i)[s:s + 1]
        ref = ball._angular_scale(g, BP, k, True)[0]
        got = views[(i, k)][0, s].double().cpu().numpy()
        e = _rel(got, ref)
        print(f"  block (i={i}, k={k}) shell {s}: rel err {e:.2e}", flush=True)
        assert e < tol


def test_ball_mixed_small():
    torch = _torch()
    import paper_2402_01282_amd as s2w
    L, N, P, B = 16, 3, 12, 3
    BP = ball.BallPlan(L, N, P)
    plan = s2w.BallPlan(L, N, P, batch=B, device=0, precision=s2w.S2W_MIXED)
    _, f = _maps(L, P, BP, B, 6)
    wav, scal = plan.analysis(torch.from_numpy(f).cuda())
    assert wav.dtype == torch.float32
    views = plan.wav_views(wav)
    wr, sr = ball.analysis(f[1], BP)
    for key, w in wr.items():
        assert _rel(views[key][1].double().cpu().numpy(), w) < 1e-6, key
    assert _rel(scal[1].cpu().numpy(), sr) < 1e-6
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    assert _rel(f2, f) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_spherical_laguerre_transform_against_oracle(prec):
    """b3w_sl_forward / b3w_sl_inverse (FP64 for either plan precision) against the
    oracle's forward and inverse spherical-Laguerre transforms, 3 maps, ragged L and P."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    L, N, P, B = 13, 3, 11, 3
    print(f"[spherical-Laguerre L={L} P={P} B={B} {prec}]", flush=True)
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, 0, 0, 0.8)
    plan = s2w.BallPlan(L, N, P, 2.0, 2.0, 0, 0, 0.8, batch=B, device=0,
                        precision=s2w.S2W_MIXED if prec == "mixed" else s2w.S2W_FP64)
    flmp, f = _maps(L, P, BP, B, 9)
    got = plan.sl_forward(torch.from_numpy(f).cuda()).cpu().numpy()
    for b in range(B):
        assert _rel(got[b], ball.sl_forward(f[b], BP)) < 1e-12, b
        assert _rel(got[b], flmp[b]) < 1e-12, b
    back = plan.sl_inverse(torch.from_numpy(np.stack(flmp))).cpu().numpy()
    assert _rel(back, f) < 1e-12


@pytest.mark.parametrize("prec_tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_ball_paper_setting_L256_P256_N1(prec_tol):
    """The ball at the setting of the paper's ball benchmark (Section 5.4, Table 2): N = 1,
    P = L = 256, lambda = nu = 2, J0 = J0' = 0, one map.  Round trip, the scaling
    coefficients' radial projection, and sampled (radial scale, angular scale, shell) blocks
    against the oracle (its per-block functions on the seeded coefficients)."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    prec, tol = prec_tol
    print(f"[ball paper setting L=P=256 N=1 {prec}]", flush=True)
    L, N, P = 256, 1, 256
    BP = ball.BallPlan(L, N, P)
    plan = s2w.BallPlan(L, N, P, batch=1, device=0,
                        precision=s2w.S2W_MIXED if prec == "mixed" else s2w.S2W_FP64)
    assert plan.Pk == BP.Pj and plan.Lk == BP.ang.Lj
    flmp = S.ball_flmp(L, P, S.stream_key(13))
    f = plan.sl_inverse(torch.from_numpy(flmp[None].copy()))
    wav, scal = plan.analysis(f)
    f2 = plan.synthesis(wav, scal)
    e = (torch.linalg.norm(f2 - f) / torch.linalg.norm(f)).item()
    print(f"  round trip rel err {e:.2e}", flush=True)
    assert e < tol
    views = plan.wav_views(wav)
    nr, na = len(BP.rscales), len(BP.ang.scales)
    for (i, k, s) in [(0, na - 1, 1), (3, na - 1, 5), (nr - 1, na - 1, 0), (nr - 1, na - 2, 200), (nr - 2, 3, 77),
                      (5, 0, 31)]:
        g = ball._shell_coeffs(flmp, BP, i)[s:s + 1]
        ref = ball._angular_scale(g, BP, k, True)[0]
        got = views[(i, k)][0, s].double().cpu().numpy()
        e = _rel(got, ref)
        print(f"  block (i={i}, k={k}) shell {s}: rel err {e:.2e}", flush=True)
        assert e < tol
