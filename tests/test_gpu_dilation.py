"""Dilations other than 2 on the device (Section 3.3: band limits L_j = ceil(lambda^(j+1)),
supports lambda^(j-1) < l < lambda^(j+1)), in both precisions, against the oracle; and the
mixed form's determinism (fixed-order sums: two runs are bitwise equal)."""
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


@pytest.mark.parametrize("prec,L,N,lam,J0,B", [(0, 64, 3, 3.0, 0, 1), (0, 100, 4, 1.5, 2, 2), (1, 96, 3, 3.0, 1, 4),
                                                (1, 128, 4, 1.5, 0, 8), (1, 300, 3, 2.5, 1, 2)])
def test_dilation_parity(prec, L, N, lam, J0, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[dilation prec={prec} L={L} N={N} lambda={lam} J0={J0} B={B}]", flush=True)
    tol = 1e-12 if prec == 0 else 1e-6
    plan = s2w.Plan(L, N, lam, J0, batch=B, precision=prec, device=0)
    P = wavelets.Plan(L, N, lam, J0)
    assert plan.Lk == P.Lj and plan.Nk == P.Nj and plan.Lphi == P.Lphi
    flm = np.stack([S.sphere_flm(L, S.stream_key(11, b)) for b in range(B)])
    f = np.stack([np.real(mw.sht_inverse(flm[b], L)) for b in range(B)])
    ft = torch.from_numpy(f).cuda()
    wav, scal = plan.analysis(ft)
    views = plan.wav_views(wav)
    for b in sorted({0, B - 1}):
        wr, sr = wavelets.analysis_lm(flm[b], P)
        es = [_rel(views[k][b].double().cpu().numpy(), w) for k, w in enumerate(wr)]
        print(f"  map {b} per-scale rel err " + " ".join(f"{e:.1e}" for e in es), flush=True)
        assert max(es) < tol
        assert _rel(scal[b].cpu().numpy(), sr) < tol
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    assert _rel(f2, f) < tol


def test_mixed_deterministic():
    """The mixed form at batch 64 with the tuned kernels: two analyses and two syntheses are
    bitwise identical (no floating-point atomics; the persistent launch's work counters
    only assign work)."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    L, N, B = 256, 4, 64
    plan = s2w.Plan(L, N, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0,
                    flags=s2w.S2W_PLAN_TUNE | s2w.S2W_PLAN_PERSISTENT)
    p64 = s2w.Plan(L, N, 2.0, 0, batch=B, device=0)
    flm = np.stack([S.sphere_flm(L, S.stream_key(12, b)) for b in range(B)])
    f = p64.sht_inverse(torch.from_numpy(flm).cuda())
    w1, s1 = plan.analysis(f)
    w1, s1 = w1.clone(), s1.clone()
    w2, s2 = plan.analysis(f)
    assert torch.equal(w1, w2) and torch.equal(s1, s2)
    g1 = plan.synthesis(w1, s1).clone()
    g2 = plan.synthesis(w1, s1)
    assert torch.equal(g1, g2)
