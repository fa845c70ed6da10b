"""Standalone SO(3) transforms (s2w_wigner_forward / s2w_wigner_inverse) and the
Wigner-Laguerre transforms of the ball (b3w_wl_forward / b3w_wl_inverse) through the C ABI,
against the oracle on seeded band-limited real functions."""
import numpy as np
import pytest

import synthetic as S
from oracle import ball, mw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec,L,N,B", [(0, 16, 3, 2), (0, 64, 4, 1), (0, 33, 1, 3), (0, 100, 2, 2), (1, 48, 3, 2),
                                        (0, 160, 4, 17)])
def test_so3_transforms_against_oracle(prec, L, N, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[so3 prec={prec} L={L} N={N} B={B}]", flush=True)
    plan = s2w.Plan(L, N, 2.0, 0, batch=B, precision=prec, device=0, flags=s2w.S2W_PLAN_WIGNER)
    c = np.stack([S.so3_flmn(L, N, S.stream_key(19, b)) for b in range(B)])
    fr = np.stack([np.real(mw.wigner_inverse(c[b], L, N)) for b in range(B)])
    f = plan.wigner_inverse(torch.from_numpy(c).cuda())
    e_inv = _rel(f.cpu().numpy(), fr)
    back = plan.wigner_forward(torch.from_numpy(fr).cuda()).cpu().numpy()
    e_fwd = _rel(back, c)
    print(f"  inverse rel err {e_inv:.1e}, forward rel err {e_fwd:.1e}", flush=True)
    assert e_inv < 1e-12 and e_fwd < 1e-12
    # coefficients outside |m|, |n| <= l are exactly zero
    for i, n in enumerate(range(-(N - 1), N)):
        for l in range(min(L, N)):
            mask = np.abs(np.arange(-(L - 1), L)) > l
            if abs(n) > l:
                assert np.all(back[:, i, l, :] == 0)
            else:
                assert np.all(back[:, i, l, mask] == 0)


@pytest.mark.parametrize("L,N,P,B", [(8, 3, 6, 1), (16, 1, 10, 2), (32, 4, 8, 1)])
def test_wigner_laguerre_against_oracle(L, N, P, B):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[wigner-laguerre L={L} N={N} P={P} B={B}]", flush=True)
    BP = ball.BallPlan(L, N, P)
    plan = s2w.BallPlan(L, N, P, batch=B, device=0, flags=s2w.S2W_PLAN_WIGNER)
    c = np.stack([S.wl_flmnp(L, N, P, S.stream_key(20, b)) for b in range(B)])
    fr = np.stack([ball.wl_inverse(c[b], BP, N) for b in range(B)])
    f = plan.wl_inverse(torch.from_numpy(c).cuda())
    e_inv = _rel(f.cpu().numpy(), fr)
    back = plan.wl_forward(torch.from_numpy(fr).cuda()).cpu().numpy()
    e_fwd = _rel(back, c)
    for b in range(B):
        assert _rel(back[b], ball.wl_forward(fr[b], BP, N)) < 1e-12
    print(f"  inverse rel err {e_inv:.1e}, forward rel err {e_fwd:.1e}", flush=True)
    assert e_inv < 1e-12 and e_fwd < 1e-12


def test_so3_transforms_need_the_flag():
    torch = _torch()
    import paper_2402_01282_amd as s2w
    plan = s2w.Plan(16, 3, 2.0, 0, device=0)
    with pytest.raises(s2w.S2WError, match="S2W_ESTATE"):
        plan.wigner_forward(torch.zeros(plan.so3_shape, dtype=torch.float64, device="cuda"))
    with pytest.raises(s2w.S2WError, match="S2W_EUNSUPPORTED"):
        s2w.Plan(32, 5, 2.0, 0, device=0, flags=s2w.S2W_PLAN_WIGNER)
