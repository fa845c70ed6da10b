"""Full-size checks at L=1024, N=8, lambda=2, J0=0 (FP64).

The spherical-harmonic transforms against the oracle, and properties that hold
at any size: exact round trip, adjoint dot products, linearity.  Every wavelet
scale is compared with the oracle element by element in test_gpu_headline.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets

pytestmark = pytest.mark.gpu

L, N, LAM, J0 = 1024, 8, 2.0, 0
TOL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def setup():
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print("[fullsize] plan L=1024 N=8", flush=True)
    plan = s2w.Plan(L, N, LAM, J0, batch=1, device=0)
    flm = S.sphere_flm(L, S.stream_key(4))
    f = plan.sht_inverse(torch.from_numpy(flm[None].copy()).cuda())
    torch.cuda.synchronize()
    return plan, flm, f


def test_fullsize_sht_against_oracle(setup):
    """GPU inverse SHT of the Gaussian field vs the oracle's, and GPU forward SHT
    recovers the coefficients (exact on MW sampling)."""
    plan, flm, f = setup
    print("[fullsize] sht", flush=True)
    fo = np.real(mw.sht_inverse(flm, L))
    assert _rel(f[0].cpu().numpy(), fo) < TOL
    back = plan.sht_forward(f)[0].cpu().numpy()
    assert _rel(back, flm) < TOL


def test_fullsize_round_trip(setup):
    """synthesis(analysis(f)) = f at L=1024 (exact reconstruction)."""
    plan, flm, f = setup
    print("[fullsize] round trip", flush=True)
    wav, scal = plan.analysis(f)
    f2 = plan.synthesis(wav, scal)
    assert _rel(f2[0].cpu().numpy(), f[0].cpu().numpy()) < TOL


def test_fullsize_adjoint_dot(setup):
    """<A x, y> = <x, A^T y> with x, y random (not band-limited) at full size."""
    torch = _torch()
    plan, flm, f = setup
    print("[fullsize] adjoint dot", flush=True)
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn(plan.map_shape, dtype=torch.float64, device="cuda", generator=g)
    yw = torch.randn(plan.wav_offset[-1], dtype=torch.float64, device="cuda", generator=g)
    ys = torch.randn(plan.scal_shape, dtype=torch.float64, device="cuda", generator=g)
    Aw, As = plan.analysis(x)
    lhs = (torch.dot(Aw, yw) + torch.sum(As * ys)).item()
    ATy = plan.analysis_adjoint(yw, ys)
    rhs = torch.sum(x * ATy).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_fullsize_linearity(setup):
    """A(f + 2 g) = A f + 2 A g for two Gaussian fields at full size."""
    torch = _torch()
    plan, flm, f = setup
    flm2 = S.sphere_flm(L, S.stream_key(44))
    f2 = plan.sht_inverse(torch.from_numpy(flm2[None].copy()).cuda())
    w1, s1 = plan.analysis(f)
    w1 = w1.clone()
    s1 = s1.clone()
    w2, s2 = plan.analysis(f2)
    w3, s3 = plan.analysis(f + 2.0 * f2)
    assert (torch.linalg.norm(w3 - (w1 + 2.0 * w2)) / torch.linalg.norm(w3)).item() < TOL
