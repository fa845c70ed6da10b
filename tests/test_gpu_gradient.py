"""Gradients through the wavelet analysis (hand-written adjoint behind
torch.autograd.Function) for the loss sum_j sum W^j^2 over the wavelet scales."""
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


def _loss(plan, x):
    import paper_2402_01282_amd as s2w
    wav, scal = s2w.analysis(x, plan)
    return (wav * wav).sum()


def test_gradient_central_differences_L16():
    """Quadratic loss: central differences are exact up to rounding."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    L, N = 16, 4
    plan = s2w.Plan(L, N, 2.0, 0, device=0)
    f = torch.from_numpy(np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(4)), L))[None].copy()).cuda()
    x = f.clone().requires_grad_(True)
    loss = _loss(plan, x)
    loss.backward()
    g = x.grad[0].cpu().numpy()
    rng = np.random.default_rng(0)
    h = 1e-3
    with torch.no_grad():
        for _ in range(12):
            i, j = int(rng.integers(L)), int(rng.integers(2 * L - 1))
            e = torch.zeros_like(f)
            e[0, i, j] = h
            fd = ((_loss(plan, f + e) - _loss(plan, f - e)) / (2 * h)).item()
            assert abs(fd - g[i, j]) < 1e-9 * max(1.0, abs(g[i, j])), (i, j, fd, g[i, j])


@pytest.mark.parametrize("L,N,J0", [(16, 4, 0), (64, 8, 0), (128, 3, 1)])
def test_gradient_against_oracle_adjoint(L, N, J0):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    plan = s2w.Plan(L, N, 2.0, J0, device=0)
    P = wavelets.Plan(L, N, 2.0, J0)
    f = np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(40, L)), L))
    x = torch.from_numpy(f[None].copy()).cuda().requires_grad_(True)
    _loss(plan, x).backward()
    wav, scal = wavelets.analysis(f, P)
    ref = wavelets.analysis_adjoint([2 * w for w in wav], np.zeros_like(scal), P)
    got = x.grad[0].cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def test_gradient_L1024_N8_directional_derivative():
    """L=1024, N=8: the gradient of sum W^2 equals 2 A^T A f; check <grad, v> against
    the directional derivative 2 <A f, A v> for a random direction v."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print("[gradient L=1024]", flush=True)
    L, N = 1024, 8
    plan = s2w.Plan(L, N, 2.0, 0, device=0)
    flm = S.sphere_flm(L, S.stream_key(4))
    f = plan.sht_inverse(torch.from_numpy(flm[None].copy()).cuda())
    x = f.clone().requires_grad_(True)
    _loss(plan, x).backward()
    gen = torch.Generator(device="cuda").manual_seed(9)
    v = torch.randn(plan.map_shape, dtype=torch.float64, device="cuda", generator=gen)
    with torch.no_grad():
        Af, _ = plan.analysis(f)
        Af = Af.clone()
        Av, _ = plan.analysis(v)
        dd = 2.0 * torch.dot(Af, Av).item()
    gv = torch.sum(x.grad * v).item()
    assert abs(gv - dd) < 1e-11 * abs(dd)


@pytest.mark.parametrize("L,N,B", [(16, 3, 2), (64, 4, 3)])
def test_mixed_gradient(L, N, B):
    """Mixed plans: the adjoint (in the forward precision split: FP32 matrix-core DFTs
    and theta sum on the FP32 cotangents, FP64 recursion and sums) is within 1e-6 of the
    oracle's adjoint of the same cotangents, and the gradient of the FP32 loss is within
    1e-6 of the exact FP64 gradient."""
    torch = _torch()
    import paper_2402_01282_amd as s2w
    plan = s2w.Plan(L, N, 2.0, 0, batch=B, precision=s2w.S2W_MIXED, device=0)
    P = wavelets.Plan(L, N, 2.0, 0)
    maps = np.stack([np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(41, b)), L)) for b in range(B)])
    x = torch.from_numpy(maps).cuda().requires_grad_(True)
    wav, scal = s2w.analysis(x, plan)
    (wav.double() ** 2).sum().backward()
    got = x.grad.cpu().numpy()
    views = plan.wav_views(wav.detach())
    for b in range(B):
        gw = [2 * v[b].double().cpu().numpy() for v in views]
        ref = wavelets.analysis_adjoint(gw, np.zeros(plan.scal_shape[1:]), P)
        assert np.linalg.norm(got[b] - ref) / np.linalg.norm(ref) < 1e-6
        wex, sex = wavelets.analysis(maps[b], P)
        exact = wavelets.analysis_adjoint([2 * w for w in wex], np.zeros_like(sex), P)
        assert np.linalg.norm(got[b] - exact) / np.linalg.norm(exact) < 1e-6
