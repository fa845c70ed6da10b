"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Bar: relative L2 error <= 1e-12 per wavelet scale and per result for the FP64
path (the tolerance the transform's exactness allows in double precision).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _plan(L, N, J0, B=1, lam=2.0):
    import paper_2402_01282_amd as s2w
    return s2w.Plan(L, N, lam, J0, batch=B, device=0)


def _map(L, key):
    return np.real(mw.sht_inverse(S.sphere_flm(L, key), L))


SMALL = [(2, 1, 0), (3, 2, 0), (8, 3, 0), (8, 4, 1), (16, 2, 0), (17, 5, 1), (32, 3, 0), (64, 8, 0), (33, 7, 2)]


@pytest.mark.parametrize("L", [2, 3, 8, 31, 64])
def test_sht_parity(L):
    torch = _torch()
    print(f"[sht L={L}]", flush=True)
    plan = _plan(L, 1, 0)
    flm = S.sphere_flm(L, S.stream_key(20, L))
    f = np.real(mw.sht_inverse(flm, L))
    ft = torch.from_numpy(f[None].copy()).cuda()
    got = plan.sht_forward(ft)[0].cpu().numpy()
    assert _rel(got, mw.sht_forward(f, L)) < TOL
    back = plan.sht_inverse(torch.from_numpy(flm[None].copy()).cuda())[0].cpu().numpy()
    assert _rel(back, f) < TOL


@pytest.mark.parametrize("L,N,J0", SMALL)
def test_analysis_parity(L, N, J0):
    torch = _torch()
    print(f"[analysis L={L} N={N} J0={J0}]", flush=True)
    plan = _plan(L, N, J0)
    P = wavelets.Plan(L, N, 2.0, J0)
    f = _map(L, S.stream_key(21, L))
    wav_ref, scal_ref = wavelets.analysis(f, P)
    wav, scal = plan.analysis(torch.from_numpy(f[None].copy()).cuda())
    views = plan.wav_views(wav)
    assert plan.Lk == P.Lj and plan.Nk == P.Nj and plan.Lphi == P.Lphi
    for k, w in enumerate(wav_ref):
        e = _rel(views[k][0].cpu().numpy(), w)
        assert e < TOL, (k, e)
    assert _rel(scal[0].cpu().numpy(), scal_ref) < TOL


@pytest.mark.parametrize("L,N,J0", SMALL)
def test_synthesis_parity_random_coefficients(L, N, J0):
    """Synthesis is a linear map defined on all sample arrays: compare on random
    (not band-limited) coefficients."""
    torch = _torch()
    print(f"[synthesis L={L} N={N} J0={J0}]", flush=True)
    plan = _plan(L, N, J0)
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L * 100 + N)
    wav = [rng.normal(size=(2 * P.Nj[k] - 1, P.Lj[k], 2 * P.Lj[k] - 1)) for k in range(len(P.scales))]
    scal = rng.normal(size=(P.Lphi, 2 * P.Lphi - 1))
    ref = wavelets.synthesis(wav, scal, P)
    packed = np.concatenate([w.reshape(-1) for w in wav])
    got = plan.synthesis(torch.from_numpy(packed).cuda(), torch.from_numpy(scal[None].copy()).cuda())
    assert _rel(got[0].cpu().numpy(), ref) < TOL


@pytest.mark.parametrize("L,N,J0", SMALL)
def test_adjoint_parity(L, N, J0):
    torch = _torch()
    print(f"[adjoint L={L} N={N} J0={J0}]", flush=True)
    plan = _plan(L, N, J0)
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L * 7 + N)
    gw = [rng.normal(size=(2 * P.Nj[k] - 1, P.Lj[k], 2 * P.Lj[k] - 1)) for k in range(len(P.scales))]
    gs = rng.normal(size=(P.Lphi, 2 * P.Lphi - 1))
    ref = wavelets.analysis_adjoint(gw, gs, P)
    packed = np.concatenate([w.reshape(-1) for w in gw])
    got = plan.analysis_adjoint(torch.from_numpy(packed).cuda(), torch.from_numpy(gs[None].copy()).cuda())
    assert _rel(got[0].cpu().numpy(), ref) < TOL


def test_round_trip_L32_N3():
    """L=32, N=3, lambda=2, J0=0: synthesis(analysis(f)) = f."""
    torch = _torch()
    plan = _plan(32, 3, 0)
    f = _map(32, S.stream_key(1))
    ft = torch.from_numpy(f[None].copy()).cuda()
    wav, scal = plan.analysis(ft)
    f2 = plan.synthesis(wav, scal)[0].cpu().numpy()
    assert _rel(f2, f) < TOL


def test_parity_L256_N4_J0_2():
    """L=256, N=4, lambda=2, J0=2, one map: every
    scale of the analysis, the synthesis and the round trip against the oracle."""
    torch = _torch()
    print("[parity L=256 N=4 J0=2]", flush=True)
    L, N, J0 = 256, 4, 2
    plan = _plan(L, N, J0)
    P = wavelets.Plan(L, N, 2.0, J0)
    f = _map(L, S.stream_key(2))
    wav_ref, scal_ref = wavelets.analysis(f, P)
    ft = torch.from_numpy(f[None].copy()).cuda()
    wav, scal = plan.analysis(ft)
    views = plan.wav_views(wav)
    for k, w in enumerate(wav_ref):
        assert _rel(views[k][0].cpu().numpy(), w) < TOL, k
    assert _rel(scal[0].cpu().numpy(), scal_ref) < TOL
    f2 = plan.synthesis(wav, scal)[0].cpu().numpy()
    assert _rel(f2, f) < TOL
    ref_syn = wavelets.synthesis(wav_ref, scal_ref, P)
    assert _rel(f2, ref_syn) < TOL


def test_batch_independent_maps():
    torch = _torch()
    L, N, J0, B = 16, 3, 0, 3
    plan = _plan(L, N, J0, B=B)
    P = wavelets.Plan(L, N, 2.0, J0)
    maps = np.stack([_map(L, S.stream_key(3, b)) for b in range(B)])
    wav, scal = plan.analysis(torch.from_numpy(maps).cuda())
    views = plan.wav_views(wav)
    for b in range(B):
        wr, sr = wavelets.analysis(maps[b], P)
        for k, w in enumerate(wr):
            assert _rel(views[k][b].cpu().numpy(), w) < TOL
        assert _rel(scal[b].cpu().numpy(), sr) < TOL
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    assert _rel(f2, maps) < TOL


def test_deterministic():
    """Two runs are bitwise identical (no floating-point atomics)."""
    torch = _torch()
    plan = _plan(64, 8, 0)
    f = torch.from_numpy(_map(64, S.stream_key(4))[None].copy()).cuda()
    w1, s1 = plan.analysis(f)
    w1 = w1.clone()
    w2, s2 = plan.analysis(f)
    assert torch.equal(w1, w2)


def test_batched_fp64_matrix_core_path():
    """Launches of 16 or more maps take the batched FP64 matrix-core contractions (one
    recursion per 32 columns); 17 maps (a ragged second column group) at L = 70 (a
    ragged theta tile, polar samples active) against the oracle, map by map."""
    torch = _torch()
    L, N, J0, B = 70, 3, 0, 17
    print(f"[batched FP64 L={L} N={N} B={B}]", flush=True)
    plan = _plan(L, N, J0, B=B)
    P = wavelets.Plan(L, N, 2.0, J0)
    maps = np.stack([_map(L, S.stream_key(5, b)) for b in range(B)])
    flm = plan.sht_forward(torch.from_numpy(maps).cuda()).cpu().numpy()
    wav, scal = plan.analysis(torch.from_numpy(maps).cuda())
    views = plan.wav_views(wav)
    for b in range(B):
        assert _rel(flm[b], mw.sht_forward(maps[b], L)) < TOL
        wr, sr = wavelets.analysis(maps[b], P)
        for k, w in enumerate(wr):
            assert _rel(views[k][b].cpu().numpy(), w) < TOL, (b, k)
        assert _rel(scal[b].cpu().numpy(), sr) < TOL
    f2 = plan.synthesis(wav, scal).cpu().numpy()
    for b in range(B):
        assert _rel(f2[b], maps[b]) < TOL
    g = plan.sht_inverse(torch.from_numpy(flm).cuda()).cpu().numpy()
    assert _rel(g, maps) < TOL
