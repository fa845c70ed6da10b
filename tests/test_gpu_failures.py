"""Error paths forced from the host, and the ordering of one plan's calls across streams.

* Allocation failure at plan creation (the library's injection hook S2W_FAIL_ALLOC_AT):
  every allocation point of a sphere and a ball plan creation returns S2W_ENOMEM and frees
  what was allocated before it, and the next creation without the hook works.
* Calls on one plan issued on two streams with no synchronisation between them give the
  results of the same calls made one after another (the plan's workspace is shared; the
  library orders the calls with an event)."""
import numpy as np
import pytest

import synthetic as S
from oracle import mw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _walk_allocations(monkeypatch, make, limit=400):
    """Creates plans with the k-th allocation failing, k = 1, 2, ... until a creation
    succeeds; returns the number of failing points seen."""
    import paper_2402_01282_amd as s2w
    torch = _torch()
    # one creation first, so that what the first plan loads once (the code object and its
    # static scratch, runtime pools) is not counted below
    monkeypatch.delenv("S2W_FAIL_ALLOC_AT", raising=False)
    del_plan = make()
    del del_plan
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(0)
    k = 1
    while k <= limit:
        monkeypatch.setenv("S2W_FAIL_ALLOC_AT", str(k))
        try:
            plan = make()
        except s2w.S2WError as e:
            assert e.status == s2w.S2W_ENOMEM, (k, str(e))
            assert "allocation" in str(e)
            k += 1
            continue
        del plan
        break
    monkeypatch.delenv("S2W_FAIL_ALLOC_AT")
    assert 1 < k <= limit, k
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(0)
    # every failed creation returned its memory (the workspaces here are tens of MB per
    # plan, so a leak of them over k failures would show)
    assert free0 - free1 < 64 << 20, (free0 - free1, k)
    return k - 1


def test_alloc_failure_sphere(monkeypatch):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print("[alloc failure sphere]", flush=True)
    n = _walk_allocations(monkeypatch, lambda: s2w.Plan(128, 4, 2.0, 0, batch=4, device=0))
    assert n > 10
    mixed = lambda: s2w.Plan(128, 3, 2.0, 0, batch=8, precision=s2w.S2W_MIXED, device=0,
                             flags=s2w.S2W_PLAN_PERSISTENT | s2w.S2W_PLAN_PRECOMPUTE)
    assert _walk_allocations(monkeypatch, mixed) > n
    # a plan made afterwards works
    plan = s2w.Plan(32, 3, 2.0, 0, device=0)
    f = torch.from_numpy(np.real(mw.sht_inverse(S.sphere_flm(32, S.stream_key(3)), 32))[None].copy()).cuda()
    wav, scal = plan.analysis(f)
    g = plan.synthesis(wav, scal)
    assert torch.max(torch.abs(g - f)).item() < 1e-10


def test_alloc_failure_ball(monkeypatch):
    _torch()
    import paper_2402_01282_amd as s2w
    print("[alloc failure ball]", flush=True)
    n = _walk_allocations(monkeypatch, lambda: s2w.BallPlan(16, 2, 8, device=0, flags=s2w.S2W_PLAN_WIGNER))
    assert n > 10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_streams_one_plan(precision):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    print(f"[two streams {precision}]", flush=True)
    L, N, B = 256, 4, 4
    prec = s2w.S2W_FP64 if precision == "fp64" else s2w.S2W_MIXED
    plan = s2w.Plan(L, N, 2.0, 0, batch=B, precision=prec, device=0)
    maps = []
    for i in range(3):
        flm = np.stack([S.sphere_flm(L, S.stream_key(70 + i, b)) for b in range(B)])
        maps.append(plan.sht_inverse(torch.from_numpy(flm).cuda()))
    # one after another on the current stream
    want = []
    for f in maps:
        wav, scal = plan.analysis(f)
        want.append((wav.clone(), scal.clone(), plan.synthesis(wav, scal).clone()))
    torch.cuda.synchronize()
    # the same calls spread over two streams, no synchronisation in between
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(2):
        for i, f in enumerate(maps):
            s = s1 if (i + rep) % 2 == 0 else s2
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                wav, scal = plan.analysis(f)
                back = plan.synthesis(wav, scal)
            outs.append((i, wav, scal, back))
    torch.cuda.synchronize()
    for i, wav, scal, back in outs:
        w, sc, b = want[i]
        assert torch.equal(wav, w) and torch.equal(scal, sc) and torch.equal(back, b), i
