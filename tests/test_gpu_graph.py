"""Plan flags: graph replay (S2W_PLAN_GRAPH) and tile-shape autotuning (S2W_PLAN_TUNE)
give the same coefficients and maps as the plain plan, replay after replay."""
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_and_tune_match_plain_plan(prec):
    torch = _torch()
    import paper_2402_01282_amd as s2w
    L, N, B = 256, 4, 3
    pr = s2w.S2W_MIXED if prec == "mixed" else s2w.S2W_FP64
    print(f"[graph+tune L={L} N={N} B={B} {prec}]", flush=True)
    plain = s2w.Plan(L, N, 2.0, 0, batch=B, precision=pr, device=0)
    fast = s2w.Plan(L, N, 2.0, 0, batch=B, precision=pr, device=0, flags=s2w.S2W_PLAN_TUNE | s2w.S2W_PLAN_GRAPH)
    f = torch.empty(plain.map_shape, dtype=torch.float64, device="cuda")
    wav, scal = fast.empty_wav(), torch.empty(fast.scal_shape, dtype=torch.float64, device="cuda")
    f2 = torch.empty_like(f)
    for rep in range(4):
        # new input each replay, written by eager work between the replays
        maps = np.stack([np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(60 + rep, b)), L)) for b in range(B)])
        f.copy_(torch.from_numpy(maps))
        torch.cuda.synchronize()
        fast.analysis(f, wav, scal)          # replays from the second iteration on
        fast.synthesis(wav, scal, f2)
        torch.cuda.synchronize()
        w_ref, s_ref = plain.analysis(f)
        g_ref = plain.synthesis(w_ref, s_ref)
        torch.cuda.synchronize()
        assert torch.equal(wav, w_ref), rep
        assert torch.equal(scal, s_ref), rep
        assert torch.equal(f2, g_ref), rep
        print(f"  replay {rep}: identical", flush=True)
