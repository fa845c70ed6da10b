"""Benchmark: directional wavelet analysis + synthesis throughput on one MI355X.

Metric: maps per second for one analysis + synthesis round trip of real maps
on McEwen-Wiaux sampling (default workload L=1024, N=8, lambda=2, J0=0; the
paper's protocol of Section 4.4 without its harmonic-space bookends).  Inputs
are synthetic Gaussian random fields (C_l = 1/(l+1)^2) synthesised on the GPU
and resident in HBM before timing starts.

Prints one JSON line.  `roofline` reports the dominant kernel: algorithmic
work per launch (counted by the library from each launch's parameters) over
its average duration measured with HIP events on the stream it runs on.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "fp64_valu": 78.6e12,
    "fp32_valu": 157.3e12,
    "fp32_mfma": 157.3e12,
    "hbm": 8.0e12,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--N", type=int, default=8)
    ap.add_argument("--lam", type=float, default=2.0)
    ap.add_argument("--J0", type=int, default=0)
    ap.add_argument("--batch", type=int, default=None, help="maps per call (default 1 for fp64, 64 for mixed)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay each transform as a HIP graph (no per-kernel timing)")
    ap.add_argument("--no-tune", action="store_true", help="skip the plan's tile-shape autotuning")
    return ap.parse_args()


def cpu_baseline(L, N, lam, J0):
    """Time the oracle on a bounded sample of the workload: the spherical-harmonic
    transform pair at full size plus the analysis and synthesis of the TOP wavelet
    scale (the largest single piece), scaled to one full round trip by the oracle's
    own cost model sum_j L_j^3 N_j over the scales."""
    import numpy as np

    import synthetic
    from oracle import mw, wavelets

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    P = wavelets.Plan(L, N, lam, J0)
    flm = synthetic.sphere_flm(L, synthetic.stream_key(4))
    mw.delta_table(L)
    t0 = time.perf_counter()
    f = np.real(mw.sht_inverse(flm, L))
    flm2 = mw.sht_forward(f, L)
    t_sht = time.perf_counter() - t0
    k = len(P.scales) - 1
    Lj, Nj = P.Lj[k], P.Nj[k]
    fl = flm2[:Lj, L - Lj:L + Lj - 1]
    lj = np.arange(Lj)
    what = (8 * np.pi ** 2 / (2 * lj + 1))[None, :, None] * fl[None] * np.conj(P.psi(k)).T[:, :, None]
    t0 = time.perf_counter()
    w = mw.wigner_inverse(what, Lj, Nj)
    _ = mw.wigner_forward(np.real(w), Lj, Nj)
    t_top = time.perf_counter() - t0
    cost = [P.Lj[i] ** 3 * P.Nj[i] for i in range(len(P.scales))]
    t_round = t_sht + t_top * sum(cost) / cost[k]
    return {"value": 1.0 / t_round, "unit": "maps/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle SHT pair at L={L} plus analysis+synthesis of the top scale "
                       f"(L_j={Lj}, N_j={Nj}) in {t_sht + t_top:.1f} s, scaled to the full round trip by "
                       f"sum_j L_j^3 N_j / (L_J^3 N_J) = {sum(cost) / cost[k]:.3f}")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2402_01282_amd as s2w
    import synthetic

    L, N, lam, J0 = args.L, args.N, args.lam, args.J0
    mixed = args.precision == "mixed"
    B = args.batch if args.batch is not None else (64 if mixed else 1)
    print(f"[bench] L={L} N={N} lambda={lam} J0={J0} batch={B} precision={args.precision}",
          file=sys.stderr, flush=True)
    flags = (0 if args.no_tune else s2w.S2W_PLAN_TUNE) | (s2w.S2W_PLAN_GRAPH if args.graph else 0)
    plan = s2w.Plan(L, N, lam, J0, batch=B, device=0, precision=s2w.S2W_MIXED if mixed else s2w.S2W_FP64,
                    flags=flags)
    # synthetic Gaussian random fields, synthesised on the GPU (FP64 inverse SHT, one map per call)
    synth = s2w.Plan(L, 1, lam, 0, batch=1, device=0)
    f = torch.empty(plan.map_shape, dtype=torch.float64, device="cuda")
    for b in range(B):
        flm = synthetic.sphere_flm(L, synthetic.stream_key(4, b))
        f[b].copy_(synth.sht_inverse(torch.from_numpy(flm[None].copy()).cuda())[0])
    del synth
    wav = plan.empty_wav()
    scal = torch.empty(plan.scal_shape, dtype=torch.float64, device="cuda")
    f2 = torch.empty_like(f)
    torch.cuda.synchronize()

    def step():
        plan.analysis(f, wav, scal)
        plan.synthesis(wav, scal, f2)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    timing = not (args.no_kernel_timing or args.graph)
    if timing:
        plan.profile(4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    kern = {}
    dropped = 0
    if timing:
        kern, dropped = plan.profile_read()
        plan.profile(0)
    err = (torch.linalg.norm(f2 - f) / torch.linalg.norm(f)).item()

    maps_per_s = B * args.steps / dt
    coeffs = plan.wav_offset[-1] // B
    out = {
        "metric": "analysis+synthesis maps/s at L=1024,N=8: FP64 vs mixed-batched @ <=1e-6 rel err",
        "value": maps_per_s,
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic Gaussian random fields, C_l = 1/(l+1)^2, synthesised on the GPU",
        "config": {"workload": f"sphere directional wavelets analysis+synthesis, "
                               f"{'mixed FP32/FP64 batched' if mixed else 'FP64'}, L={L}, N={N}, "
                               f"lambda={lam:g}, J0={J0}, batch={B}",
                   "L": L, "N": N, "lambda": lam, "J0": J0, "batch": B, "form": args.precision,
                   "tuned": not args.no_tune, "graph": args.graph},
        "coefficients_per_s": maps_per_s * coeffs,
        "round_trip_rel_err": err,
    }
    if kern:
        tot = sum(v[0] for v in kern.values())
        name, (ms, cnt, flop) = max(kern.items(), key=lambda kv: kv[1][0])
        achieved = flop / (ms * 1e-3) if ms > 0 else 0.0
        if name.endswith("_mm") or name.endswith("_f32"):
            peak, bound = PEAKS["fp32_mfma"], "mfma"
        else:
            peak, bound = PEAKS["fp64_valu"], "alu"
        out["roofline"] = {"bound": bound, "kernel": name, "achieved": achieved / 1e12, "peak": peak / 1e12,
                           "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                           "avg_launch_ms": ms / max(cnt, 1), "launches": cnt,
                           "algorithmic_flop_per_launch": flop / max(cnt, 1)}
        out["kernel_breakdown_ms_per_step"] = {k: v[0] / args.steps for k, v in
                                               sorted(kern.items(), key=lambda kv: -kv[1][0])}
        out["kernel_time_fraction_of_step"] = tot / (1e3 * dt)
        if dropped:
            out["kernel_timing_dropped_launches"] = dropped
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(L, N, lam, J0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
