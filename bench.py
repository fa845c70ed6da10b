"""Benchmark: directional wavelet analysis + synthesis throughput on one MI355X.

Metric: maps per second for one analysis + synthesis round trip of real maps
on McEwen-Wiaux sampling (default workload L=1024, N=8, lambda=2, J0=0; the
paper's protocol of Section 4.4 without its harmonic-space bookends).  Inputs
are synthetic Gaussian random fields (C_l = 1/(l+1)^2) synthesised on the GPU
and resident in HBM before timing starts.

Prints one JSON line.  By default the headline value is the mixed-precision
batched form (64 maps per call) and `fp64_form` carries the plain FP64 form
(one map per call) measured in the same run.  `roofline` reports the dominant
kernel: algorithmic work per launch (counted by the library from each launch's
parameters) over its average duration measured with HIP events on the stream
it runs on; `traffic` is the HBM bytes per launch from a committed PMC summary
(profiles/traffic.json) when it was taken on the current sources, else null.
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
    ap.add_argument("--batch", type=int, default=None, help="maps per call (default 64 for mixed, 1 for fp64)")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both",
                    help="both: the mixed batched form (the headline value) and the FP64 form beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay each transform as a HIP graph (no per-kernel timing)")
    ap.add_argument("--no-tune", action="store_true", help="skip the plan's tile-shape autotuning")
    ap.add_argument("--precompute", action="store_true",
                    help="precompute mode for every form (FP64: Wigner d tabulated for grids of band limit "
                         "<= 512; mixed: also the folded quadrature-contraction tables of the synthesis)")
    ap.add_argument("--no-precompute", action="store_true",
                    help="run the mixed form with the recursion only (by default the headline mixed form "
                         "uses precompute mode and the recursion form is reported beside it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM traffic counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="no headline line: the mixed form at batch 1, 4, 16, 64, each eager and with HIP-graph "
                         "replay, one JSON line with maps/s per setting")
    ap.add_argument("--ball", action="store_true",
                    help="no headline line: the ball transform at the setting of the paper's ball benchmark "
                         "(N=1, P=L=256 by default; --L sets L=P), FP64 and mixed, one JSON line")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats output directory of a "
                         "bench run (the per-kernel statistics, and the timed steps' launches of --family)")
    ap.add_argument("--no-gradient", action="store_true", help="skip the gradient loop (for profiled runs)")
    ap.add_argument("--family", default="lsum_mm", help="bench kernel name whose timed launches are summarised")
    ap.add_argument("--per-step", type=int, default=6, help="launches of --family per analysis + synthesis step")
    ap.add_argument("--summarize-counters", metavar="PMC_DIR",
                    help="print a markdown table of a rocprofv3 --pmc output directory of a one-step precompute "
                         "run with the SQ counters SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY "
                         "SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT, "
                         "summed per bench kernel name over the round trip's dispatches")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no benchmark: read two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; csv output) "
                         "of 'bench.py --precision mixed --steps 1 --warmup 0 --no-tune --copy-calibration' (one "
                         "round trip, so the averages are per launch of that step) and write profiles/traffic.json")
    return ap.parse_args()


# name a launch carries in the per-kernel timing -> the library kernel symbols it runs
KERNEL_NAMES = [("tsum_mm", ["k_tsum_mm<", "k_tsum_mm16<"]), ("tsum_tab", ["k_tsum_tab("]),
                ("lsum_mm", ["k_lsum_mm<", "k_lsum_bf3<", "k_lsum_bf3_list<"]),
                ("gemm_theta_bf3", ["k_gemm_bf3("]), ("gemm_theta_f32", ["k_gemm<float>"]),
                ("gemm_theta", ["k_gemm<double>"]), ("dft_c2r_f32", ["k_dft_mm<1,"]),
                ("dft_r2c_f32", ["k_dft_mm<-1,"]), ("gamma_c2r_f32", ["k_gamma_c2r<float"]),
                ("gamma_r2c_f32", ["k_gamma_r2c<float"]), ("tsum", ["k_tsum_mm64<", "k_tsum<"]),
                ("lsum", ["k_lsum_mm64<", "k_lsum<"])]


def is_mixed_kernel(name):
    """Kernels of the mixed form whose contractions run on matrix cores in FP32 accuracy
    (FP32 products, or BF16 products of three-part splits)."""
    return name.endswith(("_mm", "_f32", "_bf3")) or name == "tsum_tab"


def end_to_end(kern, steps, ms_step, L, B, nwav, scal_shape, esz):
    """The whole step against its roofline: the algorithmic work of one step on each unit
    (FP64: every flop of the FP64 kernels and the recursion inside the mixed kernels; FP32
    matrix cores: the rest of the mixed kernels' flops; HBM: reading the maps and writing
    the coefficients in analysis, reading them and writing the maps in synthesis), each
    over that unit's peak; the largest of these times over the measured step time."""
    fp64 = sum(v[3] if is_mixed_kernel(k) else v[2] for k, v in kern.items()) / steps
    mfma = sum(v[2] - v[3] for k, v in kern.items() if is_mixed_kernel(k)) / steps
    nmap = L * (2 * L - 1)
    nscal = scal_shape[1] * scal_shape[2]
    hbm = B * (2 * 8 * nmap + 2 * esz * nwav + 2 * 8 * nscal)
    t = {"fp64": fp64 / PEAKS["fp64_valu"], "fp32_mfma": mfma / PEAKS["fp32_mfma"], "hbm": hbm / PEAKS["hbm"]}
    unit = max(t, key=t.get)
    return {"bound": unit, "min_ms_per_step": 1e3 * t[unit], "ms_per_step": ms_step,
            "frac": 1e3 * t[unit] / ms_step,
            "min_ms_per_unit": {k: 1e3 * v for k, v in t.items()},
            "work_per_step": {"fp64_flop": fp64, "fp32_mfma_flop": mfma, "hbm_bytes": hbm}}


def summarize_trace(d, args):
    """Markdown summary of a profiled bench run (one form, made with --no-gradient): the kernel
    statistics of rocprofv3, and the launches of one kernel family (`--family`, matched as in
    KERNEL_NAMES) inside the timed steps, which are the family's last --steps x --per-step
    launches of the run."""
    import csv
    import glob
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    trace = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(stats)))
    print("| kernel | calls | total (ms) | average (ms) | % |")
    print("|---|---|---|---|---|")
    for r in rows[:24]:
        nm = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        print(f"| `{nm}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} |")
    syms = dict(KERNEL_NAMES).get(args.family, [])
    disp = []
    for r in csv.DictReader(open(trace)):
        nm = r["Kernel_Name"].replace(" ", "")
        if any(sy.replace(" ", "") in nm for sy in syms):
            disp.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    disp.sort()
    k, S = args.per_step, args.steps
    timed = disp[len(disp) - S * k:] if len(disp) >= S * k else []
    if timed:
        tot = sum(e - b for b, e, _ in timed) / 1e6
        names = sorted({n.split("(")[0] for _, _, n in timed})
        print(f"\n`{args.family}` in the {S} timed steps: {len(timed)} launches ({k} per step) of "
              + ", ".join(f"`{n}`" for n in names)
              + f"; {tot:.3f} ms in total, average {tot / len(timed):.4f} ms per launch, {tot / S:.3f} ms per step.")


def summarize_counters(d):
    """Markdown table of shader counters per bench kernel name, summed over the dispatches from
    the round trip's first stage on (two dispatches before the first k_sht_tab)."""
    import collections
    import csv
    import glob
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    val = collections.defaultdict(lambda: collections.defaultdict(float))
    name = {}
    for r in csv.DictReader(open(path)):
        i = int(r["Dispatch_Id"])
        val[i][r["Counter_Name"]] += float(r["Counter_Value"])
        name[i] = r["Kernel_Name"].replace(" ", "")
    ids = [i for i in name if "k_sht_tab" in name[i]]
    start = min(ids) - 2 if ids else 0
    fams = KERNEL_NAMES + [("sht_tab", ["k_sht_tab("]), ("shti_tab", ["k_shti_tab("])]
    fam = collections.defaultdict(lambda: collections.defaultdict(float))
    cnt = collections.Counter()
    for i, v in val.items():
        if i < start:
            continue
        for bname, syms in fams:
            if any(sy.replace(" ", "") in name[i] for sy in syms):
                for k, x in v.items():
                    fam[bname][k] += x
                cnt[bname] += 1
                break
    print("| kernel | dispatches | matrix cores busy | waves waiting on a counter | VALU per MFMA instruction "
          "| LDS bank-conflict cycles per LDS instruction |")
    print("|---|---|---|---|---|---|")
    for b, v in sorted(fam.items(), key=lambda kv: -kv[1]["SQ_BUSY_CYCLES"]):
        busy = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (v["SQ_BUSY_CYCLES"] * 32) if v["SQ_BUSY_CYCLES"] else 0.0
        wait = v["SQ_WAIT_INST_ANY"] / v["SQ_WAVE_CYCLES"] if v["SQ_WAVE_CYCLES"] else 0.0
        vpm = v["SQ_INSTS_VALU"] / v["SQ_INSTS_MFMA"] if v["SQ_INSTS_MFMA"] else float("nan")
        lds = v["SQ_LDS_BANK_CONFLICT"] / v["SQ_INSTS_LDS"] if v["SQ_INSTS_LDS"] else float("nan")
        print(f"| {b} | {cnt[b]} | {busy:.3f} | {wait:.3f} | {vpm:.1f} | {lds:.2f} |")


def record_traffic(fetch_dir, write_dir, args):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by
    what the same counter reads for the 1 GiB device copy of --copy-calibration."""
    import csv
    import glob
    from collections import defaultdict

    def load(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        val, name = defaultdict(float), {}
        for r in csv.DictReader(open(f)):
            val[r["Dispatch_Id"]] += float(r["Counter_Value"])
            name[r["Dispatch_Id"]] = r["Kernel_Name"].replace(" ", "")
        return val, name

    fv, fn = load(fetch_dir)
    wv, wn = load(write_dir)

    def step_window(val, name):
        # a run made with --steps 1 --warmup 0 --no-gradient in precompute mode: its round trip
        # starts two dispatches (the FP64 DFT and gamma stage of the forward SHT) before the
        # first k_sht_tab; plan creation, tuning and the input maps come before it
        ids = [int(k) for k in val if "k_sht_tab" in name[k]]
        if not ids:
            return val
        start = min(ids) - 2
        return {k: v for k, v in val.items() if int(k) >= start}

    cf = max(v for k, v in fv.items() if "copyBuffer" in fn[k])
    cw = max(v for k, v in wv.items() if "copyBuffer" in wn[k])
    fv, wv = step_window(fv, fn), step_window(wv, wn)
    gib_kib = float(1 << 20)
    # the copy is the largest device copy dispatch of the run (1 GiB read, 1 GiB written)
    ff, fw = gib_kib / cf, gib_kib / cw
    kern = {}
    for bname, syms in KERNEL_NAMES:
        ks = [k for k in fv if any(sy.replace(" ", "") in fn[k] for sy in syms)]
        kw = [k for k in wv if any(sy.replace(" ", "") in wn[k] for sy in syms)]
        if not ks or len(ks) != len(kw):
            continue
        fb = 1024.0 * ff * sum(fv[k] for k in ks) / len(ks)
        wb = 1024.0 * fw * sum(wv[k] for k in kw) / len(kw)
        pre = args.precompute or not args.no_precompute
        kern[bname] = {"workload": (f"sphere directional wavelets analysis+synthesis, mixed FP32/FP64 batched, "
                                    f"L={args.L}, N={args.N}, lambda={args.lam:g}, J0={args.J0}, batch=64"
                                    + (", precompute mode" if pre else "")),
                       "launches": len(ks), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                       "bytes_per_launch": fb + wb}
    rec = {"source_sha256": source_hash(),
           "copy_calibration": {"fetch_kib_for_1gib": cf, "write_kib_for_1gib": cw,
                                "fetch_scale": ff, "write_scale": fw},
           "command": ("cd /tmp && rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <dir> -o run --output-format csv "
                       "-- python3 bench.py --precision mixed --precompute --steps 1 --warmup 0 --no-cpu-baseline "
                       "--no-kernel-timing --no-gradient --copy-calibration; per kernel the average over the "
                       "dispatches of the round trip (from the forward SHT's first stage on)"),
           "kernels": kern}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def cpu_baseline(L, N, lam, J0):
    """Time the oracle on one map of the workload: its full round trip (forward SHT,
    analysis of every scale, synthesis), the unit the metric counts, on this host's cores."""
    import numpy as np

    import synthetic
    from oracle import mw, wavelets

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    P = wavelets.Plan(L, N, lam, J0)
    flm = synthetic.sphere_flm(L, synthetic.stream_key(4))
    f = np.real(mw.sht_inverse(flm, L))
    mw.delta_table(L)
    t0 = time.perf_counter()
    wav, scal = wavelets.analysis(f, P)
    f2 = wavelets.synthesis(wav, scal, P)
    t = time.perf_counter() - t0
    err = float(np.linalg.norm(f2 - f) / np.linalg.norm(f))
    return {"value": 1.0 / t, "unit": "maps/s", "cores": threads, "kind": "oracle",
            "sample": (f"one map at L={L}, N={N}, lambda={lam:g}, J0={J0}: the oracle's full analysis + synthesis "
                       f"round trip ({t:.1f} s, round trip rel err {err:.1e})")}


def source_hash():
    """sha256 of the library sources (kernels, host code, ABI header)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_01282_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".h", ".cpp")))
    files.append(os.path.join(ROOT, "include", "s2w.h"))
    for fn in files:
        h.update(os.path.basename(fn).encode())
        h.update(open(fn, "rb").read())
    return h.hexdigest()


def recorded_traffic_entry(kernel, workload):
    """The committed PMC record of `kernel` (bytes per launch, launches in the profiled
    round trip), if it was taken on the current sources and the same workload (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_sha256") != source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    if not ent or ent.get("workload") != workload:
        return None
    return ent


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None."""
    ent = recorded_traffic_entry(kernel, workload)
    return ent.get("bytes_per_launch") if ent else None


def run_form(args, precision, B, precompute=None):
    import torch

    import paper_2402_01282_amd as s2w
    import synthetic

    L, N, lam, J0 = args.L, args.N, args.lam, args.J0
    mixed = precision == "mixed"
    print(f"[bench] L={L} N={N} lambda={lam} J0={J0} batch={B} precision={precision}", file=sys.stderr, flush=True)
    if precompute is None:
        precompute = args.precompute
    print(f"[bench] precompute={precompute}", file=sys.stderr, flush=True)
    flags = (0 if args.no_tune else s2w.S2W_PLAN_TUNE) | (s2w.S2W_PLAN_GRAPH if args.graph else 0) \
        | (s2w.S2W_PLAN_PRECOMPUTE if precompute else 0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    plan = s2w.Plan(L, N, lam, J0, batch=B, device=0, precision=s2w.S2W_MIXED if mixed else s2w.S2W_FP64,
                    flags=flags)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    plan_bytes = free0 - torch.cuda.mem_get_info()[0]   # the plan's tables and workspace
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
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {precision}: timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    kern, dropped = {}, 0
    if timing:
        kern, dropped = plan.profile_read()
        plan.profile(0)
    err = (torch.linalg.norm(f2 - f) / torch.linalg.norm(f)).item()
    maps_per_s = B * args.steps / dt
    # gradient of sum_j sum (W^j)^2 with respect to the maps: analysis, then the transpose of
    # the analysis applied to the cotangent 2 W (timed as a separate loop of the same length)
    gf = torch.empty_like(f)
    gscal = torch.zeros_like(scal)

    def grad_step():
        plan.analysis(f, wav, scal)
        plan.analysis_adjoint(wav, gscal, gf)

    dtg = None
    if not args.no_gradient:
        grad_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            grad_step()
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
    workload = (f"sphere directional wavelets analysis+synthesis, "
                f"{'mixed FP32/FP64 batched' if mixed else 'FP64'}, L={L}, N={N}, lambda={lam:g}, J0={J0}, batch={B}"
                + (", precompute mode" if precompute else ""))
    out = {"value": maps_per_s, "ms_per_step": 1e3 * dt / args.steps,
           "dtype": "f32+f64" if mixed else "f64", "workload": workload, "batch": B,
           "coefficients_per_s": maps_per_s * (plan.wav_offset[-1] // B), "round_trip_rel_err": err,
           "plan_create_s": t_plan, "plan_device_gib": plan_bytes / 2 ** 30, "precompute": bool(precompute),
           "gradient": None if dtg is None else
           {"maps_per_s": B * args.steps / dtg, "ms_per_step": 1e3 * dtg / args.steps,
            "what": "analysis + transpose of the analysis (gradient of sum_j sum (W^j)^2)"}}
    if kern:
        tot = sum(v[0] for v in kern.values())
        name, (ms, cnt, flop, flop64, dense) = max(kern.items(), key=lambda kv: kv[1][0])
        achieved = flop / (ms * 1e-3) if ms > 0 else 0.0
        if is_mixed_kernel(name):
            peak, bound = PEAKS["fp32_mfma"], "mfma"
        else:
            peak, bound = PEAKS["fp64_valu"], "alu"
        out["roofline"] = {"bound": bound, "kernel": name, "achieved": achieved / 1e12, "peak": peak / 1e12,
                           "unit": "TFLOP/s", "frac": achieved / peak,
                           "traffic": recorded_traffic(name, workload),
                           "avg_launch_ms": ms / max(cnt, 1), "launches": cnt,
                           "algorithmic_flop_per_launch": flop / max(cnt, 1),
                           "dense_flop_per_launch": (dense / max(cnt, 1)) or None,
                           "dense_tflops": (dense / (ms * 1e-3) / 1e12) if dense and ms > 0 else None}
        out["kernel_breakdown_ms_per_step"] = {k: v[0] / args.steps for k, v in
                                               sorted(kern.items(), key=lambda kv: -kv[1][0])}
        # every timed kernel against its compute peak (algorithmic flops as for the dominant
        # one) and, where PMC traffic was recorded for this workload on the current sources,
        # against HBM
        per = {}
        for k, (kms, kcnt, kflop, kf64, kdense) in sorted(kern.items(), key=lambda kv: -kv[1][0]):
            if kms <= 0:
                continue
            kpk = PEAKS["fp32_mfma"] if is_mixed_kernel(k) else PEAKS["fp64_valu"]
            rate = kflop / (kms * 1e-3)
            e = {"ms_per_step": kms / args.steps, "tflops": rate / 1e12, "frac_of_compute_peak": rate / kpk}
            if kdense:
                e["dense_tflops"] = kdense / (kms * 1e-3) / 1e12
            # only where the profiled round trip had the same launches as a timed step (the
            # FP64 l-sum record also counts the syntheses of the input maps)
            ent = recorded_traffic_entry(k, workload)
            tb = ent.get("bytes_per_launch") if ent else None
            if tb and ent.get("launches") * args.steps == kcnt:
                bw = tb * kcnt / (kms * 1e-3)
                e["hbm_gbps"] = bw / 1e9
                e["frac_of_hbm_peak"] = bw / PEAKS["hbm"]
            per[k] = e
        out["kernel_rooflines"] = per
        out["kernel_time_fraction_of_step"] = tot / (1e3 * dt)
        out["end_to_end"] = end_to_end(kern, args.steps, 1e3 * dt / args.steps, L, B,
                                       plan.wav_offset[-1] // B, plan.scal_shape, 4 if mixed else 8)
        if dropped:
            out["kernel_timing_dropped_launches"] = dropped
    del plan, wav, scal, f, f2
    torch.cuda.empty_cache()
    return out


# The paper's ball round trip (S2BALL, one A100, FP64, N=1, P=L; Section 5.4, Table 2), ms
PAPER_BALL_MS = {8: 0.75, 16: 0.95, 32: 1.3, 64: 3.0, 128: 17.0, 256: 160.0}


def run_ball(args):
    """Ball analysis + synthesis round trips of one map at N=1, P=L (lambda = nu = 2,
    J0 = J0' = 0), FP64 and mixed, timed as the sphere forms are."""
    import torch

    import paper_2402_01282_amd as s2w
    import synthetic

    L = args.L if args.L != 1024 else 256
    P, N = L, 1
    flmp = synthetic.ball_flmp(L, P, synthetic.stream_key(13))
    rows = {}
    for prec in ("fp64", "mixed"):
        print(f"[bench] ball L=P={L} N=1 {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        plan = s2w.BallPlan(L, N, P, batch=1, device=0,
                            precision=s2w.S2W_MIXED if prec == "mixed" else s2w.S2W_FP64)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        f = plan.sl_inverse(torch.from_numpy(flmp[None].copy()))
        wav = plan.empty_wav()
        scal = torch.empty(plan.map_shape, dtype=torch.float64, device="cuda")
        f2 = torch.empty_like(f)
        for _ in range(args.warmup):
            plan.analysis(f, wav, scal)
            plan.synthesis(wav, scal, f2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.analysis(f, wav, scal)
            plan.synthesis(wav, scal, f2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        err = (torch.linalg.norm(f2 - f) / torch.linalg.norm(f)).item()
        rows[prec] = {"ms_per_round_trip": 1e3 * dt, "round_trips_per_s": 1.0 / dt, "round_trip_rel_err": err,
                      "plan_create_s": t_plan, "wavelet_coefficients": plan.wav_offset[-1]}
        del plan, wav, scal, f, f2
        torch.cuda.empty_cache()
    out = {"ball": f"ball directional wavelets analysis+synthesis, L=P={L}, N=1, lambda=nu=2, J0=J0'=0, one map",
           "forms": rows,
           "paper_context": {"S2BALL_one_A100_ms": PAPER_BALL_MS.get(L), "source": "Section 5.4, Table 2 (FP64)"}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.ball:
        if args.gpus != 1:
            sys.exit(2)
        run_ball(args)
        return
    if args.record_traffic:
        record_traffic(args.record_traffic[0], args.record_traffic[1], args)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.sweep:
        if args.gpus != 1:
            sys.exit(2)
        rows = []
        for B in (1, 4, 16, 64):
            for graph in (False, True):
                args.graph = graph
                r = run_form(args, "mixed", B, precompute=args.precompute or not args.no_precompute)
                rows.append({"batch": B, "graph": graph, "precompute": r["precompute"], "maps_per_s": r["value"],
                             "ms_per_call": r["ms_per_step"],
                             "round_trip_rel_err": r["round_trip_rel_err"]})
        print(json.dumps({"sweep": "mixed form, L=%d, N=%d, lambda=%g, J0=%d" % (args.L, args.N, args.lam, args.J0),
                          "rows": rows}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    forms = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    res = {}
    # the mixed form runs in precompute mode unless told otherwise (its tables fit the HBM of
    # one GPU at L = 1024); its recursion form is measured beside it
    mixed_pre = args.precompute or not args.no_precompute
    for form in forms:
        B = args.batch if args.batch is not None else (64 if form == "mixed" else 1)
        if form == "mixed":
            res[form] = run_form(args, form, B, precompute=mixed_pre)
            if mixed_pre and not args.precompute:
                res["mixed_recursion"] = run_form(args, form, B, precompute=False)
        else:
            res[form] = run_form(args, form, B)
    head = res[forms[0]]
    out = {
        "metric": "analysis+synthesis maps/s at L=1024,N=8: FP64 vs mixed-batched @ <=1e-6 rel err",
        "value": head["value"],
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic Gaussian random fields, C_l = 1/(l+1)^2, synthesised on the GPU",
        "config": {"workload": head["workload"], "L": args.L, "N": args.N, "lambda": args.lam, "J0": args.J0,
                   "batch": head["batch"], "form": forms[0], "tuned": not args.no_tune, "graph": args.graph,
                   "precompute": head["precompute"]},
        "plan_device_gib": head["plan_device_gib"],
        "plan_create_s": head["plan_create_s"],
        "coefficients_per_s": head["coefficients_per_s"],
        "round_trip_rel_err": head["round_trip_rel_err"],
        "gradient": head["gradient"],
    }
    for k in ("roofline", "end_to_end", "kernel_breakdown_ms_per_step", "kernel_rooflines",
              "kernel_time_fraction_of_step", "kernel_timing_dropped_launches"):
        if k in head:
            out[k] = head[k]
    if "mixed_recursion" in res:
        r = res["mixed_recursion"]
        out["mixed_recursion_form"] = {k: r[k] for k in ("value", "ms_per_step", "workload", "round_trip_rel_err",
                                                         "plan_create_s", "plan_device_gib", "roofline",
                                                         "kernel_breakdown_ms_per_step", "end_to_end") if k in r}
    if "fp64" in res and forms[0] != "fp64":
        out["fp64_form"] = res["fp64"]
        out["speedup_vs_fp64_form"] = head["value"] / res["fp64"]["value"]
    if args.copy_calibration:
        # a plain copy of known size, for scaling the HBM traffic counters of a profiled run
        n = 1 << 27
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 8 * n, "written": 8 * n}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.L, args.N, args.lam, args.J0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
