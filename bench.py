#!/usr/bin/env python3
"""Throughput benchmark: brute-force de-dispersion on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload scale_f32]

One step is one dd_execute over the whole workload (every DM trial, every
output sample, all channels), with the input already resident in HBM.
Prints ONE JSON line: DM-trial samples/s, the roofline of the dominant
kernel (algorithmic adds per launch over its HIP-event launch time) and the
CPU oracle timed on a bounded sample of the same workload.

Workloads (synthetic, seeded; see synth/):
  scale_f32      1024 ch 1214-1510 MHz, 64 us, 2^18 samples, 2048 DMs 0-1023.5
                 step 0.5, N(0,1) noise + 20 dispersed pulses, f32 in/out
  scale_u8       the same data quantised to 8 bits (128 + 16x), int32 out
  scale_f16      the same data in binary16, f32 out
  tiny_f32       64 ch 400-432 MHz, 8192 samples, 128 DMs (launch-bound)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak rates (MI355X, 256 CUs at 2.4 GHz).  The de-dispersion kernels are
# bound by plain VALU adds: 128 32-bit adds per clock per CU
# (= 157.3 TFLOP/s FP32 vector counted as 2 flops per FMA) = 78.6e12 adds/s.
PEAK_ADD_PER_S = 256 * 2.4e9 * 128
PEAK_HBM_BPS = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale_f32",
                    choices=["scale_f32", "scale_u8", "scale_f16", "tiny_f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run one plain 1 GiB device copy (for scaling "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def make_workload(name):
    """Seeded synthetic input for `name`.  Pulse arrival offsets come from the
    oracle's delay routine (the CPU-baseline leg times the oracle on this
    same input)."""
    import oracle
    import synth
    if name.startswith("scale"):
        w = synth.scale()
    else:
        w = synth.tiny()
    b = w.band
    x = synth.noise(b.nchans, w.nsamp, w.seed)
    if name.startswith("scale"):
        tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
        nout = w.nsamp - oracle.max_shift(tab)
        for p in synth.scale_pulses(w.seed, w.extra["npulses"], nout):
            off = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, [p["dm"]])[0]
            synth.add_boxcar(x, off, p["t0"], p["width"], p["amp"])
    else:
        tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
        e = w.extra
        synth.add_boxcar(x, tab[50], e["pulse_t0"], e["pulse_width"], e["pulse_amp"])
    if name.endswith("u8"):
        x = synth.quantize_u8(x)
    elif name.endswith("f16"):
        x = synth.to_f16(x)
    return w, x


def describe(name, w):
    b = w.band
    f_low = b.f_top - (b.nchans - 1) * b.df
    dt = {"f32": "f32 in, f32 out", "u8": "u8 in (128+16x), int32 out",
          "f16": "f16 in, f32 out"}[name.rsplit("_", 1)[1]]
    return (f"{name}: {b.nchans} ch {f_low:.2f}-{b.f_top:.0f} MHz, t_samp {b.t_samp * 1e6:g} us, "
            f"{w.nsamp} samples, {len(w.dms)} DMs {w.dms[0]:g}-{w.dms[-1]:g} step "
            f"{w.dms[1] - w.dms[0]:g}, N(0,1) noise + injected pulses, {dt}")


def cpu_baseline(x, w, ndms, nout, budget_s):
    """The oracle (plain C, FP64/int64 accumulation, OpenMP over DM rows) on
    a bounded sample of DM rows over the full time range."""
    import oracle
    b = w.band
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
    probe = max(threads, 8)
    rows = np.linspace(0, ndms - 1, probe).astype(np.int32)
    t0 = time.perf_counter()
    oracle.dedisperse(x, tab, rows=rows, nthreads=threads)
    dt = time.perf_counter() - t0
    nrows = int(min(ndms, max(probe, round(probe * budget_s / max(dt, 1e-3)))))
    nrows = max(threads, (nrows // threads) * threads)
    rows = np.linspace(0, ndms - 1, nrows).astype(np.int32)
    t0 = time.perf_counter()
    oracle.dedisperse(x, tab, rows=rows, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": nrows * nout / dt, "unit": "DM-trial samples/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{nrows} of {ndms} DM rows x {nout} output samples x {b.nchans} channels "
                      f"({dt:.1f} s on {threads} threads)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is "
                                   "described in DESIGN.md but not launched"}))
        sys.exit(2)
    import torch
    import paper_1107_2516_amd as dd

    name = args.workload
    w, x = make_workload(name)
    b = w.band
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    ndms, nsamp = plan.ndms, w.nsamp
    nout = plan.nout(nsamp)
    dev = torch.device("cuda:0")
    xin = torch.from_numpy(x).to(dev)
    out = torch.empty((ndms, nout), dtype=dd.out_dtype_for(xin.dtype), device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.execute(xin, out=out)
    torch.cuda.synchronize(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t_wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.execute(xin, out=out)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    t_wall = time.perf_counter() - t_wall0
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = t_wall * 1e3 / args.steps

    b_in = x.dtype.itemsize
    adds = float(ndms) * b.nchans * nout
    alg_bytes = float(b.nchans) * nsamp * b_in + float(ndms) * nout * 4
    achieved = adds / (gpu_ms * 1e-3)
    unit = "TOP/s" if name.endswith("u8") else "TFLOP/s"
    line = {
        "metric": "DM-trial samples/s",
        "value": ndms * nout / (ms_per_step * 1e-3),
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "u8": "u8", "f16": "f16"}[name.rsplit("_", 1)[1]],
        "data": "synthetic",
        "config": {"workload": describe(name, w), "nchans": b.nchans, "ndms": ndms,
                   "nsamp": nsamp, "nout": nout, "max_shift": plan.max_shift,
                   "tile": plan.tile_for(xin.dtype, nsamp)},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ADD_PER_S / 1e12,
                     "unit": unit, "frac": achieved / PEAK_ADD_PER_S, "traffic": None,
                     "kernel_ms": gpu_ms, "alg_adds_per_launch": adds,
                     "alg_bytes_per_launch": alg_bytes,
                     "hbm_gbs_algorithmic": alg_bytes / (gpu_ms * 1e-3) / 1e9,
                     "hbm_frac_algorithmic": alg_bytes / (gpu_ms * 1e-3) / PEAK_HBM_BPS},
        "real_time_factor": (gpu_ms * 1e-3) / (nout * b.t_samp),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, w, ndms, nout, args.cpu_seconds)
        line["cpu_baseline"]["gpu_over_cpu"] = line["value"] / line["cpu_baseline"]["value"]
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize(dev)
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize(dev)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
