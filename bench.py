#!/usr/bin/env python3
"""Throughput benchmark: brute-force de-dispersion on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload scale_f32] [--only]

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
  batch_u8       32 beams of uneven shapes (256-1024 ch, 2^16-2^18 samples,
                 1024-4096 DMs), 8-bit noise + 4 pulses each, one persistent
                 graph-captured launch per step
  serve_u8       64 streaming beams, 2048 ch 120-180 MHz, 327.68 us, 4096 DMs
                 step 0.125, chunks of 2^14-2^17 samples arriving as Poisson
                 processes at 1.5x real time; p50/p99 latency, RTF

By default (scale_f32) the line also carries "precision" (u8 and f16 on the
same data, with their error and the S/N of the injected pulses), "detect"
(the detection stage on the FP32 output), "corner_turn" (time-ordered
spectra to channel order for the FP32 input), "subband" (section 3.2 with
the Table 1 survey plan, against brute force over the same DMs), "batch"
and "serve" blocks;
--only drops them.
"""
import argparse
import json
import math
import os
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# Peak rates (MI355X, 256 CUs at 2.4 GHz).  The de-dispersion kernels are
# bound by plain VALU adds: 128 32-bit adds per clock per CU
# (= 157.3 TFLOP/s FP32 vector counted as 2 flops per FMA) = 78.6e12 adds/s.
PEAK_ADD_PER_S = 256 * 2.4e9 * 128
PEAK_HBM_BPS = 8.0e12

# rocprofv3 FETCH_SIZE / WRITE_SIZE of the dominant kernel per launch
# (KiB, scaled by the plain-copy calibration), keyed by workload.  Each entry
# names the kernel source hash it was taken with; it is reported only while
# the source is unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale_f32",
                    choices=["scale_f32", "scale_u8", "scale_f16", "tiny_f32", "batch_u8",
                             "serve_u8"])
    ap.add_argument("--only", action="store_true",
                    help="time only the named workload (no precision/batch/serve blocks)")
    ap.add_argument("--detect", action="store_true",
                    help="with --only: also time the detection stage on the FP32 output")
    ap.add_argument("--corner", action="store_true",
                    help="with --only: also time the corner turn of the FP32 input")
    ap.add_argument("--frontend", action="store_true",
                    help="also run the section 5 front end (channelise + de-disperse) block")
    ap.add_argument("--subband", action="store_true",
                    help="with --only: also time subband de-dispersion (Table 1 plan)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the paced (1.5x real time) serving window")
    ap.add_argument("--serve-saturate", type=int, default=128,
                    help="chunks in the unpaced (saturating) serving phase")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run one plain 1 GiB device copy (for scaling "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1107_2516_amd")
    for f in ("csrc/dd_kernels.hip", "csrc/gen_window_asm.py", "csrc/dd_internal.h",
              "csrc/dd_plan.cpp", "build.py"):
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload, launches_per_step=1):
    try:
        with open(TRAFFIC_FILE) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    e = tab.get(workload)
    if not e or e.get("kernel_source") != kernel_source_hash():
        return None
    return {"fetch_bytes": e["fetch_bytes"], "write_bytes": e["write_bytes"],
            "per": "launch", "copy_factor": e.get("copy_factor"), "source": e.get("profile")}


def timed(stream, fn, steps, warmup):
    """Run fn() warmup times, then time `steps` calls: HIP events on the
    launch stream and the host wall clock, both bracketed by syncs."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall * 1e3 / steps


def roofline(adds, in_bytes, out_bytes, kernel_ms, unit, traffic=None):
    achieved = adds / (kernel_ms * 1e-3)
    alg_bytes = in_bytes + out_bytes
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ADD_PER_S / 1e12,
            "unit": unit, "frac": achieved / PEAK_ADD_PER_S, "traffic": traffic,
            "kernel_ms": kernel_ms, "alg_adds_per_launch": adds,
            "alg_bytes_per_launch": alg_bytes,
            "hbm_gbs_algorithmic": alg_bytes / (kernel_ms * 1e-3) / 1e9,
            "hbm_frac_algorithmic": alg_bytes / (kernel_ms * 1e-3) / PEAK_HBM_BPS}


def pulse_offsets(dd, band, dm):
    """Per-channel arrival offsets of a pulse at `dm`: row 0 of the library's
    delay table for a one-trial plan."""
    p = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, [dm])
    return p.delay_table()[0]


# --------------------------------------------------------------------------
# Single-beam workloads (scale_*, tiny_f32)
# --------------------------------------------------------------------------


def make_workload(dd, name):
    """Seeded synthetic input and its plan."""
    w = synth.scale() if name.startswith("scale") else synth.tiny()
    b = w.band
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    x = synth.noise(b.nchans, w.nsamp, w.seed)
    pulses = []
    if name.startswith("scale"):
        nout = w.nsamp - plan.max_shift
        pulses = synth.scale_pulses(w.seed, w.extra["npulses"], nout)
    else:
        e = w.extra
        pulses = [dict(dm=float(w.dms[50]), width=e["pulse_width"], amp=e["pulse_amp"],
                       t0=e["pulse_t0"], snr=None)]
    for p in pulses:
        synth.add_boxcar(x, pulse_offsets(dd, b, p["dm"]), p["t0"], p["width"], p["amp"])
    return w, plan, x, pulses


def convert(x, dt):
    if dt == "u8":
        return synth.quantize_u8(x)
    if dt == "f16":
        return synth.to_f16(x)
    return x


def describe(name, w):
    b = w.band
    f_low = b.f_top - (b.nchans - 1) * b.df
    dt = {"f32": "f32 in, f32 out", "u8": "u8 in (128+16x), int32 out",
          "f16": "f16 in, f32 out"}[name.rsplit("_", 1)[1]]
    return (f"{name}: {b.nchans} ch {f_low:.2f}-{b.f_top:.0f} MHz, t_samp {b.t_samp * 1e6:g} us, "
            f"{w.nsamp} samples, {len(w.dms)} DMs {w.dms[0]:g}-{w.dms[-1]:g} step "
            f"{w.dms[1] - w.dms[0]:g}, N(0,1) noise + injected pulses, {dt}")


def run_single(dd, torch, plan, w, xh, dt, args):
    dev = torch.device("cuda:0")
    nsamp = w.nsamp
    nout = plan.nout(nsamp)
    xin = torch.from_numpy(xh).to(dev)
    out = torch.empty((plan.ndms, nout), dtype=dd.out_dtype_for(xin.dtype), device=dev)
    stream = torch.cuda.current_stream(dev)
    kms, wall_ms = timed(stream, lambda: plan.execute(xin, out=out), args.steps, args.warmup)
    adds = float(plan.ndms) * plan.nchans * nout
    unit = "TOP/s" if dt == "u8" else "TFLOP/s"
    rl = roofline(adds, float(plan.nchans) * nsamp * xh.dtype.itemsize,
                  float(plan.ndms) * nout * 4, kms, unit)
    # spread of single launches (HIP events around each one), after the timed run
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a, b in ev:
        a.record(stream)
        plan.execute(xin, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    each = np.array([a.elapsed_time(b) for a, b in ev])
    rl["kernel_ms_p10_p50_p90"] = [float(v) for v in np.percentile(each, [10, 50, 90])]
    # the same adds against 64 adds per CU per clock (39.3e12/s), a peak that
    # plain v_add_f32 was measured to exceed on this chip
    rl["frac_vs_39T_adds"] = adds / (kms * 1e-3) / (PEAK_ADD_PER_S / 2)
    return {"kernel_ms": kms, "ms_per_step": wall_ms, "value": plan.ndms * nout / (wall_ms * 1e-3),
            "roofline": rl, "tile": plan.tile_for(xin.dtype, nsamp),
            "real_time_factor": (kms * 1e-3) / (nout * w.band.t_samp)}, out


def run_copies(torch, xh, out, reps=3):
    """Host<->device copies of one step's input and output through pinned
    host memory, timed with HIP events on the current stream.  The paper
    times its kernel without them and reports them per stage (section 4;
    section 5, Table 6); they are never part of `value`."""
    dev = out.device
    stream = torch.cuda.current_stream(dev)
    hin = torch.from_numpy(xh).pin_memory()
    din = torch.empty(hin.shape, dtype=hin.dtype, device=dev)
    hout = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)

    def one(dst, src):
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize(dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            dst.copy_(src, non_blocking=True)
        b.record(stream)
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps

    h2d = one(din, hin)
    d2h = one(hout, out)
    nin = hin.numel() * hin.element_size()
    nout = out.numel() * out.element_size()
    del hin, din, hout
    return {"h2d_bytes": nin, "h2d_ms": h2d, "h2d_gbs": nin / (h2d * 1e-3) / 1e9,
            "d2h_bytes": nout, "d2h_ms": d2h, "d2h_gbs": nout / (d2h * 1e-3) / 1e9,
            "host_memory": "pinned"}


def boxcar_snr_peak(row, t0, width, search=64):
    """Peak boxcar S/N of a de-dispersed row near output sample t0, with the
    row's median and 1.4826*MAD as baseline and scale."""
    x = np.asarray(row, dtype=np.float64)
    mu = np.median(x)
    sigma = 1.482602218505602 * np.median(np.abs(x - mu))
    lo, hi = max(0, t0 - search), min(x.size, t0 + width + search)
    c = np.concatenate([[0.0], np.cumsum(x[lo:hi] - mu)])
    box = c[width:] - c[:-width]
    return float(box.max() / (sigma * math.sqrt(width)))


def pulse_snrs(out, w, pulses):
    step = float(w.dms[1] - w.dms[0])
    rows = [int(min(len(w.dms) - 1, round(p["dm"] / step))) for p in pulses]
    host = out[rows].float().cpu().numpy()
    return [boxcar_snr_peak(host[i], p["t0"], p["width"]) for i, p in enumerate(pulses)]


def time_oracle_rows(x, tab, threads, budget_s):
    """Time the oracle on an evenly spread sample of DM rows over the full time
    range, the row count sized from a probe to take about budget_s.  Returns
    (DM-trial samples/s, rows, seconds, oracle rows)."""
    import oracle
    ndms = tab.shape[0]
    nout = x.shape[1] - int(tab.max())
    probe = max(threads, 8)
    rows = np.linspace(0, ndms - 1, probe).astype(np.int32)
    t0 = time.perf_counter()
    oracle.dedisperse(x, tab, rows=rows, nthreads=threads)
    dt = time.perf_counter() - t0
    nrows = int(min(ndms, max(probe, round(probe * budget_s / max(dt, 1e-3)))))
    nrows = max(threads, (nrows // threads) * threads)
    rows = np.linspace(0, ndms - 1, nrows).astype(np.int32)
    t0 = time.perf_counter()
    ref = oracle.dedisperse(x, tab, rows=rows, nthreads=threads)
    dt = time.perf_counter() - t0
    return nrows * nout / dt, rows, dt, ref


def oracle_threads():
    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
    return threads


def cpu_baseline(w, xs, outs, budget_s):
    """The oracle (plain C, FP64/int64 accumulation, OpenMP over DM rows)
    timed on a bounded sample of DM rows over the full time range for each
    precision of the step, and the GPU results of every precision compared
    with it on those rows."""
    import oracle
    b = w.band
    tab = oracle.delay_table(b.nchans, b.f_top, b.df, b.t_samp, w.dms)
    ndms = tab.shape[0]
    x = xs["f32"]
    nout = x.shape[1] - int(tab.max())
    threads = oracle_threads()
    rate, rows, dt, ref = time_oracle_rows(x, tab, threads, budget_s)
    nrows = len(rows)
    res = {"value": rate, "unit": "DM-trial samples/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{nrows} of {ndms} DM rows x {nout} output samples x {b.nchans} channels "
                     f"({dt:.1f} s on {threads} threads)",
           "cpu_model": cpu_model()}
    # the other precisions of the same data (8-bit: int64 sums; binary16:
    # FP64 sums), a third of the budget each
    per = {}
    for pdt in ("u8", "f16"):
        if pdt in xs:
            r, rr, d, _ = time_oracle_rows(xs[pdt], tab, threads, budget_s / 3)
            per[pdt] = {"value": r, "unit": "DM-trial samples/s", "cores": threads,
                        "sample": f"{len(rr)} of {ndms} DM rows x {nout} output samples "
                                  f"({d:.1f} s on {threads} threads)"}
    if per:
        res["precisions"] = per
    # one core, as the paper's CPU baseline: a few rows
    one = rows[:: max(1, nrows // 4)][:4]
    t1 = time.perf_counter()
    oracle.dedisperse(x, tab, rows=one, nthreads=1)
    d1 = time.perf_counter() - t1
    res["single_core"] = {"value": len(one) * nout / d1, "unit": "DM-trial samples/s",
                          "sample": f"{len(one)} DM rows x {nout} output samples on 1 thread "
                                    f"({d1:.1f} s)"}
    # accuracy of each GPU result on (up to) 16 of the sampled rows
    sub = np.unique(np.linspace(0, nrows - 1, min(nrows, 16)).astype(np.int64))
    r_rows = rows[sub]
    ref_rows = ref[sub]
    den = oracle.dedisperse(np.abs(x), tab, rows=r_rows, nthreads=threads)
    acc = {"rows_checked": int(len(r_rows))}
    for dt_name, out in outs.items():
        y = out[torch_index(r_rows)].cpu().numpy().astype(np.float64)
        if dt_name == "u8":
            exact = oracle.dedisperse(xs["u8"], tab, rows=r_rows, nthreads=threads)
            acc["u8"] = {"bit_exact_vs_oracle": bool(np.array_equal(y.astype(np.int64), exact)),
                         "rel_err_vs_fp64_f32_input": normwise(
                             (y - 128.0 * b.nchans) / 16.0, ref_rows)}
        elif dt_name == "f16":
            same = oracle.dedisperse(xs["f16"], tab, rows=r_rows, nthreads=threads)
            dsame = oracle.dedisperse(np.abs(xs["f16"]), tab, rows=r_rows, nthreads=threads)
            acc["f16"] = {"scaled_err_vs_oracle": float(np.max(np.abs(y - same) / dsame)),
                          "rel_err_vs_fp64_f32_input": normwise(y, ref_rows)}
        else:
            acc["f32"] = {"scaled_err_vs_oracle": float(np.max(np.abs(y - ref_rows) / den)),
                          "rel_err_vs_fp64_f32_input": normwise(y, ref_rows)}
    res["accuracy"] = acc
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def torch_index(rows):
    import torch
    return torch.from_numpy(np.asarray(rows, dtype=np.int64)).cuda()


def normwise(y, ref):
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


# --------------------------------------------------------------------------
# Detection stage on the de-dispersed output


def run_detect(dd, torch, out, w, pulses, args, nsigma=8.0, kmax=6):
    """dd_detect over the whole FP32 output (two HBM passes: row statistics,
    then boxcars + threshold), and how many injected pulses it recovers."""
    dev = out.device
    ndms, nout = out.shape
    stats = torch.empty((ndms, 2), dtype=torch.float64, device=dev)
    max_ev = 1 << 20
    ev = torch.empty((max_ev, dd.EVENT_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    L = dd.lib()

    def step():
        st = L.dd_detect(out.data_ptr(), dd.DD_F32, ndms, nout, out.stride(0), nsigma, kmax,
                         stats.data_ptr(), ev.data_ptr(), max_ev, count.data_ptr(),
                         dd.stream_handle())
        if st != dd.DD_OK:
            raise dd.DedispError(st, dd.last_error())

    kms, wall_ms = timed(stream, step, args.steps, args.warmup)
    n = int(count.item())
    host = ev[:min(n, max_ev)].cpu().numpy().reshape(-1).view(dd.EVENT_DTYPE)
    step_dm = float(w.dms[1] - w.dms[0])
    found = 0
    for p in pulses:
        row = int(round(p["dm"] / step_dm))
        near = host[(np.abs(host["dm_row"] - row) <= 2) &
                    (np.abs(host["t"] - p["t0"]) <= p["width"] + 2)]
        found += int(len(near) > 0)
    alg = float(ndms) * nout * 4
    achieved = alg / (kms * 1e-3)
    return {"nsigma": nsigma, "widths": f"1..{1 << kmax}", "kernel_ms": kms, "ms_per_step": wall_ms,
            "events": n, "pulses_recovered": found, "pulses_injected": len(pulses),
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM_BPS / 1e9,
                         "unit": "GB/s", "frac": achieved / PEAK_HBM_BPS,
                         "alg_bytes_per_launch": alg,
                         "note": "algorithmic bytes = one read of the output; the stage reads it twice"}}


# --------------------------------------------------------------------------
# Corner turn (time-ordered spectra -> the path's channel order)


def run_corner(dd, torch, x32, args):
    """dd_corner_turn of the FP32 workload's input from spectra [nsamp,
    nchans] (as a telescope writes them) to rows [nchans, nsamp]."""
    dev = torch.device("cuda:0")
    spectra = torch.from_numpy(np.ascontiguousarray(x32.T)).to(dev)
    out = torch.empty((x32.shape[0], x32.shape[1]), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    kms, wall_ms = timed(stream, lambda: dd.corner_turn(spectra, out=out), args.steps, args.warmup)
    ok = bool(torch.equal(out[:, :4096].cpu(), torch.from_numpy(x32[:, :4096])))
    nbytes = 2.0 * x32.size * 4
    achieved = nbytes / (kms * 1e-3)
    del spectra, out
    return {"kernel_ms": kms, "ms_per_step": wall_ms, "shape": list(x32.shape[::-1]),
            "matches_input_rows": ok,
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM_BPS / 1e9,
                         "unit": "GB/s", "frac": achieved / PEAK_HBM_BPS,
                         "alg_bytes_per_launch": nbytes}}


# --------------------------------------------------------------------------
# Real-time front end (section 5) on the toy observation of its test


def run_frontend(dd, torch, args, dm_row=333, t0=20000, width=8, amp=0.5):
    """One buffer of the section 5 pipeline per step, as the paper times it:
    copy 2^19 spectra of 256 complex subbands (12.8 us) from pinned host
    memory, channelise (FFT of 8, power, channel order: 2048 channels at
    102.4 us), de-disperse 500 DMs up to 60, copy the result back.  The sum
    of the stages is compared with the buffer's duration (real time)."""
    fe = synth.FrontEnd()
    band = fe.band()
    dms = fe.dms()
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, dms)
    nt = fe.nspec // fe.nfft
    nout = plan.nout(nt)
    # a dispersed boxcar pulse, placed per subband and FFT bin of the front end
    off = pulse_offsets(dd, band, float(dms[dm_row]))
    start = np.empty((fe.nsub, fe.nfft), dtype=np.int64)
    for j in range(fe.nfft):
        start[:, (fe.nfft // 2 - 1 - j) % fe.nfft] = t0 + off[j::fe.nfft]
    v = synth.voltages_with_pulse(fe.seed, nt, fe.nsub, fe.nfft, start, width, amp)
    h_v = torch.empty((fe.nspec, fe.nsub), dtype=torch.complex64, pin_memory=True)
    h_v.numpy()[:] = v
    del v
    dev = torch.device("cuda:0")
    d_v = torch.empty_like(h_v, device=dev)
    d_p = torch.empty((band.nchans, nt), dtype=torch.float32, device=dev)
    d_out = torch.empty((plan.ndms, nout), dtype=torch.float32, device=dev)
    h_out = torch.empty((plan.ndms, nout), dtype=torch.float32, pin_memory=True)
    stream = torch.cuda.current_stream(dev)
    tile = None
    if not args.no_autotune:
        d_v.copy_(h_v)
        dd.channelise(d_v, fe.nfft, out=d_p)
        tile, _ = plan.autotune(torch.float32, nt)
    names = ["h2d", "channelise", "dedisperse", "d2h"]
    acc = np.zeros(len(names))
    steps = max(3, args.steps // 2)
    for it in range(1 + steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record(stream)
        d_v.copy_(h_v, non_blocking=True)
        ev[1].record(stream)
        dd.channelise(d_v, fe.nfft, out=d_p)
        ev[2].record(stream)
        plan.execute(d_p, out=d_out)
        ev[3].record(stream)
        h_out.copy_(d_out, non_blocking=True)
        ev[4].record(stream)
        torch.cuda.synchronize()
        if it:  # the first pass is warm-up
            acc += [ev[i].elapsed_time(ev[i + 1]) for i in range(len(names))]
    ms = acc / steps
    total = float(ms.sum())
    buffer_ms = fe.nspec * fe.t_samp * 1e3
    snr = boxcar_snr_peak(h_out[dm_row].numpy(), t0, width)
    ch_bytes = fe.nspec * fe.nsub * 8.0 + band.nchans * nt * 4.0
    ch_ach = ch_bytes / (ms[1] * 1e-3)
    # pipelined: two device voltage buffers; the next buffer's host->device
    # copy runs on its own stream while this buffer is processed
    cs = torch.cuda.Stream(dev)
    d_vv = [d_v, torch.empty_like(d_v)]
    freed = [torch.cuda.Event(), torch.cuda.Event()]
    nbuf = 2 * steps
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for k in range(nbuf):
        i = k % 2
        if k >= 2:
            cs.wait_event(freed[i])
        with torch.cuda.stream(cs):
            d_vv[i].copy_(h_v, non_blocking=True)
            landed = torch.cuda.Event()
            landed.record(cs)
        stream.wait_event(landed)
        dd.channelise(d_vv[i], fe.nfft, out=d_p, stream=stream)
        plan.execute(d_p, out=d_out, stream=stream)
        h_out.copy_(d_out, non_blocking=True)
        freed[i].record(stream)
    torch.cuda.synchronize()
    pipe_ms = (time.perf_counter() - tp) * 1e3 / nbuf
    del d_v, d_vv, d_p, d_out, h_v, h_out
    torch.cuda.empty_cache()
    return {"observation": "toy observation of the real-time test: 610 MHz centre, 20 MHz, "
                           "256 subbands at 12.8 us, 8 channels per subband, 500 DMs to 60, "
                           "buffers of 2^19 spectra (complex FP32 voltages)",
            "stage_ms": {n: float(m) for n, m in zip(names, ms)}, "total_ms": total,
            "pipelined_ms_per_buffer": pipe_ms,
            "pipelined_real_time_factor": pipe_ms / buffer_ms,
            "buffer_ms": buffer_ms, "real_time_factor": total / buffer_ms,
            "buffers_per_buffer_time": buffer_ms / total,
            "paper_c1060_total_ms": 5785.0, "tile": tile,
            "injected_pulse": {"dm": float(dms[dm_row]), "t0": t0, "width": width,
                               "power_gain": 1.0 + amp,
                               "expected_snr": amp * math.sqrt(band.nchans * width),
                               "recovered_snr": snr},
            "channelise_roofline": {"bound": "hbm", "achieved": ch_ach / 1e9,
                                    "peak": PEAK_HBM_BPS / 1e9, "unit": "GB/s",
                                    "frac": ch_ach / PEAK_HBM_BPS,
                                    "alg_bytes_per_launch": ch_bytes}}


# --------------------------------------------------------------------------
# Subband de-dispersion (section 3.2) with the paper's Table 1 survey plan

TABLE1_PASSES = [(0.0, 53.46, 0.03, 0.66, 1), (53.46, 88.26, 0.05, 1.2, 2),
                 (88.26, 150.66, 0.10, 2.4, 4)]


def run_subband(dd, torch, w, x32, pulses, args, nsub=32):
    """Subband plan over the FP32 workload (1024 channels) against brute
    force over the same fine DMs at full time resolution."""
    dev = torch.device("cuda:0")
    b = w.band
    sp = dd.SubbandPlan(b.nchans, b.f_top, b.df, b.t_samp, nsub, TABLE1_PASSES)
    xin = torch.from_numpy(x32).to(dev)
    nout, ws = sp.sizes(x32.shape[1])
    out = torch.zeros((sp.ndms, int(nout.max())), dtype=torch.float32, device=dev)
    work = torch.empty(ws, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    kms, wall_ms = timed(stream, lambda: sp.execute(xin, out=out, workspace=work),
                         max(1, args.steps // 2), 1)
    dms, pass_of = sp.dms()
    samples = float(sum(int(nout[p]) for p in pass_of))
    bf = dd.Plan(b.nchans, b.f_top, b.df, b.t_samp, dms)
    bout = torch.empty((bf.ndms, bf.nout(x32.shape[1])), dtype=torch.float32, device=dev)
    bms, _ = timed(stream, lambda: bf.execute(xin, out=bout), max(1, args.steps // 4), 1)
    ratios = []
    for p in pulses:
        if p["dm"] >= TABLE1_PASSES[-1][1]:
            continue
        r = int(np.argmin(np.abs(dms - p["dm"])))
        bin_ = TABLE1_PASSES[int(pass_of[r])][4]
        t0, wd = p["t0"], p["width"]
        sb = boxcar_snr_peak(out[r, : int(nout[pass_of[r]])].cpu().numpy(), t0 // bin_,
                             max(1, wd // bin_))
        bb = boxcar_snr_peak(bout[r].cpu().numpy(), t0, wd)
        ratios.append(sb / bb)
    del out, work, bout, xin
    torch.cuda.empty_cache()
    return {"plan": "Table 1 passes (DM 0-150.66, steps 0.03/0.05/0.10, bins 1/2/4), "
                    f"{nsub} subbands", "ndms": sp.ndms, "kernel_ms": kms, "ms_per_step": wall_ms,
            "value": samples / (wall_ms * 1e-3), "unit": "DM-trial samples/s (binned resolution)",
            "brute_force_same_dms_ms": bms, "speedup_vs_brute_force": bms / kms,
            "pulse_snr_ratio_vs_brute_force": ratios}


# --------------------------------------------------------------------------
# Many beams in one persistent launch
# --------------------------------------------------------------------------


def run_batch(dd, torch, args):
    dev = torch.device("cuda:0")
    specs = synth.batch_beams()
    plans, pulses = [], []
    for sp in specs:
        bd = sp["band"]
        p = dd.Plan(bd.nchans, bd.f_top, bd.df, bd.t_samp, synth.dm_grid(sp["ndms"], sp["step"]))
        plans.append(p)
        nout = p.nout(sp["nsamp"])
        dm_max = float(sp["ndms"] - 1) * sp["step"] * 0.98
        ps = synth.scale_pulses(sp["seed"], 4, nout, dm_max=dm_max, nchans=bd.nchans)
        pulses.append([(pulse_offsets(dd, bd, q["dm"]), q) for q in ps])

    def gen(i):
        sp = specs[i]
        x = synth.noise(sp["band"].nchans, sp["nsamp"], sp["seed"])
        for off, q in pulses[i]:
            synth.add_boxcar(x, off, q["t0"], q["width"], q["amp"])
        return synth.quantize_u8(x)

    log("batch: generating 32 beams")
    xs = []
    oracle_beams = {}  # host copies of the beams the oracle is timed on
    with ThreadPoolExecutor(8) as ex:
        for i, u8 in enumerate(ex.map(gen, range(len(specs)))):
            if i < 2:
                oracle_beams[i] = u8
            # rows start on 64-byte boundaries (pitched allocation)
            pitch = (u8.shape[1] + 63) // 64 * 64
            buf = torch.empty((u8.shape[0], pitch), dtype=torch.uint8, device=dev)
            buf[:, :u8.shape[1]].copy_(torch.from_numpy(u8))
            xs.append(buf[:, :u8.shape[1]])
    bt = dd.Batch([(p, x, None) for p, x in zip(plans, xs)])
    tuned = None
    if not args.no_autotune:
        cfg, ms = bt.autotune()
        tuned = {"tile": cfg, "ms": ms}
    info = bt.info()
    stream = torch.cuda.current_stream(dev)
    steps = max(1, min(args.steps, 10))
    kms, wall_ms = timed(stream, lambda: bt.launch(), steps, max(1, min(args.warmup, 2)))
    samples = sum(p.ndms * p.nout(x.shape[1]) for p, x in zip(plans, xs))
    adds = float(sum(p.ndms * p.nchans * p.nout(x.shape[1]) for p, x in zip(plans, xs)))
    in_bytes = float(sum(x.shape[0] * x.shape[1] for x in xs))
    # the same beams one dd_execute at a time (no batching, no graph)
    def one_by_one():
        for p, x, o in zip(plans, xs, bt.outputs):
            p.execute(x, out=o)
    seq_ms, seq_wall = timed(stream, one_by_one, 1, 1)
    res = {"beams": len(specs), "kernel_ms": kms, "ms_per_step": wall_ms,
           "value": samples / (wall_ms * 1e-3), "unit": "DM-trial samples/s",
           "dm_trial_samples_per_step": samples, "work_items": info["work_items"],
           "grid": info["grid"], "tile": info["tile"], "autotune": tuned,
           "unbatched_ms": seq_wall, "speedup_vs_unbatched": seq_wall / wall_ms,
           "roofline": roofline(adds, in_bytes, samples * 4.0, kms, "TOP/s")}
    if not args.no_cpu_baseline:
        # the oracle on two of the 32 beams (a sample of DM rows each), its add
        # rate extrapolated linearly to the whole batch
        import oracle
        threads = oracle_threads()
        t_adds, t_s, parts = 0.0, 0.0, []
        for i, xh in oracle_beams.items():
            sp = specs[i]
            bd = sp["band"]
            tab = oracle.delay_table(bd.nchans, bd.f_top, bd.df, bd.t_samp,
                                     synth.dm_grid(sp["ndms"], sp["step"]))
            _, rows, d, _ = time_oracle_rows(xh, tab, threads, args.cpu_seconds / 4)
            n_out = xh.shape[1] - int(tab.max())
            t_adds += float(len(rows)) * bd.nchans * n_out
            t_s += d
            parts.append(f"beam {i}: {len(rows)} of {sp['ndms']} DM rows x {n_out} samples x "
                         f"{bd.nchans} ch")
        add_rate = t_adds / t_s
        est_s = adds / add_rate
        res["cpu_baseline"] = {"value": samples / est_s, "unit": "DM-trial samples/s",
                               "cores": threads, "kind": "oracle", "extrapolated": True,
                               "sample": "; ".join(parts) + f" ({t_s:.1f} s); batch time "
                                         f"extrapolated from the add rate: {est_s:.0f} s",
                               "gpu_over_cpu": (samples / (wall_ms * 1e-3)) / (samples / est_s)}
    del bt, xs
    torch.cuda.empty_cache()
    return res


# --------------------------------------------------------------------------
# Streaming beams (continuous batching server)
# --------------------------------------------------------------------------


def run_serve(dd, torch, args, nbeams=64):
    dev = torch.device("cuda:0")
    band = synth.serve_band()
    seed = 2518
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.t_samp, synth.dm_grid(4096, 0.125))
    m = plan.max_shift
    max_chunk = 1 << 17
    period = 1 << 18  # each beam streams a periodic noise buffer, phase-shifted per beam
    assert period > m
    log("serve: generating the noise buffer")
    pool = synth.noise(band.nchans, period, seed)
    for q in synth.serve_pulses(seed, 16, period, nchans=band.nchans):
        synth.add_boxcar_cyclic(pool, pulse_offsets(dd, band, q["dm"]), q["t0"], q["width"],
                                q["amp"])
    pool = synth.quantize_u8(pool)
    # a second period appended so that any chunk is one column slice
    pool = np.concatenate([pool, pool[:, :max_chunk]], axis=1)
    g = synth.rng(seed + 2)
    phase = [int(v) for v in g.integers(0, period, nbeams)]

    # per beam a device ring of 2 max_shift + max_chunk (+64) samples per
    # channel; per chunk in flight its device copy and its output
    ring = (2 * m + max_chunk + 64) * band.nchans
    out_max = plan.ndms * ((max_chunk + 63) // 64 * 64) * 4
    max_inflight, nstreams = 8, 4
    arena_bytes = (nbeams * (ring + 256) + 2 * max_inflight * (out_max + max_chunk * band.nchans)
                   + (1 << 30))
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    srv = dd.Server(arena, torch.uint8, max_inflight=max_inflight, queue_capacity=512,
                    nstreams=nstreams, host_staging_bytes=4 << 30)
    # tile shape for this plan at the largest carry + chunk length (remembered
    # by the library for every execute of that size class)
    tuned_tile, tuned_ms = plan.autotune(torch.uint8, m + max_chunk)
    beams = [srv.add_beam(plan, max_chunk) for _ in range(nbeams)]
    pos = [0] * nbeams
    seq = [0] * nbeams
    stalls = {"n": 0}

    # the client: one thread submits chunks, another collects results and
    # releases their output memory as soon as they finish
    done = {}
    failed = []
    stop = threading.Event()

    def consume():
        while not stop.is_set():
            try:
                rs = srv.poll(256)
                for r in rs:
                    if r.status != dd.DD_OK:
                        failed.append(f"chunk {r.ticket} failed: {dd.status_str(r.status)}")
                    done[r.ticket] = r
                    srv.release(r.ticket)
            except Exception as e:  # reported by the submitting thread
                failed.append(repr(e))
                return
            if not rs:
                time.sleep(2e-4)

    consumer = threading.Thread(target=consume, daemon=True)
    consumer.start()

    def check():
        if failed:
            stop.set()
            raise RuntimeError(failed[0])

    def submit(b, n):
        s = (phase[b] + pos[b]) % period
        while True:
            tk = srv.submit(beams[b], pool[:, s:s + n], seq[b])
            if tk is not None:
                pos[b] += n
                seq[b] += 1
                return tk
            stalls["n"] += 1
            check()
            time.sleep(2e-4)

    def wait_all(tickets):
        while not all(t in done for t in tickets):
            check()
            time.sleep(2e-4)

    # warm-up: every beam needs max_shift samples of history before its first output
    log(f"serve: warming {nbeams} beams ({m} samples each)")
    t_w = time.perf_counter()
    warm = []
    for b in range(nbeams):
        left = m
        while left > 0:
            n = min(left, max_chunk)
            warm.append(submit(b, n))
            left -= n
    wait_all(warm)
    warm_s = time.perf_counter() - t_w

    # paced phase: Poisson arrivals at 1.5x real time
    mean_len = (2.0 ** 17 - 2.0 ** 14) / (math.log(2.0) * 3.0)
    per_beam = int(math.ceil(args.serve_seconds * 1.5 / (mean_len * band.t_samp) * 2)) + 4
    events = [e for e in synth.serve_arrivals(seed, nbeams, per_beam * nbeams, band.t_samp, 1.5)
              if e[0] < args.serve_seconds]
    log(f"serve: paced phase, {len(events)} chunks over {args.serve_seconds:g} s")
    sched = {}
    t_start = time.monotonic() + 0.2
    stalls["n"] = 0
    for (t_arr, b, _, n) in events:
        due = t_start + t_arr
        while True:
            now = time.monotonic()
            if now >= due:
                break
            time.sleep(min(5e-4, due - now))
        tk = submit(b, n)
        sched[tk] = (due, n)
    wait_all(list(sched))
    paced_wall = time.monotonic() - t_start
    lat = np.array([done[t].t_done - sched[t][0] for t in sched])
    compute = np.array([done[t].t_done - done[t].t_admit for t in sched])
    paced_samples = sum(n for _, n in sched.values())
    paced_stalls = stalls["n"]

    # saturating phase: a backlog of chunks submitted as fast as admission allows
    g2 = synth.rng(seed + 3)
    lens = [int(math.floor(2.0 ** g2.uniform(14.0, 17.0))) for _ in range(args.serve_saturate)]
    order = [int(v) for v in g2.integers(0, nbeams, args.serve_saturate)]
    log(f"serve: saturating phase, {len(lens)} chunks")
    stalls["n"] = 0
    t0 = time.monotonic()
    sat = [submit(b, n) for b, n in zip(order, lens)]
    wait_all(sat)
    sat_wall = time.monotonic() - t0
    sat_samples = float(sum(lens))
    sat_lat = np.array([done[t].t_done - done[t].t_submit for t in sat])
    stop.set()
    consumer.join()
    srv.close()

    # the plain kernel at the serving shape (carry + one maximum chunk)
    xk = torch.from_numpy(np.ascontiguousarray(pool[:, :m + max_chunk])).to(dev)
    ok = torch.empty((plan.ndms, max_chunk), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    kms, _ = timed(stream, lambda: plan.execute(xk, out=ok), 5, 1)
    kernel_rate = plan.ndms * max_chunk / (kms * 1e-3)
    adds = float(plan.ndms) * plan.nchans * max_chunk

    # the plain kernel over the saturating phase's own chunks (carry + each
    # chunk length, in the same order) back to back on one stream: the same
    # kernel work with none of the serving machinery around it
    def same_chunks():
        for n in lens:
            plan.execute(xk[:, :m + n], out=ok[:, :n])
    mix_ms, _ = timed(stream, same_chunks, 1, 1)
    mix_rate = sat_samples * plan.ndms / (mix_ms * 1e-3)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on one beam's carry + largest chunk (a sample of DM rows),
        # extrapolated to the 4096 rows of the chunk
        import oracle
        threads = oracle_threads()
        tab = oracle.delay_table(band.nchans, band.f_top, band.df, band.t_samp,
                                 synth.dm_grid(4096, 0.125))
        xo = np.ascontiguousarray(pool[:, :m + max_chunk])
        rate, rows, d, _ = time_oracle_rows(xo, tab, threads, args.cpu_seconds / 4)
        chunk_s = plan.ndms * max_chunk / rate
        cpu = {"value": rate, "unit": "DM-trial samples/s", "cores": threads, "kind": "oracle",
               "extrapolated": True,
               "sample": f"{len(rows)} of {plan.ndms} DM rows x {max_chunk} samples x "
                         f"{band.nchans} ch of one 2^17-sample chunk ({d:.1f} s); whole chunk "
                         f"extrapolated: {chunk_s:.0f} s",
               "real_time_factor_64_beams": chunk_s * nbeams / (max_chunk * band.t_samp)}
        del xo

    obs = paced_samples * band.t_samp / nbeams
    return {
        "cpu_baseline": cpu,
        "beams": nbeams, "nchans": band.nchans, "ndms": plan.ndms, "max_shift": m,
        "tile": tuned_tile,
        "chunk_samples": [1 << 14, max_chunk], "arrival_rate_x_realtime": 1.5,
        "warmup_s": warm_s,
        "paced": {"window_s": args.serve_seconds, "chunks": len(sched),
                  "p50_ms": float(np.percentile(lat, 50) * 1e3),
                  "p99_ms": float(np.percentile(lat, 99) * 1e3),
                  "max_ms": float(lat.max() * 1e3),
                  "p50_gpu_ms": float(np.percentile(compute, 50) * 1e3),
                  "wall_s": paced_wall, "observation_s_per_beam": obs,
                  "admission_stalls": paced_stalls,
                  "value": paced_samples * plan.ndms / paced_wall},
        "saturated": {"chunks": len(sat), "wall_s": sat_wall,
                      "value": sat_samples * plan.ndms / sat_wall,
                      "unit": "DM-trial samples/s",
                      "real_time_factor": sat_wall / (sat_samples * band.t_samp / nbeams),
                      "p50_ms": float(np.percentile(sat_lat, 50) * 1e3),
                      "p99_ms": float(np.percentile(sat_lat, 99) * 1e3),
                      "admission_stalls": stalls["n"]},
        "kernel_at_chunk_shape": {"kernel_ms": kms, "value": kernel_rate,
                                  "roofline": roofline(adds, float(xk.numel()),
                                                       plan.ndms * max_chunk * 4.0, kms,
                                                       "TOP/s")},
        "served_over_kernel": (sat_samples * plan.ndms / sat_wall) / kernel_rate,
        "kernel_same_chunks": {"chunks": len(lens), "kernel_ms": mix_ms, "value": mix_rate},
        "served_over_kernel_same_chunks": (sat_samples * plan.ndms / sat_wall) / mix_rate,
    }


# --------------------------------------------------------------------------


def copy_calibration(torch, args):
    """One plain device copy of 1 GiB (reads 1 GiB, writes 1 GiB), the last
    kernel of the run, for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE."""
    if not args.copy_calibration:
        return
    dev = torch.device("cuda:0")
    torch.cuda.empty_cache()
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize(dev)
    dst.copy_(src)
    torch.cuda.synchronize(dev)


def base_line(args, metric_value, ms_per_step, dtype, config, rl):
    return {
        "metric": "DM-trial samples/s",
        "value": metric_value,
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": rl,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding over several GPUs is "
                                   "designed but not launched (use --gpus 1)"}))
        sys.exit(2)
    import torch
    import paper_1107_2516_amd as dd

    name = args.workload
    if name == "batch_u8":
        r = run_batch(dd, torch, args)
        r["roofline"]["traffic"] = traffic_for(name)
        line = base_line(args, r["value"], r["ms_per_step"], "u8",
                         {"workload": "batch_u8: 32 beams, 256-1024 ch 1214-1510 MHz, 64 us, "
                                      "2^16-2^18 samples, 1024-4096 DMs, u8 noise + 4 pulses "
                                      "each, one persistent graph-captured launch",
                          "beams": r["beams"]}, r.pop("roofline"))
        line["batch"] = r
        copy_calibration(torch, args)
        print(json.dumps(line), flush=True)
        return
    if name == "serve_u8":
        r = run_serve(dd, torch, args)
        line = base_line(args, r["saturated"]["value"], r["saturated"]["wall_s"] * 1e3, "u8",
                         {"workload": "serve_u8: 64 beams, 2048 ch 120-180 MHz, 327.68 us, 4096 "
                                      "DMs step 0.125, Poisson chunks of 2^14-2^17 samples at "
                                      "1.5x real time"},
                         r["kernel_at_chunk_shape"].pop("roofline"))
        line["roofline"]["traffic"] = traffic_for(name)
        line["serve"] = r
        copy_calibration(torch, args)
        print(json.dumps(line), flush=True)
        return

    w, plan, x32, pulses = make_workload(dd, name)
    dt = name.rsplit("_", 1)[1]
    xs = {dt: convert(x32, dt)}
    log(f"{name}: timing")
    main_r, main_out = run_single(dd, torch, plan, w, xs[dt], dt, args)
    main_r["roofline"]["traffic"] = traffic_for(name)
    cfg = {"workload": describe(name, w), "nchans": w.band.nchans, "ndms": plan.ndms,
           "nsamp": w.nsamp, "nout": plan.nout(w.nsamp), "max_shift": plan.max_shift,
           "tile": main_r["tile"]}
    line = base_line(args, main_r["value"], main_r["ms_per_step"], dt, cfg, main_r["roofline"])
    line["real_time_factor"] = main_r["real_time_factor"]
    log(f"{name}: host<->device copies")
    cp = run_copies(torch, xs[dt], main_out)
    cp["value_with_copies"] = plan.ndms * plan.nout(w.nsamp) / (
        (cp["h2d_ms"] + main_r["kernel_ms"] + cp["d2h_ms"]) * 1e-3)
    line["copies"] = cp
    outs = {dt: main_out}
    extras = name == "scale_f32" and not args.only
    if extras:
        prec = {"f32": {"value": main_r["value"], "kernel_ms": main_r["kernel_ms"],
                        "frac": main_r["roofline"]["frac"],
                        "hbm_gbs_algorithmic": main_r["roofline"]["hbm_gbs_algorithmic"],
                        "pulse_snr": pulse_snrs(main_out, w, pulses)}}
        for pdt in ("u8", "f16"):
            log(f"precision {pdt}: timing")
            xs[pdt] = convert(x32, pdt)
            r, o = run_single(dd, torch, plan, w, xs[pdt], pdt, args)
            outs[pdt] = o
            prec[pdt] = {"value": r["value"], "kernel_ms": r["kernel_ms"],
                         "frac": r["roofline"]["frac"], "tile": r["tile"],
                         "hbm_gbs_algorithmic": r["roofline"]["hbm_gbs_algorithmic"],
                         "speedup_vs_f32": main_r["kernel_ms"] / r["kernel_ms"],
                         "pulse_snr": pulse_snrs(o, w, pulses)}
        prec["injected_snr"] = [p["snr"] for p in pulses]
        line["precision"] = prec
    if (extras or args.detect) and dt == "f32":
        log("detect: timing")
        line["detect"] = run_detect(dd, torch, main_out, w, pulses, args)
    if (extras or args.corner) and dt == "f32":
        log("corner turn: timing")
        line["corner_turn"] = run_corner(dd, torch, x32, args)
    if (extras or args.subband) and dt == "f32":
        log("subband: timing")
        line["subband"] = run_subband(dd, torch, w, x32, pulses, args)
    if (extras or args.frontend) and dt == "f32":
        log("front end: timing")
        line["frontend"] = run_frontend(dd, torch, args)
    if not args.no_cpu_baseline:
        if "f32" not in xs:
            xs["f32"] = x32
        log("cpu baseline: timing the oracle")
        line["cpu_baseline"] = cpu_baseline(w, xs, outs, args.cpu_seconds)
        line["cpu_baseline"]["gpu_over_cpu"] = line["value"] / line["cpu_baseline"]["value"]
        sc = line["cpu_baseline"]["single_core"]
        sc["gpu_over_single_core"] = line["value"] / sc["value"]
    del outs, main_out
    torch.cuda.empty_cache()
    if extras:
        log("batch: start")
        line["batch"] = run_batch(dd, torch, args)
        log("serve: start")
        line["serve"] = run_serve(dd, torch, args)
    copy_calibration(torch, args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
