"""Benchmark: brute-force de-dispersion throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lofar-f32]

A step is one de-dispersion of the whole workload (every trial DM x every output
sample x every channel) with the input already resident in HBM.  Prints one JSON
line with DM*channel*samples/s, the real-time factor, the roofline of the
dominant kernel (timed with HIP events on the launch stream) and the oracle's
throughput on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM·chan·samples/s + real-time factor on 1 GPU; p50/p99 block latency served"
UNIT = "DM·chan·samples/s"

# MI355X: 256 CUs x 4 SIMDs x 32 lanes per clock for a full-rate 32-bit VALU op
# (v_add_f32 / v_add_u32) at 2.4 GHz = 78.6e12 adds/s, i.e. the published
# 157.3 TFLOP/s fp32 vector peak counted as one add per FMA slot.
ALU_PEAK_TADDS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1111_6399_amd import workloads as wl
    if name == "lofar-f32":
        return wl.lofar("f32")
    if name == "lofar-u8":
        return wl.lofar("u8")
    if name == "lofar-f16":
        return wl.lofar("f16")
    if name == "small-f32":
        return wl.small_f32()
    if name == "meerkat-u8":
        return wl.meerkat_block()
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(x, shift, nsamp, ndm, nchans, target_s=12.0):
    """Time the oracle (binary64 plain loop, OpenMP) on a bounded sample of trials."""
    import oracle
    threads = oracle.num_threads()
    rows = np.linspace(0, ndm - 1, 16).astype(np.int32)
    t = time.perf_counter()
    oracle.dedisperse(x, shift, nsamp, rows=rows)
    pilot = time.perf_counter() - t
    n = int(min(ndm, max(16, 16 * target_s / max(pilot, 1e-3))))
    rows = np.linspace(0, ndm - 1, n).astype(np.int32)
    reps = 0
    t = time.perf_counter()
    while True:  # the whole grid may take less than the target: repeat it
        oracle.dedisperse(x, shift, nsamp, rows=rows)
        reps += 1
        dt = time.perf_counter() - t
        if dt >= 0.5 * target_s or reps >= 50:
            break
    return {"value": reps * n * nchans * nsamp / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": "%d x (%d of %d trials x %d output samples x %d channels), %.1f s"
                      % (reps, n, ndm, nsamp, nchans, dt)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lofar-f32")
    ap.add_argument("--variant", type=int, default=-1, help="force a kernel variant (default: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain device copy of the input (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the de-dispersion path here runs on a single device "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import oracle
    from paper_1111_6399_amd import dedisp as dd
    from paper_1111_6399_amd import workloads as wl

    w = workload(args.workload)
    b = w.band
    log("workload %s: %d ch x %d trials x %d samples (%s)" % (w.name, b.nchans, w.ndm, w.nsamp, w.dtype))
    plan = dd.Plan.for_workload(w)
    shift = plan.shift_table()
    x = wl.generate(w, shift, plan.max_shift)
    log("input generated: %.2f GB" % (x.nbytes / 1e9))
    if args.variant >= 0:
        plan.variant = args.variant
    else:
        t = time.perf_counter()
        v, ms = dd.dedisp_autotune(plan.handle, w.nsamp)
        log("autotune: variant %d, %.3f ms (%.1f s)" % (v, ms, time.perf_counter() - t))

    dev = torch.device("cuda:0")
    xin = torch.from_numpy(x).to(dev)
    odt = torch.int32 if w.dtype == "u8" else torch.float32
    out = torch.empty((w.ndm, w.nsamp), dtype=odt, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        plan.execute(xin, out, w.nsamp, stream)
    torch.cuda.synchronize()
    log("warmup done, variant %d" % plan.variant)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.execute(xin, out, w.nsamp, stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(bb) for a, bb in ev]
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = float(np.mean(kms))
    log("timed %d steps: %.3f ms/step wall, kernel %.3f ms (min %.3f)" % (args.steps, ms_per_step, kernel_ms,
                                                                          min(kms)))

    adds = float(w.ndm) * b.nchans * w.nsamp
    value = adds / (ms_per_step * 1e-3)
    rtf = w.nsamp * b.tsamp / (ms_per_step * 1e-3)
    achieved = adds / (kernel_ms * 1e-3) / 1e12
    esize = x.itemsize
    alg_bytes = (b.nchans * (w.nsamp + plan.max_shift) * esize + w.ndm * w.nsamp * 4
                 + b.nchans * w.ndm * 4)

    if args.copy_calibration:
        # a plain copy of known size, so that profiler byte counters can be scaled
        buf = torch.empty_like(xin)
        buf.copy_(xin)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (xin.numel() * xin.element_size(),
                                                                   buf.numel() * buf.element_size()))
        del buf

    # spot check of the timed output against the oracle on a few trials
    rows = np.array(sorted({0, w.ndm // 3, w.ndm - 1} | {p[0] for p in w.pulses[:2]}), dtype=np.int32)
    got = out[torch.from_numpy(rows).long().to(dev)].cpu().numpy().astype(np.float64)
    want = oracle.dedisperse(x, shift, w.nsamp, rows=rows).astype(np.float64)
    if w.dtype == "u8":
        ok = bool(np.array_equal(got, want))
    else:
        ax = np.abs(x.astype(np.float32))
        scale = oracle.dedisperse(ax, shift, w.nsamp, rows=rows)
        ok = bool(np.all(np.abs(got - want) <= 1e-5 * scale))
    log("spot check vs oracle on %d trials: %s" % (rows.size, "ok" if ok else "MISMATCH"))

    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": w.dtype, "data": "synthetic",
        "config": {"workload": w.name, "nchans": b.nchans, "ndm": w.ndm, "nsamp": w.nsamp,
                   "f_top_mhz": b.f_top, "df_mhz": b.df, "tsamp_s": b.tsamp, "max_shift": plan.max_shift,
                   "variant": plan.variant},
        "rtf": rtf, "pct_realtime": 100.0 / rtf, "parity_spot_check": ok,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TADDS, "unit": "Tadd/s",
                     "frac": achieved / ALU_PEAK_TADDS, "traffic": None,
                     "kernel_ms": kernel_ms, "hbm_alg_GBps": alg_bytes / (kernel_ms * 1e-3) / 1e9},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        res["cpu_baseline"] = cpu_baseline(x, shift, w.nsamp, w.ndm, b.nchans)
        log("oracle: %.3g %s on %d threads" % (res["cpu_baseline"]["value"], UNIT, res["cpu_baseline"]["cores"]))
    print(json.dumps(res), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
