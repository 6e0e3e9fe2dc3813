"""Benchmark: brute-force de-dispersion throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lofar-f32]

A step is one de-dispersion of the whole workload (every trial DM x every output
sample x every channel) with the input already resident in HBM.  Prints one JSON
line with DM*channel*samples/s, the real-time factor, the roofline of the
dominant kernel (timed with HIP events on the launch stream) and the CPU
baseline leg: the oracle's throughput on the host cores over a bounded sample,
beside which the timed output is checked against the oracle on a few trials
(the only place this script touches the oracle; --no-cpu-baseline skips it).
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

# MI355X published float32 vector peak, 157.3 TFLOP/s, counted as one add per
# FMA slot: 256 CUs x 2.4 GHz x 128 lane-adds per clock = 78.6e12 adds/s.
# Reaching it takes packed float32 instructions (two adds a lane), which this
# build does not use; without them the same units give half of it, 39.3e12
# (64 lane-adds per CU and clock).  Both fractions are reported.
ALU_PEAK_TADDS = 256 * 128 * 2.4e9 / 1e12
ALU_UNPACKED_TADDS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# LDS: one ds_read_b64 (512 bytes a wave) keeps a CU's LDS busy for 2 clocks
# (SQ_LDS_IDX_ACTIVE = 2 x SQ_INSTS_LDS on the tile kernels), i.e. 256 bytes
# per clock per CU, 157 TB/s for the chip.  The accumulation reads 4 bytes per
# float add and 2 bytes per add of 16-bit staged samples (half, or two 8-bit
# samples per 32-bit add), times 64/63 for the halo lane.
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12
# The paper's own estimate for its GPU kernel: about 40-50 % of the peak of an
# NVIDIA Fermi GPU (section "Conclusions"; "peak" not defined there).
PAPER_CONTEXT = ("paper: GPU kernel estimated at ~40-50% of peak on an NVIDIA Fermi GPU (section Conclusions); "
                 "CPU comparison on Sandy Bridge / Xeon with vector intrinsics; no absolute rates in the text")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1111_6399_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")


def kernel_sha() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()


def _record(path: str, key: str, variant: int):
    try:
        rec = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha256") != kernel_sha() or rec.get("variant") != variant:
        return None
    return rec


def measured_traffic(workload_name: str, variant: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (scaled by a plain copy), or None when the
    kernel source or variant differs from the one the counters were taken on."""
    rec = _record(TRAFFIC_FILE, "%s/v%d" % (workload_name, variant), variant)
    if rec is None:
        return None
    return {"bytes": rec["fetch_bytes"] + rec["write_bytes"], "fetch_bytes": rec["fetch_bytes"],
            "write_bytes": rec["write_bytes"], "source": rec.get("source")}


def measured_counters(workload_name: str, variant: int):
    """Instruction and LDS counters per launch of the dominant kernel from the
    committed rocprofv3 summary, or None when the kernel changed since."""
    return _record(COUNTERS_FILE, "%s/v%d" % (workload_name, variant), variant)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


def device_beam_input(w, max_shift, dev):
    """Input of one beam of the batched mix, drawn on the device: N(0,1) from
    torch's Philox generator seeded with the beam's seed (float32), or its
    8-bit quantisation round(clip(64 + 16 z, 0, 255))."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(int(w.seed))
    z = torch.randn((w.band.nchans, w.nsamp + int(max_shift)), generator=g, device=dev, dtype=torch.float32)
    if w.dtype == "f32":
        return z
    q = torch.clamp(torch.round(64.0 + 16.0 * z), 0.0, 255.0).to(torch.uint8)
    del z
    return q


def spot_check(x_host, shift, nsamp, out_rows, rows, dtype):
    """Compare output rows with the oracle on the same input (exact for uint8,
    per-element 1e-5 of the absolute sum for float)."""
    import oracle
    want = oracle.dedisperse(x_host, shift, nsamp, rows=rows).astype(np.float64)
    got = out_rows.astype(np.float64)
    if dtype == "u8":
        return bool(np.array_equal(got, want))
    scale = oracle.dedisperse(np.abs(x_host.astype(np.float32)), shift, nsamp, rows=rows)
    return bool(np.all(np.abs(got - want) <= 1e-5 * scale))


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
        if dt >= target_s or reps >= 50:
            break
    return {"value": reps * n * nchans * nsamp / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d x (%d of %d trials x %d output samples x %d channels), %.1f s"
                      % (reps, n, ndm, nsamp, nchans, dt)}


def cpu_vectorised(plan, x, nsamp, ndm, nchans, target_s=8.0):
    """Time the library's vectorised host search on the whole workload, with
    as many threads as the oracle uses, repeated up to about target_s seconds."""
    import oracle
    from paper_1111_6399_amd import dedisp as dd
    threads = oracle.num_threads()
    out = np.empty((ndm, nsamp), dtype=np.int32 if x.dtype == np.uint8 else np.float32)
    reps = 0
    t = time.perf_counter()
    while True:
        isa = dd.dedisp_execute_cpu(plan.handle, x, out, nsamp, threads)
        reps += 1
        dt = time.perf_counter() - t
        if dt >= 0.5 * target_s or reps >= 20:
            break
    return {"value": reps * float(ndm) * nchans * nsamp / dt, "unit": UNIT, "cores": threads, "cpu_model": cpu_model(),
            "kind": "vectorised host search (dedisp_execute_cpu)", "isa": {2: "avx512", 1: "avx2", 0: "scalar"}[isa],
            "sample": "%d x the whole workload, %.1f s" % (reps, dt)}


def oracle_leg(w, plan, shift, x, out) -> dict:
    """The CPU baseline leg of a single-beam workload: the timed output
    checked against the oracle on a few trials (and, for float16 input, the
    per-trial error against the oracle on the original float32 data), then
    the oracle and the vectorised host search timed on the host cores."""
    import torch

    import oracle
    from paper_1111_6399_amd import workloads as wl

    b = w.band
    dev = out.device
    res = {}
    rows = np.array(sorted({0, w.ndm // 3, w.ndm - 1} | {p[0] for p in w.pulses[:2]}), dtype=np.int32)
    got = out[torch.from_numpy(rows).long().to(dev)].cpu().numpy()
    res["parity_spot_check"] = spot_check(x, shift, w.nsamp, got, rows, w.dtype)
    log("spot check vs oracle on %d trials: %s" % (rows.size, "ok" if res["parity_spot_check"] else "MISMATCH"))
    if w.dtype == "f16":
        # per-trial error against the binary64 oracle on the original float32
        # data (the float16 quantisation included), on every 16th trial
        x32 = wl.generate(wl.lofar("f32", nsamp=w.nsamp, ndm=w.ndm), shift, plan.max_shift)
        rows = np.arange(0, w.ndm, 16, dtype=np.int32)
        got = out[torch.from_numpy(rows).long().to(dev)].cpu().numpy().astype(np.float64)
        want = oracle.dedisperse(x32, shift, w.nsamp, rows=rows)
        err = np.abs(got - want).max(axis=1) / np.maximum(np.abs(want).max(axis=1), 1e-30)
        res["f16_error_per_trial"] = {"min": float(err.min()), "median": float(np.median(err)),
                                      "max": float(err.max()), "trials": int(rows.size),
                                      "measure": "max_t |y - y64| / max_t |y64|, y64 on the float32 data"}
        log("float16 per-trial error vs float32 data: min %.3g median %.3g max %.3g"
            % (err.min(), np.median(err), err.max()))
        del x32
    log("timing the oracle on the host ...")
    res["cpu_baseline"] = cpu_baseline(x, shift, w.nsamp, w.ndm, b.nchans)
    log("oracle: %.3g %s on %d threads" % (res["cpu_baseline"]["value"], UNIT, res["cpu_baseline"]["cores"]))
    log("timing the vectorised host search ...")
    res["cpu_vectorised"] = cpu_vectorised(plan, x, w.nsamp, w.ndm, b.nchans)
    log("host search: %.3g %s (%s)" % (res["cpu_vectorised"]["value"], UNIT, res["cpu_vectorised"]["isa"]))
    return res


def run_batch(args) -> dict:
    """32 uneven beams (MeerKAT half-L band, nchans 256/496/1024, 2^14..2^17
    samples, 512..4096 trials, float32/uint8 mix) in one persistent launch
    replayed from a HIP graph, against the same beams launched one by one on
    one stream with each plan's own tuned variant."""
    import torch

    from paper_1111_6399_amd import dedisp as dd
    from paper_1111_6399_amd import workloads as wl

    dev = torch.device("cuda:0")
    beams = wl.batch_beams()
    plans, ins, outs = [], [], []
    t = time.perf_counter()
    for w in beams:
        p = dd.Plan.for_workload(w)
        plans.append(p)
        ins.append(device_beam_input(w, p.max_shift, dev))
        odt = torch.int32 if w.dtype == "u8" else torch.float32
        outs.append(torch.empty((w.ndm, w.nsamp), dtype=odt, device=dev))
    torch.cuda.synchronize()
    adds = float(sum(w.ndm * w.band.nchans * w.nsamp for w in beams))
    in_bytes = sum(x.numel() * x.element_size() for x in ins)
    out_bytes = sum(o.numel() * o.element_size() for o in outs)
    log("batch: %d beams, %.3g adds, inputs %.2f GB, outputs %.2f GB (set-up %.1f s)"
        % (len(beams), adds, in_bytes / 1e9, out_bytes / 1e9, time.perf_counter() - t))
    ip = [x.data_ptr() for x in ins]
    op = [o.data_ptr() for o in outs]
    stream = torch.cuda.current_stream()

    # each plan tuned on its own first: the plain form runs with these, and the
    # batch's autotune also tries the split that follows them
    t = time.perf_counter()
    for p, w in zip(plans, beams):
        if args.variant < 0:
            dd.dedisp_autotune(p.handle, w.nsamp)
    log("per-beam autotune %.1f s" % (time.perf_counter() - t))

    batch = dd.dedisp_batch_create([p.handle for p in plans], [w.nsamp for w in beams])
    try:
        t = time.perf_counter()
        if args.variant >= 0:
            dd.dedisp_batch_set_variant(batch, args.variant)
            dd.dedisp_batch_execute(batch, ip, op, stream)
        else:
            v, ms = dd.dedisp_batch_autotune(batch, ip, op, stream)
            log("batch autotune: variant %d, %.3f ms (%.1f s)" % (v, ms, time.perf_counter() - t))
        for _ in range(args.warmup):
            dd.dedisp_batch_execute(batch, ip, op, stream)
        torch.cuda.synchronize()
        items, groups = dd.dedisp_batch_info(batch)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(stream)
            dd.dedisp_batch_execute(batch, ip, op, stream)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        batch_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        variant = dd.dedisp_batch_get_variant(batch)
        layout = dd.dedisp_batch_get_layout(batch)
    finally:
        dd.dedisp_batch_destroy(batch)
    ms_per_step = wall * 1e3 / args.steps
    log("batched graph: %.3f ms/step wall, %.3f ms median (variant %d, layout %d, %d items, %d workgroups)"
        % (ms_per_step, batch_ms, variant, layout, items, groups))

    # three trials of every beam as the batch left them, to compare with the
    # plain launches below (the float sums have one order in every variant,
    # so the two agree bit for bit; parity with the oracle is the tests' part)
    check_rows = [np.array(sorted({0, w.ndm // 2, w.ndm - 1}), dtype=np.int64) for w in beams]
    kept = [o[torch.from_numpy(r).to(dev)].cpu() for o, r in zip(outs, check_rows)]

    # the plain form: one launch per beam on one stream, each plan tuned on its own

    def plain():
        for p, w, x, o in zip(plans, beams, ins, outs):
            p.execute(x, o, w.nsamp, stream)

    for _ in range(args.warmup):
        plain()
    torch.cuda.synchronize()
    evp = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        evp[i][0].record(stream)
        plain()
        evp[i][1].record(stream)
    torch.cuda.synchronize()
    plain_ms = float(np.median([a.elapsed_time(b) for a, b in evp]))
    log("plain per-beam launches: %.3f ms median" % plain_ms)
    ok = all(torch.equal(k, o[torch.from_numpy(r).to(dev)].cpu()) for k, o, r in zip(kept, outs, check_rows))
    log("batch output equals the plain launches' on 3 trials of each beam: %s" % ("yes" if ok else "NO"))

    achieved = adds / (batch_ms * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": adds / (ms_per_step * 1e-3), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+u8", "data": "synthetic",
        "config": {"workload": "batch-32-beams", "nbeams": len(beams), "adds": adds, "in_bytes": in_bytes,
                   "out_bytes": out_bytes, "variant": variant, "layout": layout, "work_items": items,
                   "workgroups": groups},
        "rtf": sum(w.nsamp * w.band.tsamp for w in beams) / (batch_ms * 1e-3),
        "batch_equals_plain": ok,
        "plain_per_beam": {"ms": plain_ms, "value": adds / (plain_ms * 1e-3)},
        "speedup_vs_plain": plain_ms / batch_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TADDS, "unit": "Tadd/s",
                     "frac": achieved / ALU_PEAK_TADDS, "traffic": None, "kernel_ms": batch_ms},
    }


# served latency targets: a quarter and a half of a 2.1 s MeerKAT block
P99_TARGET_S = 0.5
P99_TARGETS_S = (0.5, 1.0)


def served_compare(nbeams, rate_x, warmup_s, duration, inflight=8, budget_gb=128.0, pool_n=4, max_backlog=256,
                   variant=-1, plan=None):
    """64 MeerKAT-shaped beams (4096 channels, 4096 trials 0-2047.5, uint8),
    blocks of 32768 samples arriving as independent per-beam Poisson
    processes at rate_x times real time in aggregate.  Latency runs from a
    block's scheduled arrival (block already in pinned host memory) to its
    output being complete on the device.  The same arrival schedule is then
    replayed through the plain form: one FIFO, one stream, each block copied
    behind its beam's history and launched on its own.  Returns (served,
    plain, plan)."""
    import torch

    from paper_1111_6399_amd import dedisp as dd
    from paper_1111_6399_amd import workloads as wl

    dev = torch.device("cuda:0")
    B = 32768
    w = wl.meerkat_block(B)
    if plan is None:
        plan = dd.Plan.for_workload(w)
        if variant >= 0:
            plan.variant = variant
        else:
            v, ms = dd.dedisp_autotune(plan.handle, B)
            log("autotune on one block: variant %d, %.3f ms" % (v, ms))
    m = plan.max_shift
    nch, ndm = w.band.nchans, w.ndm
    block_s = B * w.band.tsamp
    work = float(ndm) * nch * B

    # a pool of distinct pinned blocks, cycled through by (beam, block)
    pool = [torch.from_numpy(wl.stream_block(5, k, 0, nch, B)).pin_memory() for k in range(pool_n)]
    rng = np.random.default_rng(5)
    rate = rate_x / block_s  # per beam, blocks/s
    horizon = warmup_s + duration
    arrivals = []
    for b in range(nbeams):
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t > horizon:
                break
            arrivals.append((t, b, k))
            k += 1
    arrivals.sort()
    log("served at %.2fx real time: %d beams, %d blocks over %.0f s (offered %.1f blocks/s = %.3g adds/s)"
        % (rate_x, nbeams, len(arrivals), horizon, len(arrivals) / horizon, work * len(arrivals) / horizon))

    def replay(submit, poll_done, nslots, label):
        """Drive one arrival schedule; submit(beam, blk, out) -> handle or None;
        poll_done(handle) -> bool.  Returns latencies of blocks arriving after
        the warm-up, the completion span and the largest backlog."""
        outs = [torch.empty((ndm, B), dtype=torch.int32, device=dev) for _ in range(nslots)]
        free = list(range(nslots))
        backlog, running, lat, sub_s = [], [], [], []
        t_start = time.perf_counter() + 0.05
        i, max_bl, overload = 0, 0, False
        first_done = last_done = None
        next_report = 15.0
        while i < len(arrivals) or backlog or running:
            now = time.perf_counter() - t_start
            if now >= next_report:
                log("  %s: %.0f s, %d of %d blocks arrived, %d done, backlog %d"
                    % (label, now, i, len(arrivals), len(lat), len(backlog)))
                next_report += 15.0
            while i < len(arrivals) and arrivals[i][0] <= now:
                backlog.append(arrivals[i])
                i += 1
            max_bl = max(max_bl, len(backlog))
            if len(backlog) > max_backlog and not overload:
                # the device cannot keep up with the offered load: stop taking
                # arrivals, finish what was admitted, report the overload
                overload = True
                backlog.clear()
                i = len(arrivals)
            progressed = False
            for r in list(running):
                h, slot, arr = r
                if poll_done(h):
                    tdone = time.perf_counter() - t_start
                    running.remove(r)
                    free.append(slot)
                    if arr[0] >= warmup_s:
                        lat.append(tdone - arr[0])
                        first_done = tdone if first_done is None else first_done
                        last_done = tdone
                    progressed = True
            while backlog and free:
                arr = backlog[0]
                slot = free[-1]
                t0 = time.perf_counter()
                h = submit(arr[1], pool[(arr[1] * 7919 + arr[2]) % len(pool)], outs[slot])
                sub_s.append(time.perf_counter() - t0)
                if h is None:
                    break
                backlog.pop(0)
                free.pop()
                running.append((h, slot, arr))
                progressed = True
            if not progressed:
                time.sleep(0.0002)
        del outs
        return np.array(lat), (first_done, last_done), (max_bl, overload, np.array(sub_s))

    def summary(lat, span, backlog, label):
        n = lat.size
        p50, p99 = (float(np.percentile(lat, 50)), float(np.percentile(lat, 99))) if n else (None, None)
        thr = (n - 1) * work / max(span[1] - span[0], 1e-9) if n > 1 else None
        sub = backlog[2]
        sub_mean, sub_max = (float(sub.mean()), float(sub.max())) if sub.size else (None, None)
        log("%s: %d blocks after warm-up, p50 %.1f ms, p99 %.1f ms, %.3g adds/s, max backlog %d, "
            "submit call %.2f ms mean %.2f ms max%s"
            % (label, n, 1e3 * (p50 or 0), 1e3 * (p99 or 0), thr or 0, backlog[0], 1e3 * (sub_mean or 0),
               1e3 * (sub_max or 0), " (OVERLOADED: arrivals stopped)" if backlog[1] else ""))
        sustained = bool(n > 1 and not backlog[1] and p99 is not None and p99 <= P99_TARGET_S)
        within = {str(t): bool(n > 1 and not backlog[1] and p99 is not None and p99 <= t) for t in P99_TARGETS_S}
        return {"rate_x_realtime": rate_x, "blocks": n, "p50_s": p50, "p99_s": p99, "value": thr,
                "max_backlog": backlog[0], "overloaded": backlog[1], "sustained_at_p99_target": sustained,
                "p99_within": within, "submit_mean_s": sub_mean, "submit_max_s": sub_max}

    server = dd.dedisp_server_create(int(budget_gb * (1 << 30)), inflight)
    try:
        bids = [dd.dedisp_server_add_beam(server, plan.handle, B) for _ in range(nbeams)]

        def s_submit(beam, blk, out):
            return dd.dedisp_submit(server, bids[beam], blk.data_ptr(), out.data_ptr())

        def s_poll(tk):
            return dd.dedisp_poll(server, tk)[0]

        lat, span, backlog = replay(s_submit, s_poll, inflight, "served")
        dd.dedisp_server_drain(server)
        p50s, p99s, rate_s = dd.dedisp_server_stats(server)
    finally:
        dd.dedisp_server_destroy(server)
    served = summary(lat, span, backlog, "served")
    served["server_p50_s"], served["server_p99_s"], served["server_rate"] = p50s, p99s, rate_s

    # plain FIFO: one stream, per beam one history buffer shifted in place
    stream = torch.cuda.Stream()
    hist = {}

    def p_submit(beam, blk, out):
        h = hist.get(beam)
        with torch.cuda.stream(stream):
            if h is None:
                h = torch.zeros((nch, m + B), dtype=torch.uint8, device=dev)
                hist[beam] = h
            else:
                h[:, :m] = h[:, B:B + m].clone()
            h[:, m:].copy_(blk, non_blocking=True)
            plan.execute(h, out, B, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    lat, span, backlog = replay(p_submit, lambda ev: ev.query(), 1, "plain FIFO")
    torch.cuda.synchronize()
    plain = summary(lat, span, backlog, "plain FIFO")
    hist.clear()
    del pool
    torch.cuda.empty_cache()
    return served, plain, plan


def run_served(args) -> dict:
    """The served MeerKAT stream at each rate of --rates (x real time): the
    server and the plain FIFO on the same arrival schedule, p50/p99 latency
    and throughput, and the highest rate each form sustains with p99 within
    P99_TARGET_S."""
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    rows, plan = [], None
    for r in rates:
        served, plain, plan = served_compare(args.beams, r, args.warmup_s, args.duration, args.inflight,
                                             args.budget_gb, args.pool, args.max_backlog, args.variant, plan)
        rows.append({"rate_x_realtime": r, "served": served, "plain_fifo": plain})
    best = {str(t): {form: max([row["rate_x_realtime"] for row in rows if row[form]["p99_within"][str(t)]],
                               default=None) for form in ("served", "plain_fifo")} for t in P99_TARGETS_S}
    for t in P99_TARGETS_S:
        log("highest rate sustained with p99 <= %.0f ms: served %s, plain %s"
            % (1e3 * t, best[str(t)]["served"], best[str(t)]["plain_fifo"]))
    top = rows[0]["served"]
    from paper_1111_6399_amd import workloads as wl
    w = wl.meerkat_block(32768)
    work = float(w.ndm) * w.band.nchans * 32768
    value = top["value"] or 0.0
    achieved = value / 1e12
    return {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": top["blocks"],
        "warmup": args.warmup_s, "ms_per_step": None if not value else work / value * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "served-meerkat", "nbeams": args.beams, "block": 32768, "ndm": w.ndm,
                   "nchans": w.band.nchans, "max_shift": plan.max_shift, "rates_x_realtime": rates,
                   "duration_s": args.duration, "inflight": args.inflight, "variant": plan.variant},
        "p99_targets_s": list(P99_TARGETS_S), "sweep": rows, "highest_sustained_rate_x": best,
        "rtf": None if not value else value / work * 32768 * w.band.tsamp,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TADDS, "unit": "Tadd/s",
                     "frac": achieved / ALU_PEAK_TADDS, "traffic": None},
    }


def run_pipeline(args) -> dict:
    """One MeerKAT-shaped uint8 block through the whole per-block pipeline:
    ingestion (corner turn of the block, time-major as a filterbank stores it,
    into the plan's input behind the history), the search (4096 channels x 4096
    trials x 32768 samples) and detection (boxcar widths 1-512, threshold 8);
    each stage timed alone with HIP events on the launch stream (median over
    --steps), the search against the ALU add peak and the other two against
    the HBM bandwidth of what they must move."""
    import torch

    from paper_1111_6399_amd import dedisp as dd
    from paper_1111_6399_amd import workloads as wl

    dev = torch.device("cuda:0")
    w = wl.meerkat_block()
    nch, n = w.band.nchans, w.nsamp
    plan = dd.Plan.for_workload(w)
    if args.variant >= 0:
        plan.variant = args.variant
    else:
        dd.dedisp_autotune(plan.handle, n)
    m = plan.max_shift
    g = torch.Generator(device=dev)
    g.manual_seed(int(w.seed))
    z = torch.randn((n, nch), generator=g, device=dev)
    block = torch.clamp(torch.round(64.0 + 16.0 * z), 0.0, 255.0).to(torch.uint8)  # time-major
    del z
    x = torch.zeros((nch, n + m), dtype=torch.uint8, device=dev)  # zero history, then the block
    out = torch.empty((w.ndm, n), dtype=torch.int32, device=dev)
    nw, thr, cap = 10, 8.0, 1 << 16
    stats = torch.empty((w.ndm, 2), dtype=torch.float64, device=dev)
    snr = torch.empty((w.ndm, nw), dtype=torch.float64, device=dev)
    tb = torch.empty((w.ndm, nw), dtype=torch.int32, device=dev)
    cand = torch.empty(cap * 4, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    stages = [
        lambda: dd.dedisp_corner_turn(block.data_ptr(), x.data_ptr() + m, n, nch, n + m, "u8", False, stream),
        lambda: plan.execute(x, out, n, stream),
        lambda: dd.dedisp_detect(plan.handle, out.data_ptr(), n, nw, thr, stats.data_ptr(), snr.data_ptr(),
                                 tb.data_ptr(), cand.data_ptr(), cap, count.data_ptr(), stream),
    ]
    for _ in range(max(1, args.warmup)):
        for f in stages:
            f()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)] for _ in stages]
    for i in range(args.steps):
        for k, f in enumerate(stages):
            ev[k][2 * i].record(stream)
            f()
            ev[k][2 * i + 1].record(stream)
    torch.cuda.synchronize()
    ms = [float(np.median([ev[k][2 * i].elapsed_time(ev[k][2 * i + 1]) for i in range(args.steps)]))
          for k in range(len(stages))]
    ncand = int(count.item())
    adds = float(w.ndm) * nch * n
    ingest_gbs = 2.0 * block.numel() / (ms[0] * 1e-3) / 1e9  # read and write every sample once
    detect_gbs = out.numel() * 4 / (ms[2] * 1e-3) / 1e9       # read the block once
    log("ingest %.3f ms (%.0f GB/s), search %.3f ms, detection %.3f ms (%.0f GB/s), %d candidates above S/N %.0f"
        % (ms[0], ingest_gbs, ms[1], ms[2], detect_gbs, ncand, thr))
    total = sum(ms)
    achieved = adds / (ms[1] * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": adds / (total * 1e-3), "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "meerkat-u8 block: ingest + search + detection", "nchans": nch, "ndm": w.ndm,
                   "nsamp": n, "widths": [1 << k for k in range(nw)], "threshold": thr, "variant": plan.variant},
        "stages_ms": {"ingest": ms[0], "search": ms[1], "detect": ms[2]}, "candidates": ncand,
        "rtf": n * w.band.tsamp / (total * 1e-3),
        "roofline": {"bound": "alu", "kernel": "dedisp_tiled", "achieved": achieved, "peak": ALU_PEAK_TADDS,
                     "unit": "Tadd/s", "frac": achieved / ALU_PEAK_TADDS, "traffic": None},
        "stage_rooflines": {
            "ingest": {"bound": "hbm", "achieved": ingest_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ingest_gbs / HBM_PEAK_GBS},
            "detect": {"bound": "hbm", "achieved": detect_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": detect_gbs / HBM_PEAK_GBS}},
    }


def run_fig4(args) -> dict:
    """Both timing sweeps of the paper's Figure 4 on the stand-in band: as many
    trials as channels, equally spaced up to a maximum DM (the library's grid
    planner); (a) 256-4096 channels at a maximum DM of 200, (b) 2000 channels
    with the maximum DM from 25 to 800.  Each point: tuned variant, median
    kernel time over --steps launches (HIP events on the launch stream), and
    that time as a percentage of the data's duration (the paper's axis)."""
    import torch

    from paper_1111_6399_amd import dedisp as dd
    from paper_1111_6399_amd import workloads as wl

    dev = torch.device("cuda:0")
    nsamp = 65536
    points = []
    for sweep, nchans, dm_max in wl.fig4_points():
        band = wl.fig4_band(nchans)
        plan = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dd.dedisp_dm_grid(dm_max, nchans), "f32")
        m = plan.max_shift
        in_bytes, out_bytes, _ = dd.dedisp_plan_footprint(plan.handle, nsamp)
        g = torch.Generator(device=dev)
        g.manual_seed(100000 * nchans + int(dm_max))
        x = torch.randn((nchans, nsamp + m), generator=g, device=dev)
        out = torch.empty((nchans, nsamp), dtype=torch.float32, device=dev)
        stream = torch.cuda.current_stream()
        if args.variant >= 0:
            plan.variant = args.variant
        else:
            dd.dedisp_autotune(plan.handle, nsamp)
        for _ in range(max(1, args.warmup)):
            plan.execute(x, out, nsamp, stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        ev[0].record(stream)
        for i in range(args.steps):
            plan.execute(x, out, nsamp, stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]))
        adds = float(nchans) * nchans * nsamp
        pt = {"sweep": sweep, "nchans": nchans, "ndm": nchans, "dm_max": dm_max, "max_shift": m,
              "input_gb": in_bytes / 1e9, "output_gb": out_bytes / 1e9, "variant": plan.variant,
              "kernel_ms": ms, "adds_per_s": adds / (ms * 1e-3),
              "pct_realtime": 100.0 * ms * 1e-3 / (nsamp * band.tsamp)}
        points.append(pt)
        log("fig4 %-8s nchans=ndm %4d  max DM %5.0f  max_shift %8d  input %6.2f GB  variant %2d  %8.3f ms  "
            "%.3g adds/s  %.3f %% of real time" % (sweep, nchans, dm_max, m, in_bytes / 1e9, plan.variant, ms,
                                                 adds / (ms * 1e-3), pt["pct_realtime"]))
        del x, out
        torch.cuda.empty_cache()
    ref = [p for p in points if p["sweep"] == "channels" and p["nchans"] == 2048][0]
    achieved = ref["adds_per_s"] / 1e12
    return {
        "metric": METRIC, "value": ref["adds_per_s"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ref["kernel_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fig4-sweeps", "reference_point": "2048 channels = trials, max DM 200",
                   "nsamp": nsamp, "band": "150 MHz top, 96.875 MHz wide, 327.68 us"},
        "rtf": 100.0 / ref["pct_realtime"], "sweeps": points,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TADDS, "unit": "Tadd/s",
                     "frac": achieved / ALU_PEAK_TADDS, "traffic": None},
    }


def roofline(w, adds, alg_bytes, kernel_ms, variant) -> dict:
    """Achieved add rate of the timed launches (median of HIP events on their
    stream) against the ALU add peak (and its unpacked half), with the LDS
    read rate the accumulation needs (and the one the counters measured) and
    the HBM traffic from the committed counters."""
    achieved = adds / (kernel_ms * 1e-3) / 1e12
    lds_bytes_per_add = (4.0 if w.dtype == "f32" else 2.0) * 64.0 / 63.0
    lds_tbs = achieved * lds_bytes_per_add
    tr = measured_traffic(w.name, variant)
    ctr = measured_counters(w.name, variant)
    lds = {"model_TBps": lds_tbs, "peak_TBps": LDS_PEAK_TBS, "model_frac": lds_tbs / LDS_PEAK_TBS,
           "bytes_per_add": lds_bytes_per_add}
    if ctr is not None:
        # bytes the counters saw per launch, over this run's median launch time
        meas = ctr["lds_read_bytes"] / (kernel_ms * 1e-3) / 1e12
        lds.update({"measured_TBps": meas, "measured_frac": meas / LDS_PEAK_TBS, "counters": ctr.get("source")})
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TADDS, "unit": "Tadd/s",
            "frac": achieved / ALU_PEAK_TADDS, "frac_unpacked": achieved / ALU_UNPACKED_TADDS,
            "traffic": None if tr is None else tr["bytes"],
            "traffic_detail": tr, "kernel_ms": kernel_ms, "kernel_ms_stat": "median", "alg_bytes": alg_bytes,
            "traffic_over_alg": None if tr is None else tr["bytes"] / alg_bytes,
            "hbm_alg_GBps": alg_bytes / (kernel_ms * 1e-3) / 1e9, "lds": lds,
            "counters": None if ctr is None else {k: v for k, v in ctr.items() if k.startswith(("SQ_", "per_"))},
            "context": PAPER_CONTEXT}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lofar-f32")
    ap.add_argument("--variant", type=int, default=-1, help="force a kernel variant (default: autotune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--beams", type=int, default=64, help="served: number of beams")
    ap.add_argument("--rate", type=float, default=1.5, help="served: aggregate arrival rate, x real time per beam")
    ap.add_argument("--rates", default="", help="served: comma-separated rates to sweep (x real time)")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg of the default workload")
    ap.add_argument("--served-duration", type=float, default=20.0, help="served leg: measured seconds")
    ap.add_argument("--duration", type=float, default=60.0, help="served: measured seconds after the warm-up")
    ap.add_argument("--warmup-s", type=float, default=10.0, help="served: warm-up seconds")
    ap.add_argument("--inflight", type=int, default=8, help="served: requests in flight")
    ap.add_argument("--budget-gb", type=float, default=128.0, help="served: device memory budget")
    ap.add_argument("--pool", type=int, default=4, help="served: distinct pinned blocks cycled through")
    ap.add_argument("--max-backlog", type=int, default=256, help="served: backlog that counts as overload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain device copy of the input (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the de-dispersion path here runs on a single device "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    if args.workload in ("batch-32", "served-meerkat", "fig4", "pipeline-meerkat"):
        res = {"batch-32": run_batch, "served-meerkat": run_served, "fig4": run_fig4,
               "pipeline-meerkat": run_pipeline}[args.workload](args)
        print(json.dumps(res), flush=True)
        return 0 if res.get("batch_equals_plain", True) else 1

    import torch

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
    kernel_ms = float(np.median(kms))
    log("timed %d steps: %.3f ms/step wall, kernel %.3f ms median (min %.3f, mean %.3f)"
        % (args.steps, ms_per_step, kernel_ms, min(kms), float(np.mean(kms))))

    adds = float(w.ndm) * b.nchans * w.nsamp
    value = adds / (ms_per_step * 1e-3)
    rtf = w.nsamp * b.tsamp / (ms_per_step * 1e-3)
    esize = x.itemsize
    # algorithmic bytes: the input region the trials reference (each channel
    # up to its own largest delay), read once; the output written once; the
    # delay table read once
    alg_bytes = (int(b.nchans * w.nsamp + shift.max(axis=1).astype(np.int64).sum()) * esize
                 + w.ndm * w.nsamp * 4 + b.nchans * w.ndm * 4)

    if args.copy_calibration:
        # a plain copy of known size, so that profiler byte counters can be scaled
        buf = torch.empty_like(xin)
        buf.copy_(xin)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (xin.numel() * xin.element_size(),
                                                                   buf.numel() * buf.element_size()))
        del buf

    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": w.dtype, "data": "synthetic",
        "config": {"workload": w.name, "nchans": b.nchans, "ndm": w.ndm, "nsamp": w.nsamp,
                   "f_top_mhz": b.f_top, "df_mhz": b.df, "tsamp_s": b.tsamp, "max_shift": plan.max_shift,
                   "variant": plan.variant},
        "rtf": rtf, "pct_realtime": 100.0 / rtf, "parity_spot_check": None,
        "roofline": roofline(w, adds, alg_bytes, kernel_ms, plan.variant),
    }
    if not args.no_cpu_baseline:
        # the CPU baseline leg (the oracle on the host cores), with the timed
        # output checked against the oracle on a few trials beside it
        res.update(oracle_leg(w, plan, shift, x, out))
    if w.name == "lofar-f32" and not args.no_served:
        # a short served leg: the MeerKAT-shaped stream at 1.5x real time,
        # server against the plain FIFO on the same arrivals
        del xin, out
        torch.cuda.empty_cache()
        log("served leg ...")
        served, plain, splan = served_compare(64, 1.5, 5.0, args.served_duration)
        res["served"] = {"workload": "served-meerkat: 64 beams, 4096 ch x 4096 trials, blocks of 32768 uint8",
                         "rate_x_realtime": 1.5, "p99_target_s": P99_TARGET_S, "variant": splan.variant,
                         "server": served, "plain_fifo": plain}
    print(json.dumps(res), flush=True)
    return 0 if res["parity_spot_check"] in (True, None) else 1


if __name__ == "__main__":
    sys.exit(main())
