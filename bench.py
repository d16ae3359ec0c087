"""Benchmark: UTF-16 toWellFormed throughput on one MI355X.

One step = one pass of the repair over the single-buffer workload: five
buffers of 268,435,456 uint16 units (512 MiB each) — pure ASCII, the
character mix at lone-surrogate rates 0, 1e-6 and 1e-2, and all units uniform
over the surrogate range — each repaired out of place by one launch. The
inputs are resident in HBM before timing starts. ``value`` is GB/s of input
(2 bytes per unit) over the whole job.

The JSON line also carries
  * ``roofline``: the repair kernel's algorithmic bytes (4 per unit: read and
    write) divided by its mean launch time from HIP events on its stream,
    against the 8 TB/s HBM peak; ``traffic`` comes from the rocprofv3 counter
    summary under profiles/ when it was taken on the current kernel source;
  * ``cpu_baseline``: the scalar CPU oracle on one host core over the same
    five buffers, timed by the paper's method (best iteration, error margin);
  * per-variant GB/s for copy, in place and isWellFormed, the copy ceiling,
    the 1,048,576-unit string's latency, the ragged batch in one launch
    against one launch per string (all 1,000,000), the autotuned
    large-batch numbers, the paper's own workloads (the 1M-unit runs, the
    128-point size sweep beside the oracle, the JavaScript strings) flat,
    batched and served, and the serving loop's p50/p99 latency over its
    configured 60 s (skip these with --no-extras).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "toWellFormed GB/s input and % HBM peak; batched vs per-string; serve p99"
PEAK_HBM_GBS = 8000.0
N_UNITS = 1 << 28
KERNEL_SRC = os.path.join(ROOT, "paper_2601_06349_amd", "csrc", "kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "flat_to_single268M_pmc.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch from the committed counter summary, or None when
    missing or taken on a different kernel source."""
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


class Timer:
    """HIP events recorded on the stream the kernels are launched on."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream
        self.pairs = []

    def run(self, fn):
        a = self.torch.cuda.Event(enable_timing=True)
        b = self.torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        fn()
        b.record(self.stream)
        self.pairs.append((a, b))

    def times_ms(self):
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.pairs]


def median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2] if xs else float("nan")


def time_fn(torch, stream, fn, reps=10, setup=None):
    """Median and best event time (ms) of fn over reps, setup untimed."""
    fn()
    torch.cuda.synchronize()
    t = Timer(torch, stream)
    for _ in range(reps):
        if setup:
            setup()
        t.run(fn)
    ts = t.times_ms()
    return median(ts), min(ts)


def paper_timing(fn, iterations=100, min_s=1e-3, budget_s=None):
    """The paper's timing method (Sec. 4): each iteration repeats fn until at
    least min_s has passed and takes the time per call; the result is the
    best iteration, with the median, the mean and the error margin
    (mean - best) / best. With budget_s, stops early (after at least 3
    iterations) once that much time has been spent."""
    times, t_start = [], time.perf_counter()
    for _ in range(iterations):
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            el = time.perf_counter() - t0
            if el >= min_s:
                break
        times.append(el / reps)
        if budget_s is not None and len(times) >= 3 and time.perf_counter() - t_start >= budget_s:
            break
    best = min(times)
    mean = sum(times) / len(times)
    return {"best_s": best, "median_s": median(times), "mean_s": mean,
            "error_margin": (mean - best) / best, "iterations": len(times)}


def cpu_baseline(inputs, names, budget_s=15.0):
    """The oracle as it stands (single-threaded scalar C) over the
    benchmark's own five buffers, timed by the paper's method (Sec. 4): per
    buffer, the best of up to 100 iterations (each at least 1 ms, here one
    whole-buffer repair), within about budget_s of CPU work in all."""
    import oracle
    lib = oracle._load()
    out = np.empty(inputs[0].size, dtype=np.uint16)
    per, best_total, med_total, mean_total = {}, 0.0, 0.0, 0.0
    for name, s in zip(names, inputs):
        r = paper_timing(lambda: lib.wf_to_seq(s.ctypes.data, out.ctypes.data, s.size),
                         budget_s=budget_s / len(inputs))
        best_total += r["best_s"]
        med_total += r["median_s"]
        mean_total += r["mean_s"]
        per[name] = {"best_GBps": round(2 * s.size / r["best_s"] / 1e9, 3),
                     "median_GBps": round(2 * s.size / r["median_s"] / 1e9, 3),
                     "error_margin": round(r["error_margin"], 4), "iterations": r["iterations"]}
    units = sum(x.size for x in inputs)
    return {
        "value": round(2.0 * units / best_total / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "the benchmark's five 268,435,456-unit buffers, each repaired out of place by the "
                  "single-threaded scalar oracle (gcc -O2 -fno-tree-vectorize); per buffer the best of up to 100 "
                  "whole-buffer repairs within a 15 s budget (the paper's method, Sec. 4)",
        "method": "paper: best iteration, each >= 1 ms; error margin = (mean - best) / best",
        "median_value": round(2.0 * units / med_total / 1e9, 3),
        "error_margin": round((mean_total - best_total) / best_total, 4),
        "per_buffer": per,
    }


def cpu_baseline_mt(inputs, passes=3):
    """The chunked multi-threaded oracle over the same five buffers, on this
    process's CPU share (at most 16 threads): best of a few passes."""
    import oracle
    lib = oracle._load()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    out = np.empty(inputs[0].size, dtype=np.uint16)
    units = sum(s.size for s in inputs)
    best = float("inf")
    for _ in range(passes):
        t0 = time.perf_counter()
        for s in inputs:
            if lib.wf_to_chunked_mt(s.ctypes.data, out.ctypes.data, s.size, threads) < 0:
                raise RuntimeError("oracle threads could not be created")
        best = min(best, time.perf_counter() - t0)
    return {"value": round(2.0 * units / best / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"the five buffers ({units} units), chunked multi-threaded oracle, best of {passes} passes"}


def per_string_vs_batched(torch, wf, stream):
    """Ragged batch of 1,000,000 log-normal strings: one persistent launch
    against one flat launch per string, every string launched."""
    from paper_2601_06349_amd import workloads as W
    buf, off = W.ragged_batch()
    n = int(off[-1])
    t_in = torch.from_numpy(buf.view(np.int16)).cuda()
    t_off = torch.from_numpy(off).cuda()
    t_out = torch.empty_like(t_in)
    med, best = time_fn(torch, stream, lambda: wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out,
                                                                units_hint=n), reps=20)
    plan = wf.BatchPlan(wf.OP_TO, t_in, t_off, out=t_out)
    med_plan, _ = time_fn(torch, stream, plan.launch, reps=20)
    plan.close()
    L = wf.lib()
    base_in, base_out, sh = t_in.data_ptr(), t_out.data_ptr(), stream.cuda_stream
    starts, lens = off[:-1].tolist(), np.diff(off).tolist()
    fn = L.utf16_to_well_formed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, ln in zip(starts, lens):
        fn(base_in + 2 * a, base_out + 2 * a, ln, sh)
    torch.cuda.synchronize()
    per_string_ms = (time.perf_counter() - t0) * 1e3
    return {
        "workload": "1,000,000 strings, log-normal lengths (median 32, sigma 1.5), "
                    f"{n} units, mix at 1e-3 plus forced edge surrogates",
        "seed": W.SEEDS["ragged_1m"],
        "batched_ms": round(med, 4),
        "batched_best_ms": round(best, 4),
        "batched_plan_ms": round(med_plan, 4),
        "batched_input_GBps": round(2 * n / (med * 1e-3) / 1e9, 1),
        "batched_pct_hbm": round(100 * (4 * n + 8 * off.size) / (med * 1e-3) / 1e9 / PEAK_HBM_GBS, 1),
        "per_string_ms": round(per_string_ms, 1),
        "per_string_launches": len(lens),
        "per_string_note": "every string one flat launch on the same stream, host time from the first launch to "
                           "the stream's end (synchronised before and after)",
        "speedup": round(per_string_ms / med, 1),
    }


def zipf_tuned_vs_default(torch, wf, tune, stream):
    """The 4096-string Zipf(1.1) batch (up to 2^24 units per string): copy
    repair, in-place repair and isWellFormed with early exit, each called
    with its size hint, with the autotuned launch shape and with the built-in
    default; and, tuned, without the hint (the shape for unknown sizes)."""
    from paper_2601_06349_amd import workloads as W
    buf, off, kind = W.zipf_batch()
    n = int(off[-1])
    t_in = torch.from_numpy(buf.view(np.int16)).cuda()
    t_off = torch.from_numpy(off).cuda()
    t_out = torch.empty_like(t_in)
    t_ip = torch.empty_like(t_in)
    res = torch.empty(off.size - 1, dtype=torch.uint8, device="cuda")
    def calls(hint):
        return {
            "to": (lambda: wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out, units_hint=hint), None, 4 * n),
            "to_inplace": (lambda: wf.utf16wf_batch(wf.OP_TO_INPLACE, t_ip, t_off, out=t_ip, units_hint=hint),
                           lambda: t_ip.copy_(t_in), 2 * n),
            "is": (lambda: wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=res, units_hint=hint), None, 2 * n),
        }
    lens = np.diff(off)
    ascii_units = int(lens[~kind].sum())
    out = {"workload": f"4096 strings, Zipf(1.1) lengths over 1..2^24, {n} units, "
                       f"{int(kind.sum())} strings mix(1e-2), the rest ({ascii_units} units) ASCII"}
    unhinted = calls(0)
    for name, (fn, setup, algo_bytes) in calls(n).items():
        wf.reset_params()
        d_ms, _ = time_fn(torch, stream, fn, reps=5, setup=setup)
        tune.apply_cache()
        t_ms, _ = time_fn(torch, stream, fn, reps=5, setup=setup)
        u_ms, _ = time_fn(torch, stream, unhinted[name][0], reps=5, setup=setup)
        out[name] = {"default_ms": round(d_ms, 4), "tuned_ms": round(t_ms, 4),
                     "tuned_input_GBps": round(2 * n / (t_ms * 1e-3) / 1e9, 1),
                     "tuned_no_hint_ms": round(u_ms, 4)}
        if name == "is":
            # early exit: only the well-formed (ASCII) strings must be read whole
            out[name]["must_read_bytes"] = 2 * ascii_units
            out[name]["pct_hbm_of_must_read"] = round(
                100 * 2 * ascii_units / (t_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 1)
        else:
            out[name]["pct_hbm_full_pass"] = round(100 * algo_bytes / (t_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 1)
    del t_in, t_out, t_ip
    torch.cuda.empty_cache()
    return out


def paper_workloads(torch, wf, stream):
    """The paper's own shapes (Sec. 4, Sec. 4.1): 1,000,000 units at 0.1 %
    pairs with 0 % and 0.1 % mismatched; the 128-point size sweep up to
    1,000,000 units, a fresh string per point, with the oracle timed beside
    the GPU at every point (the paper's figure compares two
    implementations per size); the 1024-unit JavaScript string with 5 %
    lows and 5 % highs. Each as one flat launch and as a batch of many such
    strings in one launch."""
    import oracle
    from paper_2601_06349_amd import workloads as W
    lib = oracle._load()
    res = {}
    for label, mis in (("1M_pairs0.1_mis0", 0.0), ("1M_pairs0.1_mis0.1", 0.1)):
        s = W.paper_mix(1_000_000, 0.1, mis, W.SEEDS["paper_1m"])
        d = torch.from_numpy(s.view(np.int16)).cuda()
        o = torch.empty_like(d)
        med, best = time_fn(torch, stream, lambda: wf.utf16_to_well_formed(d, o), reps=100)
        big, offs_h = W.paper_1m_batch(mis)
        offs = torch.from_numpy(offs_h).cuda()
        db = torch.from_numpy(big.view(np.int16)).cuda()
        ob = torch.empty_like(db)
        bmed, _ = time_fn(torch, stream, lambda: wf.utf16wf_batch(wf.OP_TO, db, offs, out=ob,
                                                                  units_hint=big.size), reps=20)
        out_h = np.empty_like(s)
        cpu = paper_timing(lambda: lib.wf_to_seq(s.ctypes.data, out_h.ctypes.data, s.size), budget_s=1.0)
        res[label] = {"seed": W.SEEDS["paper_1m"], "flat_us": round(med * 1e3, 2), "flat_best_us": round(best * 1e3, 2),
                      "flat_input_GBps": round(2e6 / (med * 1e-3) / 1e9, 1),
                      "flat_best_input_GBps": round(2e6 / (best * 1e-3) / 1e9, 1),
                      "batch_of_64_input_GBps": round(2 * big.size / (bmed * 1e-3) / 1e9, 1),
                      "oracle_1core_best_GBps": round(2e6 / cpu["best_s"] / 1e9, 3),
                      "oracle_error_margin": round(cpu["error_margin"], 4)}
        del db, ob
    sizes = W.paper_sweep_sizes()
    gpu_best, gpu_med, cpu_best, margins = [], [], [], []
    for i in range(sizes.size):
        s = W.paper_sweep_string(i, sizes)
        x = torch.from_numpy(s.view(np.int16)).cuda()
        y = torch.empty_like(x)
        med, best = time_fn(torch, stream, lambda: wf.utf16_to_well_formed(x, y), reps=20)
        gpu_best.append(round(2 * s.size / (best * 1e-3) / 1e9, 1))
        gpu_med.append(round(2 * s.size / (med * 1e-3) / 1e9, 1))
        out_h = np.empty_like(s)
        cpu = paper_timing(lambda: lib.wf_to_seq(s.ctypes.data, out_h.ctypes.data, s.size), iterations=20)
        cpu_best.append(round(2 * s.size / cpu["best_s"] / 1e9, 3))
        margins.append(round(cpu["error_margin"], 4))
    res["size_sweep_128"] = {
        "sizes_units": sizes.tolist(),
        "strings": "a fresh string per point: 0.1 % pairs, 0.1 % mismatched, seed [paper_sweep, point]",
        "seed": W.SEEDS["paper_sweep"],
        "gpu_flat_best_input_GBps": gpu_best,
        "gpu_flat_median_input_GBps": gpu_med,
        "oracle_1core_best_input_GBps": cpu_best,
        "oracle_error_margin": margins,
        "timing": "GPU: HIP events per launch, best and median of 20; oracle: best of 20 iterations of >= 1 ms",
    }
    js = W.js_string()
    d = torch.from_numpy(js.view(np.int16)).cuda()
    o = torch.empty_like(d)
    med, best = time_fn(torch, stream, lambda: wf.utf16_to_well_formed(d, o), reps=100)
    many, offs_h = W.js_batch()
    k = offs_h.size - 1
    offs = torch.from_numpy(offs_h).cuda()
    db = torch.from_numpy(many.view(np.int16)).cuda()
    ob = torch.empty_like(db)
    bmed, _ = time_fn(torch, stream, lambda: wf.utf16wf_batch(wf.OP_TO, db, offs, out=ob, units_hint=many.size),
                      reps=20)
    res["js_1024_5pct_low_5pct_high"] = {
        "seed": W.SEEDS["js_1024"],
        "flat_us": round(med * 1e3, 2), "flat_input_GiBps": round(2048 / (med * 1e-3) / 2**30, 2),
        "batch_of_262144_input_GiBps": round(2 * many.size / (bmed * 1e-3) / 2**30, 1),
        "batch_us_per_string": round(bmed * 1e3 / k, 5)}
    del db, ob
    torch.cuda.empty_cache()
    return res


def small_string_latency(torch, wf, stream):
    """The 1,048,576-unit string (lone low forced first, lone high last):
    out-of-place repair and isWellFormed, each one launch; device time per
    call from HIP events (best and median of 200), and the host's round trip
    of a synchronising isWellFormed call."""
    from paper_2601_06349_amd import workloads as W
    s = W.small_string()
    d = torch.from_numpy(s.view(np.int16)).cuda()
    o = torch.empty_like(d)
    res = torch.empty(1, dtype=torch.int32, device="cuda")
    to_med, to_best = time_fn(torch, stream, lambda: wf.utf16_to_well_formed(d, o), reps=200)
    is_med, is_best = time_fn(torch, stream, lambda: wf.utf16_is_well_formed(d, res), reps=200)
    host = []
    for _ in range(200):
        t0 = time.perf_counter()
        wf.is_well_formed(d)
        host.append(time.perf_counter() - t0)
    return {"workload": "1,048,576 units, mix at 1e-3, lone low at 0 and lone high at the end",
            "seed": W.SEEDS["small"],
            "to_well_formed_us": {"best": round(to_best * 1e3, 2), "median": round(to_med * 1e3, 2)},
            "is_well_formed_us": {"best": round(is_best * 1e3, 2), "median": round(is_med * 1e3, 2)},
            "is_well_formed_host_round_trip_us": {"best": round(min(host) * 1e6, 1),
                                                  "median": round(median(host) * 1e6, 1)}}


def host_resident(torch, wf, host_input):
    """The same 512 MiB repair when the string lives in pinned host memory:
    chunked copy in, repair and copy out on overlapping streams (PCIe-bound;
    never the headline value)."""
    n = host_input.size
    pin_in = torch.empty(n, dtype=torch.int16, pin_memory=True)
    pin_out = torch.empty(n, dtype=torch.int16, pin_memory=True)
    a = pin_in.numpy().view(np.uint16)
    b = pin_out.numpy().view(np.uint16)
    a[:] = host_input
    # the first two calls of a process pay one-time costs (the staging
    # allocation, then the first transfers over freshly pinned pages); they
    # are reported apart and the steady state is timed after them
    first = []
    for _ in range(2):
        t0 = time.perf_counter()
        wf.utf16_to_well_formed_host(a, out=b)
        first.append(time.perf_counter() - t0)
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        wf.utf16_to_well_formed_host(a, out=b)
        times.append(time.perf_counter() - t0)
    best = min(times)
    median = float(np.median(times))
    # the link itself: plain copies of the same pinned buffers, one direction
    # at a time and both at once on two streams
    d = torch.empty(n, dtype=torch.int16, device="cuda")
    d2 = torch.empty(n, dtype=torch.int16, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    h2d = timed(lambda: d.copy_(pin_in, non_blocking=True))
    d2h = timed(lambda: pin_out.copy_(d, non_blocking=True))

    def both():
        with torch.cuda.stream(s1):
            d2.copy_(pin_in, non_blocking=True)
        with torch.cuda.stream(s2):
            pin_out.copy_(d, non_blocking=True)

    duplex = timed(both)
    del d, d2
    return {"units": n, "best_s": round(best, 4), "input_GBps": round(2 * n / best / 1e9, 2),
            "median_input_GBps": round(2 * n / median / 1e9, 2),
            "first_two_calls_input_GBps": [round(2 * n / t / 1e9, 2) for t in first],
            "link_h2d_GBps": round(2 * n / h2d / 1e9, 2), "link_d2h_GBps": round(2 * n / d2h / 1e9, 2),
            "link_both_directions_GBps_each": round(2 * n / duplex / 1e9, 2),
            "note": "pinned host in and out, 8 Mi-unit chunks, copies in on one stream, repair and copies out "
                    "on another; includes both PCIe transfers"}


def profile_batches(torch, wf, W, reps=5):
    """Short run for rocprofv3 over the batch workloads, in a fixed order:
    for the 1,000,000-string batch and then the 4096-string Zipf batch, each
    with its size hint, 1 + `reps` calls each of the out-of-place repair, the
    check and the locate (the first of each a warm-up, as the benchmark's
    timed calls follow warm-up calls); then one copy-kernel launch over
    268,435,456 units (the counters' calibration)."""
    for label, (buf, off), hinted in (("ragged 1M", W.ragged_batch(), True),
                                      ("zipf 4096", W.zipf_batch()[:2], True)):
        log(f"profile: {label}")
        t_in = torch.from_numpy(buf.view(np.int16)).cuda()
        t_off = torch.from_numpy(off).cuda()
        t_out = torch.empty_like(t_in)
        b = off.size - 1
        res = torch.empty(b, dtype=torch.uint8, device="cuda")
        first = torch.empty(b, dtype=torch.int64, device="cuda")
        count = torch.empty(b, dtype=torch.int64, device="cuda")
        hint = int(off[-1]) if hinted else 0
        for op, kw in ((wf.OP_TO, {"out": t_out}), (wf.OP_IS, {"results": res}),
                       (wf.OP_LOCATE, {"first": first, "count": count})):
            for _ in range(1 + reps):
                wf.utf16wf_batch(op, t_in, t_off, units_hint=hint, **kw)
            torch.cuda.synchronize()
        del t_in, t_out
        torch.cuda.empty_cache()
    a = torch.zeros(N_UNITS, dtype=torch.int16, device="cuda")
    wf.utf16wf_copy_units(a, torch.empty_like(a))
    torch.cuda.synchronize()


def profile_flat(torch, wf, d_in, d_out, reps=2):
    """Short run for rocprofv3 over the one-buffer kernels other than the
    out-of-place repair: for each of the five 268,435,456-unit variants in
    order, `reps` times: restore a scratch copy of the input (a torch copy,
    untimed by the summaries), repair it in place, then check the input;
    finally one copy-kernel launch over one buffer (the counters'
    calibration)."""
    scratch = d_out[0]
    res = torch.empty(1, dtype=torch.int32, device="cuda")
    for x in d_in:
        for _ in range(reps):
            scratch.copy_(x)
            wf.utf16_to_well_formed_inplace(scratch)
            wf.utf16_is_well_formed(x, res)
        torch.cuda.synchronize()
    wf.utf16wf_copy_units(d_in[0], d_out[1])
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="only the timed steps, roofline and CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run at 50,000 requests/s (the configured 60 s by default)")
    ap.add_argument("--compare-seconds", type=float, default=5.0,
                    help="length of the serving runs that compare batch paths and the check")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: the steps plus one copy-kernel launch, no extras")
    ap.add_argument("--profile-batches", action="store_true",
                    help="run for rocprofv3 over the batch workloads only (no JSON line)")
    ap.add_argument("--profile-flat", action="store_true",
                    help="run for rocprofv3: in-place repair and isWellFormed over the five single-buffer "
                         "variants, then one copy-kernel launch (no JSON line)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_06349_amd as wf
    from paper_2601_06349_amd import tune
    from paper_2601_06349_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    wf.lib()  # fails loudly when the HIP library is missing
    tuned = tune.apply_cache()
    if args.profile_batches:
        profile_batches(torch, wf, W)
        return
    stream = torch.cuda.current_stream()

    log("generating inputs")
    host_inputs = [W.single_buffer(v) for v in W.SINGLE_VARIANTS]
    d_in = [torch.from_numpy(s.view(np.int16)).cuda() for s in host_inputs]
    d_out = [torch.empty_like(x) for x in d_in]
    torch.cuda.synchronize()
    if args.profile_flat:
        profile_flat(torch, wf, d_in, d_out)
        return

    def step(timer=None):
        for x, y in zip(d_in, d_out):
            if timer is None:
                wf.utf16_to_well_formed(x, y)
            else:
                timer.run(lambda x=x, y=y: wf.utf16_to_well_formed(x, y))

    # The timed region: one HIP event pair around each step (an event pair
    # around every launch adds about 7 us of stream work per launch). The
    # roofline's launch duration is the step's event time over its five
    # launches, the short gaps between them included.
    steps = Timer(torch, stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        steps.run(step)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if args.profile:
        wf.utf16wf_copy_units(d_in[0], d_out[0])
        torch.cuda.synchronize()

    step_ms = steps.times_ms()
    mean_launch_s = sum(step_ms) / len(step_ms) / len(d_in) * 1e-3
    in_bytes = 2 * N_UNITS * len(d_in) * args.steps
    value = in_bytes / el / 1e9
    achieved = 4 * N_UNITS / mean_launch_s / 1e9
    traffic = read_traffic()
    # per-variant rates: a second pass of the same steps, after the timed
    # region, with an event pair around every launch
    launches = Timer(torch, stream)
    if not args.profile:
        for _ in range(args.steps):
            step(launches)
    launch_ms = launches.times_ms()
    per_variant = {}
    for i, v in enumerate(W.SINGLE_VARIANTS):
        ts = launch_ms[i::len(d_in)]
        if ts:
            per_variant[v] = round(2 * N_UNITS / (median(ts) * 1e-3) / 1e9, 1)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": "single buffer of 268,435,456 uint16 units (512 MiB) in five seeded variants "
                        "(ascii, mix r=0, mix r=1e-6, mix r=1e-2, all surrogates); one step = "
                        "out-of-place toWellFormed of all five",
            "units_per_buffer": N_UNITS,
            "buffers": len(d_in),
            "launch_params": wf.get_params(wf.OP_TO, 0, N_UNITS),
            "tuning_cache": tuned,
            "seeds": {v: W.SEEDS["single_" + v] for v in W.SINGLE_VARIANTS},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "wf_kernel<OP_TO, flat> (out-of-place repair)",
            "algorithmic_bytes_per_launch": 4 * N_UNITS,
            "mean_launch_us": round(mean_launch_s * 1e6, 2),
            "launch_timing": "HIP events around each step of the timed region (5 launches on the benchmark's "
                             "stream); launch duration = step time / 5, gaps between launches included",
        },
        "per_variant_input_GBps": per_variant,
        "per_variant_timing": "a second pass of the same steps after the timed region, HIP events around "
                              "each launch (median per variant)",
    }

    if not args.no_cpu and not args.profile:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(host_inputs, W.SINGLE_VARIANTS)
        result["cpu_baseline_multithread"] = cpu_baseline_mt(host_inputs)

    if not args.no_extras and not args.profile:
        log("extras: in place, isWellFormed, copy ceiling")
        ex = {}
        ex["small_string_latency"] = small_string_latency(torch, wf, stream)
        inplace, isw = {}, {}
        res = torch.empty(1, dtype=torch.int32, device="cuda")
        scratch = torch.empty_like(d_in[0])
        for i, v in enumerate(W.SINGLE_VARIANTS):
            med, _ = time_fn(torch, stream, lambda: wf.utf16_to_well_formed_inplace(scratch), reps=10,
                             setup=lambda: scratch.copy_(d_in[i]))
            inplace[v] = round(2 * N_UNITS / (med * 1e-3) / 1e9, 1)
            med, _ = time_fn(torch, stream, lambda: wf.utf16_is_well_formed(d_in[i], res), reps=10)
            isw[v] = round(2 * N_UNITS / (med * 1e-3) / 1e9, 1)
        ex["inplace_input_GBps"] = inplace
        ex["is_well_formed_input_GBps"] = isw
        med, _ = time_fn(torch, stream, lambda: wf.utf16wf_copy_units(d_in[0], d_out[0]), reps=20)
        med_t, _ = time_fn(torch, stream, lambda: d_out[0].copy_(d_in[0]), reps=20)
        ex["copy_ceiling"] = {"library_copy_GBps_rw": round(4 * N_UNITS / (med * 1e-3) / 1e9, 1),
                              "torch_copy_GBps_rw": round(4 * N_UNITS / (med_t * 1e-3) / 1e9, 1)}
        del scratch
        log("extras: batched vs per-string")
        ex["ragged_batch"] = per_string_vs_batched(torch, wf, stream)
        del d_out
        torch.cuda.empty_cache()
        log("extras: Zipf batch, tuned vs default")
        ex["zipf_batch"] = zipf_tuned_vs_default(torch, wf, tune, stream)
        log("extras: the paper's workloads")
        ex["paper_workloads"] = paper_workloads(torch, wf, stream)
        log("extras: host-resident input")
        ex["host_resident"] = host_resident(torch, wf, host_inputs[2])
        log(f"extras: serving loop, {args.serve_seconds:.0f} s")
        from paper_2601_06349_amd import serve as S
        sv = S.serve_workload(duration_s=args.serve_seconds, rate_hz=50_000, num_streams=4,
                              arena_bytes=64 << 30, window_s=10.0, log=log)
        ex["serve"] = sv
        result["serve_p99_ms"] = sv.get("p99_ms")
        result["serve_p50_ms"] = sv.get("p50_ms")
        result["serve_seconds"] = args.serve_seconds
        log("extras: serving loop, separate strings vs every batch packed (the ragged-batch path alone)")
        ex["serve_compare_separate"] = S.serve_workload(duration_s=args.compare_seconds, rate_hz=50_000,
                                                        num_streams=4, arena_bytes=64 << 30, log=log)
        ex["serve_all_packed"] = S.serve_workload(duration_s=args.compare_seconds, rate_hz=50_000, num_streams=4,
                                                  arena_bytes=64 << 30, separate_max=-1, log=log)
        log("extras: serving loop, isWellFormed requests")
        ex["serve_check"] = S.serve_workload(duration_s=2.0, rate_hz=50_000, num_streams=4,
                                             arena_bytes=64 << 30, op=wf.OP_IS, log=log)
        log("extras: the paper's 1024-unit strings, served")
        ex["paper_workloads"]["js_1024_served"] = S.serve_js_strings(duration_s=1.0, rate_hz=1_000_000, log=log)
        log("extras: the paper's 1,000,000-unit runs, served")
        ex["paper_workloads"]["1M_runs_served"] = S.serve_paper_1m(duration_s=1.0, rate_hz=10_000, log=log)
        result["extras"] = ex

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
