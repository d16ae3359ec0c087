"""Python front-end of the serving loop (include/utf16wf_serve.h).

The loop itself is native (``utf16wf_serve_run``): arrivals replayed from a
schedule, admission against an HBM arena, continuous batching over several
streams, completion by event polling. This module builds request arrays,
calls it, and summarises latencies (measured from each request's scheduled
arrival, so a slow server cannot hide queueing delay).
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import OP_IS, OP_TO, check, lib

REQUEST_DTYPE = np.dtype([("arrival_ns", "<i8"), ("src", "<u8"), ("length", "<i8"), ("dst", "<u8")])
OUTCOME_DTYPE = np.dtype([("launch_ns", "<i8"), ("done_ns", "<i8"), ("status", "<i4"), ("batch", "<i4"),
                          ("slot", "<i4"), ("well_formed", "<i4")])


class ServeConfig(ctypes.Structure):
    _fields_ = [("num_streams", ctypes.c_int32), ("op", ctypes.c_int32), ("arena_bytes", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int64), ("max_batch_units", ctypes.c_int64),
                ("timeout_ns", ctypes.c_int64), ("separate_max", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("batches", "completed", "rejected", "timed_out", "failed",
                                               "max_inflight", "max_queue", "arena_peak_bytes", "wall_ns",
                                               "direct_batches")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def make_config(num_streams=4, op=OP_TO, arena_bytes=64 << 30, max_batch_requests=4096,
                max_batch_units=1 << 26, timeout_ns=0, separate_max=0) -> ServeConfig:
    """separate_max: batches of at most this many requests run as separate
    strings (0 = the most, 32; -1 = every batch packed)."""
    return ServeConfig(num_streams, op, arena_bytes, max_batch_requests, max_batch_units, timeout_ns,
                       separate_max)


def run(requests: np.ndarray, config: ServeConfig):
    """Run the loop on the current device. ``requests`` is an array of
    REQUEST_DTYPE (device pointers as integers). Returns (outcomes, stats)."""
    requests = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE)
    outcomes = np.zeros(requests.size, dtype=OUTCOME_DTYPE)
    st = ServeStats()
    check(lib().utf16wf_serve_run(ctypes.addressof(config), requests.ctypes.data, requests.size,
                                  outcomes.ctypes.data, ctypes.addressof(st)))
    return outcomes, st.as_dict()


def simulate(arrival_ns, lengths, config: ServeConfig, lat_base_ns=20_000, lat_ns_per_unit=0.001,
             fail_every=0):
    """The same scheduler on a simulated device with a virtual clock."""
    arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
    lens = np.ascontiguousarray(lengths, dtype=np.int64)
    outcomes = np.zeros(arr.size, dtype=OUTCOME_DTYPE)
    st = ServeStats()
    check(lib().utf16wf_serve_simulate(ctypes.addressof(config), arr.ctypes.data, lens.ctypes.data, arr.size,
                                       int(lat_base_ns), float(lat_ns_per_unit), int(fail_every),
                                       outcomes.ctypes.data, ctypes.addressof(st)))
    return outcomes, st.as_dict()


def latency_summary(outcomes, arrival_ns, lengths, window_s=None):
    """p50 / p99 / mean / max latency (ms) of completed requests, from their
    scheduled arrival to the host seeing their batch complete; throughput in
    GB/s of input over the run; fraction of the run with at least one batch
    in flight (launch to completion seen by the host). With window_s, also
    p50 / p99 per window of that many seconds of arrivals (their spread shows
    how much one run's tail varies)."""
    ok = outcomes["status"] == 0
    lat = (outcomes["done_ns"][ok] - np.asarray(arrival_ns)[ok]) / 1e6
    res = {"completed": int(ok.sum())}
    if lat.size:
        res.update(p50_ms=round(float(np.percentile(lat, 50)), 4), p99_ms=round(float(np.percentile(lat, 99)), 4),
                   mean_ms=round(float(lat.mean()), 4), max_ms=round(float(lat.max()), 4))
        if window_s:
            arr = np.asarray(arrival_ns)[ok]
            win = (arr - arr.min()) // int(window_s * 1e9)
            p50w, p99w = [], []
            for w in range(int(win.max()) + 1):
                x = lat[win == w]
                if x.size:
                    p50w.append(round(float(np.percentile(x, 50)), 4))
                    p99w.append(round(float(np.percentile(x, 99)), 4))
            res.update(window_s=window_s, p50_ms_by_window=p50w, p99_ms_by_window=p99w)
        t_end = float(outcomes["done_ns"][ok].max())
        t_start = float(np.asarray(arrival_ns)[ok].min())
        res["input_GBps"] = round(2.0 * float(np.asarray(lengths)[ok].sum()) / max(t_end - t_start, 1.0), 3)
        # union of [launch, done] over batches
        b = outcomes[ok]
        _, first = np.unique(b["batch"], return_index=True)
        busy, cur_s, cur_e = 0, None, None
        for s, e in sorted(map(tuple, np.stack([b["launch_ns"][first], b["done_ns"][first]], axis=1))):
            if cur_e is None or s > cur_e:
                if cur_e is not None:
                    busy += cur_e - cur_s
                cur_s, cur_e = s, e
            else:
                cur_e = max(cur_e, e)
        if cur_e is not None:
            busy += cur_e - cur_s
        res["inflight_frac"] = round(float(busy) / max(t_end - t_start, 1.0), 4)
        res["batches"] = int(first.size)
        res["mean_batch_requests"] = round(float(ok.sum()) / max(first.size, 1), 2)
    return res


def serve_workload(duration_s=5.0, rate_hz=50_000.0, num_streams=4, arena_bytes=64 << 30,
                   max_batch_requests=4096, max_batch_units=1 << 26, op=OP_TO, seed=None,
                   pool_len=1 << 24, n_pools=16, separate_max=0, window_s=None, log=None):
    """The serving workload: Poisson arrivals at ``rate_hz`` for
    ``duration_s``, Zipf(1.1) lengths up to ``pool_len`` units, per-request
    lone-surrogate rate 10^U(-6,-1), payloads sliced from device-resident
    pools of mix(r_j) at log-spaced r_j. Returns a summary dict."""
    import torch

    from . import workloads as W
    kw = {} if seed is None else {"seed": seed}
    sch = W.serve_schedule(duration_s, rate_hz=rate_hz, n_pools=n_pools, pool_len=pool_len,
                           max_len=pool_len, **kw)
    if log:
        log(f"serve: {sch['length'].size} requests, {int(sch['length'].sum())} units")
    pools = W.serve_pools(sch["pool_rates"], pool_len=pool_len)
    d_pools = [torch.from_numpy(p.view(np.int16)).cuda() for p in pools]
    base = np.array([p.data_ptr() for p in d_pools], dtype=np.uint64)
    reqs = np.zeros(sch["length"].size, dtype=REQUEST_DTYPE)
    reqs["arrival_ns"] = sch["arrival_ns"]
    reqs["src"] = base[sch["pool"]] + 2 * sch["pool_offset"].astype(np.uint64)
    reqs["length"] = sch["length"]
    torch.cuda.synchronize()
    cfg = make_config(num_streams=num_streams, op=op, arena_bytes=arena_bytes,
                      max_batch_requests=max_batch_requests, max_batch_units=max_batch_units,
                      separate_max=separate_max)
    out, st = run(reqs, cfg)
    summ = latency_summary(out, sch["arrival_ns"], sch["length"], window_s=window_s)
    summ.update({"requests": int(sch["length"].size), "duration_s": duration_s, "rate_hz": rate_hz,
                 "seed": W.SEEDS["serve"] if seed is None else seed,
                 "num_streams": num_streams, "arena_bytes": arena_bytes, "separate_max": separate_max,
                 "stats": st})
    del d_pools
    return summ


def js_requests(duration_s=1.0, rate_hz=1_000_000.0, n_distinct=4096, seed=1601):
    """The paper's JavaScript shape as a request stream: Poisson arrivals of
    1024-unit strings with 5 % lone lows and 5 % lone highs (the rest
    ASCII), each one of ``n_distinct`` strings. Returns (pool, arrival_ns,
    which): the host pool of n_distinct * 1024 units, arrival times, and the
    pool string of each request."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    pool = np.concatenate([W.js_string(seed=rng) for _ in range(n_distinct)])
    count = int(rng.poisson(rate_hz * duration_s))
    arrival = (np.cumsum(rng.exponential(1.0 / rate_hz, size=count)) * 1e9).astype(np.int64)
    which = rng.integers(0, n_distinct, size=count)
    return pool, arrival, which


def paper_1m_requests(duration_s=0.1, rate_hz=10_000.0, seed=1701):
    """The paper's two 1,000,000-unit runs (0.1 % pairs; 0 % and 0.1 %
    mismatched) as a request stream: Poisson arrivals, each request one of
    the two strings. Returns (pool, arrival_ns, which): the host pool (the
    two strings back to back), arrival times and each request's string."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    pool = np.concatenate([W.paper_mix(1_000_000, 0.1, mis, W.SEEDS["paper_1m"]) for mis in (0.0, 0.1)])
    count = int(rng.poisson(rate_hz * duration_s))
    arrival = (np.cumsum(rng.exponential(1.0 / rate_hz, size=count)) * 1e9).astype(np.int64)
    which = rng.integers(0, 2, size=count)
    return pool, arrival, which


def serve_fixed_length(pool, arrival, which, length, num_streams=4, arena_bytes=1 << 30,
                       max_batch_requests=65536, dst=None, log=None, label=""):
    """Serve requests that are each `length` units of the host `pool` at
    string index `which[i]` (a device copy of the pool is made). With a
    device `dst` tensor of len(which) * length units, request i repairs into
    dst[i * length, (i + 1) * length). Returns a summary dict."""
    import torch
    d_pool = torch.from_numpy(pool.view(np.int16)).cuda()
    count = which.size
    reqs = np.zeros(count, dtype=REQUEST_DTYPE)
    reqs["arrival_ns"] = arrival
    reqs["src"] = np.uint64(d_pool.data_ptr()) + (2 * length * which).astype(np.uint64)
    reqs["length"] = length
    if dst is not None:
        if dst.numel() < count * length:
            raise ValueError("dst is smaller than the requests' outputs")
        reqs["dst"] = np.uint64(dst.data_ptr()) + (2 * length * np.arange(count)).astype(np.uint64)
    if log:
        rate = count / max((arrival[-1] - arrival[0]) * 1e-9, 1e-9) if count > 1 else 0.0
        log(f"serve {label}: {count} requests of {length} units at {rate:.0f}/s")
    torch.cuda.synchronize()
    cfg = make_config(num_streams=num_streams, op=OP_TO, arena_bytes=arena_bytes,
                      max_batch_requests=max_batch_requests, max_batch_units=1 << 26)
    out, st = run(reqs, cfg)
    summ = latency_summary(out, arrival, reqs["length"])
    summ.update({"requests": int(count), "num_streams": num_streams, "stats": st,
                 "all_completed": bool(np.all(out["status"] == 0))})
    del d_pool
    return summ


def serve_js_strings(duration_s=1.0, rate_hz=1_000_000.0, num_streams=4, arena_bytes=1 << 30,
                     max_batch_requests=65536, n_distinct=4096, seed=1601, dst=None, log=None):
    """The paper's JavaScript shape served (js_requests); see
    serve_fixed_length for `dst`. Returns a summary dict."""
    pool, arrival, which = js_requests(duration_s, rate_hz, n_distinct, seed)
    summ = serve_fixed_length(pool, arrival, which, 1024, num_streams=num_streams, arena_bytes=arena_bytes,
                              max_batch_requests=max_batch_requests, dst=dst, log=log, label="js 1024")
    summ.update({"duration_s": duration_s, "rate_hz": rate_hz})
    return summ


def serve_paper_1m(duration_s=0.1, rate_hz=10_000.0, num_streams=4, arena_bytes=4 << 30, seed=1701, dst=None,
                   log=None):
    """The paper's 1,000,000-unit runs served (paper_1m_requests); see
    serve_fixed_length for `dst`. Returns a summary dict."""
    pool, arrival, which = paper_1m_requests(duration_s, rate_hz, seed)
    summ = serve_fixed_length(pool, arrival, which, 1_000_000, num_streams=num_streams, arena_bytes=arena_bytes,
                              dst=dst, log=log, label="paper 1M")
    summ.update({"duration_s": duration_s, "rate_hz": rate_hz})
    return summ
