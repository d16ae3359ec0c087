"""Autotuner for the launch parameters of the repair and check kernels.

For each (operation, flat or batch, size class) it times every launch shape
in a grid — 16-byte loads per lane per tile (rows), waves per workgroup,
workgroups per compute unit, streaming cache hints — with HIP events on
synthetic inputs of that size, and keeps the fastest. The untuned default is
timed beside it and both are written to the cache, so the gain is visible.

The cache is JSON keyed by GPU architecture and compute-unit count, stored in
``paper_2601_06349_amd/tuning/``. ``apply_cache()`` loads the entry for the
current device into the library (``UTF16WF_TUNING_CACHE`` names another
file; ``UTF16WF_NO_TUNING=1`` keeps the built-in defaults).

Run on the GPU:  python -m paper_2601_06349_amd.tune [--quick] [--out PATH]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")

ROWS = (1, 2, 4, 8)
WG_WAVES = (2, 4, 8, 16)
GRID_PER_CU = (2, 4, 8, 16, 32, 64)
NONTEMPORAL = (0, 1)


def device_key():
    import torch

    import paper_2601_06349_amd as wf
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}_{wf.device_cus()}cu"


def cache_path(key=None):
    env = os.environ.get("UTF16WF_TUNING_CACHE")
    if env:
        return env
    return os.path.join(TUNING_DIR, f"{key or device_key()}.json")


def apply_cache(path=None):
    """Load tuned parameters for this device into the library. Returns the
    file name used, or None when there is none (defaults stay)."""
    import paper_2601_06349_amd as wf
    if os.environ.get("UTF16WF_NO_TUNING") == "1":
        return None
    path = path or cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    for e in data.get("entries", []):
        p = e["params"]
        wf.set_params(e["op"], e["batch"], e["size_class"], p["rows"], p["wg_waves"], p["grid_per_cu"],
                      p["nontemporal"])
    return os.path.basename(path)


def _timer(torch):
    stream = torch.cuda.current_stream()

    def run(fn, reps):
        fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in evs)
        return ts[len(ts) // 2]

    return run


def shapes(quick=False):
    if quick:
        return list(itertools.product((1, 4, 8), (4, 8), (8, 16, 32), (0, 1)))
    return list(itertools.product(ROWS, WG_WAVES, GRID_PER_CU, NONTEMPORAL))


def _sweep(wf, run, op, batch, size_class, call, reps, quick):
    """Time every shape for one key; returns (best_params, best_ms, default_ms)."""
    wf.reset_params()
    default = wf.get_params(op, batch, 1 << size_class if size_class < 40 else 1 << 40)
    default_ms = run(call, reps)
    best = (default_ms, default)
    for rows, wg, gpc, nt in shapes(quick):
        wf.set_params(op, batch, size_class, rows, wg, gpc, nt)
        ms = run(call, reps)
        if ms < best[0]:
            best = (ms, {"rows": rows, "wg_waves": wg, "grid_per_cu": gpc, "nontemporal": nt})
    wf.reset_params()
    return best[1], best[0], default_ms


def tune(quick=False, flat_classes=None, out=None, log=print):
    import torch

    import paper_2601_06349_amd as wf
    from paper_2601_06349_amd import workloads as W

    run = _timer(torch)
    entries = []
    flat_classes = flat_classes or (list(range(10, 29, 2)) if quick else list(range(10, 29)))
    names = {wf.OP_IS: "is", wf.OP_TO: "to", wf.OP_TO_INPLACE: "to_inplace", wf.OP_LOCATE: "locate"}
    t_start = time.time()
    big = W.mix(1 << max(flat_classes), 1e-3, 4242)
    clean = W.mix(1 << max(flat_classes), 0.0, 4243)
    d_mix = torch.from_numpy(big.view(np.int16)).cuda()
    d_clean = torch.from_numpy(clean.view(np.int16)).cuda()
    d_out = torch.empty_like(d_mix)
    d_tmp = torch.empty_like(d_mix)
    res = torch.empty(4, dtype=torch.int64, device="cuda")
    for c in flat_classes:
        n = 1 << c
        reps = 10 if n >= 1 << 24 else 20
        x, y, z, cl = d_mix[:n], d_out[:n], d_tmp[:n], d_clean[:n]
        z.copy_(x)
        calls = {
            wf.OP_TO: lambda: wf.utf16_to_well_formed(x, y),
            wf.OP_TO_INPLACE: lambda: wf.utf16_to_well_formed_inplace(z),
            wf.OP_IS: lambda: wf.utf16_is_well_formed(cl, res[:1].view(torch.int32)),
            wf.OP_LOCATE: lambda: wf.utf16_locate_ill_formed(x),
        }
        for op, call in calls.items():
            params, ms, dms = _sweep(wf, run, op, 0, c, call, reps, quick)
            entries.append({"op": op, "op_name": names[op], "batch": 0, "size_class": c, "params": params,
                            "tuned_ms": round(ms, 5), "default_ms": round(dms, 5)})
            log(f"flat {names[op]:10s} 2^{c:2d}: tuned {ms * 1e3:9.1f} us  default {dms * 1e3:9.1f} us  {params}")
    del d_mix, d_clean, d_out, d_tmp

    # batches: the Zipf(1.1) 4096-string workload (launched without a size
    # hint, so it sets the parameters for unknown sizes) and the 1,000,000
    # log-normal strings (launched with their size hint)
    zb, zoff, _ = W.zipf_batch()
    rb, roff = W.ragged_batch()
    for label, buf, off, hinted in (("zipf_4096", zb, zoff, False), ("ragged_1m", rb, roff, True)):
        t_in = torch.from_numpy(buf.view(np.int16)).cuda()
        t_off = torch.from_numpy(off).cuda()
        t_out = torch.empty_like(t_in)
        t_ip = t_in.clone()
        nunits = int(off[-1])
        hint = nunits if hinted else 0
        cls = 40 if not hinted else int(np.floor(np.log2(nunits)))
        results = torch.empty(off.size - 1, dtype=torch.uint8, device="cuda")
        calls = {
            wf.OP_TO: lambda: wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out, units_hint=hint),
            wf.OP_TO_INPLACE: lambda: wf.utf16wf_batch(wf.OP_TO_INPLACE, t_ip, t_off, out=t_ip,
                                                       units_hint=hint),
            wf.OP_IS: lambda: wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=results, units_hint=hint),
        }
        for op, call in calls.items():
            params, ms, dms = _sweep(wf, run, op, 1, cls, call, 5, quick)
            entries.append({"op": op, "op_name": names[op], "batch": 1, "size_class": cls, "params": params,
                            "tuned_ms": round(ms, 5), "default_ms": round(dms, 5), "workload": label,
                            "units": nunits})
            log(f"batch {label} {names[op]:10s}: tuned {ms:8.3f} ms  default {dms:8.3f} ms  {params}")
        del t_in, t_off, t_out, t_ip
        torch.cuda.empty_cache()

    data = {"device": device_key(), "created_unix": int(time.time()),
            "sweep": "quick" if quick else "full", "seconds": round(time.time() - t_start, 1),
            "entries": entries}
    out = out or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as f:
        json.dump(data, f, indent=1)
    log(f"wrote {out}")
    return data


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    tune(quick=args.quick, out=args.out, log=lambda m: print(m, flush=True))
    return 0


if __name__ == "__main__":
    sys.exit(main())
