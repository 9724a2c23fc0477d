#!/usr/bin/env python3
"""Autotuner for the planner's launch shapes (the ks_tune_* tunables of include/ks.h).

    python -m paper_0712_4046_amd.autotune --workload batch_mixed_10000 [--variant ks4] [--out tuning.json]

For one workload it times the whole run (HIP events on the stream the library launches on,
median of a few runs after warm-up) for candidate values of each tunable in turn -- a
coordinate descent, repeated while it still improves.  Each candidate is timed next to the
current best, re-timed right before it, and kept only if it beats that pair partner: a GPU
whose clocks drift over a long sweep (power or heat) then cannot pass drift off as a gain.
It keeps the fastest value of each tunable, and
writes them as JSON together with the default and tuned times to the library's cache file
(read by every later process at plan time; --out names another file, which KS_TUNING_FILE can
point the library at), and `ks.apply_tuning(table)` sets them in the running process.  The shapes change only how work
is cut into launches and blocks, never the result: tests/test_gpu_autotune.py checks a tuned
run bit for bit against the default one.

Workloads: product_4096_s64 (one product, L = 4096, signed 64-bit), batch_mixed_10000 (the 10,000-product batch),
batch_mod_64x65536 (the 64-product modular batch, L = 65536), or `small` (a 300-product batch for tests).
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys

from . import ks

CANDIDATES = {
    "KS_NTT_MIN_LIMBS": [0, 4000, 8000, 12000, 20000, 40000, 80000],
    "KS_CHAIN_K": [0, 4, 8, 16, 32, 64, 128, 256, 512, 1024],
    "KS_MFMA_MIN_LIMBS": [2000, 4000, 6000, 10000, 20000, 1 << 30],
    "KS_MFMA_RT": [0, 4, 8],
    "KS_KARATSUBA_MIN_LIMBS": [0, 8192, 16384, 32768],
    "KS_MFMA_BLOCKS": [256, 512, 1024, 2048, 4096],
    "KS_MFMA_MIN_PART": [32, 64, 128, 256, 512],
    "KS_MUL_WAVE_MAX": [0, 256, 512, 1024, 2048, 4096],
    "KS_SCAN_SMALL": [0, 64, 128],
}


def cache_path() -> str:
    """The JSON cache the library reads at plan time (include/ks.h, ks_tune_set): KS_TUNING_FILE,
    else $XDG_CACHE_HOME/ksmul/tuning.json or ~/.cache/ksmul/tuning.json."""
    import os
    if os.environ.get("KS_TUNING_FILE"):
        return os.environ["KS_TUNING_FILE"]
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "ksmul", "tuning.json")


def save(res: dict, path: str | None = None) -> str:
    """Write a tuning result (its "tunables" table is what the library reads) to the cache."""
    import os
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "w") as fh:
        fh.write(json.dumps(res) + "\n")
    return path


def time_ms(run, warmup: int = 2, reps: int = 5) -> float:
    """Median time of `run()` in milliseconds, from events on the current stream."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return statistics.median(out)


def workload(name: str, variant: str):
    """A factory: called after the tunables are set, it plans the workload and returns a
    zero-argument callable that runs it once (results on the device)."""
    import torch
    from . import workloads as wl
    if name == "product_4096_s64":
        P = wl.product_4096_s64()
        tf, tg = ks.to_device(P.f), ks.to_device(P.g)
        out = torch.empty((2 * P.f.shape[0] - 1, ks.out_limbs(P.f.shape[0], P.g.shape[0], P.bits)),
                          dtype=torch.int32, device="cuda")

        def make():
            return lambda: ks.mul(tf, tg, P.bits, variant, P.signed, out=out)
        return make
    B = ks.Batch()
    if name == "batch_mod_64x65536":
        p, pairs = wl.batch_mod_64x65536()
        for f, g in pairs:
            B.add_mod(f, g, p)
    else:
        prods = wl.batch_mixed_10000() if name == "batch_mixed_10000" else wl.batch_mixed_10000(count=300, seed=36)
        for Q in prods:
            B.add(Q.f, Q.g, Q.bits, Q.signed)
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    descs = B.desc_array()
    state = {}

    def make():
        if "plan" in state:
            state["plan"].close()
        plan = ks.BatchPlan(descs, variant)
        ws = ks.alloc_workspace(plan.workspace_bytes)
        state.update(plan=plan, ws=ws)
        return lambda: plan.run(ain, aout, ws)
    make.batch = B
    make.arenas = (ain, aout)
    make.state = state
    return make


def tune(make, candidates=None, max_passes: int = 2, warmup: int = 2, reps: int = 5, log=None) -> dict:
    """Coordinate descent over the tunables; returns the best table and the timings."""
    candidates = candidates or CANDIDATES
    ks.tune_reset()
    best = {k: ks.tune_get(k) for k in candidates}
    base = time_ms(make(), warmup, reps)
    best_ms = base
    for _ in range(max_passes):
        improved = False
        for name, values in candidates.items():
            for v in values:
                if v == best[name]:
                    continue
                ks.tune_set(name, best[name])
                ref = time_ms(make(), warmup, reps)  # the current best, timed just before
                ks.tune_set(name, v)
                ms = time_ms(make(), warmup, reps)
                if log:
                    log(f"{name}={v}: {ms:.4f} ms (best {ref:.4f} now)")
                if ms < ref * 0.995:
                    best_ms, best[name], improved = ms, v, True
                ks.tune_set(name, best[name])
        if not improved:
            break
    final = time_ms(make(), warmup, reps)  # every tunable is at its best value here
    return {"tunables": best, "ms": final, "default_ms": base}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch_mixed_10000", choices=["product_4096_s64", "batch_mixed_10000", "batch_mod_64x65536", "small"])
    ap.add_argument("--variant", default="ks4")
    ap.add_argument("--out", default=None, help="where to write the result (default: the library's cache)")
    ap.add_argument("--passes", type=int, default=2)
    a = ap.parse_args(argv)
    make = workload(a.workload, a.variant)
    res = tune(make, max_passes=a.passes, log=lambda s: print(s, file=sys.stderr, flush=True))
    res.update(workload=a.workload, variant=a.variant)
    res["cache"] = save(res, a.out)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
