#!/usr/bin/env python3
"""Benchmark: exact dense products in Z[x] by multipoint Kronecker substitution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload product_4096_s64|product_256_u32] [--no-batch]

A step is one whole product f*g through the library's hot path (pack -> integer products ->
carry resolution and halving -> reconstruction / read-off), with the inputs already in HBM.
Workload (default): one product of two length-4096 polynomials with signed 64-bit
coefficients drawn from seed 2 (the single-product configuration the paper's comparison is
quoted on, at a size that fits one GPU).  The four-point variant (paper Section 3.4) is the
reported value; the standard substitution (3.1), the negated variant (3.3) and the two-point
reciprocal variant (3.2) are timed the same way for the speedups; each product runs on the engine the planner picks (vector ALU or
int8 matrix cores).  Extra fields: per-kernel durations and the dominant kernel's roofline,
the CPU oracle's rate on the host cores, and the two batched workloads (10,000 mixed products;
64 products mod a 60-bit prime of length 65536) with their own rooflines.  Prints ONE JSON line.
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

# vector-ALU peak for the limb multiplier: one limb-mult is a v_mad_u64_u32 (32x32+64 -> 64)
# plus a v_addc (carry into the top word of a 96-bit column sum), both issuing at full rate:
# 256 CUs x 64 lanes x 2.4 GHz / 2 instructions = 19.66e12 limb-mults/s
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 2 / 1e12
# int8 matrix cores (dense, no sparsity): 5.0e15 operations/s, one multiply-add = 2 operations
MFMA_I8_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE + WRITE_SIZE (copy-calibrated: FETCH x2,
# WRITE x1) for the four-point product of the L=4096 workload (profiles/product_4096_s64_ks4_hbm_traffic.txt)
# and for the 64-product modular batch (profiles/batch_mod_64x65536_ks4_hbm_traffic.txt).  A kernel whose
# code changed after the counters were taken has no entry (traffic: null).  "pack" is the fused
# pack-and-anchor launch, "recon" the reconstruction chain.
MEASURED_TRAFFIC = {"pack": 1000619, "digitize": 1021819, "mul_mfma": 5861019, "normalize": 1407366, "recon": 778348,
                    "finish": 441720}
MEASURED_TRAFFIC_CONFIG4 = {"pack": 2236843379, "digitize": 814250784, "mul_mfma": 4348159197,
                            "normalize": 2348495456, "recon": 1779810943, "finish": 612164503}
KERNELS = ("kara", "pack", "mul_valu", "digitize", "mul_mfma", "normalize", "anchor", "recon", "finish", "extract",
           "p2_eval", "p2_recon")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="product_4096_s64", choices=["product_256_u32", "product_4096_s64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workloads")
    ap.add_argument("--no-paper", action="store_true", help="skip the (Z/nZ)[x] sweep of the paper's figures")
    ap.add_argument("--no-poly2", action="store_true", help="skip the bivariate (Z/pZ)[x, y] workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    return ap.parse_args()


def time_variant(ks, torch, tf, tg, bits, variant, signed, steps, warmup, out):
    for _ in range(warmup):
        ks.mul(tf, tg, bits, variant, signed, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ks.mul(tf, tg, bits, variant, signed, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def poly2_line(ks, torch, wl, reps=20):
    """The paper's polynomial case (Section 2) on the bivariate workload: h = f g in
    (Z/pZ)[x, y], L_x = 16, L_y = 4096, p a random odd 60-bit modulus, through the standard,
    reciprocal, negated and four-point substitutions into (Z/pZ)[x] (ks_mul_poly2), timed with
    inputs resident on the device; each substitution's result must equal the standard one's
    (checked on the device; the oracle checks sampled coefficients in the GPU tests)."""
    p, f, g = wl.poly2_workload()
    tf = torch.from_numpy(f.view(np.int64)).cuda()
    tg = torch.from_numpy(g.view(np.int64)).cuda()
    ms, res = {}, {}
    for v in ("ks1", "recip2", "neg2", "ks4"):
        o = torch.empty((2 * f.shape[0] - 1, 2 * f.shape[1] - 1), dtype=torch.int64, device="cuda")
        for _ in range(3):
            ks.mul_poly2(tf, tg, p, v, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ks.mul_poly2(tf, tg, p, v, out=o)
        torch.cuda.synchronize()
        ms[v] = (time.perf_counter() - t0) / reps * 1e3
        res[v] = o
    ks.check()
    if not all(torch.equal(res[v], res["ks1"]) for v in res):
        raise SystemExit("bivariate workload: substitutions disagree")
    kern = kernel_times(ks, lambda: ks.mul_poly2(tf, tg, p, "ks4", out=res["ks4"]), 5)
    return {"workload": f"(Z/pZ)[x, y], L_x = {f.shape[1]}, L_y = {f.shape[0]}, p = {p} (60-bit odd), "
                        f"residues uniform in [0, p), seed 7",
            "ms": ms, "products_per_s": {v: 1e3 / ms[v] for v in ms},
            "speedup_vs_ks1": {v: ms["ks1"] / ms[v] for v in ("recip2", "neg2", "ks4")},
            "ks4_kernels_us_per_run": {k: x["per_run_us"] for k, x in kern.items()}}


def paper_sweep(ks, torch, wl):
    """The paper's example timings redone on this GPU: (Z/nZ)[x] products through every variant
    for a random 4-bit and a random 48-bit odd modulus n at L = 4 .. 65536 (powers of 4), as
    t(KS1) / t(variant) -- the quantity of the paper's Figures 1 and 2.  Each variant's result
    must equal KS1's (checked on the device); the oracle checks these moduli in the GPU tests."""
    out = {}
    for nb in wl.PAPER_FIG_BITS:
        rows = []
        for L in wl.PAPER_FIG_LENGTHS:
            n, f, g = wl.paper_fig_pair(nb, L)
            tf = torch.from_numpy(f.view(np.int64)).cuda()
            tg = torch.from_numpy(g.view(np.int64)).cuda()
            res, ms = {}, {}
            for v in ("ks1", "recip2", "neg2", "ks4"):
                o = torch.empty(2 * L - 1, dtype=torch.int64, device="cuda")
                ks.mul_mod(tf, tg, n, v, out=o)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ks.mul_mod(tf, tg, n, v, out=o)
                torch.cuda.synchronize()
                reps = max(5, min(200, int(0.03 / max(time.perf_counter() - t0, 1e-6))))
                for _ in range(3):
                    ks.mul_mod(tf, tg, n, v, out=o)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    ks.mul_mod(tf, tg, n, v, out=o)
                torch.cuda.synchronize()
                ms[v] = (time.perf_counter() - t0) / reps * 1e3
                res[v] = o
            ks.check()
            same = all(torch.equal(res[v], res["ks1"]) for v in res)
            if not same:
                raise SystemExit(f"paper sweep: variants disagree at n of {nb} bits, L = {L}")
            rows.append({"L": L, "ms": ms, "ks1_over": {v: ms["ks1"] / ms[v] for v in ("recip2", "neg2", "ks4")}})
        out[f"n_{nb}_bit"] = {"n": n, "rows": rows}
    return out


def kernel_times(ks, run, reps):
    """Per stage: launches per run, average launch duration and the stage's time per run (its
    launches added up), from the HIP events that every launch of the library records at its own
    start and end on the stream it runs on (hipExtLaunchKernelGGL, via ks_profile_*)."""
    ks.profile_reset()
    ks.profile_enable(True)
    for _ in range(reps):
        run()
    import torch
    torch.cuda.synchronize()
    ks.profile_enable(False)
    out = {}
    for name in KERNELS:
        n, ms = ks.profile_read(name)
        if n:
            out[name] = {"launches": n, "launches_per_run": n / reps, "avg_us": 1000.0 * ms / n,
                         "per_run_us": 1000.0 * ms / reps}
    return out


def roofline(kern, info, traffic_table=None):
    """The dominant stage's achieved rate against its bound: the stage's algorithmic work in one
    run (limb products of the vector-ALU products, int8 operations of the matrix-core products,
    or the stage's bytes) over the stage's time in one run.  A single product launches each
    stage once, so there this is work per launch over the launch's duration; a batch may launch
    a stage twice (block- and wave-mode multipliers, wide and one-wave scans)."""
    dom = max(kern, key=lambda k: kern[k]["per_run_us"])
    sec = kern[dom]["per_run_us"] * 1e-6
    traffic = (traffic_table or {}).get(dom)
    lpr = kern[dom]["launches_per_run"]
    if dom == "mul_mfma":
        ops = info["mfma_ops"]
        achieved = ops / sec / 1e12
        return {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / MFMA_I8_PEAK_TOPS, "traffic": traffic, "launches_per_run": lpr,
                "op": "int8 multiply-add of balanced 8-bit digits (2 operations)", "ops_per_run": ops}
    if dom in ("mul_valu", "anchor"):
        ops = info["valu_limb_mults"] if dom == "mul_valu" else info["anchor_limb_mults"]
        achieved = ops / sec / 1e12
        return {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic, "launches_per_run": lpr,
                "op": "32x32->64-bit limb multiply-accumulate", "ops_per_run": ops}
    nbytes = {"pack": info["pack_bytes"], "normalize": info["normalize_bytes"]}.get(dom, info["finish_bytes"])
    achieved = nbytes / sec / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "launches_per_run": lpr, "bytes_per_run": nbytes}


def batch_line(ks, torch, B, count, variant, reps, traffic=None):
    """One batched workload through ks_batch_run: products/s, limb-mults/s, stage times and the
    dominant stage's roofline."""
    plan = ks.BatchPlan(B.desc_array(), variant)
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    plan.run(ain, aout, ws)
    torch.cuda.synchronize()
    rc = plan.status(ws)
    if rc != ks.KS_OK:
        raise SystemExit(f"batch status: {ks.strerror(rc)}")
    info = plan.info()
    kern = kernel_times(ks, lambda: plan.run(ain, aout, ws), 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(ain, aout, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # the same run captured once in a hipGraph and replayed (its launches issued by the graph)
    eager = aout.clone()
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.run(ain, aout, ws, stream=s)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    dtg = (time.perf_counter() - t0) / reps
    if plan.status(ws) != ks.KS_OK or not torch.equal(aout, eager):
        raise SystemExit("batch graph replay differs from the eager run")
    del graph
    plan.close()
    eng = {ks.KS_ENGINE_VALU: "valu", ks.KS_ENGINE_MFMA: "mfma"}.get(info["engine"], "valu+mfma")
    return {"variant": variant, "engine": eng, "ms_per_batch": dt * 1e3, "products_per_s": count / dt,
            "ms_per_batch_graph": dtg * 1e3, "products_per_s_graph": count / dtg,
            "limb_mults_per_s": info["limb_mults"] / dt, "mfma_ops_per_s": info["mfma_ops"] / dt,
            "kernels_us_per_run": {k: v["per_run_us"] for k, v in kern.items()},
            "roofline": roofline(kern, info, traffic)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); across GPUs the batched and "
              "serving products would shard by instance and a four-point product by its four sub-products",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_0712_4046_amd import ks
    from paper_0712_4046_amd import workloads as wl

    P = wl.product_4096_s64() if args.workload == "product_4096_s64" else wl.product_256_u32()
    L, bits, signed = P.f.shape[0], P.bits, P.signed
    tf, tg = ks.to_device(P.f), ks.to_device(P.g)
    wo = ks.out_limbs(L, L, bits)
    variants = ("ks4", "ks1", "neg2", "recip2")
    outs = {v: torch.empty((2 * L - 1, wo), dtype=torch.int32, device="cuda") for v in variants}

    t = {}
    for v in variants:
        t[v] = time_variant(ks, torch, tf, tg, bits, v, signed, args.steps, args.warmup, outs[v])
    rc = ks.status()
    if rc != ks.KS_OK:
        raise SystemExit(f"device status after timing: {ks.strerror(rc)}")
    plans = {v: ks.plan(L, L, bits, v, signed) for v in variants}
    engine_name = {ks.KS_ENGINE_VALU: "valu", ks.KS_ENGINE_MFMA: "mfma"}

    # spread of single calls: each of 100 calls bracketed by its own events on the stream
    def spread(v, n=100):
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record(s)
            ks.mul(tf, tg, bits, v, signed, out=outs[v])
            b.record(s)
        torch.cuda.synchronize()
        ms_each = sorted(a.elapsed_time(b) for a, b in ev)
        return {"p10": ms_each[n // 10], "p50": ms_each[n // 2], "p90": ms_each[(9 * n) // 10]}
    dist = {v: spread(v) for v in variants}

    # per-kernel durations of the four-point product on the library's own stream
    kern = kernel_times(ks, lambda: ks.mul(tf, tg, bits, "ks4", signed, out=outs["ks4"]), args.steps)
    roof = roofline(kern, plans["ks4"], MEASURED_TRAFFIC if args.workload == "product_4096_s64" else None)

    # bit-exact check of every variant against the oracle (also the CPU baseline sample)
    cpu = None
    exact = None
    if not args.no_cpu:
        from oracle import oracle as O
        t0 = time.perf_counter()
        n = 0
        exp = None
        while True:
            exp = O.mul_classical(P.f, P.g, signed, wo)
            n += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        cpu = {"value": n / el, "unit": "products/s", "cores": O.threads(), "kind": "oracle",
               "sample": f"{n} full products of the same workload (classical convolution, OpenMP over coefficients)"}
        exact = all(np.array_equal(ks.to_host(outs[v]), exp) for v in outs)
        if not exact:
            raise SystemExit("GPU result differs from the oracle")

    # the batched workloads (throughput; their results are checked by the GPU tests)
    batch = None
    if not args.no_batch:
        batch = {}
        prods = wl.batch_mixed_10000()
        B = ks.Batch()
        for Q in prods:
            B.add(Q.f, Q.g, Q.bits, Q.signed)
        for v in ("ks4", "ks1"):
            batch[f"batch_mixed_10000_{v}"] = batch_line(ks, torch, B, len(prods), v, 10)
        del B
        p, pairs = wl.batch_mod_64x65536()
        B = ks.Batch()
        for f, g in pairs:
            B.add_mod(f, g, p)
        for v in ("ks4", "ks1"):
            batch[f"batch_mod_64x65536_{v}"] = batch_line(ks, torch, B, len(pairs), v, 3,
                                               MEASURED_TRAFFIC_CONFIG4 if v == "ks4" else None)
        del B
        batch["speedup_ks4_vs_ks1"] = {c: batch[f"{c}_ks1"]["ms_per_batch"] / batch[f"{c}_ks4"]["ms_per_batch"]
                                       for c in ("batch_mixed_10000", "batch_mod_64x65536")}
        batch["workloads"] = {
            "batch_mixed_10000": "10,000 signed products, L log-uniform in [16, 1024], b in {16, 32, 64, 128}, seed 3",
            "batch_mod_64x65536": "64 products mod a 60-bit odd p, L = 65536, residues uniform in [0, p), seed 4"}

    paper = None if args.no_paper else paper_sweep(ks, torch, wl)
    bivariate = None if args.no_poly2 else poly2_line(ks, torch, wl)

    p4 = plans["ks4"]
    ms = t["ks4"] * 1000.0
    rec = {
        "metric": "polynomial products/s + limb-mults/s at 1 GPU; KS4 vs KS1 speedup, bit-exact",
        "value": 1.0 / t["ks4"],
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: one Z[x] product, L={L}, {'signed' if signed else 'unsigned'} "
                               f"{bits}-bit coefficients, four-point Kronecker substitution",
                   "len": L, "coeff_bits": bits, "signed": signed, "variant": "ks4"},
        "limb_mults_per_s": p4["limb_mults"] / t["ks4"],
        "schoolbook_limb_mults_per_s": p4["schoolbook_limb_mults"] / t["ks4"],
        "variants_ms": {v: t[v] * 1000.0 for v in t},
        "variants_ms_single_call": dist,
        "variants_products_per_s": {v: 1.0 / t[v] for v in t},
        "variants_engine": {v: engine_name.get(plans[v]["engine"], "?") for v in variants},
        "speedup_ks4_vs_ks1": t["ks1"] / t["ks4"],
        "speedup_neg2_vs_ks1": t["ks1"] / t["neg2"],
        "speedup_recip2_vs_ks1": t["ks1"] / t["recip2"],
        "bit_exact": exact,
        "kernels_us": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "batch": batch,
        "paper_figures": paper,
        "poly2": bivariate,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
