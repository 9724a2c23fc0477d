#!/usr/bin/env python3
"""Helpers for rocprofv3 measurements of the library (used to make the files in profiles/).

    python -m paper_0712_4046_amd.prof_tools workload [product_4096_s64[_variants]|batch_mixed_10000|batch_mod_64x65536|poly2] [valu|mfma|ntt]
    python -m paper_0712_4046_amd.prof_tools summarize DB "cmd"  # kernel-trace summary table
    python -m paper_0712_4046_amd.prof_tools counters FETCH_DB WRITE_DB   # HBM bytes per kernel
    python -m paper_0712_4046_amd.prof_tools valu   # vector-ALU instruction rates (libksprobe.so)
    python -m paper_0712_4046_amd.prof_tools issue DB [DB ...]   # per-kernel counters, VALU issue rate

The workload is a plain device copy of known size (to calibrate FETCH_SIZE / WRITE_SIZE) and
then the benchmark product (one Z[x] product, L = 4096, signed 64-bit coefficients, seed 2)
through the four-point variant, or one four-point run of a batched workload.
"""
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_MIB = 256


def workload(name: str = "product_4096_s64", reps: int = 5, engine=None):
    """A plain device copy of COPY_MIB MiB (the FETCH_SIZE / WRITE_SIZE calibration), then
    product_4096_s64: `reps` four-point products of the L = 4096 signed 64-bit workload (seed 2);
    product_4096_s64_variants: 50 products of the same workload through each of ks4, ks1, neg2, recip2;
    batch_mixed_10000: one four-point run of the 10,000-product batch (seed 3);
    batch_mod_64x65536: one four-point run of the 64-product modular batch (seed 4);
    poly2: `reps` four-point bivariate products of the (Z/pZ)[x, y] workload (seed 7)."""
    sys.path.insert(0, ROOT)
    import torch
    from paper_0712_4046_amd import ks
    from paper_0712_4046_amd import workloads as wl
    src = torch.ones(COPY_MIB * 1024 * 1024 // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # known traffic: COPY_MIB MiB read and COPY_MIB MiB written
    torch.cuda.synchronize()
    if name in ("product_4096_s64", "product_4096_s64_variants"):
        P = wl.product_4096_s64()
        tf, tg = ks.to_device(P.f), ks.to_device(P.g)
        variants = ("ks4",) if name == "product_4096_s64" else ("ks4", "ks1", "neg2", "recip2")
        for v in variants:
            for _ in range(reps if name == "product_4096_s64" else 50):
                ks.mul(tf, tg, P.bits, v, P.signed, engine=engine)
        ks.check()
    elif name == "poly2":
        import numpy as np
        p, f, g = wl.poly2_workload()
        tf = torch.from_numpy(f.view(np.int64)).cuda()
        tg = torch.from_numpy(g.view(np.int64)).cuda()
        for _ in range(reps):
            ks.mul_poly2(tf, tg, p, "ks4")
        ks.check()
    else:
        B = ks.Batch()
        if name == "batch_mixed_10000":
            for P in wl.batch_mixed_10000():
                B.add(P.f, P.g, P.bits, P.signed)
        else:
            p, pairs = wl.batch_mod_64x65536()
            for f, g in pairs:
                B.add_mod(f, g, p)
        plan = ks.BatchPlan(B.desc_array(), "ks4", engine)
        ain = ks.to_device(B.arena_in())
        aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
        ws = ks.alloc_workspace(plan.workspace_bytes)
        plan.run(ain, aout, ws)
        if plan.status(ws) != ks.KS_OK:
            raise SystemExit("batch status not OK")
        plan.close()
    print("workload done", flush=True)


def _table(rows):
    print(f"{'kernel':60s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}")
    for name, n, tot, avg, mn, mx in rows:
        short = name if len(name) <= 60 else name[:57] + "..."
        print(f"{short:60s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f}")


def summarize(db: str, cmd: str = "", last: int = 0):
    """Per-kernel durations of a --kernel-trace run; last > 0 adds a table over the last `last`
    dispatches of each kernel (the calls a run profiles at its end)."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    print("# rocprofv3 --kernel-trace --stats summary")
    print(f"# command: {cmd}")
    print("# durations in microseconds")
    _table(rows)
    if last > 0:
        print(f"# the last {last} dispatches of each kernel")
        tail = []
        for (name,) in con.execute("select distinct name from kernels"):
            d = [r[0] for r in con.execute("select duration from kernels where name = ? order by start desc limit ?",
                                            (name, last))]
            if len(d) == last:
                tail.append((name, len(d), sum(d), sum(d) / len(d), min(d), max(d)))
        _table(sorted(tail, key=lambda r: -r[2]))


def counter_per_kernel(db: str):
    """(kernel name -> list of per-dispatch counter values) from a --pmc run."""
    con = sqlite3.connect(db)
    out = {}
    for k, v in con.execute("select kernel_name, value from counters_collection order by dispatch_id"):
        out.setdefault(k, []).append(float(v))
    return out


def counters(fetch_db: str, write_db: str):
    f, w = counter_per_kernel(fetch_db), counter_per_kernel(write_db)
    copy = [k for k in f if "copyBuffer" in k]
    skip = set(copy) | {k for k in f if "FillFunctor" in k or "fillBuffer" in k}
    print("# HBM traffic from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch),")
    print(f"# scaled by the same counters on a plain {COPY_MIB} MiB device copy in the same run")
    kib = COPY_MIB * 1024
    fk = max((max(f[k]) for k in copy), default=0.0)
    wk = max((max(w.get(k, [0.0])) for k in copy), default=0.0)
    cal = (kib / fk if fk else 1.0, kib / wk if wk else 1.0)
    print(f"# calibration copy: FETCH {fk:.0f} KiB, WRITE {wk:.0f} KiB for {kib} KiB each way")
    print(f"# factors: fetch x{cal[0]:.3f}, write x{cal[1]:.3f}")
    print(f"{'kernel':60s} {'n':>4s} {'fetch_KiB':>10s} {'write_KiB':>10s} {'bytes':>12s}")
    for k in f:
        if k in skip:
            continue
        fa = sum(f[k]) / len(f[k])
        wa = sum(w.get(k, [0])) / max(len(w.get(k, [1])), 1)
        tot = (fa * cal[0] + wa * cal[1]) * 1024
        short = k if len(k) <= 60 else k[:57] + "..."
        print(f"{short:60s} {len(f[k]):4d} {fa:10.1f} {wa:10.1f} {tot:12.0f}")


def pmc_table(db: str, cmd: str = ""):
    """Every counter of a --pmc run, averaged per dispatch, per kernel."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                       "group by kernel_name, counter_name order by kernel_name, counter_name").fetchall()
    print("# rocprofv3 --pmc counters, average per dispatch")
    print(f"# command: {cmd}")
    last = None
    for k, c, v, n in rows:
        if k != last:
            print(k if len(k) <= 100 else k[:97] + "...")
            last = k
        print(f"    {c:32s} {v:20.1f}   (dispatches: {n})")


def issue_table(dbs, cus: int = 256, xcds: int = 8):
    """Per kernel, the counters of several --pmc runs of one workload (one dispatch each) and the
    vector-ALU issue rate: SQ_INSTS_VALU (wave instructions) / (CUs x GRBM_GUI_ACTIVE / XCDs).
    GRBM_GUI_ACTIVE adds up the busy cycles of the XCDs; a CU issues at most one wave64 vector
    instruction per cycle (four SIMDs, four cycles each), so the rate is the fraction of the
    vector ALUs' issue slots used."""
    rows = {}
    for db in dbs:
        con = sqlite3.connect(db)
        for k, c, v in con.execute("select kernel_name, counter_name, avg(value) from counters_collection "
                                   "group by kernel_name, counter_name"):
            rows.setdefault(k, {})[c] = v
    print("# rocprofv3 --pmc counters per dispatch and the vector-ALU issue rate")
    print(f"# issue = SQ_INSTS_VALU / ({cus} CUs x GRBM_GUI_ACTIVE / {xcds} XCDs); "
          "wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES; conflicts = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS")
    print(f"{'kernel':60s} {'VALU (M)':>9s} {'LDS (M)':>8s} {'issue':>6s} {'wait':>6s} {'conflicts':>9s}")
    for k, c in rows.items():
        if "ks::" not in k or "fill_zero" in k or "GRBM_GUI_ACTIVE" not in c or "SQ_INSTS_VALU" not in c:
            continue
        clk = c["GRBM_GUI_ACTIVE"] / xcds
        issue = c["SQ_INSTS_VALU"] / (cus * clk) if clk else 0.0
        wait = c.get("SQ_WAIT_ANY", 0.0) / c["SQ_WAVE_CYCLES"] if c.get("SQ_WAVE_CYCLES") else 0.0
        conf = (c.get("SQ_LDS_BANK_CONFLICT", 0.0) / c["SQ_ACTIVE_INST_LDS"]) if c.get("SQ_ACTIVE_INST_LDS") else 0.0
        short = k if len(k) <= 60 else k[:57] + "..."
        print(f"{short:60s} {c['SQ_INSTS_VALU'] / 1e6:9.1f} {c.get('SQ_INSTS_LDS', 0.0) / 1e6:8.1f} "
              f"{issue:6.2f} {wait:6.2f} {conf:9.2f}")


def valu_rates(blocks: int = 4096, iters: int = 4096, reps: int = 5):
    """Issue rate of each probe operation (probe/valu_rates.hip): lane-operations per second
    over the whole chip, and the lanes per SIMD per clock that rate means at the nominal
    2.4 GHz (256 CUs, 4 SIMDs each).  A wave64 instruction at 16 lanes per clock takes four
    clocks (the fp64 FMA rate); at 32 lanes, two (the fp32 rate)."""
    import ctypes
    import torch
    torch.cuda.init()
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_0712_4046_amd", "libksprobe.so"))
    lib.ks_probe_name.restype = ctypes.c_char_p
    print("# vector-ALU issue rates (paper_0712_4046_amd/probe/valu_rates.hip)")
    print(f"# command: python -m paper_0712_4046_amd.prof_tools valu   ({blocks} blocks x 256 threads, "
          f"{iters} steps of 8 chains, mean of {reps} launches)")
    print("# (for the ds_read patterns: lanes/SIMD/clk x 4 = words a CU reads per clock)")
    print(f"{'operation':76s} {'ms':>8s} {'T inst/s':>9s} {'lanes/SIMD/clk @2.4GHz':>23s}")
    for op in range(lib.ks_probe_count()):
        ms = ctypes.c_float()
        if lib.ks_probe_valu(op, blocks, iters, reps, ctypes.byref(ms)) != 0:
            raise SystemExit(f"probe {op} failed")
        inst = blocks * 256 * iters * 8 * lib.ks_probe_insts(op)
        rate = inst / (ms.value * 1e-3)
        print(f"{lib.ks_probe_name(op).decode():76s} {ms.value:8.3f} {rate / 1e12:9.2f} "
              f"{rate / (256 * 4 * 2.4e9):23.1f}")


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else "workload"
    if cmd == "workload":
        workload(sys.argv[2] if len(sys.argv) > 2 else "product_4096_s64",
                 engine=sys.argv[3] if len(sys.argv) > 3 else None)
    elif cmd == "summarize":
        summarize(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "", int(sys.argv[4]) if len(sys.argv) > 4 else 0)
    elif cmd == "counters":
        counters(sys.argv[2], sys.argv[3])
    elif cmd == "pmc":
        pmc_table(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
    elif cmd == "valu":
        valu_rates()
    elif cmd == "issue":
        issue_table(sys.argv[2:])
