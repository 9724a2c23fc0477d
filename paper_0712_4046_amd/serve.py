"""Serving loop: a stream of Z[x] product requests on one GPU, with continuous admission.

Requests arrive at given times (a Poisson process in the measured workload).  The server
admits them in arrival order whenever a slot and enough device memory are free, copies the
operands to the device, and enqueues the product (libksmul's ks_mul) on one of several HIP
streams, so products admitted while others are still running overlap on the GPU.  Finished
requests are retired by polling their completion events; their slot and memory return to the
pool and their results stay on the device until the caller fetches them.

Latency of a request = time its completion is observed minus its arrival time.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import ks


@dataclass
class Request:
    idx: int
    arrival: float          # seconds from the start of the run
    f: np.ndarray           # (L, W) uint32 limbs
    g: np.ndarray
    bits: int
    signed: bool


@dataclass
class Done:
    idx: int
    arrival: float
    admitted: float
    finished: float
    out: object             # device tensor holding h

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Stats:
    completed: int
    wall_s: float
    products_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    limb_mults: float
    max_inflight: int
    results: list = field(repr=False, default_factory=list)


def request_bytes(r: Request) -> int:
    """Device bytes a request holds while in flight: operands, output and scratch."""
    lf, lg = r.f.shape[0], r.g.shape[0]
    p = ks.plan(lf, lg, r.bits, "auto", r.signed)
    ops = 4 * (p["operand_limbs_f"] + p["operand_limbs_g"]) * p["n_products"]
    cols = 12 * (p["operand_limbs_f"] + p["operand_limbs_g"] + 128) * p["n_products"]
    out = 4 * (lf + lg - 1) * p["out_limbs"]
    inputs = 4 * (r.f.size + r.g.size)
    return inputs + out + 2 * ops + cols


class Server:
    def __init__(self, slots: int = 16, streams: int = 4, mem_budget: int | None = None, variant: str = "auto"):
        import torch
        self.torch = torch
        self.slots = slots
        self.variant = variant
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        if mem_budget is None:
            free, _total = torch.cuda.mem_get_info()
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget

    def warm(self, reqs):
        """Grow every stream's scratch pool to the largest request, outside the timed run."""
        torch = self.torch
        big = max(reqs, key=lambda r: r.f.shape[0] * r.f.shape[1])
        for s in self.streams:
            with torch.cuda.stream(s):
                tf, tg = ks.to_device(big.f), ks.to_device(big.g)
                ks.mul(tf, tg, big.bits, self.variant, big.signed, stream=s)
        torch.cuda.synchronize()
        for s in self.streams:
            ks.check(s)

    def run(self, reqs: list[Request], poll_s: float = 50e-6) -> Stats:
        torch = self.torch
        pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
        inflight = []   # (req, admitted, event, nbytes, out, device inputs)
        done: list[Done] = []
        used = 0
        rr = 0
        max_inflight = 0
        limb_mults = 0.0
        t0 = time.perf_counter()
        while pending or inflight:
            now = time.perf_counter() - t0
            # retire finished requests
            still = []
            for item in inflight:
                req, adm, ev, nb, out, _inputs = item
                if ev.query():
                    done.append(Done(req.idx, req.arrival, adm, now, out))
                    used -= nb
                else:
                    still.append(item)
            inflight = still
            # admit arrived requests while a slot and memory are free (arrival order)
            admitted_any = False
            while pending and pending[0].arrival <= now and len(inflight) < self.slots:
                req = pending[0]
                nb = request_bytes(req)
                if used + nb > self.mem_budget and inflight:
                    break
                pending.popleft()
                s = self.streams[rr % len(self.streams)]
                rr += 1
                with torch.cuda.stream(s):
                    tf = ks.to_device(req.f)
                    tg = ks.to_device(req.g)
                    out = ks.mul(tf, tg, req.bits, self.variant, req.signed, stream=s)
                    ev = torch.cuda.Event()
                    ev.record(s)
                p = ks.plan(req.f.shape[0], req.g.shape[0], req.bits, self.variant, req.signed)
                limb_mults += p["limb_mults"]
                inflight.append((req, now, ev, nb, out, (tf, tg)))
                used += nb
                admitted_any = True
                max_inflight = max(max_inflight, len(inflight))
            if not admitted_any:
                # nothing admitted: wait for the next arrival or a completion
                nxt = pending[0].arrival - (time.perf_counter() - t0) if pending else poll_s
                time.sleep(max(0.0, min(poll_s, nxt)))
        wall = time.perf_counter() - t0
        for s in self.streams:
            rc = ks.status(s)
            if rc != ks.KS_OK:
                raise ks.KSError(rc, "serving run")
        lat = np.array([d.latency for d in done]) * 1000.0
        done.sort(key=lambda d: d.idx)
        return Stats(completed=len(done), wall_s=wall, products_per_s=len(done) / wall,
                     p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                     mean_ms=float(lat.mean()), limb_mults=limb_mults, max_inflight=max_inflight, results=done)


def make_requests(count: int, rate_per_s: float, seed: int = 5, max_len: int = 65536, max_bits: int = 256):
    """The serving mix: L log-uniform in [8, max_len], b uniform in [8, max_bits], signed values,
    Poisson arrivals at `rate_per_s` (rate 0 or less: all arrive at time 0, a closed loop)."""
    from . import workloads as wl
    lens, bits, seeds = wl.serving_requests(count, seed, max_len, max_bits)
    arr = wl.poisson_arrivals(count, rate_per_s, seed) if rate_per_s > 0 else np.zeros(count)
    reqs = []
    for i in range(count):
        P = wl.request_product(int(lens[i]), int(bits[i]), int(seeds[i]))
        reqs.append(Request(i, float(arr[i]), P.f, P.g, P.bits, True))
    return reqs


def main(argv=None):
    """Measure the serving mix: closed-loop saturated throughput, then Poisson arrivals at
    0.7 of it; prints one JSON line (products/s, p50/p99 latency, the rate used)."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--max-len", type=int, default=65536)
    ap.add_argument("--max-bits", type=int, default=256)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--variant", default="auto")
    a = ap.parse_args(argv)
    closed = make_requests(a.requests, 0.0, 5, a.max_len, a.max_bits)
    srv = Server(slots=a.slots, streams=a.streams, variant=a.variant)
    srv.warm(closed)
    sat = srv.run(closed)
    rate = 0.7 * sat.products_per_s
    reqs = make_requests(a.requests, rate, 5, a.max_len, a.max_bits)
    st = srv.run(reqs)
    print(json.dumps({
        "workload": f"serving: {a.requests} signed Z[x] products, L log-uniform in [8, {a.max_len}], "
                    f"b uniform in [8, {a.max_bits}], Poisson arrivals (seed 5)",
        "saturated_products_per_s": sat.products_per_s, "rate_per_s": rate,
        "products_per_s": st.products_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
        "limb_mults_per_s": st.limb_mults / st.wall_s, "max_inflight": st.max_inflight,
        "slots": a.slots, "streams": a.streams, "variant": a.variant}))


if __name__ == "__main__":
    main()
