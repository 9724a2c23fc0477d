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


def request_io_bytes(r: Request) -> int:
    """Device bytes a request's own tensors hold while it is in flight: operands and output."""
    lf, lg = r.f.shape[0], r.g.shape[0]
    return 4 * (r.f.size + r.g.size) + 4 * (lf + lg - 1) * ks.out_limbs(lf, lg, r.bits)


class Server:
    """Continuous admission over `streams` HIP streams and at most `slots` requests in flight.

    Device memory is accounted as the library holds it: each in-flight request's operands and
    output, plus the scratch pool that ks_mul keeps per stream, which grows to the largest
    product run on that stream (ks_plan's scratch_bytes) and stays.  A request goes to a stream
    whose pool already fits it when there is one (no growth, so no synchronisation inside the
    library), else to the stream whose pool needs the least growth; it is admitted when the
    operands, output and any growth fit in the budget (or when nothing else is in flight)."""

    def __init__(self, slots: int = 16, streams: int = 4, mem_budget: int | None = None, variant: str = "auto"):
        import torch
        self.torch = torch
        self.slots = slots
        self.variant = variant
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.pool = [0] * streams  # bytes of the library's scratch pool on each stream
        if mem_budget is None:
            free, _total = torch.cuda.mem_get_info()
            mem_budget = int(free * 0.5)
        self.mem_budget = mem_budget

    def warm(self, reqs):
        """Grow every stream's scratch pool to the largest request, outside the timed run."""
        torch = self.torch
        big = max(reqs, key=lambda r: ks.plan(r.f.shape[0], r.g.shape[0], r.bits, self.variant,
                                               r.signed)["scratch_bytes"])
        need = ks.plan(big.f.shape[0], big.g.shape[0], big.bits, self.variant, big.signed)["scratch_bytes"]
        for i, s in enumerate(self.streams):
            with torch.cuda.stream(s):
                tf, tg = ks.to_device(big.f), ks.to_device(big.g)
                ks.mul(tf, tg, big.bits, self.variant, big.signed, stream=s)
            self.pool[i] = max(self.pool[i], need)
        torch.cuda.synchronize()
        for s in self.streams:
            ks.check(s)

    def _pick_stream(self, scratch: int, rr: int) -> int:
        n = len(self.streams)
        for k in range(n):
            i = (rr + k) % n
            if self.pool[i] >= scratch:
                return i
        return max(range(n), key=lambda i: self.pool[i])

    def run(self, reqs: list[Request]) -> Stats:
        torch = self.torch
        pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
        inflight = []   # (req, admitted, event, io bytes, out, device inputs)
        done: list[Done] = []
        used_io = 0
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
                    used_io -= nb
                else:
                    still.append(item)
            inflight = still
            # admit arrived requests while a slot and memory are free (arrival order)
            while pending and pending[0].arrival <= now and len(inflight) < self.slots:
                req = pending[0]
                pl = ks.plan(req.f.shape[0], req.g.shape[0], req.bits, self.variant, req.signed)
                nb = request_io_bytes(req)
                si = self._pick_stream(pl["scratch_bytes"], rr)
                grow = max(0, pl["scratch_bytes"] - self.pool[si])
                if used_io + sum(self.pool) + grow + nb > self.mem_budget and inflight:
                    break
                pending.popleft()
                rr += 1
                s = self.streams[si]
                with torch.cuda.stream(s):
                    tf = ks.to_device(req.f)
                    tg = ks.to_device(req.g)
                    out = ks.mul(tf, tg, req.bits, self.variant, req.signed, stream=s)
                    ev = torch.cuda.Event()
                    ev.record(s)
                self.pool[si] += grow
                limb_mults += pl["limb_mults"]
                inflight.append((req, now, ev, nb, out, (tf, tg)))
                used_io += nb
                max_inflight = max(max_inflight, len(inflight))
            if not inflight and pending:
                # idle until the next arrival
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
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


# ---- result check: h(r) = f(r) g(r) mod q at random points (Schwartz-Zippel) ------------------
# Primes below 2^31, so that a residue times a limb (< 2^32) or a residue times a residue stays
# below 2^63 in numpy's uint64.  A wrong h passes one check with probability at most (D-1)/q.
SZ_PRIMES = (2147483629, 2147483587)


def _residues(limbs: np.ndarray, q: int, signed: bool) -> np.ndarray:
    """(L, W) little-endian uint32 limbs (two's complement when signed) -> values mod q."""
    limbs = np.asarray(limbs, dtype=np.uint32)
    if limbs.ndim == 1:
        limbs = limbs.reshape(-1, 1)
    Q = np.uint64(q)
    acc = np.zeros(limbs.shape[0], dtype=np.uint64)
    for t in range(limbs.shape[1]):
        acc = (acc + (limbs[:, t].astype(np.uint64) * np.uint64(pow(2, 32 * t, q))) % Q) % Q
    if signed:
        neg = (limbs[:, -1] >> np.uint32(31)).astype(bool)
        acc[neg] = (acc[neg] + np.uint64(q - pow(2, 32 * limbs.shape[1], q))) % Q
    return acc


class PointCheck:
    """Evaluations at seeded random points r mod each q of SZ_PRIMES (powers of r cached)."""

    def __init__(self, seed: int = 2024):
        gen = np.random.Generator(np.random.PCG64(seed))
        self.points = [(q, int(gen.integers(2, q - 1))) for q in SZ_PRIMES]
        self.pw = [np.ones(1, dtype=np.uint64) for _ in SZ_PRIMES]

    def _powers(self, j: int, n: int) -> np.ndarray:
        q, r = self.points[j]
        pw = self.pw[j]
        while pw.size < n:
            pw = np.concatenate([pw, (pw * np.uint64(pow(r, pw.size, q))) % np.uint64(q)])
        self.pw[j] = pw
        return pw[:n]

    def value(self, limbs: np.ndarray, signed: bool, j: int) -> int:
        q = self.points[j][0]
        c = _residues(limbs, q, signed)
        return int(((c * self._powers(j, c.size)) % np.uint64(q)).sum(dtype=np.uint64) % np.uint64(q))

    def holds(self, f: np.ndarray, g: np.ndarray, h: np.ndarray, signed: bool) -> bool:
        for j, (q, _r) in enumerate(self.points):
            if self.value(h, True, j) != self.value(f, signed, j) * self.value(g, signed, j) % q:
                return False
        return True


def check_results(reqs: list[Request], runs: list[Stats], checker: PointCheck | None = None,
                  workers: int = 16) -> dict:
    """Every served result of every run checked on the host at the random points (in a thread
    pool: numpy releases the interpreter lock on whole arrays); f(r) and g(r) are evaluated
    once per request.  Counts of checked and failed results (failures listed by index)."""
    import concurrent.futures as cf
    checker = checker or PointCheck()
    for j in range(len(checker.points)):  # fill the power caches before the threads read them
        checker._powers(j, 2 * max(r.f.shape[0] for r in reqs))
    npts = len(checker.points)

    def fg(r):
        return [checker.value(r.f, r.signed, j) * checker.value(r.g, r.signed, j) % checker.points[j][0]
                for j in range(npts)]

    def ok(args):
        want, h = args
        return all(checker.value(h, True, j) == want[j] for j in range(npts))

    bad = []
    checked = 0
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        wants = list(ex.map(fg, reqs))
        for st in runs:
            items = [(d.idx, ks.to_host(d.out)) for d in st.results]
            res = ex.map(ok, [(wants[i], h) for i, h in items])
            for (i, _h), good in zip(items, res):
                checked += 1
                if not good:
                    bad.append(i)
    return {"checked": checked, "failed": len(bad), "failed_idx": bad[:20],
            "points": [{"q": q, "r": r} for q, r in checker.points]}


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


def with_arrivals(reqs: list[Request], rate_per_s: float, seed: int = 5) -> list[Request]:
    """The same requests (same operands) with Poisson arrival times at `rate_per_s`."""
    from . import workloads as wl
    arr = wl.poisson_arrivals(len(reqs), rate_per_s, seed)
    return [Request(r.idx, float(arr[i]), r.f, r.g, r.bits, r.signed) for i, r in enumerate(reqs)]


def measure(count: int = 10000, max_len: int = 65536, max_bits: int = 256, slots: int = 16, streams: int = 4,
            variant: str = "auto", check: bool = True) -> dict:
    """The serving measurement: a closed loop (every request queued at t = 0) gives the saturated
    throughput; the same requests then arrive as a Poisson stream at 0.7 of it.  Every result of
    both runs is checked at random points afterwards (outside the timed runs)."""
    import torch
    closed = make_requests(count, 0.0, 5, max_len, max_bits)
    srv = Server(slots=slots, streams=streams, variant=variant)
    srv.warm(closed)
    sat = srv.run(closed)
    rate = 0.7 * sat.products_per_s
    reqs = with_arrivals(closed, rate, 5)
    st = srv.run(reqs)
    chk = None
    if check:
        chk = check_results(closed, [sat, st])
        if chk["failed"]:
            raise SystemExit(f"serving: results fail the point check: {chk}")
    del sat.results, st.results
    torch.cuda.synchronize()
    return {
        "workload": f"serving_requests: {count} signed Z[x] products, L log-uniform in [8, {max_len}], "
                    f"b uniform in [8, {max_bits}], Poisson arrivals (seed 5)",
        "requests": count, "saturated_products_per_s": sat.products_per_s, "rate_per_s": rate,
        "products_per_s": st.products_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
        "closed_loop_p50_ms": sat.p50_ms, "closed_loop_p99_ms": sat.p99_ms,
        "limb_mults_per_s": st.limb_mults / st.wall_s, "max_inflight": st.max_inflight,
        "slots": slots, "streams": streams, "variant": variant,
        "latency": "arrival to completion observed on the host (completion events polled without sleeping)",
        "point_check": chk}


def main(argv=None):
    """Measure the serving mix (see measure) and print one JSON line."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--max-len", type=int, default=65536)
    ap.add_argument("--max-bits", type=int, default=256)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--variant", default="auto")
    a = ap.parse_args(argv)
    print(json.dumps(measure(a.requests, a.max_len, a.max_bits, a.slots, a.streams, a.variant)))


if __name__ == "__main__":
    main()
