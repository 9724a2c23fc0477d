"""Host logic of the serving harness (no GPU): the random-point check that bench.py applies to
every served result accepts exact products and rejects wrong ones."""
import numpy as np

from paper_0712_4046_amd import serve
from paper_0712_4046_amd import workloads as wl


def test_point_check_accepts_exact_products(oracle):
    chk = serve.PointCheck(seed=7)
    gen = wl.rng(70)
    for L, bits, signed in [(1, 8, True), (5, 33, True), (300, 64, True), (257, 256, True), (40, 32, False)]:
        f, g = wl.random_coeffs(gen, L, bits, signed), wl.random_coeffs(gen, L + 3, bits, signed)
        h = oracle.mul_classical(f, g, signed, oracle.out_limbs(L, L + 3, bits))
        assert chk.holds(f, g, h, signed), (L, bits, signed)


def test_point_check_rejects_wrong_products(oracle):
    chk = serve.PointCheck(seed=8)
    gen = wl.rng(71)
    f, g = wl.random_coeffs(gen, 200, 100, True), wl.random_coeffs(gen, 200, 100, True)
    h = oracle.mul_classical(f, g, True, oracle.out_limbs(200, 200, 100))
    for k, t, delta in [(0, 0, 1), (199, 3, 1 << 31), (398, 6, 1), (57, 2, 0xFFFF)]:
        bad = h.copy()
        bad[k, t] ^= np.uint32(delta)
        assert not chk.holds(f, g, bad, True), (k, t)
    # a dropped top limb (the sign of a coefficient flipped to its unsigned reading)
    bad = h.copy()
    bad[10, -1] = 0
    assert not chk.holds(f, g, bad, True)


def test_residues_of_signed_limbs():
    q = serve.SZ_PRIMES[0]
    vals = [0, 1, -1, 2**95 - 1, -2**95, 123456789012345678901234567]
    from oracle import oracle as O
    limbs = O.ints_to_limbs(vals, 3)
    got = serve._residues(limbs, q, True)
    assert [int(x) for x in got] == [v % q for v in vals]


def test_request_stream_shapes():
    # the serving mix is drawn on the host: lengths and widths in range, arrivals ordered, and the
    # same operands re-timed for the Poisson run
    reqs = serve.make_requests(50, 0.0, seed=5, max_len=4096, max_bits=256)
    assert len(reqs) == 50 and all(r.arrival == 0.0 for r in reqs)
    for r in reqs:
        assert 8 <= r.f.shape[0] <= 4096 and r.f.shape == r.g.shape
        assert 8 <= r.bits <= 256 and r.f.shape[1] == (r.bits + 31) // 32
    timed = serve.with_arrivals(reqs, 1000.0, seed=5)
    arr = [r.arrival for r in timed]
    assert arr == sorted(arr) and arr[0] > 0
    assert all(a.f is b.f and a.idx == b.idx for a, b in zip(reqs, timed))
