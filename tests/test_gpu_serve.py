"""GPU tests of the serving loop: products admitted while others run give the same bits as
the same product computed alone, and the oracle agrees on a sample; a tight memory budget
makes requests queue instead of failing."""
import numpy as np
import pytest

from paper_0712_4046_amd import ks
from paper_0712_4046_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.lib()
    return torch


def test_results_in_mix_equal_results_alone(torch_dev, oracle):
    reqs = serve.make_requests(160, rate_per_s=20000.0, seed=51, max_len=2048, max_bits=256)
    srv = serve.Server(slots=8, streams=4)
    st = srv.run(reqs)
    assert st.completed == len(reqs)
    assert st.max_inflight > 1, "requests never overlapped"
    for d in st.results:
        r = reqs[d.idx]
        alone = ks.mul(ks.to_device(r.f), ks.to_device(r.g), r.bits, "auto", True)
        ks.check()
        assert np.array_equal(ks.to_host(d.out), ks.to_host(alone)), d.idx
    for d in st.results[::8]:
        r = reqs[d.idx]
        exp = oracle.mul_classical(r.f, r.g, True, oracle.out_limbs(r.f.shape[0], r.g.shape[0], r.bits))
        assert np.array_equal(ks.to_host(d.out), exp), d.idx
    assert st.p99_ms >= st.p50_ms > 0


def test_small_memory_budget_queues(torch_dev):
    reqs = serve.make_requests(40, rate_per_s=0.0, seed=52, max_len=512, max_bits=64)
    srv = serve.Server(slots=8, streams=2, mem_budget=1)  # one request at a time
    st = srv.run(reqs)
    assert st.completed == len(reqs)
    assert st.max_inflight == 1


def test_large_mix_equals_alone(torch_dev, oracle):
    # long products of every size on four streams, each stream's scratch reused by products of
    # different layouts: every result equals the same product computed alone (regression: the
    # look-back status words of a product once lived in that reused scratch, where data of an
    # earlier product could read as a fresh status word)
    reqs = serve.make_requests(1100, rate_per_s=0.0, seed=5, max_len=65536, max_bits=256)
    srv = serve.Server(slots=16, streams=4)
    srv.warm(reqs)
    st = srv.run(reqs)
    assert st.completed == len(reqs)
    for d in st.results:
        r = reqs[d.idx]
        alone = ks.mul(ks.to_device(r.f), ks.to_device(r.g), r.bits, "auto", True)
        ks.check()
        assert torch_dev.equal(d.out, alone), d.idx
    # the 20 largest requests (limbs per input) against the classical oracle: the first and last
    # coefficients and 200 random ones each
    big = sorted(st.results, key=lambda d: -reqs[d.idx].f.size)[:20]
    gen = np.random.Generator(np.random.PCG64(53))
    for d in big:
        r = reqs[d.idx]
        L = r.f.shape[0]
        D = 2 * L - 1
        idx = np.unique(np.concatenate([[0, D - 1], gen.integers(0, D, 200)]))
        exp = oracle.coeffs_classical(r.f, r.g, True, idx, oracle.out_limbs(L, L, r.bits))
        assert np.array_equal(ks.to_host(d.out)[idx], exp), (d.idx, L, r.bits)


def test_every_served_result_passes_the_point_check(torch_dev):
    # the check bench.py applies to every served result, on a small stream
    reqs = serve.make_requests(200, rate_per_s=0.0, seed=54, max_len=4096, max_bits=256)
    srv = serve.Server(slots=16, streams=4)
    st = srv.run(reqs)
    chk = serve.check_results(reqs, [st])
    assert chk["checked"] == len(reqs) and chk["failed"] == 0, chk
