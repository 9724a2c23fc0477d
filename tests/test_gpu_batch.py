"""GPU parity of the batch ABI (ks_batch_plan_create / ks_batch_run) against the CPU oracle.

* a mixed batch (unequal lengths, signed and unsigned, every variant) checked product by product;
* the 10,000-product workload (lengths log-uniform in [16, 1024], b in {16, 32, 64, 128},
  signed, seed 3) with every product compared against the classical oracle;
* the modular workload (64 products mod a 60-bit odd p, L = 65536) on sampled coefficients;
* a run captured in a hipGraph, replayed several times with eager work in between;
* descriptor validation and device range errors.
"""
import numpy as np
import pytest

from paper_0712_4046_amd import ks
from paper_0712_4046_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.lib()
    return torch


def run_batch(torch, B, variant="auto", engine=None):
    descs = B.desc_array()
    plan = ks.BatchPlan(descs, variant, engine)
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    plan.run(ain, aout, ws)
    rc = plan.status(ws)
    assert rc == ks.KS_OK, ks.strerror(rc)
    out = ks.to_host(aout)
    plan.close()
    return out


@pytest.mark.parametrize("engine", [None, "valu", "mfma"])
@pytest.mark.parametrize("variant", ["ks1", "neg2", "recip2", "ks4", "auto"])
def test_mixed_batch(torch_dev, oracle, variant, engine):
    gen = wl.rng(31)
    B = ks.Batch()
    cases = []
    for _ in range(120):
        lf, lg = int(gen.integers(1, 300)), int(gen.integers(1, 300))
        bits = int(gen.choice([1, 7, 16, 32, 33, 64, 100, 128, 200]))
        signed = bool(gen.integers(0, 2))
        f, g = wl.random_coeffs(gen, lf, bits, signed), wl.random_coeffs(gen, lg, bits, signed)
        cases.append((B.add(f, g, bits, signed), f, g, bits, signed))
    out = run_batch(torch_dev, B, variant, engine)
    for i, f, g, bits, signed in cases:
        exp = oracle.mul_classical(f, g, signed, oracle.out_limbs(f.shape[0], g.shape[0], bits))
        assert np.array_equal(B.result(out, i), exp), (variant, i, f.shape[0], g.shape[0], bits, signed)


def test_mixed_batch_full(torch_dev, oracle):
    prods = wl.batch_mixed_10000()
    B = ks.Batch()
    for P in prods:
        B.add(P.f, P.g, P.bits, P.signed)
    out = run_batch(torch_dev, B, "ks4")
    for i, P in enumerate(prods):
        exp = oracle.mul_classical(P.f, P.g, P.signed, oracle.out_limbs(P.f.shape[0], P.g.shape[0], P.bits))
        assert np.array_equal(B.result(out, i), exp), i


def test_mixed_batch_unequal_lengths(torch_dev, oracle):
    prods = wl.batch_mixed_10000(count=600, independent_lengths=True, seed=33)
    B = ks.Batch()
    for P in prods:
        B.add(P.f, P.g, P.bits, P.signed)
    out = run_batch(torch_dev, B, "auto")
    for i, P in enumerate(prods):
        exp = oracle.mul_classical(P.f, P.g, P.signed, oracle.out_limbs(P.f.shape[0], P.g.shape[0], P.bits))
        assert np.array_equal(B.result(out, i), exp), i


def test_modular_batch_sampled(torch_dev, oracle):
    p, pairs = wl.batch_mod_64x65536()
    B = ks.Batch()
    for f, g in pairs:
        B.add_mod(f, g, p)
    out = run_batch(torch_dev, B, "ks4", "mfma")
    D = 2 * 65536 - 1
    gen = wl.rng(44)
    for i, (f, g) in enumerate(pairs):
        kidx = np.unique(np.concatenate([[0, 1, 65535, 65536, D - 2, D - 1], gen.integers(0, D, 24)]))
        assert np.array_equal(B.result(out, i)[kidx], oracle.coeffs_mod(f, g, p, kidx)), i


def test_graph_capture_replays(torch_dev, oracle):
    torch = torch_dev
    prods = wl.batch_mixed_10000(count=300, seed=35)
    B = ks.Batch()
    for P in prods:
        B.add(P.f, P.g, P.bits, P.signed)
    plan = ks.BatchPlan(B.desc_array(), "ks4")
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    plan.run(ain, aout, ws)
    assert plan.status(ws) == ks.KS_OK
    eager = aout.clone()
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.run(ain, aout, ws, stream=s)
    for rep in range(4):
        aout.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(aout, eager), f"replay {rep}"
        _ = torch.arange(1000, device="cuda").sum().item()  # eager work between replays
    assert plan.status(ws) == ks.KS_OK
    out = ks.to_host(aout)
    for i, P in enumerate(prods[:50]):
        exp = oracle.mul_classical(P.f, P.g, P.signed, oracle.out_limbs(P.f.shape[0], P.g.shape[0], P.bits))
        assert np.array_equal(B.result(out, i), exp), i
    plan.close()


def test_invalid_descriptor_named(torch_dev):
    B = ks.Batch()
    f = np.zeros((4, 1), dtype=np.uint32)
    B.add(f, f, 8, False)
    B.add(f, f, 8, False)
    descs = B.desc_array()
    descs[1].coeff_bits = 0
    with pytest.raises(ks.KSError) as ei:
        ks.BatchPlan(descs)
    assert ei.value.code == ks.KS_EINVAL
    assert ks.lib().ks_batch_plan_bad_index() == 1


def test_batch_range_error_reported(torch_dev):
    torch = torch_dev
    B = ks.Batch()
    good = np.array([[1], [2], [3]], dtype=np.uint32)
    bad = np.array([[1], [999], [3]], dtype=np.uint32)  # 999 does not fit in 8 bits
    B.add(good, good, 8, False)
    B.add(bad, good, 8, False)
    plan = ks.BatchPlan(B.desc_array(), "ks4")
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    plan.run(ain, aout, ws)
    assert plan.status(ws) == ks.KS_ERANGE
    assert plan.status(ws) == ks.KS_OK
    plan.close()
