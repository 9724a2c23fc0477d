"""GPU parity of the batch ABI (ks_batch_plan_create / ks_batch_run) against the CPU oracle.

* a mixed batch (unequal lengths, signed and unsigned, every variant) checked product by product;
* the 10,000-product workload (lengths log-uniform in [16, 1024], b in {16, 32, 64, 128},
  signed, seed 3) through KS4 and KS1 with every product compared against the classical oracle;
* the modular workload (64 products mod a 60-bit odd p, L = 65536) as the bench runs it: three
  products in full and every product sampled, for KS4 and KS1 (equal everywhere);
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


@pytest.mark.parametrize("engine", [None, "valu", "mfma", "ntt"])
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


@pytest.mark.parametrize("variant", ["ks4", "ks1"])
def test_mixed_batch_full(torch_dev, oracle, variant):
    # the 10,000-product workload as the bench runs it, every product compared in full
    prods = wl.batch_mixed_10000()
    B = ks.Batch()
    for P in prods:
        B.add(P.f, P.g, P.bits, P.signed)
    out = run_batch(torch_dev, B, variant)
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


def kara_levels(torch, B, variant, engine=None):
    """Run the batch with per-launch timing on; Karatsuba levels = the split and combination
    launches of one run / 2."""
    plan = ks.BatchPlan(B.desc_array(), variant, engine)
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    ks.profile_reset()
    ks.profile_enable(True)
    plan.run(ain, aout, ws)
    torch.cuda.synchronize()
    ks.profile_enable(False)
    n, _ms = ks.profile_read("kara")
    ks.profile_reset()
    rc = plan.status(ws)
    assert rc == ks.KS_OK, ks.strerror(rc)
    out = ks.to_host(aout)
    plan.close()
    return out, n // 2


def test_modular_batch_full(torch_dev, oracle):
    # the 64-product modular workload exactly as the bench runs it (default plan: the transform
    # engine's products, no Karatsuba split): three products compared in full (all 131,071
    # coefficients) for KS4 and KS1, every product sampled, and KS4 equal to KS1 everywhere
    p, pairs = wl.batch_mod_64x65536()
    B = ks.Batch()
    for f, g in pairs:
        B.add_mod(f, g, p)
    out4, _ = kara_levels(torch_dev, B, "ks4")
    out1, _ = kara_levels(torch_dev, B, "ks1")
    assert np.array_equal(out4, out1)
    for i in (0, 31, 63):
        f, g = pairs[i]
        exp = oracle.mul_mod(f, g, p)
        assert np.array_equal(B.result(out4, i), exp), ("ks4", i)
        assert np.array_equal(B.result(out1, i), exp), ("ks1", i)
    D = 2 * 65536 - 1
    gen = wl.rng(45)
    for i, (f, g) in enumerate(pairs):
        kidx = np.unique(np.concatenate([[0, 1, 32767, 32768, 65535, 65536, D - 2, D - 1], gen.integers(0, D, 24)]))
        assert np.array_equal(B.result(out1, i)[kidx], oracle.coeffs_mod(f, g, p, kidx)), i


@pytest.mark.parametrize("variant", ["ks4", "ks1"])
def test_modular_batch_matrix_cores_sampled(torch_dev, oracle, variant):
    # the same workload on the matrix cores, where the default plan splits every product by
    # Karatsuba on the polynomials (recursively): every product sampled
    p, pairs = wl.batch_mod_64x65536()
    B = ks.Batch()
    for f, g in pairs:
        B.add_mod(f, g, p)
    out, levels = kara_levels(torch_dev, B, variant, "mfma")
    assert levels >= 1, levels
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


def test_transform_rows_of_two_sizes_in_one_batch(torch_dev, oracle):
    # one batch whose transform products have rows of 2048 (2^22 terms) and of 4096 (2^23, the
    # longest transform), sampled against the oracle
    gen = wl.rng(4242)
    B = ks.Batch()
    prods = []
    for L in (65536, 98304):
        f, g = wl.random_coeffs(gen, L, 256, True), wl.random_coeffs(gen, L, 256, True)
        prods.append((B.add(f, g, 256, True), f, g))
    out = run_batch(torch_dev, B, "ks1", "ntt")
    for i, f, g in prods:
        L = f.shape[0]
        D = 2 * L - 1
        idx = np.unique(np.concatenate([np.arange(0, 4), np.arange(D - 4, D), gen.integers(0, D, 24)]))
        exp = oracle.coeffs_classical(f, g, True, idx, oracle.out_limbs(L, L, 256))
        assert np.array_equal(B.result(out, i)[idx], exp), L


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


# ---- polynomial-level Karatsuba of modular batches ------------------------------------------

KARA_LENGTHS = [2, 3, 4, 5, 17, 64, 257, 1000, 4097]


@pytest.fixture
def karatsuba_from(request):
    """Lower the split threshold (KS_KARATSUBA_MIN_LIMBS, operand limbs) for one test, restored
    afterwards; the split recurses while the halves' operands keep that many limbs."""
    def set_(n):
        ks.tune_set("KS_KARATSUBA_MIN_LIMBS", n)
        ks.tune_set("KS_NTT_MIN_LIMBS", 0)  # products on the transform engine are never split
    yield set_
    ks.tune_reset()


def mod_batch(lengths, p, seed):
    gen = wl.rng(seed)
    B = ks.Batch()
    pairs = []
    for L in lengths:
        f = gen.integers(0, p, size=L, dtype=np.uint64)
        g = gen.integers(0, p, size=L, dtype=np.uint64)
        B.add_mod(f, g, p)
        pairs.append((f, g))
    return B, pairs


@pytest.mark.parametrize("variant", ["ks1", "neg2", "recip2", "ks4", "auto"])
def test_karatsuba_split_against_oracle(torch_dev, oracle, karatsuba_from, variant):
    # every length from the smallest that splits (2) through odd and even halves, in one plan
    karatsuba_from(2)
    p = wl.paper_fig_modulus(60, 9)
    B, pairs = mod_batch(KARA_LENGTHS, p, 61)
    out = run_batch(torch_dev, B, variant)
    for i, (f, g) in enumerate(pairs):
        assert np.array_equal(B.result(out, i), oracle.mul_mod(f, g, p)), (variant, len(f))


@pytest.mark.parametrize("variant", ["ks1", "neg2", "recip2", "ks4"])
def test_karatsuba_three_levels_against_oracle(torch_dev, oracle, karatsuba_from, variant):
    # lengths of about 1000, the threshold set from the variant's own operand length at a
    # quarter of it: the split recurses exactly three times (leaves of 125-138 terms), which the
    # number of split and combination launches shows, and every product matches the oracle
    lengths = [1000, 1001, 1024, 1100]
    p = wl.paper_fig_modulus(60, 13)
    quarter = min(ks.plan((L + 3) // 4, (L + 3) // 4, 60, variant)["operand_limbs_f"] for L in lengths)
    karatsuba_from(quarter)
    B, pairs = mod_batch(lengths, p, 65)
    out, levels = kara_levels(torch_dev, B, variant)
    assert levels == 3, levels
    for i, (f, g) in enumerate(pairs):
        assert np.array_equal(B.result(out, i), oracle.mul_mod(f, g, p)), (variant, len(f))


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_karatsuba_split_equals_unsplit(torch_dev, karatsuba_from, engine):
    # operands of ~3200-4800 limbs split while the halves keep 500: three levels
    p = (1 << 61) - 1
    B, _ = mod_batch([3000, 3000, 4500], p, 62)
    karatsuba_from(0)
    plain = run_batch(torch_dev, B, "ks4", engine)
    karatsuba_from(500)
    split = run_batch(torch_dev, B, "ks4", engine)
    assert np.array_equal(plain, split)


def test_karatsuba_extreme_residues(torch_dev, oracle, karatsuba_from):
    # all p - 1 (the halves' sums wrap mod p) and all 0
    karatsuba_from(2)
    p = wl.paper_fig_modulus(60, 10)
    B = ks.Batch()
    pairs = []
    for L, fill in [(7, p - 1), (64, p - 1), (65, 0), (9, 1)]:
        f = np.full(L, fill, dtype=np.uint64)
        B.add_mod(f, f, p)
        pairs.append((f, f))
    out = run_batch(torch_dev, B, "ks4")
    for i, (f, g) in enumerate(pairs):
        assert np.array_equal(B.result(out, i), oracle.mul_mod(f, g, p)), i


def test_karatsuba_not_applied_to_mixed_batches(torch_dev, oracle, karatsuba_from):
    # a batch with unequal lengths (or integer products) is planned unsplit and stays exact
    karatsuba_from(2)
    p = wl.paper_fig_modulus(60, 11)
    gen = wl.rng(63)
    B = ks.Batch()
    f, g = gen.integers(0, p, size=40, dtype=np.uint64), gen.integers(0, p, size=33, dtype=np.uint64)
    B.add_mod(f, g, p)
    out = run_batch(torch_dev, B, "ks4")
    assert np.array_equal(B.result(out, 0), oracle.mul_mod(f, g, p))


def test_karatsuba_graph_capture_replays(torch_dev, oracle, karatsuba_from):
    torch = torch_dev
    karatsuba_from(100)
    p = wl.paper_fig_modulus(60, 12)
    B, pairs = mod_batch([500, 777, 1024], p, 64)
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
    for rep in range(3):
        aout.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(aout, eager), f"replay {rep}"
        _ = torch.arange(1000, device="cuda").sum().item()
    out = ks.to_host(aout)
    for i, (f, g) in enumerate(pairs):
        assert np.array_equal(B.result(out, i), oracle.mul_mod(f, g, p)), i
    plan.close()


def test_karatsuba_range_error_reported(torch_dev, karatsuba_from):
    torch = torch_dev
    karatsuba_from(2)
    p = 1_000_003
    B = ks.Batch()
    good = np.arange(1, 65, dtype=np.uint64)
    bad = good.copy()
    bad[50] = p  # not a residue (in the upper half)
    B.add_mod(good, good, p)
    B.add_mod(bad, good, p)
    plan = ks.BatchPlan(B.desc_array(), "ks4")
    ain = ks.to_device(B.arena_in())
    aout = torch.zeros(B.out_words(), dtype=torch.int32, device="cuda")
    ws = ks.alloc_workspace(plan.workspace_bytes)
    plan.run(ain, aout, ws)
    assert plan.status(ws) == ks.KS_ERANGE
    plan.close()
