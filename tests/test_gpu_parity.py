"""GPU parity: every product through the C ABI is bit-exact against the CPU oracle.

Inputs come from the seeded generators in paper_0712_4046_amd.workloads; expected values come
only from oracle/ (classical convolution).  Sizes span several tiles and scan blocks and
include ragged tails; the edge grid covers lengths 1..3, unequal lengths with an odd and an
even number of output coefficients, bit sizes around limb boundaries, and structured inputs.
"""
import numpy as np
import pytest

from paper_0712_4046_amd import ks
from paper_0712_4046_amd import workloads as wl

pytestmark = pytest.mark.gpu

VARIANTS = ["ks1", "neg2", "recip2", "ks4"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.lib()
    return torch


ENGINES = ["valu", "mfma", "ntt"]


def gpu_mul(f, g, bits, variant, signed, engine=None):
    tf, tg = ks.to_device(f), ks.to_device(g)
    h = ks.mul(tf, tg, bits, variant, signed, engine=engine)
    rc = ks.status()
    assert rc == ks.KS_OK, ks.strerror(rc)
    return ks.to_host(h)


def want(oracle, f, g, bits, signed):
    return oracle.mul_classical(f, g, signed, oracle.out_limbs(f.shape[0], g.shape[0], bits))


def assert_same(got, exp, label):
    if not np.array_equal(got, exp):
        bad = np.nonzero((got != exp).any(axis=1))[0]
        raise AssertionError(f"{label}: {len(bad)} coefficients differ, first at {bad[:8].tolist()}")


def test_paper_example(torch_dev, oracle):
    f = oracle.ints_to_limbs([274, 610, 887, 621], 1)
    g = oracle.ints_to_limbs([553, 298, 424, 790], 1)
    for v in VARIANTS + ["auto"]:
        got = oracle.limbs_to_ints(gpu_mul(f, g, 10, v, False), False)
        assert got == [151522, 418982, 788467, 1082839, 1043046, 964034, 490590], v


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_product_256_u32_full(torch_dev, oracle, variant, engine):
    P = wl.product_256_u32()
    assert_same(gpu_mul(P.f, P.g, P.bits, variant, P.signed, engine), want(oracle, P.f, P.g, P.bits, P.signed),
                f"product_256_u32 {variant} {engine}")


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_product_4096_s64_full(torch_dev, oracle, variant, engine):
    P = wl.product_4096_s64()
    assert_same(gpu_mul(P.f, P.g, P.bits, variant, P.signed, engine), want(oracle, P.f, P.g, P.bits, P.signed),
                f"product_4096_s64 {variant} {engine}")


EDGE_LENGTHS = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 3), (3, 5), (5, 3), (4, 7), (17, 16), (33, 2), (64, 64)]
EDGE_BITS = [1, 2, 31, 32, 33, 60, 64, 65, 128, 256]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("bits", EDGE_BITS)
def test_edge_grid(torch_dev, oracle, bits, engine):
    for lf, lg in EDGE_LENGTHS:
        for signed in (False, True):
            gen = wl.rng(lf * 100 + lg + bits)
            f = wl.random_coeffs(gen, lf, bits, signed)
            g = wl.random_coeffs(gen, lg, bits, signed)
            exp = want(oracle, f, g, bits, signed)
            for v in VARIANTS:
                assert_same(gpu_mul(f, g, bits, v, signed, engine), exp,
                            f"{v} {engine} lf={lf} lg={lg} b={bits} s={signed}")


@pytest.mark.parametrize("kind", ["max", "min", "zero", "onehot", "sparse", "tiny"])
@pytest.mark.parametrize("bits,signed", [(32, False), (64, True), (128, True), (17, False), (200, True)])
def test_structured_inputs(torch_dev, oracle, kind, bits, signed):
    gen = wl.rng(7)
    f = wl.special_coeffs(kind, 301, bits, signed, gen)
    g = wl.special_coeffs(kind, 300, bits, signed, gen)
    exp = want(oracle, f, g, bits, signed)
    for v in VARIANTS:
        for e in ENGINES:
            assert_same(gpu_mul(f, g, bits, v, signed, e), exp, f"{kind} {v} {e} b={bits} s={signed}")


@pytest.mark.parametrize("lf,lg,bits,signed", [(5000, 4999, 128, True), (3000, 1001, 64, False), (3000, 1000, 64, True),
                                               (20000, 20000, 8, False), (7, 9000, 100, True)])
def test_multi_block_sizes(torch_dev, oracle, lf, lg, bits, signed):
    # operands and products span many carry-scan blocks and multiplier tiles/splits
    gen = wl.rng(lf + lg + bits)
    f = wl.random_coeffs(gen, lf, bits, signed)
    g = wl.random_coeffs(gen, lg, bits, signed)
    exp = want(oracle, f, g, bits, signed)
    for v in VARIANTS:
        for e in ENGINES:
            assert_same(gpu_mul(f, g, bits, v, signed, e), exp, f"{v} {e} lf={lf} lg={lg} b={bits}")


@pytest.mark.parametrize("lf,lg,bits,signed", [(4096, 4096, 64, True), (3000, 1001, 64, False), (7, 9000, 100, True),
                                               (300, 300, 17, False)])
def test_single_product_with_batch_scan_blocks(torch_dev, oracle, monkeypatch, lf, lg, bits, signed):
    # KS_SCAN_BIG = 1: every single product takes a batch's carry-scan blocks (8 limbs per
    # thread in pack, 4 in the recombination), as large single products do by default
    monkeypatch.setenv("KS_SCAN_BIG", "1")
    gen = wl.rng(3 * lf + lg + bits)
    f = wl.random_coeffs(gen, lf, bits, signed)
    g = wl.random_coeffs(gen, lg, bits, signed)
    exp = want(oracle, f, g, bits, signed)
    for v in VARIANTS:
        for e in ENGINES:
            assert_same(gpu_mul(f, g, bits, v, signed, e), exp, f"{v} {e} lf={lf} lg={lg} b={bits} batch scan blocks")


def test_deterministic(torch_dev):
    P = wl.product_4096_s64()
    a = gpu_mul(P.f, P.g, P.bits, "ks4", True)
    b = gpu_mul(P.f, P.g, P.bits, "ks4", True)
    assert np.array_equal(a, b)


def test_other_stream(torch_dev, oracle):
    torch = torch_dev
    P = wl.product_256_u32()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tf, tg = ks.to_device(P.f), ks.to_device(P.g)
        h = ks.mul(tf, tg, P.bits, "ks4", False, stream=s)
        assert ks.status(s) == ks.KS_OK
    assert_same(ks.to_host(h), want(oracle, P.f, P.g, P.bits, False), "side stream")


def test_mod_small(torch_dev, oracle):
    torch = torch_dev
    # odd and even moduli: Section 4 lifts, multiplies and reduces modulo any word-sized n
    for p in (2, 3, 10, 65537, (1 << 31) - 1, 1 << 32, wl.batch_mod_modulus(), (1 << 61) - 1, 1 << 61,
              (1 << 62) - 2):
        gen = wl.rng(p % 1000)
        for lf, lg in ((1, 1), (2, 3), (300, 257), (1000, 1000)):
            f = gen.integers(0, p, size=lf, dtype=np.uint64)
            g = gen.integers(0, p, size=lg, dtype=np.uint64)
            exp = oracle.mul_mod(f, g, p)
            for v in VARIANTS:
                tf = torch.from_numpy(f.view(np.int64)).cuda()
                tg = torch.from_numpy(g.view(np.int64)).cuda()
                h = ks.mul_mod(tf, tg, p, v, engine="mfma" if lf >= 300 else None)
                assert ks.status() == ks.KS_OK
                got = h.cpu().numpy().view(np.uint64)
                assert np.array_equal(got, exp), (p, lf, lg, v)


def test_mod_one_product_of_the_modular_batch_sampled(torch_dev, oracle):
    torch = torch_dev
    p, pairs = wl.batch_mod_64x65536(count=1)
    f, g = pairs[0]
    tf = torch.from_numpy(f.view(np.int64)).cuda()
    tg = torch.from_numpy(g.view(np.int64)).cuda()
    D = len(f) + len(g) - 1
    ks_idx = np.unique(np.concatenate([np.arange(0, 40), np.arange(D - 40, D), wl.rng(11).integers(0, D, 400)]))
    exp = oracle.coeffs_mod(f, g, p, ks_idx)
    for v, e in (("ks4", "mfma"), ("ks4", "valu"), ("ks1", None)):
        h = ks.mul_mod(tf, tg, p, v, engine=e)
        assert ks.status() == ks.KS_OK
        got = h.cpu().numpy().view(np.uint64)[ks_idx]
        assert np.array_equal(got, exp), (v, e)


@pytest.mark.parametrize("nbits", [4, 48])
def test_mod_paper_moduli(torch_dev, oracle, nbits):
    # the moduli and lengths of the paper's example timings (random odd 4-bit and 48-bit n):
    # every variant against the oracle, in full up to L = 4096, sampled at L = 65536
    torch = torch_dev
    for L in wl.PAPER_FIG_LENGTHS:
        n, f, g = wl.paper_fig_pair(nbits, L)
        tf = torch.from_numpy(f.view(np.int64)).cuda()
        tg = torch.from_numpy(g.view(np.int64)).cuda()
        if L <= 4096:
            idx = None
            exp = oracle.mul_mod(f, g, n)
        elif L == 65536:
            D = 2 * L - 1
            idx = np.unique(np.concatenate([np.arange(0, 30), np.arange(D - 30, D), wl.rng(L).integers(0, D, 200)]))
            exp = oracle.coeffs_mod(f, g, n, idx)
        else:
            continue
        for v in VARIANTS:
            h = ks.mul_mod(tf, tg, n, v)
            assert ks.status() == ks.KS_OK
            got = h.cpu().numpy().view(np.uint64)
            assert np.array_equal(got if idx is None else got[idx], exp), (nbits, L, v)


@pytest.mark.parametrize("bits", [128, 256])
def test_long_wide_product_sampled(torch_dev, oracle, bits):
    # one signed product of length 65536 with 128- or 256-bit coefficients (the largest requests
    # of the serving mix) through every variant: the first and last 20 coefficients and 200
    # random ones against the classical oracle; the variants agree everywhere
    gen = wl.rng(900 + bits)
    L = 65536
    f, g = wl.random_coeffs(gen, L, bits, True), wl.random_coeffs(gen, L, bits, True)
    D = 2 * L - 1
    wo = oracle.out_limbs(L, L, bits)
    idx = np.unique(np.concatenate([np.arange(0, 20), np.arange(D - 20, D), gen.integers(0, D, 200)]))
    exp = oracle.coeffs_classical(f, g, True, idx, wo)
    tf, tg = ks.to_device(f), ks.to_device(g)
    first = None
    for v in VARIANTS:
        h = ks.mul(tf, tg, bits, v, True)
        rc = ks.status()
        assert rc == ks.KS_OK, (v, ks.strerror(rc))
        got = ks.to_host(h)
        assert np.array_equal(got[idx], exp), (bits, v)
        if first is None:
            first = got
        else:
            assert np.array_equal(got, first), (bits, v)


@pytest.mark.parametrize("kind,signed", [("max", False), ("min", True), ("max", True)])
def test_transform_engine_extreme_terms(torch_dev, oracle, kind, signed):
    # the largest convolution terms the transform engine meets: all-max (or all-min) 256-bit
    # coefficients at L = 65536 through the standard substitution (one product of ~1.08M-limb
    # operands, a transform of 2^22 terms), sampled against the oracle
    L, bits = 65536, 256
    f = wl.special_coeffs(kind, L, bits, signed)
    D = 2 * L - 1
    idx = np.unique(np.concatenate([np.arange(0, 8), np.arange(D - 8, D), wl.rng(5).integers(0, D, 60)]))
    exp = oracle.coeffs_classical(f, f, signed, idx, oracle.out_limbs(L, L, bits))
    tf = ks.to_device(f)
    h = ks.mul(tf, tf, bits, "ks1", signed, engine="ntt")
    assert ks.status() == ks.KS_OK
    assert np.array_equal(ks.to_host(h)[idx], exp)


def test_transform_engine_longest_transform(torch_dev, oracle):
    # L = 98304 signed 256-bit coefficients through the standard substitution: the planner
    # reaches the longest transform (2^23 terms, rows of 4096 in the row step), sampled against
    # the oracle
    L, bits = 98304, 256
    plan = ks.plan(L, L, bits, "ks1", True, "ntt")
    assert plan["ntt_k1"] + plan["ntt_k2"] == 23 and plan["ntt_k2"] == 12
    gen = wl.rng(2323)
    f, g = wl.random_coeffs(gen, L, bits, True), wl.random_coeffs(gen, L, bits, True)
    D = 2 * L - 1
    idx = np.unique(np.concatenate([np.arange(0, 8), np.arange(D - 8, D), gen.integers(0, D, 40)]))
    exp = oracle.coeffs_classical(f, g, True, idx, oracle.out_limbs(L, L, bits))
    h = ks.mul(ks.to_device(f), ks.to_device(g), bits, "ks1", True, engine="ntt")
    assert ks.status() == ks.KS_OK
    assert np.array_equal(ks.to_host(h)[idx], exp)


def test_invalid_arguments(torch_dev):
    torch = torch_dev
    t = torch.zeros((4, 1), dtype=torch.int32, device="cuda")
    h = torch.zeros((7, 2), dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert ks.mul_raw(t.data_ptr(), t.data_ptr(), 0, 4, 8, 1, s, h.data_ptr()) == ks.KS_EINVAL
    assert ks.mul_raw(t.data_ptr(), t.data_ptr(), 4, 4, 0, 1, s, h.data_ptr()) == ks.KS_EINVAL
    assert ks.mul_raw(t.data_ptr(), t.data_ptr(), 4, 4, 300, 1, s, h.data_ptr()) == ks.KS_EINVAL
    assert ks.mul_raw(t.data_ptr(), t.data_ptr(), 4, 4, 8, 5, s, h.data_ptr()) == ks.KS_EINVAL
    assert ks.mul_raw(0, t.data_ptr(), 4, 4, 8, 1, s, h.data_ptr()) == ks.KS_EINVAL
    assert ks.status() == ks.KS_OK


def test_out_of_range_coefficient_is_reported(torch_dev, oracle):
    f = oracle.ints_to_limbs([1, 2, 300, 4], 1)  # 300 does not fit in 8 bits
    g = oracle.ints_to_limbs([5, 6, 7, 8], 1)
    for v in VARIANTS:
        ks.mul(ks.to_device(f), ks.to_device(g), 8, v, False)
        assert ks.status() == ks.KS_ERANGE
        assert ks.status() == ks.KS_OK  # cleared after reading
    fs = oracle.ints_to_limbs([1, -2, 127, -128], 1)
    ks.mul(ks.to_device(fs), ks.to_device(fs), 8, "ks4", True)
    assert ks.status() == ks.KS_OK
    fb = oracle.ints_to_limbs([1, 200, 3, 4], 1)  # 200 is not an 8-bit signed value
    ks.mul(ks.to_device(fb), ks.to_device(fs), 8, "ks4", True)
    assert ks.status() == ks.KS_ERANGE


@pytest.mark.parametrize("blocks,min_part", [("1", "1000000"), ("4096", "32"), ("1024", "128"), ("40", "128"),
                                             ("0", "128"), ("0", "1")])
def test_mfma_part_splits(torch_dev, oracle, monkeypatch, blocks, min_part):
    # the matrix-core multiplier cuts each row group's shift range into parts, and each part
    # into residue groups, whose column sums meet in 64-bit atomics: one block per group, many
    # short parts over four residue groups, two residue groups (40 blocks), the launch-shape
    # model (0)
    monkeypatch.setenv("KS_MFMA_BLOCKS", blocks)
    monkeypatch.setenv("KS_MFMA_MIN_PART", min_part)
    P = wl.product_4096_s64()
    exp = want(oracle, P.f, P.g, P.bits, P.signed)
    for v in VARIANTS:
        assert_same(gpu_mul(P.f, P.g, P.bits, v, P.signed, "mfma"), exp, f"product_4096_s64 {v} blocks={blocks} part>={min_part}")


@pytest.mark.parametrize("pattern", [0x7F, 0x80, 0xFF])
@pytest.mark.parametrize("L", [1, 7, 300])
def test_mfma_balanced_digit_carries(torch_dev, oracle, pattern, L):
    # the matrix-core digits are balanced base-256 digits, whose carries run through every
    # byte 0x7f: coefficients of 0x7f bytes over a low byte `pattern` (0x80 and 0xff start a
    # carry that must cross the whole run, within a wave's limbs and across waves)
    bits = 256
    w = bits // 32
    one = np.full((L, w), 0x7F7F7F7F, dtype=np.uint32)
    one[:, 0] = (one[:, 0] & np.uint32(0xFFFFFF00)) | np.uint32(pattern)
    other = np.full((L, w), 0x7F7F7F7F, dtype=np.uint32)
    for f, g in ((one, other), (one, one)):
        exp = want(oracle, f, g, bits, False)
        for v in VARIANTS:
            assert_same(gpu_mul(f, g, bits, v, False, "mfma"), exp, f"0x7f runs over {pattern:#x} L={L} {v}")


@pytest.mark.parametrize("variant", ["ks1", "neg2"])
def test_mfma_long_shift_ranges_sampled(torch_dev, oracle, variant):
    # L = 65536 signed 64-bit: the standard substitution's operands hold ~295k limbs (~1.35M
    # digits), more block shifts per row group than one part may take (32768), so every row
    # group is split; checked on the first and last coefficients and a random sample
    L, bits = 65536, 64
    gen = wl.rng(41)
    f = wl.random_coeffs(gen, L, bits, True)
    g = wl.random_coeffs(gen, L, bits, True)
    tf, tg = ks.to_device(f), ks.to_device(g)
    h = ks.mul(tf, tg, bits, variant, True, engine="mfma")
    assert ks.status() == ks.KS_OK
    got = ks.to_host(h)
    D = 2 * L - 1
    idx = np.unique(np.concatenate([np.arange(0, 40), np.arange(D - 40, D), np.arange(L - 20, L + 20),
                                    wl.rng(42).integers(0, D, 300)]))
    exp = oracle.coeffs_classical(f, g, True, idx, got.shape[1])
    assert_same(got[idx], exp, f"L=65536 {variant} mfma sampled")


@pytest.mark.parametrize("rt", ["4", "8"])
def test_mfma_tiles_per_block(torch_dev, oracle, monkeypatch, rt):
    # the matrix-core blocks own 4 or 8 tiles of 32 output rows (the planner picks per product)
    monkeypatch.setenv("KS_MFMA_RT", rt)
    P = wl.product_4096_s64()
    exp = want(oracle, P.f, P.g, P.bits, P.signed)
    for v in VARIANTS:
        assert_same(gpu_mul(P.f, P.g, P.bits, v, P.signed, "mfma"), exp, f"product_4096_s64 {v} rt={rt}")
    for blocks, part in (("1", "1000000"), ("4096", "32")):
        monkeypatch.setenv("KS_MFMA_BLOCKS", blocks)
        monkeypatch.setenv("KS_MFMA_MIN_PART", part)
        assert_same(gpu_mul(P.f, P.g, P.bits, "ks4", P.signed, "mfma"), exp, f"product_4096_s64 ks4 rt={rt} blocks={blocks}")


@pytest.mark.parametrize("rt", ["4", "8"])
def test_mfma_tiles_unequal_modular(torch_dev, oracle, monkeypatch, rt):
    # both tile counts on unequal lengths and a modular product (the reversed operands of the
    # four-point and reciprocal variants have their own lengths)
    monkeypatch.setenv("KS_MFMA_RT", rt)
    gen = wl.rng(41)
    f = wl.random_coeffs(gen, 3001, 64, True)
    g = wl.random_coeffs(gen, 1777, 64, True)
    exp = want(oracle, f, g, 64, True)
    for v in VARIANTS:
        assert_same(gpu_mul(f, g, 64, v, True, "mfma"), exp, f"unequal {v} rt={rt}")
    p = 2**61 - 1
    fm = gen.integers(0, p, size=2500, dtype=np.uint64)
    gm = gen.integers(0, p, size=4100, dtype=np.uint64)
    expm = oracle.mul_mod(fm, gm, p)
    tf = torch_dev.from_numpy(fm.view(np.int64)).cuda()
    tg = torch_dev.from_numpy(gm.view(np.int64)).cuda()
    for v in VARIANTS:
        h = ks.mul_mod(tf, tg, p, v, engine="mfma")
        assert ks.status() == ks.KS_OK
        assert np.array_equal(h.cpu().numpy().view(np.uint64), expm), f"modular {v} rt={rt}"
