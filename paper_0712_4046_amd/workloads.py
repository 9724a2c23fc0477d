"""Seeded synthetic inputs for the workloads the library is measured and tested on.

This module only draws random coefficients and lays them out; it holds none of the
multiplication's arithmetic, so both the GPU path and the CPU oracle can take their inputs
from it.  All draws use ``numpy.random.Generator(PCG64(seed))``.

Layout: a polynomial of length L with b-bit coefficients is a (L, W) uint32 array,
W = ceil(b / 32), coefficient i in row i as little-endian limbs; signed values are stored in
two's complement (sign-extended to 32 W bits).

The paper measured random polynomials over random moduli (Section 4); these generators
stand in for those inputs with the shapes listed in ``CONFIGS``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def limbs_for_bits(bits: int) -> int:
    return (bits + 31) // 32


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_coeffs(gen: np.random.Generator, length: int, bits: int, signed: bool) -> np.ndarray:
    """Uniform b-bit coefficients: [0, 2^b) unsigned, [-2^(b-1), 2^(b-1)) signed."""
    w = limbs_for_bits(bits)
    a = gen.integers(0, 1 << 32, size=(length, w), dtype=np.uint64).astype(np.uint32)
    top = bits - 32 * (w - 1)  # bits used in the top limb, 1..32
    if top < 32:
        a[:, w - 1] &= np.uint32((1 << top) - 1)
    if signed:
        # reinterpret the b-bit pattern as two's complement and sign-extend to 32 w bits
        neg = ((a[:, w - 1] >> np.uint32(top - 1)) & np.uint32(1)).astype(bool)
        if top < 32:
            a[neg, w - 1] |= np.uint32((0xFFFFFFFF << top) & 0xFFFFFFFF)
    return a


def special_coeffs(kind: str, length: int, bits: int, signed: bool, gen=None) -> np.ndarray:
    """Structured inputs for edge cases: all-max, all-min, zero, one-hot, sparse, tiny."""
    w = limbs_for_bits(bits)
    a = np.zeros((length, w), dtype=np.uint32)
    top = bits - 32 * (w - 1)
    if kind == "max":           # 2^b - 1 (unsigned) or 2^(b-1) - 1 (signed)
        a[:] = 0xFFFFFFFF
        keep = top - 1 if signed else top
        if keep == 0 and w > 1:
            a[:, w - 1] = 0
        else:
            a[:, w - 1] = np.uint32((1 << keep) - 1) if keep < 32 else np.uint32(0xFFFFFFFF)
    elif kind == "min":         # -2^(b-1) (signed) or 0
        if signed:
            a[:, w - 1] = np.uint32((0xFFFFFFFF << (top - 1)) & 0xFFFFFFFF)
    elif kind == "zero":
        pass
    elif kind == "onehot":
        gen = gen or rng(0)
        i = int(gen.integers(0, length))
        a[i] = random_coeffs(gen, 1, bits, signed)[0]
    elif kind == "sparse":
        gen = gen or rng(0)
        full = random_coeffs(gen, length, bits, signed)
        keep = gen.random(length) < 0.05
        a[keep] = full[keep]
    elif kind == "tiny":        # small values under a large declared b (near-tie carries)
        gen = gen or rng(0)
        vals = gen.integers(0, 4, size=length)
        a[:, 0] = vals.astype(np.uint32)
    else:
        raise ValueError(kind)
    return a


@dataclass
class Product:
    f: np.ndarray
    g: np.ndarray
    bits: int
    signed: bool


# ---- the named workloads -------------------------------------------------------------------

def product_256_u32() -> Product:
    """One product, L = 256, coefficients uniform unsigned 32-bit."""
    gen = rng(1)
    return Product(random_coeffs(gen, 256, 32, False), random_coeffs(gen, 256, 32, False), 32, False)


def product_4096_s64() -> Product:
    """One product, L = 4096, coefficients uniform signed in [-2^63, 2^63) (b = 64 with sign)."""
    gen = rng(2)
    return Product(random_coeffs(gen, 4096, 64, True), random_coeffs(gen, 4096, 64, True), 64, True)


def batch_mixed_10000(count: int = 10000, independent_lengths: bool = False, seed: int = 3) -> list:
    """Batch: L log-uniform in [16, 1024] per instance, b uniform in {16, 32, 64, 128}, signed."""
    gen = rng(seed)
    out = []
    for _ in range(count):
        lf = int(round(float(np.exp(gen.uniform(np.log(16), np.log(1024))))))
        lg = int(round(float(np.exp(gen.uniform(np.log(16), np.log(1024)))))) if independent_lengths else lf
        b = int(gen.choice([16, 32, 64, 128]))
        out.append(Product(random_coeffs(gen, lf, b, True), random_coeffs(gen, lg, b, True), b, True))
    return out


def batch_mod_modulus(seed: int = 4) -> int:
    """Odd modulus 2^59 <= p < 2^60: p = 2^59 + 2 U[0, 2^58) + 1."""
    gen = rng(seed)
    return (1 << 59) + 2 * int(gen.integers(0, 1 << 58, dtype=np.uint64)) + 1


# The paper's example timings (its Section 4, Figures 1-2): (Z/nZ)[x] with a random 4-bit and a
# random 48-bit modulus n, across degrees; n is a random number of the stated bit length (odd
# or even: the modular entry point lifts, multiplies and reduces modulo any such n).
PAPER_FIG_BITS = (4, 48)
PAPER_FIG_LENGTHS = tuple(4 ** k for k in range(1, 9))  # 4 .. 65536


def paper_fig_modulus(bits: int, seed: int = 6) -> int:
    """Random odd n with exactly `bits` bits: 2^(bits-1) + 2 U[0, 2^(bits-2)) + 1 (the
    bivariate products and the tests that need 2 invertible draw theirs here)."""
    gen = rng(seed + bits)
    return (1 << (bits - 1)) + 2 * int(gen.integers(0, 1 << (bits - 2), dtype=np.uint64)) + 1


def random_modulus(bits: int, seed: int) -> int:
    """Random n with exactly `bits` bits, odd or even: 2^(bits-1) + U[0, 2^(bits-1))."""
    gen = rng(seed + 7919 * bits)
    return (1 << (bits - 1)) + int(gen.integers(0, 1 << (bits - 1), dtype=np.uint64))


def paper_fig_pair(bits: int, length: int, seed: int = 6):
    """(n, f, g): n a random `bits`-bit modulus (see random_modulus), residues uniform in
    [0, n), f and g of the given length."""
    n = random_modulus(bits, seed)
    gen = rng(seed * 1000 + bits * 100 + length)
    return n, gen.integers(0, n, size=length, dtype=np.uint64), gen.integers(0, n, size=length, dtype=np.uint64)


def poly2_pair(ly: int, lx: int, p: int, seed: int):
    """(f, g): bivariate polynomials over Z/pZ as (ly, lx) uint64 arrays of residues uniform in
    [0, p) (row i: the coefficients of f_i(x))."""
    gen = rng(seed)
    return (gen.integers(0, p, size=(ly, lx), dtype=np.uint64), gen.integers(0, p, size=(ly, lx), dtype=np.uint64))


# Bivariate workload of the paper's polynomial case (Section 2): products in (Z/pZ)[x, y] of
# the shape of polynomials of length 4096 over an extension field of degree 16 (coefficients
# of x-degree < 16), p a random odd 60-bit modulus
POLY2_LX, POLY2_LY = 16, 4096


def poly2_workload(seed: int = 7):
    """(p, f, g) of the bivariate workload: p the first random odd 60-bit modulus (seeds
    seed, seed + 1, ...) prime to 3, so that every substitution applies (the cube roots of
    Section 2.5 divide by 6)."""
    s = seed
    while paper_fig_modulus(60, s) % 3 == 0:
        s += 1
    p = paper_fig_modulus(60, s)
    f, g = poly2_pair(POLY2_LY, POLY2_LX, p, seed)
    return p, f, g


def batch_mod_64x65536(count: int = 64, length: int = 65536, seed: int = 4):
    """Modular batch: `count` products in (Z/pZ)[x], f, g uniform in [0, p), length 65536."""
    gen = rng(seed)
    p = (1 << 59) + 2 * int(gen.integers(0, 1 << 58, dtype=np.uint64)) + 1
    pairs = []
    for _ in range(count):
        f = gen.integers(0, p, size=length, dtype=np.uint64)
        g = gen.integers(0, p, size=length, dtype=np.uint64)
        pairs.append((f, g))
    return p, pairs


def serving_requests(count: int = 10000, seed: int = 5, max_len: int = 65536, max_bits: int = 256):
    """Serving mix: L log-uniform in [8, max_len], b uniform in [8, max_bits], signed values.

    Returns (lengths, bits, seeds) per request; coefficients are drawn lazily with
    ``request_product`` so that a long stream does not hold every operand in host memory.
    """
    gen = rng(seed)
    lens = np.rint(np.exp(gen.uniform(np.log(8), np.log(max_len), size=count))).astype(np.int64)
    bits = gen.integers(8, max_bits + 1, size=count).astype(np.int64)
    seeds = gen.integers(0, 1 << 62, size=count, dtype=np.int64)
    return lens, bits, seeds


def request_product(length: int, bits: int, seed: int) -> Product:
    gen = rng(int(seed))
    return Product(random_coeffs(gen, int(length), int(bits), True),
                   random_coeffs(gen, int(length), int(bits), True), int(bits), True)


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream."""
    gen = rng(seed + 1000)
    return np.cumsum(gen.exponential(1.0 / rate_per_s, size=count))
