"""Pins of the bivariate oracle (oracle/poly2.py) against facts other than itself, and its
paper-ordered variants (Section 2) against the definition.  CPU only."""
import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle import poly2

PRIMES = [3, 5, 97, 2**31 - 1, 2**61 - 1]
ODD = PRIMES + [(1 << 59) + 2 * 123456789 + 1, 15, (1 << 62) - 1]


def rnd(seed, ly, lx, p):
    return poly2.random_poly2(np.random.default_rng(seed), ly, lx, p)


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("ly,lx", [(1, 1), (2, 3), (4, 1), (3, 5), (6, 4)])
def test_direct_values_at_points(p, ly, lx):
    # h(a, b) = f(a, b) g(a, b) in Z/pZ at random points: a dropped term, a wrong index or a
    # transposed operand in the definition changes some value
    f, g = rnd(1, ly, lx, p), rnd(2, ly, lx, p)
    h = poly2.mul_direct(f, g, p)
    assert len(h) == 2 * ly - 1 and all(len(r) == 2 * lx - 1 for r in h)
    rng = np.random.default_rng(3)
    for _ in range(6):
        a, b = (int(v) for v in rng.integers(0, p, size=2, dtype=np.uint64))
        assert poly2.evaluate(h, a, b, p) == poly2.evaluate(f, a, b, p) * poly2.evaluate(g, a, b, p) % p


def test_direct_reduces_to_univariate_products():
    # L_y = 1 is a product in (Z/pZ)[x]; L_x = 1 one in (Z/pZ)[y] (numpy's polymul on integers)
    p = 2**61 - 1
    f, g = rnd(4, 1, 9, p), rnd(5, 1, 7, p)
    h = poly2.mul_direct(f, g, p)
    want = P.polymul(np.array(f[0], dtype=object), np.array(g[0], dtype=object))
    assert h[0] == [int(v) % p for v in want]
    f, g = rnd(6, 8, 1, p), rnd(7, 8, 1, p)
    h = poly2.mul_direct(f, g, p)
    want = P.polymul(np.array([r[0] for r in f], dtype=object), np.array([r[0] for r in g], dtype=object))
    assert [r[0] for r in h] == [int(v) % p for v in want]


@pytest.mark.parametrize("ly,lx", [(1, 1), (3, 4), (5, 2)])
def test_direct_all_ones_closed_form(ly, lx):
    # f = g = sum x^a y^i: h_k[c] = T(k; L_y) T(c; L_x), T(t; L) = min(t, 2L - 2 - t) + 1
    p = 1_000_003
    ones = [[1] * lx for _ in range(ly)]
    h = poly2.mul_direct(ones, ones, p)
    T = lambda t, L: min(t, 2 * L - 2 - t) + 1  # noqa: E731
    assert h == [[T(k, ly) * T(c, lx) for c in range(2 * lx - 1)] for k in range(2 * ly - 1)]


def test_coeff_direct_matches():
    p = 2**31 - 1
    f, g = rnd(8, 5, 6, p), rnd(9, 5, 6, p)
    h = poly2.mul_direct(f, g, p)
    for k in range(9):
        for c in range(11):
            assert poly2.coeff_direct(f, g, p, k, c) == h[k][c]


@pytest.mark.parametrize("variant", sorted(poly2.VARIANTS))
@pytest.mark.parametrize("p", ODD)
@pytest.mark.parametrize("ly,lx", [(1, 1), (1, 4), (4, 1), (2, 2), (2, 3), (3, 5), (5, 8), (7, 7), (8, 3)])
def test_variants_equal_definition(variant, p, ly, lx):
    if variant == "cube" and p % 3 == 0:
        pytest.skip("the cube-root points divide by 6 (Section 2.5): 3 must be invertible")
    f, g = rnd(10 + ly, ly, lx, p), rnd(20 + lx, ly, lx, p)
    assert poly2.VARIANTS[variant](f, g, p) == poly2.mul_direct(f, g, p)


def test_variants_at_extreme_residues():
    p = 2**61 - 1
    for fill in (0, 1, p - 1):
        f = [[fill] * 6 for _ in range(5)]
        for name, fn in poly2.VARIANTS.items():
            assert fn(f, f, p) == poly2.mul_direct(f, f, p), (name, fill)


def test_planted_mistakes_are_caught(monkeypatch):
    # a variant with a step changed must disagree with the definition somewhere
    p = 2**61 - 1
    f, g = rnd(30, 4, 5, p), rnd(31, 4, 5, p)
    want = poly2.mul_direct(f, g, p)
    with monkeypatch.context() as m:  # halving dropped (Sections 2.3, 2.4)
        m.setattr(poly2, "_half", lambda v, q: v % q)
        assert poly2.neg(f, g, p) != want
        assert poly2.four(f, g, p) != want
    real = poly2.substitute
    with monkeypatch.context() as m:  # the reciprocal points not reversed (Section 2.2)
        m.setattr(poly2, "substitute", lambda ff, n, s, r, q: real(ff, n, s, False, q))
        with pytest.raises(AssertionError):
            assert poly2.recip(f, g, p) == want
    with monkeypatch.context() as m:  # no alternating sign at -x^N (Section 2.3)
        m.setattr(poly2, "substitute", lambda ff, n, s, r, q: real(ff, n, 1, r, q))
        assert poly2.neg(f, g, p) != want


def test_extension_points_planted_mistakes(monkeypatch):
    # Section 2.5: a wrong product in the extension ring or a wrong conjugation must break the
    # reconstruction (the cube-root variant also checks that the second components vanish)
    p = 2**61 - 1
    f, g = rnd(40, 5, 7, p), rnd(41, 5, 7, p)
    want = poly2.mul_direct(f, g, p)
    assert poly2.cplx(f, g, p) == want and poly2.cube(f, g, p) == want
    with monkeypatch.context() as m:  # i^2 = +1 instead of -1
        m.setattr(poly2, "_cmul", lambda u, v, q: ((u[0] * v[0] + u[1] * v[1]) % q, (u[0] * v[1] + u[1] * v[0]) % q))
        assert poly2.cplx(f, g, p) != want
    with monkeypatch.context() as m:  # w^2 = -1 (the complex rule) instead of -1 - w
        m.setattr(poly2, "_wmul", lambda u, v, q: ((u[0] * v[0] - u[1] * v[1]) % q, (u[0] * v[1] + u[1] * v[0]) % q))
        with pytest.raises(AssertionError):
            assert poly2.cube(f, g, p) == want


def test_extension_points_fewer_longer_products():
    # the sizes Section 2.5 states: complex points multiply polynomials of length
    # ceil(L_x / 2)(L_y - 1) + L_x (five of them); cube roots of length ceil(L_x / 3)(L_y - 1)
    # + L_x (eight), a sixth of the standard substitution's length for large L_x
    p = 97
    ly, lx = 6, 30
    f = rnd(42, ly, lx, p)
    a, _ = poly2.substitute_ext(f, (lx + 1) // 2, (0, 1), poly2._cmul, p)
    b, _ = poly2.substitute_ext(f, (lx + 2) // 3, (0, 1), poly2._wmul, p)
    std_len = len(poly2.substitute(f, 2 * lx - 1, 1, False, p))
    assert len(a) == 15 * (ly - 1) + lx and len(b) == 10 * (ly - 1) + lx
    assert std_len == (2 * lx - 1) * (ly - 1) + lx
