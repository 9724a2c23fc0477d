"""Bivariate products over Z/pZ by Kronecker substitution (test infrastructure only).

The paper's Section 2 multiplies f, g in R[x, y] by substituting y = x^N (or -x^N, x^-N,
-x^-N) and multiplying in R[x].  Here R = Z/pZ and everything is plain Python integers.

A bivariate polynomial is a list of L_y rows, row i the L_x coefficients of f_i(x) (x^0
first), so f = sum_i f_i(x) y^i; the product h has 2 L_y - 1 rows of 2 L_x - 1 coefficients.

  mul_direct  -- h = f g written out: h_k[c] = sum_{i+j=k} sum_{a+b=c} f_i[a] g_j[b] mod p
                 (the plain definition, Section 2, first paragraph)
  coeff_direct-- one coefficient of the same sum, for sampled checks
  std         -- standard substitution y = x^N, N = 2 L_x - 1, one product, read off
                 (Section 2.1)
  recip       -- y = x^N and x^-N, N = L_x, two products, halves glued and subtracted in turn
                 (Section 2.2)
  neg         -- y = +-x^N, N = L_x, two products, even and odd parts by halving
                 (Section 2.3; needs 2 invertible, p odd)
  four        -- y = +-x^N, +-x^-N, N = ceil(L_x / 2), four products, halving, then the
                 Section 2.2 gluing on the even and the odd parts at x^(2N) (Section 2.4)
  cplx        -- y = x^M, -x^M, i x^M over R[i], M = ceil(L_x / 2): five products, the rows
                 read off by residue mod 4 (Section 2.5; p odd)
  cube        -- y = +-x^M, +-w x^M over R[w] (w a primitive cube root of unity),
                 M = ceil(L_x / 3): eight products, the rows read off by residue mod 6
                 (Section 2.5; 6 invertible)

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use this
module.  The variants follow the paper's steps in its order; the tests pin ``mul_direct`` to
identities it must satisfy (values at points, the univariate special cases, a closed form) and
check every variant against it.
"""
from __future__ import annotations

import numpy as np


def _rows(f):
    return [[int(c) for c in row] for row in f]


def pmul(a, b, p: int) -> list:
    """Product in (Z/pZ)[x] by the classical convolution (the multiplications in R[x] that
    every variant performs)."""
    if not len(a) or not len(b):
        return []
    out = np.convolve(np.array([int(v) for v in a], dtype=object), np.array([int(v) for v in b], dtype=object))
    return [int(v) % p for v in out]


def mul_direct(f, g, p: int) -> list:
    """h = f g in (Z/pZ)[x, y] from the definition."""
    f, g = _rows(f), _rows(g)
    ly, lx = len(f), len(f[0])
    hy, hx = len(f) + len(g) - 1, lx + len(g[0]) - 1
    h = [[0] * hx for _ in range(hy)]
    for i, fi in enumerate(f):
        for j, gj in enumerate(g):
            row = np.convolve(np.array(fi, dtype=object), np.array(gj, dtype=object))
            hij = h[i + j]
            for c, v in enumerate(row):
                hij[c] += int(v)
    return [[v % p for v in row] for row in h]


def coeff_direct(f, g, p: int, k: int, c: int) -> int:
    """Coefficient of x^c y^k of f g (mod p)."""
    ly_f, ly_g = len(f), len(g)
    lx_f, lx_g = len(f[0]), len(g[0])
    s = 0
    for i in range(max(0, k - ly_g + 1), min(k, ly_f - 1) + 1):
        fi, gj = f[i], g[k - i]
        for a in range(max(0, c - lx_g + 1), min(c, lx_f - 1) + 1):
            s += int(fi[a]) * int(gj[c - a])
    return s % p


def evaluate(f, x: int, y: int, p: int) -> int:
    """f(x, y) mod p."""
    acc = 0
    for row in reversed(_rows(f)):
        r = 0
        for c in reversed(row):
            r = (r * x + c) % p
        acc = (acc * y + r) % p
    return acc


# ---- the substitutions ------------------------------------------------------------------------

def substitute(f, n: int, sign: int, reverse: bool, p: int) -> list:
    """x^(N (L_y - 1)) f(x, sign x^-N) if reverse, else f(x, sign x^N), as a list of
    coefficients mod p: sum_i s^i f_i(x) x^(i N) with f_i taken in reversed order for the
    reciprocal points.  Rows overlap when N < L_x (Section 2.4), so positions add up."""
    f = _rows(f)
    ly, lx = len(f), len(f[0])
    out = [0] * (n * (ly - 1) + lx)
    for i in range(ly):
        row = f[ly - 1 - i] if reverse else f[i]
        s = sign ** i
        for c, v in enumerate(row):
            out[i * n + c] += s * v
    return [v % p for v in out]


def std(f, g, p: int) -> list:
    """Section 2.1: N = 2 L_x - 1, one product, h_i read off at x^(i N)."""
    ly, lx = len(f), len(f[0])
    n = 2 * lx - 1
    F, G = substitute(f, n, 1, False, p), substitute(g, n, 1, False, p)
    assert len(F) == 2 * lx * ly - lx - ly + 1  # the proposition's length
    H = pmul(F, G, p)
    H += [0] * ((2 * ly - 1) * n - len(H))
    return [H[i * n:i * n + 2 * lx - 1] for i in range(2 * ly - 1)]


def glue(plus, minus, count: int, m: int, width: int, p: int) -> list:
    """The gluing of Section 2.2 at block M: plus = sum_i u_i x^(i M) and
    minus = sum_i u_(count-1-i) x^(i M), each u_i of length <= 2 M - 1.  The lowest M terms of
    plus are those of u_0 and the highest M - 1 terms of minus are those of u_0; u_0 is then
    subtracted from both, which uncovers u_1, and so on.  Returns u_0 .. u_(count-1), each cut
    to `width` coefficients (the part above must vanish)."""
    size = (count + 1) * m
    A = list(plus) + [0] * max(0, size - len(plus))
    B = list(minus) + [0] * max(0, size - len(minus))
    out = []
    for i in range(count):
        low = A[i * m:i * m + m]
        top = (count - i) * m  # where u_i's upper half lies in minus
        high = B[top:top + m - 1]
        u = [v % p for v in low + high]
        for t, v in enumerate(u):
            A[i * m + t] -= v
            B[(count - 1 - i) * m + t] -= v
        assert all(v == 0 for v in u[width:]), "coefficients beyond the product's length"
        out.append(u[:width])
    return out


def recip(f, g, p: int) -> list:
    """Section 2.2: N = L_x, products at x^N and (normalised) x^-N of length L_x L_y."""
    ly, lx = len(f), len(f[0])
    n = lx
    Fp, Gp = substitute(f, n, 1, False, p), substitute(g, n, 1, False, p)
    Fm, Gm = substitute(f, n, 1, True, p), substitute(g, n, 1, True, p)
    assert len(Fp) == len(Fm) == lx * ly
    return glue(pmul(Fp, Gp, p), pmul(Fm, Gm, p), 2 * ly - 1, n, 2 * lx - 1, p)


def _half(v: int, p: int) -> int:
    return v * pow(2, -1, p) % p


def neg(f, g, p: int) -> list:
    """Section 2.3: N = L_x, products at +-x^N; h^(0)(x, x^(2N)) = (H+ + H-) / 2 and
    h^(1)(x, x^(2N)) = (H+ - H-) / (2 x^N); h_(2i) and h_(2i+1) read off at x^(2 i N)."""
    ly, lx = len(f), len(f[0])
    n = lx
    Hp = pmul(substitute(f, n, 1, False, p), substitute(g, n, 1, False, p), p)
    Hm = pmul(substitute(f, n, -1, False, p), substitute(g, n, -1, False, p), p)
    even = [_half(a + b, p) for a, b in zip(Hp, Hm)]
    odd = [_half(a - b, p) for a, b in zip(Hp, Hm)][n:]
    even += [0] * (2 * n * ly)
    odd += [0] * (2 * n * ly)
    h = []
    for k in range(2 * ly - 1):
        src = even if k % 2 == 0 else odd
        h.append(src[(k // 2) * 2 * n:(k // 2) * 2 * n + 2 * lx - 1])
    return h


def four(f, g, p: int) -> list:
    """Section 2.4: N = ceil(L_x / 2), products at +-x^N and (normalised) +-x^-N of length
    N (L_y - 1) + L_x; the even and odd parts at x^(2N) and x^(-2N) by halving, then the
    gluing of Section 2.2 at block 2N (L_y even-index rows, L_y - 1 odd-index rows)."""
    ly, lx = len(f), len(f[0])
    n = (lx + 1) // 2
    H = [pmul(substitute(f, n, s, r, p), substitute(g, n, s, r, p), p) for r in (False, True) for s in (1, -1)]
    assert all(len(substitute(f, n, 1, r, p)) == n * (ly - 1) + lx for r in (False, True))
    ep = [_half(a + b, p) for a, b in zip(H[0], H[1])]
    op = [_half(a - b, p) for a, b in zip(H[0], H[1])][n:]
    em = [_half(a + b, p) for a, b in zip(H[2], H[3])]
    om = [_half(a - b, p) for a, b in zip(H[2], H[3])][n:]
    evens = glue(ep, em, ly, 2 * n, 2 * lx - 1, p)
    odds = glue(op, om, ly - 1, 2 * n, 2 * lx - 1, p) if ly > 1 else []
    h = []
    for k in range(2 * ly - 1):
        h.append(evens[k // 2] if k % 2 == 0 else odds[k // 2])
    return h


# ---- Section 2.5: evaluation points in an extension of R -----------------------------------------
# Elements of S = R[i] (i^2 = -1) or S = R[w] (w^2 + w + 1 = 0) are pairs (a, b) = a + b i or
# a + b w; a polynomial over S is the pair of its two coefficient lists in R[x].

def _cmul(u, v, p):
    """(a + b i)(c + d i) in R[i]."""
    a, b = u
    c, d = v
    return ((a * c - b * d) % p, (a * d + b * c) % p)


def _wmul(u, v, p):
    """(a + b w)(c + d w) in R[w], w^2 = -1 - w."""
    a, b = u
    c, d = v
    return ((a * c - b * d) % p, (a * d + b * c - b * d) % p)


def substitute_ext(f, m: int, z, mul, p: int):
    """f(x, z x^M) for z in S: sum_i f_i(x) z^i x^(i M), as the pair (real part, other part)
    of polynomials in R[x] of length M (L_y - 1) + L_x."""
    f = _rows(f)
    ly, lx = len(f), len(f[0])
    re, im = [0] * (m * (ly - 1) + lx), [0] * (m * (ly - 1) + lx)
    zi = (1, 0)
    for i in range(ly):
        for c, v in enumerate(f[i]):
            re[i * m + c] += zi[0] * v
            im[i * m + c] += zi[1] * v
        zi = mul(zi, z, p)
    return [v % p for v in re], [v % p for v in im]


def _addp(a, b, p):
    return [(x + y) % p for x, y in zip(a, b)]


def _subp(a, b, p):
    return [(x - y) % p for x, y in zip(a, b)]


def cplx(f, g, p: int) -> list:
    """Section 2.5, complex points: M = ceil(L_x / 2), S = R[i]; h evaluated at y = x^M, -x^M
    (products in R[x]) and i x^M (a product in S[x], three products in R[x]: ac, bd and
    (a + b)(c + d)).  The value at -i x^M is the conjugate of the one at i x^M, so the four
    values are h at the fourth roots of unity times x^M; their inverse transform of length 4
    gives A_r = sum over rows j = r (mod 4) of h_j x^(j M), whose terms do not overlap (4 M >=
    2 L_x), and h_j is read off A_(j mod 4) at x^(j M).  Five products in R[x]; needs 2
    invertible (p odd)."""
    ly, lx = len(f), len(f[0])
    m = (lx + 1) // 2
    one, mone, ii = (1, 0), (p - 1, 0), (0, 1)
    Fp, _ = substitute_ext(f, m, one, _cmul, p)
    Gp, _ = substitute_ext(g, m, one, _cmul, p)
    Fm, _ = substitute_ext(f, m, mone, _cmul, p)
    Gm, _ = substitute_ext(g, m, mone, _cmul, p)
    Fa, Fb = substitute_ext(f, m, ii, _cmul, p)
    Ga, Gb = substitute_ext(g, m, ii, _cmul, p)
    H1 = pmul(Fp, Gp, p)
    H2 = pmul(Fm, Gm, p)
    ac, bd = pmul(Fa, Ga, p), pmul(Fb, Gb, p)
    ad_bc = _subp(_subp(pmul(_addp(Fa, Fb, p), _addp(Ga, Gb, p), p), ac, p), bd, p)
    re, im = _subp(ac, bd, p), ad_bc  # h(x, i x^M) = re + i im
    q = pow(4, -1, p)
    A = [[(h1 + h2 + 2 * r) * q % p for h1, h2, r in zip(H1, H2, re)],
         [(h1 - h2 + 2 * t) * q % p for h1, h2, t in zip(H1, H2, im)],
         [(h1 + h2 - 2 * r) * q % p for h1, h2, r in zip(H1, H2, re)],
         [(h1 - h2 - 2 * t) * q % p for h1, h2, t in zip(H1, H2, im)]]
    for a in A:
        a += [0] * ((2 * ly) * m + 2 * lx)
    return [A[j % 4][j * m:j * m + 2 * lx - 1] for j in range(2 * ly - 1)]


def cube(f, g, p: int) -> list:
    """Section 2.5, cube roots of unity: M = ceil(L_x / 3), S = R[w] with w^2 + w + 1 = 0; h
    evaluated at y = x^M, -x^M (products in R[x]) and w x^M, -w x^M (products in S[x], three
    products in R[x] each).  With z = 1 + w, a primitive sixth root of unity (z^2 = w,
    z^3 = -1), these are h at z^0, z^3, z^2, z^5 times x^M; the conjugation w -> w^2 of S gives
    the values at z^4 and z^1.  The inverse transform of length 6 gives A_r = sum over rows
    j = r (mod 6) of h_j x^(j M) (non-overlapping: 6 M >= 2 L_x), whose second component
    vanishes, and h_j is read off A_(j mod 6) at x^(j M).  Eight products in R[x], each about a
    sixth of the standard substitution's; needs 6 invertible."""
    ly, lx = len(f), len(f[0])
    m = (lx + 2) // 3
    w, mw = (0, 1), (0, p - 1)

    def val(z):  # h(x, z x^M) as a pair of polynomials, through three products in R[x]
        Fa, Fb = substitute_ext(f, m, z, _wmul, p)
        Ga, Gb = substitute_ext(g, m, z, _wmul, p)
        ac, bd = pmul(Fa, Ga, p), pmul(Fb, Gb, p)
        s = pmul(_addp(Fa, Fb, p), _addp(Ga, Gb, p), p)
        # (a + b w)(c + d w) = (ac - bd) + (ad + bc - bd) w, ad + bc = s - ac - bd
        return _subp(ac, bd, p), [(x - y - 2 * z2) % p for x, y, z2 in zip(s, ac, bd)]

    Fp, _ = substitute_ext(f, m, (1, 0), _wmul, p)
    Gp, _ = substitute_ext(g, m, (1, 0), _wmul, p)
    Fm, _ = substitute_ext(f, m, (p - 1, 0), _wmul, p)
    Gm, _ = substitute_ext(g, m, (p - 1, 0), _wmul, p)
    n = 2 * (m * (ly - 1) + lx) - 1
    V = [None] * 6
    V[0] = (pmul(Fp, Gp, p), [0] * n)
    V[3] = (pmul(Fm, Gm, p), [0] * n)
    V[2] = val(w)
    V[5] = val(mw)

    def conj(u):  # a + b w -> a + b w^2 = (a - b) - b w
        return ([(a - b) % p for a, b in zip(*u)], [(-b) % p for b in u[1]])

    V[4], V[1] = conj(V[2]), conj(V[5])
    z = (1, 1)  # 1 + w
    zinv = (0, p - 1)  # z^5 = -w
    zp = [(1, 0)]
    for _ in range(5):
        zp.append(_wmul(zp[-1], zinv, p))  # z^(-k)
    six = pow(6, -1, p)
    A = []
    for r in range(6):
        acc_a, acc_b = [0] * n, [0] * n
        for k in range(6):
            c = zp[(r * k) % 6]
            for t in range(n):
                e = _wmul(c, (V[k][0][t], V[k][1][t]), p)
                acc_a[t] += e[0]
                acc_b[t] += e[1]
        assert all(v % p == 0 for v in acc_b), "the inverse transform left a second component"
        A.append([v * six % p for v in acc_a] + [0] * ((2 * ly) * m + 2 * lx))
    assert _wmul(z, zinv, p) == (1, 0)
    return [A[j % 6][j * m:j * m + 2 * lx - 1] for j in range(2 * ly - 1)]


VARIANTS = {"ks1": std, "recip2": recip, "neg2": neg, "ks4": four, "cplx": cplx, "cube": cube}


def random_poly2(rng: np.random.Generator, ly: int, lx: int, p: int) -> list:
    """Residues uniform in [0, p), as Python integers."""
    return [[int(v) for v in rng.integers(0, p, size=lx, dtype=np.uint64)] for _ in range(ly)]
