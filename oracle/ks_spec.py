"""Kronecker-substitution variants written out in the paper's order (test infrastructure only).

This is the executable description of *how* each variant reaches the product; the plain
definition of *what* it reaches (h = f g) is the C oracle.  Everything here is Python
integers and works in any radix R: the evaluation point is X = R^N, so the paper's decimal
worked examples (R = 10) and the binary algorithms (R = 2) run through the same lines.

Variants (paper, Section 3):
  ks1      -- evaluate at X, one product, read the coefficients off      (Section 3.1)
  recip2   -- evaluate at X and 1/X, two products, carry-aware
              reconstruction of overlapping halves                        (Section 3.2)
  neg2     -- evaluate at X and -X, two products, halve, read even and
              odd coefficients off at X^2                                 (Section 3.3)
  ks4      -- evaluate at +-X and +-1/X, four products, halve, run the
              Section 3.2 reconstruction twice at Y = X^2                 (Section 3.4)

The paper states the integer algorithms for equal lengths and non-negative coefficients.
Two readings extend them; both are exercised by the tests against the C oracle:
  * unequal lengths: each input is reversed at its own length, so the reversed product is
    the reversal of h with D = len_f + len_g - 1 coefficients; when D is even the even part
    of the reversed product is the reversal of the *odd* part of h and vice versa;
  * signed coefficients (|c| <= 2^(b-1)): the evaluations are taken of the signed values and
    a constant C = 2^(2b-2+e) >= max |h_k| is added to every coefficient slot before reading
    off or reconstructing, so every slot holds h_k + C in [0, 2C]; C is removed at the end.
"""
from __future__ import annotations

from dataclasses import dataclass, field


def evaluate(coeffs, x: int) -> int:
    """sum_i c_i x^i (Horner)."""
    acc = 0
    for c in reversed(list(coeffs)):
        acc = acc * x + int(c)
    return acc


def digits(value: int, base: int, count: int) -> list:
    """The lowest `count` base-`base` digits of a non-negative integer."""
    assert value >= 0
    out = []
    for _ in range(count):
        value, d = divmod(value, base)
        out.append(d)
    return out


def e_of(len_f: int, len_g: int) -> int:
    """e = ceil(log2 L) (Section 3), with L the smaller length (at most that many terms meet)."""
    return (min(len_f, len_g) - 1).bit_length()


def slot_bits(variant: str, b: int, e: int) -> int:
    """N per variant: 2b+e (3.1); b+ceil(e/2) (3.2, 3.3); ceil((2b+e)/4) (3.4)."""
    if variant == "ks1":
        return 2 * b + e
    if variant in ("recip2", "neg2"):
        return b + (e + 1) // 2
    if variant == "ks4":
        return (2 * b + e + 3) // 4
    raise ValueError(variant)


def offset_for(b: int, e: int, signed: bool) -> int:
    """Constant added to each slot for signed inputs (0 for the paper's non-negative case)."""
    return 1 << (2 * b - 2 + e) if signed else 0


@dataclass
class Trace:
    """Intermediate values, named as in the paper, for comparison with its examples."""
    values: dict = field(default_factory=dict)

    def __setitem__(self, k, v):
        self.values[k] = v

    def __getitem__(self, k):
        return self.values[k]


# ---- Section 3.2: reconstruction from two overlapping expansions ---------------------------

def recip_reconstruct(A: int, B: int, m: int, X: int, trace: Trace | None = None) -> list:
    """Recover h_0..h_{m-1} from A = sum h_i X^i and B = sum h_i X^(m-1-i).

    Requires 0 <= h_i < X (X - 1) (the paper's bound on beta).  Digits: A = sum_{i<=m} u_i X^i,
    B = sum_{i<=m} w_{m-i} X^i; split h_i = alpha_i + X beta_i; delta_i / eps_i are the carries
    of eqs. (carry-1) / (carry-2).  Procedure of Section 3.2, in its order.
    """
    u = digits(A, X, m + 1)
    wd = digits(B, X, m + 1)
    w = [wd[m - i] for i in range(m + 1)]  # w_i is the digit of B at position m - i
    assert A < X ** (m + 1) and B < X ** (m + 1)
    alpha = [0] * m
    beta = [0] * m
    alpha[0] = u[0]
    alpha_prev = 0  # alpha_{-1}
    delta = 0       # delta_0
    for j in range(0, m - 1):
        # eps_j from (carry-2) at i = j: beta_{j+1} + eps_{j+1} = (w_{j+1} - alpha_j) + X eps_j
        eps_j = 1 if alpha[j] > w[j + 1] else 0
        beta[j] = (w[j] - alpha_prev - eps_j) % X
        alpha[j + 1] = (u[j + 1] - beta[j] - delta) % X
        # delta_{j+1} from (carry-1): beta_j + alpha_{j+1} + delta_j = u_{j+1} + X delta_{j+1}
        t = beta[j] + alpha[j + 1] + delta - u[j + 1]
        assert t in (0, X)
        delta = t // X
        alpha_prev = alpha[j]
        if trace is not None and j == 0:
            trace["eps_0"] = eps_j
    # final top half from (carry-2) with i = m-2 and eps_{m-1} = 0
    beta[m - 1] = (w[m - 1] - (alpha[m - 2] if m >= 2 else 0)) % X
    h = [alpha[i] + X * beta[i] for i in range(m)]
    if trace is not None:
        trace["u"], trace["w"] = u, w
        trace["alpha"], trace["beta"] = alpha, beta
        # the two relations the procedure leaves unused hold as checks
        trace["check_top_alpha"] = alpha[m - 1] == w[m]
        trace["check_top_carry"] = beta[m - 1] + delta == u[m]
    return h


# ---- the variants -------------------------------------------------------------------------

def ks1(f, g, R: int, N: int, C: int = 0, trace: Trace | None = None) -> list:
    """Section 3.1: one evaluation point X = R^N; requires 0 <= h_k + C < X."""
    X = R ** N
    D = len(f) + len(g) - 1
    F, G = evaluate(f, X), evaluate(g, X)
    H = F * G
    ones = sum(X ** k for k in range(D))
    h = [d - C for d in digits(H + C * ones, X, D)]
    if trace is not None:
        trace["f(X)"], trace["g(X)"], trace["h(X)"] = F, G, H
    return h


def neg2(f, g, R: int, N: int, C: int = 0, trace: Trace | None = None) -> list:
    """Section 3.3: points X and -X; even and odd coefficients read off at X^2."""
    X = R ** N
    Y = X * X
    D = len(f) + len(g) - 1
    m0, m1 = (D + 1) // 2, D // 2
    Fp, Fm = evaluate(f, X), evaluate(f, -X)
    Gp, Gm = evaluate(g, X), evaluate(g, -X)
    Hp, Hm = Fp * Gp, Fm * Gm
    assert (Hp + Hm) % 2 == 0 and (Hp - Hm) % (2 * X) == 0
    E = (Hp + Hm) // 2          # h^(0)(X^2)
    O = (Hp - Hm) // (2 * X)    # h^(1)(X^2)
    even = [d - C for d in digits(E + C * sum(Y ** k for k in range(m0)), Y, m0)]
    odd = [d - C for d in digits(O + C * sum(Y ** k for k in range(m1)), Y, m1)] if m1 else []
    if trace is not None:
        trace["f(X)"], trace["f(-X)"], trace["g(X)"], trace["g(-X)"] = Fp, Fm, Gp, Gm
        trace["h(X)"], trace["h(-X)"] = Hp, Hm
        trace["h0(X^2)"], trace["X h1(X^2)"] = E, (Hp - Hm) // 2
        # the paper's route for f(-X) with a non-negative packing routine: f0(X^2) - X f1(X^2)
        trace["f0(X^2)"], trace["X f1(X^2)"] = evaluate(f[0::2], Y), X * evaluate(f[1::2], Y)
    h = [0] * D
    h[0::2], h[1::2] = even, odd
    return h


def recip2(f, g, R: int, N: int, C: int = 0, trace: Trace | None = None) -> list:
    """Section 3.2: points X and 1/X (the latter through the reversed inputs)."""
    X = R ** N
    D = len(f) + len(g) - 1
    ones = sum(X ** k for k in range(D))
    F, Fr = evaluate(f, X), evaluate(list(reversed(f)), X)
    G, Gr = evaluate(g, X), evaluate(list(reversed(g)), X)
    A, B = F * G, Fr * Gr
    h = [c - C for c in recip_reconstruct(A + C * ones, B + C * ones, D, X, trace)]
    if trace is not None:
        trace["f(X)"], trace["X^(L-1) f(1/X)"] = F, Fr
        trace["g(X)"], trace["X^(L-1) g(1/X)"] = G, Gr
        trace["h(X)"], trace["X^(2L-2) h(1/X)"] = A, B
    return h


def ks4(f, g, R: int, N: int, C: int = 0, trace: Trace | None = None) -> list:
    """Section 3.4: points +-X and +-1/X; Section 3.2's reconstruction twice at Y = X^2."""
    X = R ** N
    Y = X * X
    D = len(f) + len(g) - 1
    m0, m1 = (D + 1) // 2, D // 2
    fr, gr = list(reversed(f)), list(reversed(g))
    H1 = evaluate(f, X) * evaluate(g, X)
    H2 = evaluate(f, -X) * evaluate(g, -X)
    H3 = evaluate(fr, X) * evaluate(gr, X)     # X^(D-1) h(1/X)
    H4 = evaluate(fr, -X) * evaluate(gr, -X)   # reversed product at -X
    assert (H1 + H2) % 2 == 0 and (H1 - H2) % (2 * X) == 0
    assert (H3 + H4) % 2 == 0 and (H3 - H4) % (2 * X) == 0
    P0, P1 = (H1 + H2) // 2, (H1 - H2) // (2 * X)   # h^(0)(Y), h^(1)(Y)
    Q0, Q1 = (H3 + H4) // 2, (H3 - H4) // (2 * X)   # even / odd parts of the reversed product
    # reversal of h swaps parity roles when D is even
    Qe, Qo = (Q0, Q1) if D % 2 == 1 else (Q1, Q0)
    ones0 = sum(Y ** k for k in range(m0))
    ones1 = sum(Y ** k for k in range(m1))
    even = [c - C for c in recip_reconstruct(P0 + C * ones0, Qe + C * ones0, m0, Y)]
    odd = [c - C for c in recip_reconstruct(P1 + C * ones1, Qo + C * ones1, m1, Y)] if m1 else []
    if trace is not None:
        trace["f(X)"], trace["f(-X)"] = evaluate(f, X), evaluate(f, -X)
        trace["f^rev(X)"], trace["f^rev(-X)"] = evaluate(fr, X), evaluate(fr, -X)
        trace["g(X)"], trace["g(-X)"] = evaluate(g, X), evaluate(g, -X)
        trace["g^rev(X)"], trace["g^rev(-X)"] = evaluate(gr, X), evaluate(gr, -X)
        trace["H1"], trace["H2"], trace["H3"], trace["H4"] = H1, H2, H3, H4
        trace["P0"], trace["X P1"], trace["Q0"], trace["X Q1"] = P0, (H1 - H2) // 2, Q0, (H3 - H4) // 2
    h = [0] * D
    h[0::2], h[1::2] = even, odd
    return h


VARIANTS = {"ks1": ks1, "neg2": neg2, "recip2": recip2, "ks4": ks4}


def multiply(f, g, b: int, variant: str, signed: bool = False) -> list:
    """Binary (R = 2) product through one variant, with N from the paper's formula."""
    e = e_of(len(f), len(g))
    N = slot_bits(variant, b, e)
    return VARIANTS[variant](list(f), list(g), 2, N, offset_for(b, e, signed))
