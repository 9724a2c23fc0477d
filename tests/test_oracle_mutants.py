"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each one.

Each mutant is built from a textual edit of oracle/oracle.c into a temporary library; the
committed oracle is never changed.  A mutant that survives every pin would mean the pins do
not constrain that part of the oracle.
"""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as pins

MUTANTS = {
    "classical drops the last term": ("for (int64_t i = lo; i <= hi; i++) {\n        int64_t j = k - i;",
                                      "for (int64_t i = lo; i < hi; i++) {\n        int64_t j = k - i;"),
    "classical sign of a product": ("if (fs[i] ^ gs[j])", "if (fs[i] | gs[j])"),
    "classical window upper index": ("memset(acc, 0, sizeof(uint32_t) * (size_t)w_out);\n    int64_t lo = k - (lg - 1) > 0 ? k - (lg - 1) : 0;\n    int64_t hi = k < lf - 1 ? k : lf - 1;",
                                     "memset(acc, 0, sizeof(uint32_t) * (size_t)w_out);\n    int64_t lo = k - (lg - 1) > 0 ? k - (lg - 1) : 0;\n    int64_t hi = k < lf - 1 ? k : lf - 2;"),
    "carry dropped in addition": ("        acc[i] = (uint32_t)s;\n        c = s >> 32;", "        acc[i] = (uint32_t)s;\n        c = 0;"),
    "ks1 slot one bit too narrow": ("int64_t N = 2 * (int64_t)b + e;", "int64_t N = 2 * (int64_t)b + e - 1;"),
    "ks1 balanced carry lost": ("if (carry) mp_add(v, wv, one, 1);", "if (0) mp_add(v, wv, one, 1);"),
    "ks1 second operand transposed": ("add_shifted(G, nG, mag, w_in, s, N * i);", "add_shifted(G, nG, mag, w_in, s, N * (lg - 1 - i));"),
    "mod reduction skipped": ("if (++cnt == 2) { acc %= p; cnt = 0; }", "if (++cnt == 2) { cnt = 0; }"),
}


def _battery(oracle):
    """A quick pass over the pins; returns the list of pins that failed."""
    failed = []
    checks = [
        ("example", lambda: pins.test_example_product_classical_and_ks1(oracle)),
        ("all-max", lambda: [pins.test_all_max_unsigned_bound_is_tight(oracle, b, lf, lg)
                             for b in (32, 64) for lf, lg in ((16, 16), (37, 20))]),
        ("signed extremes", lambda: [pins.test_signed_extremes(oracle, b, 9, 30) for b in (16, 64)]),
        ("binomials", lambda: pins.test_binomials(oracle, 30, 33)),
        ("monomials", lambda: pins.test_monomials(oracle)),
        ("geometric", lambda: pins.test_geometric_row(oracle)),
        ("invariants", lambda: pins.test_invariants_random(oracle, 300, 301, 64, True)),
        ("invariants unequal", lambda: pins.test_invariants_random(oracle, 64, 17, 128, True)),
        ("mod", lambda: pins.test_mod_p(oracle)),
    ]
    for name, fn in checks:
        try:
            fn()
        except Exception:
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(O.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mutant.c")
        so = os.path.join(d, "libmutant.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", c, "-o", so], check=True)
        try:
            O.use_library(so)
            failed = _battery(O)
        finally:
            O.use_library(None)
    assert failed, f"mutant '{name}' survived every pin"


def test_unmutated_oracle_passes_battery():
    O.use_library(None)
    assert _battery(O) == []
