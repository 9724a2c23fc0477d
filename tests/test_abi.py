"""Host-side checks of the C-ABI library (no GPU work): it loads, exports every symbol that
include/ks.h declares, and its planner follows the paper's formulas for N and operand sizes.
"""
import ctypes
import os
import re

import pytest

from paper_0712_4046_amd import ks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ks.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ks_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ks.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_messages():
    assert ks.lib().ks_version() >= 100
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert ks.strerror(code) and ks.strerror(code) != "unknown status code"


@pytest.mark.parametrize("lf,lg,b", [(1, 1, 1), (256, 256, 32), (4096, 4096, 64), (17, 1000, 60), (65536, 65536, 60),
                                     (8, 9, 256)])
def test_out_limbs_follow_the_bound(lf, lg, b):
    # coefficients of h have length <= 2b + e (Section 3), plus one sign bit
    e = (min(lf, lg) - 1).bit_length()
    assert ks.out_limbs(lf, lg, b) == (2 * b + e + 1 + 31) // 32


def test_invalid_sizes_rejected():
    L = ks.lib()
    assert L.ks_out_limbs(0, 5, 32) == ks.KS_EINVAL
    assert L.ks_out_limbs(5, 5, 0) == ks.KS_EINVAL
    assert L.ks_out_limbs(5, 5, ks.KS_MAX_BITS + 1) == ks.KS_EINVAL
    for bad in [(0, 4, 8, "ks1"), (4, 4, 0, "ks4"), (4, 4, 300, "neg2")]:
        with pytest.raises(ks.KSError) as ei:
            ks.plan(bad[0], bad[1], bad[2], bad[3])
        assert ei.value.code == ks.KS_EINVAL
    info = ks.PlanInfo()
    assert L.ks_plan(4, 4, 8, 5, info) == ks.KS_EINVAL       # not a variant
    assert L.ks_plan(4, 4, 8, 0x3000 | 1, info) == ks.KS_EINVAL  # both engines


@pytest.mark.parametrize("lf,lg,b,signed", [(256, 256, 32, False), (4096, 4096, 64, True), (1, 1, 7, False),
                                            (100, 3, 128, True), (65536, 65536, 60, False), (1000, 999, 16, True)])
def test_planner_slot_widths_and_operand_lengths(lf, lg, b, signed):
    e = (min(lf, lg) - 1).bit_length()
    for variant, N, k in (("ks1", 2 * b + e, 1), ("neg2", b + (e + 1) // 2, 2), ("recip2", b + (e + 1) // 2, 2),
                          ("ks4", (2 * b + e + 3) // 4, 4)):
        p = ks.plan(lf, lg, b, variant, signed)
        assert p["slot_bits"] == N and p["n_products"] == k and p["e"] == e
        # operand length N (L-1) + b of the propositions, plus one carry bit and one sign bit
        assert p["operand_limbs_f"] == (N * (lf - 1) + b + 2 + 31) // 32
        assert p["operand_limbs_g"] == (N * (lg - 1) + b + 2 + 31) // 32
        assert p["schoolbook_limb_mults"] == k * p["operand_limbs_f"] * p["operand_limbs_g"]


def test_product_4096_s64_slot_width():
    # L = 4096, b = 64 (sign included): KS1 N = 2b + e = 140, KS4 N = 35
    assert ks.plan(4096, 4096, 64, "ks1", True)["slot_bits"] == 140
    assert ks.plan(4096, 4096, 64, "ks4", True)["slot_bits"] == 35


def test_tunables_round_trip_and_reach_the_planner():
    L = ks.lib()
    ks.tune_reset()
    try:
        assert ks.tune_get("KS_MFMA_MIN_LIMBS") == 2500
        assert L.ks_tune_set(b"NO_SUCH_TUNABLE", 3) == ks.KS_EINVAL
        assert L.ks_tune_set(b"KS_CHAIN_K", -1) == ks.KS_EINVAL
        # engine threshold: a 2,241-limb product moves to the matrix cores when it is lowered
        assert ks.plan(2048, 2048, 64, "ks4", True)["engine"] == ks.KS_ENGINE_VALU
        ks.tune_set("KS_MFMA_MIN_LIMBS", 1)
        assert ks.tune_get("KS_MFMA_MIN_LIMBS") == 1
        assert ks.plan(2048, 2048, 64, "ks4", True)["engine"] == ks.KS_ENGINE_MFMA
        # segment length: longer segments, fewer anchors
        ks.tune_set("KS_CHAIN_K", 4)
        a4 = ks.plan(4096, 4096, 64, "ks4", True)["anchor_limb_mults"]
        ks.tune_set("KS_CHAIN_K", 64)
        a64 = ks.plan(4096, 4096, 64, "ks4", True)["anchor_limb_mults"]
        assert a4 > 10 * a64 > 0
    finally:
        ks.tune_reset()
    assert ks.tune_get("KS_MFMA_MIN_LIMBS") == 2500


def test_poly2_arguments_checked_on_the_host():
    # ks_mul_poly2 rejects bad arguments before touching the device (null buffers, lengths
    # below 1, an even or too large modulus, an unknown substitution, signed inner products)
    L = ks.lib()
    P = ctypes.c_void_p
    buf = P(256)  # never dereferenced: every call below fails validation first
    ok = dict(f=buf, g=buf, lx=4, ly=3, p=(1 << 61) - 1, v=ks.KS_VARIANT["ks4"], inner=0)

    def call(**kw):
        a = dict(ok, **kw)
        return L.ks_mul_poly2(a["f"], a["g"], a["lx"], a["ly"], a["p"], a["v"], a["inner"], None, a.get("h", buf))

    assert call(f=P(0)) == ks.KS_EINVAL
    assert call(h=P(0)) == ks.KS_EINVAL
    assert call(lx=0) == ks.KS_EINVAL
    assert call(ly=0) == ks.KS_EINVAL
    assert call(p=1 << 40) == ks.KS_EINVAL
    assert call(p=1 << 62 | 1) == ks.KS_EINVAL
    assert call(p=1) == ks.KS_EINVAL
    assert call(v=0x55) == ks.KS_EINVAL
    assert call(inner=ks.KS_SIGNED) == ks.KS_EINVAL
    assert call(v=ks.P2_VARIANT["cube"], p=3 * 1_000_003) == ks.KS_EINVAL  # the cube roots divide by 6
    assert call(v=7) == ks.KS_EINVAL


def test_tuning_cache_file_read_at_plan_time(tmp_path):
    # the autotuner's JSON cache (KS_TUNING_FILE) sets tunables in a fresh process, below
    # ks_tune_set and the environment; unknown keys are ignored
    import json
    import subprocess
    import sys
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"tunables": {"KS_CHAIN_K": 77, "KS_NTT_MIN_LIMBS": 5000, "NOT_A_TUNABLE": 3},
                                "workload": "x"}))
    code = ("from paper_0712_4046_amd import ks; "
            "print(ks.tune_get('KS_CHAIN_K'), ks.tune_get('KS_NTT_MIN_LIMBS'), ks.tune_get('KS_MFMA_RT')); "
            "ks.tune_set('KS_CHAIN_K', 9); print(ks.tune_get('KS_CHAIN_K'))")
    env = dict(os.environ, KS_TUNING_FILE=str(path))
    env.pop("KS_CHAIN_K", None)
    env.pop("KS_NTT_MIN_LIMBS", None)
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, check=True)
    assert out.stdout.split() == ["77", "5000", "0", "9"]
    env["KS_CHAIN_K"] = "12"  # the environment wins over the file
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, check=True)
    assert out.stdout.split()[0] == "12"


@pytest.mark.parametrize("L,bits,variant", [(65536, 60, "ks4"), (65536, 256, "ks1"), (32768, 64, "neg2")])
def test_planner_takes_the_transforms_for_long_operands(L, bits, variant):
    # long operands go to the transform engine; its exactness condition fixes the piece width
    p = ks.plan(L, L, bits, variant, True)
    assert p["engine"] == ks.KS_ENGINE_NTT
    assert p["ntt_butterflies"] > 0 and p["mfma_ops"] == 0
    forced = ks.plan(L, L, bits, variant, True, engine="mfma")
    assert forced["engine"] == ks.KS_ENGINE_MFMA and forced["ntt_butterflies"] == 0
