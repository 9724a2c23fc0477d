"""The autotuner changes launch shapes only: a tuned batch run is bit-identical to the default
run (and to the oracle on a sample)."""
import numpy as np
import pytest

from paper_0712_4046_amd import autotune, ks

pytestmark = pytest.mark.gpu


def test_tuned_batch_equals_default(oracle):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.tune_reset()
    make = autotune.workload("small", "ks4")
    make()()
    torch.cuda.synchronize()
    ain, aout = make.arenas
    plan, ws = make.state["plan"], make.state["ws"]
    assert plan.status(ws) == ks.KS_OK
    default = aout.clone()
    cands = {"KS_CHAIN_K": [4, 64], "KS_MFMA_MIN_LIMBS": [1, 6000]}
    try:
        res = autotune.tune(make, candidates=cands, max_passes=1, warmup=1, reps=2)
        assert set(res["tunables"]) == set(cands) and res["ms"] > 0
        # every candidate shape gives the same bits
        for k, v in (("KS_CHAIN_K", 4), ("KS_MFMA_MIN_LIMBS", 1)):
            ks.tune_reset()
            ks.tune_set(k, v)
            aout.fill_(-1)
            make()()
            torch.cuda.synchronize()
            assert make.state["plan"].status(make.state["ws"]) == ks.KS_OK
            assert torch.equal(aout, default), (k, v)
    finally:
        ks.tune_reset()
        make.state["plan"].close()
    out = ks.to_host(default)
    from paper_0712_4046_amd import workloads as wl
    prods = wl.batch_mixed_10000(count=300, seed=36)
    for i in (0, 1, 150, 299):
        P = prods[i]
        exp = oracle.mul_classical(P.f, P.g, P.signed, oracle.out_limbs(P.f.shape[0], P.g.shape[0], P.bits))
        assert np.array_equal(make.batch.result(out, i), exp), i
