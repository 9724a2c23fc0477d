"""GPU test of ks_mul_noalloc (the entry point that allocates nothing): through the C ABI its
results equal ks_mul's, bit for bit, on two calls in a row (the second smaller, so the array
holds the first call's data), on every variant; a range error is reported through
ks_stream_status; a product beyond the fixed array is refused on the host."""
import ctypes

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


def noalloc(torch, f, g, bits, variant, signed):
    tf, tg = ks.to_device(f), ks.to_device(g)
    lf, lg = f.shape[0], g.shape[0]
    h = torch.full((lf + lg - 1, ks.out_limbs(lf, lg, bits)), -1, dtype=torch.int32, device="cuda")
    flags = ks.KS_VARIANT[variant] | (ks.KS_SIGNED if signed else 0)
    rc = ks.lib().ks_mul_noalloc(ctypes.c_void_p(tf.data_ptr()), ctypes.c_void_p(tg.data_ptr()), lf, lg, bits,
                                 flags, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 ctypes.c_void_p(h.data_ptr()))
    assert rc == ks.KS_OK, ks.strerror(rc)
    assert ks.status() == ks.KS_OK
    return ks.to_host(h)


def pooled(f, g, bits, variant, signed):
    h = ks.mul(ks.to_device(f), ks.to_device(g), bits, variant, signed)
    assert ks.status() == ks.KS_OK
    return ks.to_host(h)


@pytest.mark.parametrize("variant", ["ks1", "neg2", "recip2", "ks4", "auto"])
def test_noalloc_equals_ks_mul_twice(torch_dev, variant):
    # a large signed product (matrix cores, anchored reconstruction), then a smaller unsigned one
    # of unequal lengths that reuses the array the first one filled
    gen = wl.rng(7000)
    big = (wl.random_coeffs(gen, 4096, 64, True), wl.random_coeffs(gen, 4096, 64, True), 64, True)
    small = (wl.random_coeffs(gen, 300, 33, False), wl.random_coeffs(gen, 171, 33, False), 33, False)
    for f, g, bits, signed in (big, small):
        assert np.array_equal(noalloc(torch_dev, f, g, bits, variant, signed), pooled(f, g, bits, variant, signed)), \
            (variant, f.shape[0], bits)


def test_noalloc_range_error_reported(torch_dev):
    good = np.array([[1], [2], [3]], dtype=np.uint32)
    bad = np.array([[1], [999], [3]], dtype=np.uint32)  # 999 does not fit in 8 bits
    torch = torch_dev
    tf, tg = ks.to_device(bad), ks.to_device(good)
    h = torch.zeros((5, ks.out_limbs(3, 3, 8)), dtype=torch.int32, device="cuda")
    rc = ks.lib().ks_mul_noalloc(ctypes.c_void_p(tf.data_ptr()), ctypes.c_void_p(tg.data_ptr()), 3, 3, 8,
                                 ks.KS_VARIANT["ks4"], ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 ctypes.c_void_p(h.data_ptr()))
    assert rc == ks.KS_OK
    assert ks.status() == ks.KS_ERANGE
    assert ks.status() == ks.KS_OK
    # the next call is clean again
    f = np.array([[5], [7]], dtype=np.uint32)
    assert np.array_equal(noalloc(torch, f, f, 8, "ks4", False), pooled(f, f, 8, "ks4", False))


def test_noalloc_refuses_beyond_its_array(torch_dev):
    torch = torch_dev
    L, bits = 1 << 20, 256
    assert ks.plan(L, L, bits, "ks1", True)["scratch_bytes"] > ks.KS_NOALLOC_SCRATCH_BYTES
    t = torch.zeros(8, dtype=torch.int32, device="cuda")  # never read: refused before any launch
    rc = ks.lib().ks_mul_noalloc(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), L, L, bits,
                                 ks.KS_VARIANT["ks1"] | ks.KS_SIGNED,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.c_void_p(t.data_ptr()))
    assert rc == ks.KS_ESCRATCH
