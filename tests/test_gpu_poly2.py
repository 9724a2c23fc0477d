"""GPU parity of the bivariate products over Z/pZ (ks_mul_poly2, paper Section 2): every
substitution against the oracle's definition, element by element at sizes the oracle finishes
in seconds, and on sampled coefficients at the bivariate workload's full size."""
import numpy as np
import pytest

from paper_0712_4046_amd import ks
from paper_0712_4046_amd import workloads as wl

pytestmark = pytest.mark.gpu

VARIANTS = ["ks1", "recip2", "neg2", "ks4", "auto"]
MODULI = [3, 2**31 - 1, 2**61 - 1, wl.paper_fig_modulus(60, 7), (1 << 62) - 1]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.lib()
    return torch


@pytest.fixture(scope="module")
def poly2():
    from oracle import poly2 as o
    return o


def gpu(torch, f, g, p, variant, inner="auto", engine=None):
    tf = torch.from_numpy(f.astype(np.int64)).cuda()
    tg = torch.from_numpy(g.astype(np.int64)).cuda()
    h = ks.mul_poly2(tf, tg, p, variant, inner, engine)
    rc = ks.status()
    assert rc == ks.KS_OK, ks.strerror(rc)
    return h.cpu().numpy().astype(np.uint64)


def rows(a):
    return [[int(v) for v in r] for r in a]


@pytest.mark.parametrize("p", MODULI)
@pytest.mark.parametrize("ly,lx", [(1, 1), (1, 5), (5, 1), (2, 2), (3, 4), (4, 7), (8, 3), (16, 16), (33, 9),
                                   (64, 16)])
def test_poly2_against_definition(torch_dev, poly2, ly, lx, p):
    f, g = wl.poly2_pair(ly, lx, p, seed=100 * ly + lx)
    want = poly2.mul_direct(rows(f), rows(g), p)
    for v in VARIANTS:
        got = gpu(torch_dev, f, g, p, v)
        assert got.shape == (2 * ly - 1, 2 * lx - 1), v
        assert rows(got) == want, f"{v} ly={ly} lx={lx} p={p}"


@pytest.mark.parametrize("inner", ["ks1", "neg2", "recip2", "ks4"])
@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_poly2_inner_products(torch_dev, poly2, inner, engine):
    p = 2**61 - 1
    f, g = wl.poly2_pair(40, 12, p, seed=5)
    want = poly2.mul_direct(rows(f), rows(g), p)
    for v in ["ks1", "recip2", "neg2", "ks4"]:
        assert rows(gpu(torch_dev, f, g, p, v, inner, engine)) == want, (v, inner, engine)


@pytest.mark.parametrize("ly,lx", [(3000, 1), (1, 3000), (700, 2), (2, 700)])
def test_poly2_thin_shapes(torch_dev, poly2, ly, lx):
    # a single row or column reduces to a univariate product; two rows or columns are the
    # smallest overlaps of the four-point evaluation
    p = wl.paper_fig_modulus(60, 7)
    f, g = wl.poly2_pair(ly, lx, p, seed=ly + lx)
    rng = np.random.default_rng(1)
    for v in VARIANTS:
        got = gpu(torch_dev, f, g, p, v)
        for _ in range(60):
            k, c = int(rng.integers(0, 2 * ly - 1)), int(rng.integers(0, 2 * lx - 1))
            assert int(got[k, c]) == poly2.coeff_direct(f, g, p, k, c), (v, k, c)


def test_poly2_workload_sampled(torch_dev, poly2):
    # the bivariate workload at full size (L_x = 16, L_y = 4096, 60-bit p): 300 sampled
    # coefficients of every substitution against the definition, the first and last rows and
    # columns among them, and all substitutions equal everywhere
    p, f, g = wl.poly2_workload()
    ly, lx = f.shape
    outs = {v: gpu(torch_dev, f, g, p, v) for v in VARIANTS}
    rng = np.random.default_rng(2)
    picks = [(0, 0), (0, 2 * lx - 2), (2 * ly - 2, 0), (2 * ly - 2, 2 * lx - 2), (ly - 1, lx - 1)]
    picks += [(int(rng.integers(0, 2 * ly - 1)), int(rng.integers(0, 2 * lx - 1))) for _ in range(295)]
    fl, gl = rows(f), rows(g)
    for k, c in picks:
        w = poly2.coeff_direct(fl, gl, p, k, c)
        for v, h in outs.items():
            assert int(h[k, c]) == w, (v, k, c)
    for v in VARIANTS[1:]:
        assert np.array_equal(outs[v], outs["ks1"]), v


def test_poly2_errors(torch_dev):
    import torch
    f = torch.zeros((3, 4), dtype=torch.int64, device="cuda")
    with pytest.raises(ks.KSError):
        ks.mul_poly2(f, f, 2**20, "ks4")  # even modulus
    with pytest.raises(ks.KSError):
        ks.mul_poly2(f, f, 1 << 62, "ks4")  # too large
    bad = torch.full((3, 4), 7, dtype=torch.int64, device="cuda")
    ks.mul_poly2(bad, bad, 5, "neg2")  # residues >= p
    assert ks.status() == ks.KS_ERANGE
    assert ks.status() == ks.KS_OK


# ---- Section 2.5: evaluation points in an extension of R ---------------------------------------

@pytest.mark.parametrize("p", MODULI)
@pytest.mark.parametrize("ly,lx", [(1, 1), (1, 5), (5, 1), (2, 2), (3, 4), (4, 7), (7, 3), (8, 6), (16, 16),
                                   (33, 9), (64, 17)])
def test_poly2_extension_points_against_definition(torch_dev, poly2, ly, lx, p):
    # the complex points (five products, rows by residue mod 4) and the cube roots of unity
    # (eight products, rows by residue mod 6; p must not be divisible by 3) element by element
    f, g = wl.poly2_pair(ly, lx, p, seed=300 * ly + lx)
    want = poly2.mul_direct(rows(f), rows(g), p)
    for v in ("cplx", "cube"):
        if v == "cube" and p % 3 == 0:
            continue
        got = gpu(torch_dev, f, g, p, v)
        assert got.shape == (2 * ly - 1, 2 * lx - 1), v
        assert rows(got) == want, f"{v} ly={ly} lx={lx} p={p}"


def test_poly2_extension_points_workload_sampled(torch_dev, poly2):
    # the bivariate workload's shape (L_x = 16, L_y = 4096, 60-bit p): both extension-point
    # substitutions equal the standard one everywhere and the definition on 200 samples
    p, f, g = wl.poly2_workload()
    ref = gpu(torch_dev, f, g, p, "ks1")
    rng = np.random.default_rng(9)
    for v in ("cplx", "cube"):
        got = gpu(torch_dev, f, g, p, v)
        assert np.array_equal(got, ref), v
    for _ in range(200):
        k, c = int(rng.integers(0, 2 * f.shape[0] - 1)), int(rng.integers(0, 2 * f.shape[1] - 1))
        assert int(ref[k, c]) == poly2.coeff_direct(f, g, p, k, c), (k, c)


def test_poly2_extension_points_range_error(torch_dev):
    torch = torch_dev
    p = 1_000_003
    f = torch.ones((4, 5), dtype=torch.int64, device="cuda")
    g = f.clone()
    g[2, 3] = p  # not a residue
    for v in ("cplx", "cube"):
        ks.mul_poly2(f, g, p, v)
        assert ks.status() == ks.KS_ERANGE, v
