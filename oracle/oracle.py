"""Python view of the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import this
module.  It loads ``oracle/liboracle.so`` (built from ``oracle/oracle.c`` with gcc) through
ctypes and adds small helpers that move between Python integers and the limb layout used by
both the oracle and the library: coefficient i of a polynomial occupies ``w`` little-endian
32-bit limbs, two's complement when signed.

Routes (see ``oracle.c``):
  * ``mul_classical``  -- h_k = sum_{i+j=k} f_i g_j written out (paper, Section 3);
  * ``mul_ks1``        -- standard Kronecker substitution over a schoolbook bignum
                          (paper, Section 3.1);
  * ``coeffs_classical`` / ``coeffs_mod`` -- single coefficients, for sampled checks;
  * ``mul_mod``        -- (Z/pZ)[x] product by lifting and reducing (paper, Section 4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, OpenMP across coefficients)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", SRC_PATH, "-o", LIB_PATH + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def _configure(L):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    L.or_mul_classical.argtypes = [P, P, i64, i64, ci, ci, P, ci]
    L.or_coeffs_classical.argtypes = [P, P, i64, i64, ci, ci, P, i64, P, ci]
    L.or_mul_ks1.argtypes = [P, P, i64, i64, ci, ci, ci, P, ci]
    L.or_mul_mod.argtypes = [P, P, i64, i64, ctypes.c_uint64, P]
    L.or_coeffs_mod.argtypes = [P, P, i64, i64, ctypes.c_uint64, P, i64, P]
    L.or_threads.argtypes = []
    for fn in (L.or_mul_classical, L.or_coeffs_classical, L.or_mul_ks1, L.or_mul_mod,
               L.or_coeffs_mod, L.or_threads):
        fn.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _configure(ctypes.CDLL(LIB_PATH))
    return _lib


def use_library(path):
    """Point this module at another build of oracle.c (the mutation tests use this)."""
    global _lib
    _lib = _configure(ctypes.CDLL(path)) if path else None


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# ---- format helpers (no arithmetic of the method) ----------------------------------------

def limbs_for_bits(bits: int) -> int:
    return (bits + 31) // 32


def ints_to_limbs(vals, w: int) -> np.ndarray:
    """Python ints -> (len, w) uint32 array, two's complement modulo 2^(32 w)."""
    out = np.zeros((len(vals), w), dtype=np.uint32)
    mask = (1 << (32 * w)) - 1
    for i, v in enumerate(vals):
        x = int(v) & mask
        for t in range(w):
            out[i, t] = (x >> (32 * t)) & 0xFFFFFFFF
    return out


def limbs_to_ints(arr: np.ndarray, signed: bool = True) -> list:
    """(len, w) uint32 array -> Python ints (two's complement when signed)."""
    arr = np.asarray(arr, dtype=np.uint32)
    if arr.ndim == 1:
        arr = arr.reshape(-1, 1)
    w = arr.shape[1]
    out = []
    for row in arr:
        x = 0
        for t in range(w - 1, -1, -1):
            x = (x << 32) | int(row[t])
        if signed and (x >> (32 * w - 1)) & 1:
            x -= 1 << (32 * w)
        out.append(x)
    return out


def out_limbs(len_f: int, len_g: int, b: int) -> int:
    """Output width in limbs: coefficients of h have length <= 2b + e (Section 3), plus a sign bit."""
    e = (min(len_f, len_g) - 1).bit_length()
    return limbs_for_bits(2 * b + e + 1)


# ---- the routes ---------------------------------------------------------------------------

def mul_classical(f: np.ndarray, g: np.ndarray, signed: bool, w_out: int) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    lf, w = f.shape
    lg, w2 = g.shape
    assert w == w2
    h = np.zeros((lf + lg - 1, w_out), dtype=np.uint32)
    _check(lib().or_mul_classical(_ptr(f), _ptr(g), lf, lg, w, int(signed), _ptr(h), w_out), "classical")
    return h


def coeffs_classical(f: np.ndarray, g: np.ndarray, signed: bool, ks, w_out: int) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    out = np.zeros((len(ks), w_out), dtype=np.uint32)
    _check(lib().or_coeffs_classical(_ptr(f), _ptr(g), f.shape[0], g.shape[0], f.shape[1], int(signed),
                                     _ptr(ks), len(ks), _ptr(out), w_out), "coeffs")
    return out


def mul_ks1(f: np.ndarray, g: np.ndarray, b: int, signed: bool, w_out: int) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    lf, w = f.shape
    lg, _ = g.shape
    h = np.zeros((lf + lg - 1, w_out), dtype=np.uint32)
    _check(lib().or_mul_ks1(_ptr(f), _ptr(g), lf, lg, w, b, int(signed), _ptr(h), w_out), "ks1")
    return h


def mul_mod(f: np.ndarray, g: np.ndarray, p: int) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.uint64)
    g = np.ascontiguousarray(g, dtype=np.uint64)
    h = np.zeros(len(f) + len(g) - 1, dtype=np.uint64)
    _check(lib().or_mul_mod(_ptr(f), _ptr(g), len(f), len(g), p, _ptr(h)), "mod")
    return h


def coeffs_mod(f: np.ndarray, g: np.ndarray, p: int, ks) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.uint64)
    g = np.ascontiguousarray(g, dtype=np.uint64)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    out = np.zeros(len(ks), dtype=np.uint64)
    _check(lib().or_coeffs_mod(_ptr(f), _ptr(g), len(f), len(g), p, _ptr(ks), len(ks), _ptr(out)), "coeffs_mod")
    return out


def threads() -> int:
    return int(lib().or_threads())
