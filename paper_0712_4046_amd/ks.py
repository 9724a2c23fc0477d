"""Python binding of libksmul (argument marshalling only).

Every step of a product runs in the library's HIP kernels; this module only checks shapes,
allocates output tensors, and passes device pointers and the current HIP stream through
the C ABI declared in include/ks.h.  PyTorch supplies device memory and streams.

There is no fallback: if libksmul.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksmul.so")

KS_VARIANT = {"auto": 0, "ks1": 1, "neg2": 2, "recip2": 3, "ks4": 4}
# substitutions of the bivariate products: the variants above and Section 2.5's points in an
# extension of R (complex points, cube roots of unity)
P2_VARIANT = {**KS_VARIANT, "cplx": 5, "cube": 6}
KS_SIGNED = 0x100
KS_ENGINE_VALU, KS_ENGINE_MFMA, KS_ENGINE_NTT = 0x1000, 0x2000, 0x4000
KS_ENGINE = {None: 0, "valu": KS_ENGINE_VALU, "mfma": KS_ENGINE_MFMA, "ntt": KS_ENGINE_NTT}
KS_MOD = 0x10000
KS_OK, KS_EINVAL, KS_ENOMEM, KS_EHIP, KS_ERANGE, KS_EUNSUPPORTED, KS_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
KS_ESCRATCH = -7
KS_NOALLOC_SCRATCH_BYTES = 64 << 20
KS_MAX_BITS = 256


class KSError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class PlanInfo(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("engine", ctypes.c_int32), ("e", ctypes.c_int32),
                ("slot_bits", ctypes.c_int32), ("n_products", ctypes.c_int32), ("out_limbs", ctypes.c_int32),
                ("operand_limbs_f", ctypes.c_int64), ("operand_limbs_g", ctypes.c_int64),
                ("limb_mults", ctypes.c_double), ("schoolbook_limb_mults", ctypes.c_double),
                ("hbm_bytes", ctypes.c_double), ("pack_bytes", ctypes.c_double),
                ("normalize_bytes", ctypes.c_double), ("finish_bytes", ctypes.c_double),
                ("anchor_limb_mults", ctypes.c_double), ("mfma_ops", ctypes.c_double),
                ("valu_limb_mults", ctypes.c_double), ("scratch_bytes", ctypes.c_int64),
                ("ntt_butterflies", ctypes.c_double), ("ntt_k1", ctypes.c_int32), ("ntt_k2", ctypes.c_int32)]


class Desc(ctypes.Structure):
    _fields_ = [("f_off", ctypes.c_uint64), ("g_off", ctypes.c_uint64), ("h_off", ctypes.c_uint64),
                ("len_f", ctypes.c_int32), ("len_g", ctypes.c_int32), ("coeff_bits", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("mod_p", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libksmul.so not built ({LIB_PATH}); run `python -m paper_0712_4046_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "ks_version": ([], i32),
        "ks_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "ks_out_limbs": ([i64, i64, i32], i64),
        "ks_mul": ([P, P, i64, i64, i32, i32, P, P], ctypes.c_int),
        "ks_mul_mod": ([P, P, i64, i64, u64, i32, P, P], ctypes.c_int),
        "ks_mul_noalloc": ([P, P, i64, i64, i32, i32, P, P], ctypes.c_int),
        "ks_mul_poly2": ([P, P, i64, i64, u64, i32, i32, P, P], ctypes.c_int),
        "ks_stream_status": ([P], ctypes.c_int),
        "ks_plan": ([i64, i64, i32, i32, ctypes.POINTER(PlanInfo)], ctypes.c_int),
        "ks_profile_enable": ([i32], ctypes.c_int),
        "ks_profile_read": ([ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "ks_profile_reset": ([], ctypes.c_int),
        "ks_tune_set": ([ctypes.c_char_p, i64], ctypes.c_int),
        "ks_tune_get": ([ctypes.c_char_p, ctypes.POINTER(i64)], ctypes.c_int),
        "ks_tune_reset": ([], ctypes.c_int),
        "ks_batch_plan_create": ([P, i64, i32, ctypes.POINTER(P)], ctypes.c_int),
        "ks_batch_plan_bad_index": ([], i64),
        "ks_batch_plan_workspace_bytes": ([P], sz),
        "ks_batch_plan_info": ([P, ctypes.POINTER(PlanInfo)], ctypes.c_int),
        "ks_batch_run": ([P, P, P, P, sz, P], ctypes.c_int),
        "ks_batch_status": ([P, P, P], ctypes.c_int),
        "ks_batch_plan_destroy": ([P], None),
        "ks_batch_workspace_bytes": ([P, i64, i32], sz),
        "ks_mul_batch": ([P, P, P, i64, i32, P, sz, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().ks_strerror(code).decode()
    except Exception:
        return "unknown"


def _check(rc: int, what: str):
    if rc != KS_OK:
        raise KSError(rc, what)


def _flags(variant: str, signed: bool, engine) -> int:
    if variant not in KS_VARIANT:
        raise ValueError(f"unknown variant {variant!r}")
    return KS_VARIANT[variant] | (KS_SIGNED if signed else 0) | KS_ENGINE[engine]


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def limbs_for_bits(bits: int) -> int:
    return (bits + 31) // 32


def out_limbs(len_f: int, len_g: int, bits: int) -> int:
    r = lib().ks_out_limbs(len_f, len_g, bits)
    if r < 0:
        raise KSError(int(r), "ks_out_limbs")
    return int(r)


def plan(len_f: int, len_g: int, bits: int, variant: str = "auto", signed: bool = False, engine=None) -> dict:
    info = PlanInfo()
    _check(lib().ks_plan(len_f, len_g, bits, _flags(variant, signed, engine), ctypes.byref(info)), "ks_plan")
    return {k: getattr(info, k) for k, _ in PlanInfo._fields_}


def to_device(arr: np.ndarray, device="cuda"):
    """uint32 limb array -> int32 torch tensor on the device (same bits)."""
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def mul(f, g, bits: int, variant: str = "auto", signed: bool = False, engine=None, stream=None, out=None):
    """h = f g; f, g are (L, W) int32 CUDA tensors of limbs (W = ceil(bits/32))."""
    import torch
    W = limbs_for_bits(bits)
    if f.dim() != 2 or g.dim() != 2 or f.shape[1] != W or g.shape[1] != W:
        raise ValueError(f"inputs must be (L, {W}) limb tensors")
    if not (f.is_cuda and g.is_cuda and f.is_contiguous() and g.is_contiguous()):
        raise ValueError("inputs must be contiguous CUDA tensors")
    lf, lg = f.shape[0], g.shape[0]
    wo = out_limbs(lf, lg, bits)
    if out is None:
        out = torch.empty((lf + lg - 1, wo), dtype=torch.int32, device=f.device)
    elif tuple(out.shape) != (lf + lg - 1, wo) or not out.is_contiguous():
        raise ValueError("out has the wrong shape")
    rc = lib().ks_mul(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), lf, lg, bits,
                      _flags(variant, signed, engine), _stream_ptr(stream), ctypes.c_void_p(out.data_ptr()))
    _check(rc, "ks_mul")
    return out


def mul_noalloc(f, g, bits: int, variant: str = "auto", signed: bool = False, engine=None, stream=None, out=None):
    """h = f g through ks_mul_noalloc (scratch from the library's fixed device array; the output
    tensor is the caller's: pass `out` to allocate nothing at all)."""
    import torch
    W = limbs_for_bits(bits)
    if f.dim() != 2 or g.dim() != 2 or f.shape[1] != W or g.shape[1] != W:
        raise ValueError(f"inputs must be (L, {W}) limb tensors")
    if not (f.is_cuda and g.is_cuda and f.is_contiguous() and g.is_contiguous()):
        raise ValueError("inputs must be contiguous CUDA tensors")
    lf, lg = f.shape[0], g.shape[0]
    wo = out_limbs(lf, lg, bits)
    if out is None:
        out = torch.empty((lf + lg - 1, wo), dtype=torch.int32, device=f.device)
    elif tuple(out.shape) != (lf + lg - 1, wo) or not out.is_contiguous():
        raise ValueError("out has the wrong shape")
    rc = lib().ks_mul_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), lf, lg, bits,
                              _flags(variant, signed, engine), _stream_ptr(stream), ctypes.c_void_p(out.data_ptr()))
    _check(rc, "ks_mul_noalloc")
    return out


def mul_raw(f_ptr: int, g_ptr: int, lf: int, lg: int, bits: int, flags: int, stream_ptr: int, h_ptr: int) -> int:
    """Direct call with integer pointers (returns the status code)."""
    return lib().ks_mul(ctypes.c_void_p(f_ptr), ctypes.c_void_p(g_ptr), lf, lg, bits, flags,
                        ctypes.c_void_p(stream_ptr), ctypes.c_void_p(h_ptr))


def mul_mod(f, g, p: int, variant: str = "auto", engine=None, stream=None, out=None):
    """h = f g in (Z/pZ)[x]; f, g are int64 CUDA tensors of residues in [0, p)."""
    import torch
    if f.dim() != 1 or g.dim() != 1 or f.dtype != torch.int64 or g.dtype != torch.int64:
        raise ValueError("inputs must be 1-D int64 tensors of residues")
    lf, lg = f.shape[0], g.shape[0]
    if out is None:
        out = torch.empty(lf + lg - 1, dtype=torch.int64, device=f.device)
    rc = lib().ks_mul_mod(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), lf, lg, p,
                          _flags(variant, False, engine), _stream_ptr(stream), ctypes.c_void_p(out.data_ptr()))
    _check(rc, "ks_mul_mod")
    return out


def mul_poly2(f, g, p: int, variant: str = "auto", inner: str = "auto", engine=None, stream=None, out=None):
    """h = f g in (Z/pZ)[x, y] (ks_mul_poly2); f, g are (len_y, len_x) int64 CUDA tensors of
    residues in [0, p) (row i: the coefficients of f_i(x)); h is (2 len_y - 1, 2 len_x - 1)."""
    import torch
    if f.dim() != 2 or f.shape != g.shape or f.dtype != torch.int64 or g.dtype != torch.int64:
        raise ValueError("inputs must be 2-D int64 tensors of residues of the same shape")
    if not (f.is_contiguous() and g.is_contiguous()):
        raise ValueError("inputs must be contiguous")
    ly, lx = f.shape
    if out is None:
        out = torch.empty((2 * ly - 1, 2 * lx - 1), dtype=torch.int64, device=f.device)
    rc = lib().ks_mul_poly2(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), lx, ly, p,
                            P2_VARIANT[variant], _flags(inner, False, engine), _stream_ptr(stream),
                            ctypes.c_void_p(out.data_ptr()))
    _check(rc, "ks_mul_poly2")
    return out


def status(stream=None) -> int:
    """Synchronise the stream and return (and clear) the device status code."""
    return int(lib().ks_stream_status(_stream_ptr(stream)))


def check(stream=None):
    rc = status(stream)
    if rc != KS_OK:
        raise KSError(rc, "device status")


def profile_enable(on: bool = True):
    _check(lib().ks_profile_enable(1 if on else 0), "ks_profile_enable")


def profile_reset():
    _check(lib().ks_profile_reset(), "ks_profile_reset")


TUNABLES = ("KS_MFMA_MIN_LIMBS", "KS_MFMA_BLOCKS", "KS_MFMA_MIN_PART", "KS_MFMA_BLOCK_COST", "KS_CHAIN_K",
            "KS_MUL_WAVE_MAX", "KS_SCAN_SMALL", "KS_MFMA_RT", "KS_KARATSUBA_MIN_LIMBS", "KS_NTT_MIN_LIMBS", "KS_SCAN_BIG")


def tune_set(name: str, value: int):
    """Override a planner tunable (ks_tune_set); see include/ks.h for names and defaults."""
    _check(lib().ks_tune_set(name.encode(), int(value)), f"ks_tune_set({name})")


def tune_get(name: str) -> int:
    v = ctypes.c_int64()
    _check(lib().ks_tune_get(name.encode(), ctypes.byref(v)), f"ks_tune_get({name})")
    return int(v.value)


def tune_reset():
    _check(lib().ks_tune_reset(), "ks_tune_reset")


def apply_tuning(table: dict):
    """Set every tunable of a table written by paper_0712_4046_amd.autotune."""
    for k, v in table.items():
        if k in TUNABLES:
            tune_set(k, v)


def profile_read(name: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().ks_profile_read(name.encode(), ctypes.byref(n), ctypes.byref(ms)), "ks_profile_read")
    return int(n.value), float(ms.value)


# ---- batches ---------------------------------------------------------------------------------

class Batch:
    """Host-side layout of many products in two arenas (marshalling only).

    add(f, g, bits, signed) appends limb arrays; add_mod(f, g, p) appends residues.  The
    arena_in / descriptor arrays then go to BatchPlan; out_slice(i) locates product i's output.
    """

    def __init__(self):
        self._in = []
        self._in_len = 0
        self._out_len = 0
        self.descs = []
        self._out = []  # (offset, count, width, kind)

    def _push(self, a: np.ndarray) -> int:
        off = self._in_len
        a = np.ascontiguousarray(a).view(np.uint32).reshape(-1)
        if off % 2:
            self._in.append(np.zeros(1, dtype=np.uint32))
            self._in_len += 1
            off += 1
        self._in.append(a)
        self._in_len += a.size
        return off

    def add(self, f: np.ndarray, g: np.ndarray, bits: int, signed: bool) -> int:
        lf, lg = f.shape[0], g.shape[0]
        fo, go = self._push(f), self._push(g)
        wo = out_limbs(lf, lg, bits)
        ho = self._out_len
        self._out_len += (lf + lg - 1) * wo
        self.descs.append((fo, go, ho, lf, lg, bits, KS_SIGNED if signed else 0, 0))
        self._out.append((ho, lf + lg - 1, wo, "z"))
        return len(self.descs) - 1

    def add_mod(self, f: np.ndarray, g: np.ndarray, p: int) -> int:
        lf, lg = len(f), len(g)
        fo, go = self._push(np.asarray(f, dtype=np.uint64)), self._push(np.asarray(g, dtype=np.uint64))
        if self._out_len % 2:
            self._out_len += 1
        ho = self._out_len
        self._out_len += 2 * (lf + lg - 1)
        self.descs.append((fo, go, ho, lf, lg, 0, KS_MOD, p))
        self._out.append((ho, lf + lg - 1, 2, "mod"))
        return len(self.descs) - 1

    def arena_in(self) -> np.ndarray:
        return np.concatenate(self._in) if self._in else np.zeros(1, dtype=np.uint32)

    def out_words(self) -> int:
        return max(self._out_len, 1)

    def desc_array(self):
        arr = (Desc * len(self.descs))()
        for i, d in enumerate(self.descs):
            arr[i] = Desc(*d)
        return arr

    def result(self, arena_out: np.ndarray, i: int) -> np.ndarray:
        off, count, width, kind = self._out[i]
        a = arena_out[off:off + count * width]
        return a.view(np.uint64) if kind == "mod" else a.reshape(count, width)


class BatchPlan:
    """A planned batch (ks_batch_plan_*): tables live on the device until close()."""

    def __init__(self, descs, variant: str = "auto", engine=None):
        self._descs = descs
        h = ctypes.c_void_p()
        flags = KS_VARIANT[variant] | KS_ENGINE[engine]
        rc = lib().ks_batch_plan_create(ctypes.cast(descs, ctypes.c_void_p), len(descs), flags, ctypes.byref(h))
        if rc != KS_OK:
            raise KSError(rc, f"ks_batch_plan_create (descriptor {lib().ks_batch_plan_bad_index()})")
        self.handle = h
        self.workspace_bytes = int(lib().ks_batch_plan_workspace_bytes(h))

    def info(self) -> dict:
        info = PlanInfo()
        _check(lib().ks_batch_plan_info(self.handle, ctypes.byref(info)), "ks_batch_plan_info")
        return {k: getattr(info, k) for k, _ in PlanInfo._fields_}

    def run(self, arena_in, arena_out, workspace, stream=None):
        rc = lib().ks_batch_run(self.handle, ctypes.c_void_p(arena_in.data_ptr()), ctypes.c_void_p(arena_out.data_ptr()),
                                ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream))
        _check(rc, "ks_batch_run")

    def status(self, workspace, stream=None) -> int:
        return int(lib().ks_batch_status(self.handle, ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream)))

    def close(self):
        if self.handle:
            lib().ks_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def alloc_workspace(nbytes: int, device="cuda"):
    """A 256-byte aligned device buffer (torch allocations are at least 512-byte aligned)."""
    import torch
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
