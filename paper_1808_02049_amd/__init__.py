"""Python binding of the MI355X Epstein-Nesbet PT2 engine (libpt2.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI declared in include/pt2.h.  PyTorch is used for
device memory (an optional allocator hook into its caching allocator) and
streams; arrays may be numpy (host) or torch CUDA tensors (device-resident
inputs go through ``pt2_evaluate_device``).

There is no CPU fallback: importing this package fails if the shared
library has not been built (``python paper_1808_02049_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt2.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP engine first "
                      "(python paper_1808_02049_amd/build.py)")

_lib = C.CDLL(LIB_PATH)

PT2_OK, PT2_NOT_READY = 0, 1
PT2_E_INVALID, PT2_E_NOMEM, PT2_E_DEVICE = -1, -2, -3
PT2_E_BUSY, PT2_E_SINGULAR, PT2_E_UNKNOWN_REQ = -4, -5, -6
PT2_FP64, PT2_FP32_PAYLOAD, PT2_FP32_ARITH = 0, 1, 2

_ERRNAMES = {PT2_E_INVALID: "PT2_E_INVALID", PT2_E_NOMEM: "PT2_E_NOMEM",
             PT2_E_DEVICE: "PT2_E_DEVICE", PT2_E_BUSY: "PT2_E_BUSY",
             PT2_E_SINGULAR: "PT2_E_SINGULAR", PT2_E_UNKNOWN_REQ: "PT2_E_UNKNOWN_REQ"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("precision", C.c_int), ("cutoff", C.c_double),
                ("device_budget_bytes", C.c_uint64), ("max_partition_bytes", C.c_uint64),
                ("log2_partitions", C.c_int), ("device", C.c_int), ("n_streams", C.c_int),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", C.c_void_p),
                ("stream", C.c_void_p), ("timing", C.c_int), ("compress_keys", C.c_int),
                ("exclusion", C.c_int), ("hash_bits", C.c_int), ("spin_flip", C.c_int),
                ("string_reuse", C.c_int), ("compact_refs", C.c_int)]


class Result(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("e_pt2", C.c_double), ("n_contrib", C.c_uint64),
                ("n_after_cutoff", C.c_uint64), ("n_unique", C.c_uint64),
                ("n_external", C.c_uint64), ("n_in_ref_hit", C.c_uint64),
                ("n_partitions", C.c_uint32), ("n_sort_passes", C.c_uint32),
                ("record_bytes", C.c_uint32),
                ("min_abs_denom", C.c_double), ("n_nonneg_denom", C.c_uint64),
                ("ref_cross", C.c_double), ("key_xor", C.c_uint64), ("key_sum", C.c_uint64),
                ("ms_total", C.c_double), ("ms_gen", C.c_double), ("ms_sort", C.c_double),
                ("ms_sort_scatter", C.c_double), ("ms_reduce", C.c_double), ("ms_hist", C.c_double),
                ("ms_sort_pass_max", C.c_double), ("bytes_gen", C.c_double),
                ("bytes_sort", C.c_double), ("bytes_reduce", C.c_double), ("key_bits", C.c_uint32),
                ("n_alpha_groups", C.c_uint64), ("n_beta_groups", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "struct_size"}


_u64p, _f64p, _u32p = C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.POINTER(C.c_uint32)
_vp, _i64p, _u8p = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_uint8)
_CTX = C.c_void_p

_SIGS = {
    "pt2_default_options": (None, [C.POINTER(Options)]),
    "pt2_key_words": (C.c_int, [C.c_int]),
    "pt2_key_form": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(Options), C.POINTER(C.c_int),
                               C.POINTER(C.c_int)]),
    "pt2_create": (C.c_int, [_f64p, _f64p, C.c_int, C.c_int, C.c_int, C.POINTER(Options),
                             C.POINTER(_CTX)]),
    "pt2_evaluate": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, C.POINTER(Result)]),
    "pt2_evaluate_device": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, C.POINTER(Result)]),
    "pt2_evaluate_parts": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, C.c_int, _u32p,
                                     C.c_int, _f64p, C.POINTER(Result)]),
    "pt2_evaluate_device_noalloc": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, C.POINTER(Result)]),
    "pt2_evaluate_parts_device": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, C.c_int, _u32p,
                                            C.c_int, _f64p, C.POINTER(Result)]),
    "pt2_submit": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_double, _i64p]),
    "pt2_poll": (C.c_int, [_CTX, C.c_int64, C.POINTER(Result)]),
    "pt2_wait": (C.c_int, [_CTX, C.c_int64, C.POINTER(Result)]),
    "pt2_destroy": (C.c_int, [_CTX]),
    "pt2_last_error": (C.c_char_p, []),
    "pt2_dump_records": (C.c_int, [_CTX, _vp, _vp, C.c_int64, C.c_int, _u64p, _f64p,
                                   C.c_int64, _i64p]),
    "pt2_dump_numerators": (C.c_int, [_CTX, _vp, _vp, C.c_int64, _u64p, _f64p, _u8p,
                                      C.c_int64, _i64p]),
    "pt2_sort_records": (C.c_int, [C.c_int, C.c_int, C.c_int, _u64p, _vp, C.c_int, C.c_int64]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class PT2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


_PRECISIONS = {"fp64": PT2_FP64, "fp32": PT2_FP32_PAYLOAD, "fp32-arith": PT2_FP32_ARITH}


def _check(rc):
    if rc not in (PT2_OK, PT2_NOT_READY):
        raise PT2Error(rc, (_lib.pt2_last_error() or b"").decode(errors="replace"))
    return rc


def key_words(norb: int) -> int:
    return _lib.pt2_key_words(norb)


KEY_FORMS = ("bitstring", "rank", "hash")


def key_form(norb, nalpha, nbeta, precision="fp64", compress_keys=-1, hash_bits=0):
    """(form, key bits) of the records a context of these sizes and options
    takes (``pt2_key_form``; host only)."""
    o = default_options()
    o.precision = _PRECISIONS[precision]
    o.compress_keys = int(compress_keys)
    o.hash_bits = int(hash_bits)
    form, bits = C.c_int(), C.c_int()
    _check(_lib.pt2_key_form(int(norb), int(nalpha), int(nbeta), C.byref(o), C.byref(form), C.byref(bits)))
    return KEY_FORMS[form.value], bits.value


def default_options() -> Options:
    o = Options()
    _lib.pt2_default_options(C.byref(o))
    return o


def _is_torch_cuda(x):
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def _host_u64(a, W):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).reshape(-1, W)
    return a


def _host_f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)


class _TorchAllocator:
    """Allocator hook routing the engine's device memory to torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}

        def _alloc(nbytes, user):
            try:
                p = int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device))
            except Exception:
                return None
            self.live[p] = nbytes
            return p

        def _free(ptr, nbytes, user):
            if ptr:
                self.live.pop(int(ptr), None)
                self.torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class Context:
    """One Hamiltonian resident on the device (``pt2_create``)."""

    def __init__(self, h, eri, norb, nalpha, nbeta, precision="fp64", cutoff=0.0,
                 log2_partitions=-1, device=0, n_streams=4, device_budget_bytes=0,
                 max_partition_bytes=0, timing=False, stream=None, allocator=None, compress_keys=-1,
                 exclusion="search", hash_bits=0, spin_flip=False, string_reuse=1, compact_refs=True):
        self.norb, self.nalpha, self.nbeta = int(norb), int(nalpha), int(nbeta)
        self.W = key_words(self.norb)
        o = default_options()
        o.precision = _PRECISIONS[precision]
        o.cutoff = float(cutoff)
        o.log2_partitions = int(log2_partitions)
        o.device = int(device)
        o.n_streams = int(n_streams)
        o.device_budget_bytes = int(device_budget_bytes)
        o.max_partition_bytes = int(max_partition_bytes)
        o.timing = 1 if timing else 0
        o.compress_keys = int(compress_keys)
        o.exclusion = {"search": 0, "subtract": 1}[exclusion]
        o.hash_bits = int(hash_bits)
        o.spin_flip = 1 if spin_flip else 0
        o.string_reuse = int(string_reuse)
        o.compact_refs = 1 if compact_refs else 0
        if stream is not None:
            o.stream = int(getattr(stream, "cuda_stream", stream))
        self._alloc = None
        if allocator == "torch":
            self._alloc = _TorchAllocator(o.device)
            o.alloc, o.free = self._alloc.alloc, self._alloc.free
        self.options = o
        hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(norb, norb))
        ee = np.ascontiguousarray(np.asarray(eri, dtype=np.float64).reshape(-1))
        if ee.size != self.norb ** 4:
            raise ValueError("eri must have norb^4 entries")
        ctx = _CTX()
        _check(_lib.pt2_create(hh.ctypes.data_as(_f64p), ee.ctypes.data_as(_f64p), self.norb,
                               self.nalpha, self.nbeta, C.byref(o), C.byref(ctx)))
        self._ctx = ctx

    # -- evaluation ---------------------------------------------------------
    def _args(self, dets, coeffs):
        if _is_torch_cuda(dets) or _is_torch_cuda(coeffs):
            if not (_is_torch_cuda(dets) and _is_torch_cuda(coeffs)):
                raise ValueError("dets and coeffs must both be host arrays or both CUDA tensors")
            import torch
            if dets.dtype not in (torch.int64, torch.uint64) or coeffs.dtype != torch.float64:
                raise ValueError("device dets must be int64/uint64 and coeffs float64")
            if not (dets.is_contiguous() and coeffs.is_contiguous()):
                raise ValueError("device tensors must be contiguous")
            n = coeffs.numel()
            if dets.numel() != n * self.W:
                raise ValueError("dets must have ndets x W words")
            return True, dets.data_ptr(), coeffs.data_ptr(), n, (dets, coeffs)
        d = _host_u64(dets, self.W)
        c = _host_f64(coeffs)
        if len(c) != len(d):
            raise ValueError("dets and coeffs differ in length")
        return False, d.ctypes.data, c.ctypes.data, len(c), (d, c)

    def evaluate(self, dets, coeffs, e0):
        """E_PT2 and diagnostics (dict) for the reference (dets, coeffs) and E0."""
        dev, dp, cp, n, _keep = self._args(dets, coeffs)
        r = Result()
        r.struct_size = C.sizeof(Result)
        fn = _lib.pt2_evaluate_device if dev else _lib.pt2_evaluate
        _check(fn(self._ctx, dp, cp, n, float(e0), C.byref(r)))
        return r.as_dict()

    def evaluate_noalloc(self, dets, coeffs, e0):
        """As evaluate on device tensors, through the allocation-free entry
        point (the library's static device scratch)."""
        dev, dp, cp, n, _keep = self._args(dets, coeffs)
        if not dev:
            raise ValueError("evaluate_noalloc takes device tensors")
        r = Result()
        r.struct_size = C.sizeof(Result)
        _check(_lib.pt2_evaluate_device_noalloc(self._ctx, dp, cp, n, float(e0), C.byref(r)))
        return r.as_dict()

    def evaluate_parts(self, dets, coeffs, e0, log2p, parts):
        """Energies of the listed subsets of a 2^log2p hash split (host arrays,
        or CUDA tensors resident on the device)."""
        if not (_is_torch_cuda(dets) or _is_torch_cuda(coeffs)):
            dets, coeffs = np.asarray(dets), np.asarray(coeffs)
        dev, dp, cp, n, _keep = self._args(dets, coeffs)
        pp = np.ascontiguousarray(np.asarray(parts, dtype=np.uint32))
        ep = np.zeros(len(pp), dtype=np.float64)
        r = Result()
        r.struct_size = C.sizeof(Result)
        fn = _lib.pt2_evaluate_parts_device if dev else _lib.pt2_evaluate_parts
        _check(fn(self._ctx, dp, cp, n, float(e0), int(log2p), pp.ctypes.data_as(_u32p), len(pp),
                  ep.ctypes.data_as(_f64p), C.byref(r)))
        return r.as_dict(), ep

    # -- serving -------------------------------------------------------------
    def submit(self, dets, coeffs, e0):
        _dev, dp, cp, n, _keep = self._args(np.asarray(dets), np.asarray(coeffs))
        rid = C.c_int64()
        _check(_lib.pt2_submit(self._ctx, dp, cp, n, float(e0), C.byref(rid)))
        return rid.value

    def poll(self, rid):
        """None while running, else the result dict."""
        r = Result()
        r.struct_size = C.sizeof(Result)
        rc = _check(_lib.pt2_poll(self._ctx, int(rid), C.byref(r)))
        return None if rc == PT2_NOT_READY else r.as_dict()

    def wait(self, rid):
        r = Result()
        r.struct_size = C.sizeof(Result)
        _check(_lib.pt2_wait(self._ctx, int(rid), C.byref(r)))
        return r.as_dict()

    # -- inspection ------------------------------------------------------------
    def dump_records(self, dets, coeffs, sorted=False, cap=None):
        _dev, dp, cp, n, _keep = self._args(np.asarray(dets), np.asarray(coeffs))
        if cap is None:
            cap = n * self._nper()
        keys = np.zeros((max(cap, 1), self.W), dtype=np.uint64)
        vals = np.zeros(max(cap, 1), dtype=np.float64)
        cnt = C.c_int64()
        _check(_lib.pt2_dump_records(self._ctx, dp, cp, n, 1 if sorted else 0,
                                     keys.ctypes.data_as(_u64p), vals.ctypes.data_as(_f64p), cap,
                                     C.byref(cnt)))
        m = min(cnt.value, cap)
        return keys[:m], vals[:m]

    def dump_numerators(self, dets, coeffs, cap=None):
        _dev, dp, cp, n, _keep = self._args(np.asarray(dets), np.asarray(coeffs))
        if cap is None:
            cap = n * self._nper()
        keys = np.zeros((max(cap, 1), self.W), dtype=np.uint64)
        nums = np.zeros(max(cap, 1), dtype=np.float64)
        inref = np.zeros(max(cap, 1), dtype=np.uint8)
        cnt = C.c_int64()
        _check(_lib.pt2_dump_numerators(self._ctx, dp, cp, n, keys.ctypes.data_as(_u64p),
                                        nums.ctypes.data_as(_f64p), inref.ctypes.data_as(_u8p), cap,
                                        C.byref(cnt)))
        m = min(cnt.value, cap)
        return keys[:m], nums[:m], inref[:m].astype(bool)

    def _nper(self):
        n, a, b = self.norb, self.nalpha, self.nbeta
        va, vb = n - a, n - b
        c2 = lambda x: x * (x - 1) // 2
        return a * va + b * vb + c2(a) * c2(va) + c2(b) * c2(vb) + a * va * b * vb

    def close(self):
        if getattr(self, "_ctx", None):
            _check(_lib.pt2_destroy(self._ctx))
            self._ctx = None

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                _lib.pt2_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass


def sort_records(keys, payload, key_bits, device=0):
    """The engine's stable LSD radix sort on host arrays (returns sorted copies)."""
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    if k.ndim == 1:
        k = k.reshape(-1, 1)
    W = k.shape[1]
    p = np.ascontiguousarray(np.array(payload))
    if p.dtype.itemsize not in (4, 8) or len(p) != len(k):
        raise ValueError("payload must be 4- or 8-byte elements, one per key")
    _check(_lib.pt2_sort_records(int(device), W, int(key_bits), k.ctypes.data_as(_u64p),
                                 p.ctypes.data, p.dtype.itemsize, len(k)))
    return k, p
