"""ctypes front end of the FP64 CPU oracle and the brute-force FCI checker.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the HIP engine never imports it.

* ``Oracle`` wraps ``pt2_oracle.c``: the Epstein-Nesbet PT2 energy by
  excitation loops, grouping by bitstring and a single pass (Algorithm 1 and
  Algorithm 2 of arXiv:1808.02049), plus Slater-Condon matrix elements used to
  build synthetic inputs (diagonal energies, H_RR, <c|H|c>).
* ``Brute`` wraps ``fci_brute.c``: the literal second-quantised Hamiltonian
  applied operator by operator over the full-CI space; ``Brute.pt2`` assembles
  sum over the complement of (H c)_a^2 / (E0 - H_aa) with numpy.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

_u64p = C.POINTER(C.c_uint64)
_f64p = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)


class _System(C.Structure):
    _fields_ = [("norb", C.c_int), ("nalpha", C.c_int), ("nbeta", C.c_int),
                ("h", _f64p), ("eri", _f64p)]


class _Result(C.Structure):
    _fields_ = [("e_pt2", C.c_double), ("n_contrib", C.c_uint64), ("n_kept", C.c_uint64),
                ("n_unique", C.c_uint64), ("n_external", C.c_uint64),
                ("n_in_ref_hit", C.c_uint64), ("min_abs_denom", C.c_double),
                ("n_nonneg_denom", C.c_uint64), ("ref_cross", C.c_double),
                ("key_xor", C.c_uint64), ("key_sum", C.c_uint64)]


def _load(name):
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    return C.CDLL(path)


_pt2 = None
_fci = None


def _libs():
    global _pt2, _fci
    if _pt2 is None:
        _pt2 = _load("liborc_pt2.so")
        S = C.POINTER(_System)
        _pt2.orc_key_words.argtypes = [C.c_int]
        _pt2.orc_key_words.restype = C.c_int
        _pt2.orc_diag.argtypes = [S, _u64p]
        _pt2.orc_diag.restype = C.c_double
        _pt2.orc_hij.argtypes = [S, _u64p, _u64p]
        _pt2.orc_hij.restype = C.c_double
        _pt2.orc_pt2.argtypes = [S, _u64p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_int,
                                 _u32p, C.c_int, C.c_int, C.POINTER(_Result), _f64p]
        _pt2.orc_pt2.restype = C.c_int
        _pt2.orc_emit.argtypes = [S, _u64p, _f64p, C.c_int64, C.c_double, C.c_int, C.c_uint32,
                                  _u64p, _f64p, C.c_int64]
        _pt2.orc_emit.restype = C.c_int64
        _pt2.orc_numerators.argtypes = [S, _u64p, _f64p, C.c_int64, C.c_int, C.c_uint32,
                                        _u64p, _f64p, C.c_int64]
        _pt2.orc_numerators.restype = C.c_int64
        _pt2.orc_diag_many.argtypes = [S, _u64p, C.c_int64, _f64p, C.c_int]
        _pt2.orc_diag_many.restype = None
        _pt2.orc_denominator_many.argtypes = [S, _u64p, C.c_int64, C.c_double, _f64p]
        _pt2.orc_denominator_many.restype = None
        _pt2.orc_hrr.argtypes = [S, _u64p, C.c_int64, _f64p]
        _pt2.orc_hrr.restype = None
        _pt2.orc_expectation.argtypes = [S, _u64p, _f64p, C.c_int64, C.c_int]
        _pt2.orc_expectation.restype = C.c_double
        _pt2.orc_parts.argtypes = [C.c_int, _u64p, C.c_int64, C.c_int, _u32p]
        _pt2.orc_parts.restype = None
        _pt2.orc_zobrist_table.argtypes = [C.c_int, _u64p]
        _pt2.orc_zobrist_table.restype = None
        _pt2.orc_splitmix64_stream.argtypes = [C.c_uint64, C.c_int, _u64p]
        _pt2.orc_splitmix64_stream.restype = None
        _pt2.orc_key_mix.argtypes = [_u64p, C.c_int]
        _pt2.orc_key_mix.restype = C.c_uint64
    if _fci is None:
        _fci = _load("liborc_fci.so")
        S = C.POINTER(_System)
        _fci.fb_dim.argtypes = [C.c_int, C.c_int, C.c_int]
        _fci.fb_dim.restype = C.c_int64
        _fci.fb_index_of_key.argtypes = [S, _u64p]
        _fci.fb_index_of_key.restype = C.c_int64
        _fci.fb_key_of_index.argtypes = [S, C.c_int64, _u64p]
        _fci.fb_key_of_index.restype = None
        _fci.fb_h_times.argtypes = [S, _u64p, _f64p, C.c_int64, _f64p]
        _fci.fb_h_times.restype = None
        _fci.fb_diag_many.argtypes = [S, _i64p, C.c_int64, _f64p, C.c_int]
        _fci.fb_diag_many.restype = None
        _fci.fb_dense.argtypes = [S, _f64p]
        _fci.fb_dense.restype = None
    return _pt2, _fci


def _ptr(a, t):
    return a.ctypes.data_as(t)


def key_words(norb: int) -> int:
    return (2 * norb + 63) // 64


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class _Base:
    def __init__(self, h, eri, norb, nalpha, nbeta):
        _libs()
        self.h = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(norb, norb))
        self.eri = np.ascontiguousarray(np.asarray(eri, dtype=np.float64).reshape(-1))
        assert self.eri.size == norb ** 4
        self.norb, self.nalpha, self.nbeta = norb, nalpha, nbeta
        self.W = key_words(norb)
        self._sys = _System(norb, nalpha, nbeta, _ptr(self.h, _f64p), _ptr(self.eri, _f64p))

    def _keys(self, keys):
        k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
        return k.reshape(-1, self.W)


class Oracle(_Base):
    """Plain FP64 PT2 oracle (Algorithm 1 and Algorithm 2 of the paper)."""

    def pt2(self, dets, c, e0, cutoff=0.0, log2p=0, parts=None, nthreads=None):
        """Returns (result dict, per-subset energies in the order of `parts`)."""
        lib, _ = _libs()
        d = self._keys(dets)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        assert len(cc) == len(d)
        nthreads = nthreads or default_threads()
        if parts is None:
            np_ = 1 << log2p
            pp = None
        else:
            pp = np.ascontiguousarray(np.asarray(parts, dtype=np.uint32))
            np_ = len(pp)
        res = _Result()
        ep = np.zeros(np_, dtype=np.float64)
        rc = lib.orc_pt2(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d), float(e0),
                         float(cutoff), int(log2p), None if pp is None else _ptr(pp, _u32p),
                         np_, int(nthreads), C.byref(res), _ptr(ep, _f64p))
        if rc == -2:
            raise ValueError("duplicate reference determinants")
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        out = {f: getattr(res, f) for f, _ in _Result._fields_}
        return out, ep

    def emit(self, dets, c, cutoff=0.0, log2p=0, part=0):
        lib, _ = _libs()
        d = self._keys(dets)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        n = lib.orc_emit(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d), cutoff,
                         log2p, part, None, None, 0)
        keys = np.zeros((max(n, 1), self.W), dtype=np.uint64)
        vals = np.zeros(max(n, 1), dtype=np.float64)
        lib.orc_emit(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d), cutoff,
                     log2p, part, _ptr(keys, _u64p), _ptr(vals, _f64p), n)
        return keys[:n], vals[:n]

    def numerators(self, dets, c, log2p=0, part=0):
        lib, _ = _libs()
        d = self._keys(dets)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        n = lib.orc_numerators(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d),
                               log2p, part, None, None, 0)
        keys = np.zeros((max(n, 1), self.W), dtype=np.uint64)
        nums = np.zeros(max(n, 1), dtype=np.float64)
        lib.orc_numerators(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d),
                           log2p, part, _ptr(keys, _u64p), _ptr(nums, _f64p), n)
        return keys[:n], nums[:n]

    def diag(self, keys, nthreads=None):
        lib, _ = _libs()
        k = self._keys(keys)
        out = np.zeros(len(k), dtype=np.float64)
        if len(k):
            lib.orc_diag_many(C.byref(self._sys), _ptr(k, _u64p), len(k), _ptr(out, _f64p),
                              int(nthreads or default_threads()))
        return out

    def denominators(self, keys, e0):
        """E0 - H_aa of each key as one compensated sum (exact to a few ulps
        of the difference itself)."""
        lib, _ = _libs()
        k = self._keys(keys)
        out = np.zeros(len(k), dtype=np.float64)
        if len(k):
            lib.orc_denominator_many(C.byref(self._sys), _ptr(k, _u64p), len(k), float(e0),
                                     _ptr(out, _f64p))
        return out

    def hij(self, ki, kj):
        lib, _ = _libs()
        a = self._keys(ki)[0].copy()
        b = self._keys(kj)[0].copy()
        return lib.orc_hij(C.byref(self._sys), _ptr(a, _u64p), _ptr(b, _u64p))

    def hrr(self, dets):
        lib, _ = _libs()
        d = self._keys(dets)
        H = np.zeros((len(d), len(d)), dtype=np.float64)
        lib.orc_hrr(C.byref(self._sys), _ptr(d, _u64p), len(d), _ptr(H, _f64p))
        return H

    def expectation(self, dets, c, nthreads=None):
        lib, _ = _libs()
        d = self._keys(dets)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        return lib.orc_expectation(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d),
                                   int(nthreads or default_threads()))


def zobrist_table(norb: int) -> np.ndarray:
    lib, _ = _libs()
    R = np.zeros(2 * norb, dtype=np.uint64)
    lib.orc_zobrist_table(norb, _ptr(R, _u64p))
    return R


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    lib, _ = _libs()
    out = np.zeros(n, dtype=np.uint64)
    lib.orc_splitmix64_stream(seed, n, _ptr(out, _u64p))
    return out


def parts_of(norb: int, keys, log2p: int) -> np.ndarray:
    lib, _ = _libs()
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).reshape(-1, key_words(norb))
    out = np.zeros(len(k), dtype=np.uint32)
    lib.orc_parts(norb, _ptr(k, _u64p), len(k), log2p, _ptr(out, _u32p))
    return out


def key_mix(keys, norb: int) -> np.ndarray:
    lib, _ = _libs()
    W = key_words(norb)
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).reshape(-1, W)
    return np.array([lib.orc_key_mix(_ptr(k[i].copy(), _u64p), W) for i in range(len(k))],
                    dtype=np.uint64)


class Brute(_Base):
    """Literal second-quantised H over the full-CI space (pins the oracle)."""

    def dim(self):
        _, lib = _libs()
        return lib.fb_dim(self.norb, self.nalpha, self.nbeta)

    def index_of(self, keys):
        _, lib = _libs()
        k = self._keys(keys)
        return np.array([lib.fb_index_of_key(C.byref(self._sys), _ptr(k[i].copy(), _u64p))
                         for i in range(len(k))], dtype=np.int64)

    def keys_of(self, idx):
        _, lib = _libs()
        idx = np.asarray(idx, dtype=np.int64)
        out = np.zeros((len(idx), self.W), dtype=np.uint64)
        for i, x in enumerate(idx):
            row = np.zeros(self.W, dtype=np.uint64)
            lib.fb_key_of_index(C.byref(self._sys), int(x), _ptr(row, _u64p))
            out[i] = row
        return out

    def h_times(self, dets, c):
        _, lib = _libs()
        d = self._keys(dets)
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        v = np.zeros(self.dim(), dtype=np.float64)
        lib.fb_h_times(C.byref(self._sys), _ptr(d, _u64p), _ptr(cc, _f64p), len(d), _ptr(v, _f64p))
        return v

    def diag(self, idx, nthreads=None):
        _, lib = _libs()
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        out = np.zeros(len(idx), dtype=np.float64)
        if len(idx):
            lib.fb_diag_many(C.byref(self._sys), _ptr(idx, _i64p), len(idx), _ptr(out, _f64p),
                             int(nthreads or default_threads()))
        return out

    def dense(self):
        _, lib = _libs()
        n = self.dim()
        H = np.zeros((n, n), dtype=np.float64)
        lib.fb_dense(C.byref(self._sys), _ptr(H, _f64p))
        return H

    def pt2(self, dets, c, e0):
        """sum over a outside R with (Hc)_a != 0 of (Hc)_a^2 / (E0 - H_aa)."""
        v = self.h_times(dets, c)
        ref_idx = self.index_of(dets)
        mask = np.ones(len(v), dtype=bool)
        mask[ref_idx] = False
        ext = np.nonzero(mask & (v != 0.0))[0]
        haa = self.diag(ext)
        return float(np.sum(v[ext] ** 2 / (e0 - haa))), len(ext)
