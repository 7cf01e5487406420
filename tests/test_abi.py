"""The C-ABI library: it loads, exports every entry point of include/pt2.h,
and rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pt2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt2_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    import paper_1808_02049_amd as pt2
    lib = C.CDLL(pt2.LIB_PATH)
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pt2.EXPORTED)


def test_struct_sizes_match_header_layout():
    import paper_1808_02049_amd as pt2
    o = pt2.default_options()
    assert o.struct_size == C.sizeof(pt2.Options)
    assert o.log2_partitions == -1 and o.precision == pt2.PT2_FP64 and o.cutoff == 0.0


def test_field_offsets_match_header(tmp_path):
    """Every field of the ctypes mirrors of pt2_options and pt2_result sits at
    the offset the C compiler gives it from include/pt2.h, and the sizes agree
    (a field missing on either side moves an offset or the size)."""
    import shutil
    import subprocess
    import paper_1808_02049_amd as pt2
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = (("pt2_options", pt2.Options), ("pt2_result", pt2.Result))
    lines = ["#include <stdio.h>", '#include "pt2.h"', "int main(void) {"]
    for name, cls in structs:
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {(a, b): int(c) for a, b, c in (line.split() for line in out.splitlines())}
    for name, cls in structs:
        assert got[(name, "sizeof")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def test_import_fails_without_the_library(tmp_path):
    """No CPU fallback: the binding refuses to import when libpt2.so is absent."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1808_02049_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1808_02049_amd", "__init__.py"), pkg)
    r = subprocess.run([sys.executable, "-c", "import paper_1808_02049_amd"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is missing" in r.stderr


def test_key_words():
    import paper_1808_02049_amd as pt2
    assert [pt2.key_words(n) for n in (1, 12, 32, 33, 40, 64, 76, 100, 128)] == [1, 1, 1, 2, 2, 2, 3, 4, 4]


def test_key_form_rule():
    """The record form a context takes (pt2_key_form, host only): each form is
    priced by the bytes its records move through the digit passes, and a
    compressed form is taken only when it saves 30% against the bitstring."""
    import paper_1808_02049_amd as pt2
    kf = pt2.key_form
    # (4a,4b)/12: 18-bit ranks sort in as many passes as the 24-bit strings
    assert kf(12, 4, 4) == ("bitstring", 24) and kf(12, 4, 4, "fp32") == ("bitstring", 24)
    # (10a,10b)/40, FP64: 16-byte rank records in 8 passes save 29% of ten
    # 18-byte bitstring passes; FP32: 60-bit ranks (eight 12-byte passes) tie
    # with six packed 16-byte hash passes, and a tie takes hash records
    assert kf(40, 10, 10) == ("bitstring", 80)
    assert kf(40, 10, 10, "fp32") == ("hash", 64)
    # an explicit hash width leaves the unpacked 20-byte FP32 records
    assert kf(40, 10, 10, "fp32", hash_bits=40) == ("rank", 60)
    # (14a,14b)/76 and (18a,18b)/100: hash records in both precisions
    for norb, n in ((76, 14), (100, 18)):
        for prec in ("fp64", "fp32", "fp32-arith"):
            assert kf(norb, n, n, prec) == ("hash", 64)
    # served shapes
    assert kf(24, 5, 5, "fp32") == ("rank", 32)
    assert kf(28, 6, 6, "fp32") == ("bitstring", 56)
    assert kf(54, 12, 12, "fp32") == ("hash", 64)
    assert kf(54, 12, 12) == ("rank", 78)
    # forced forms, and rank keys where the ranks do not fit 64 bits
    assert kf(40, 10, 10, compress_keys=0) == ("bitstring", 80)
    assert kf(40, 10, 10, compress_keys=1) == ("rank", 60)
    assert kf(40, 10, 10, compress_keys=2) == ("hash", 64)
    assert kf(100, 18, 18, compress_keys=1) == ("bitstring", 200)
    for bad in (dict(norb=0, nalpha=0, nbeta=0), dict(norb=12, nalpha=13, nbeta=0),
                dict(norb=12, nalpha=4, nbeta=4, compress_keys=3), dict(norb=12, nalpha=4, nbeta=4, hash_bits=65)):
        with pytest.raises(pt2.PT2Error):
            kf(**bad)


def test_key_forms_of_the_served_workload():
    """The 200 served requests (FP32 payloads): 83 take packed hash records
    (83% of the contributions), 73 rank keys and 44 bitstrings."""
    import collections
    import paper_1808_02049_amd as pt2
    import synth
    count, share = collections.Counter(), collections.Counter()
    for r in synth.serving_requests():
        form, _ = pt2.key_form(r.norb, r.nalpha, r.nalpha, "fp32")
        count[form] += 1
        share[form] += r.n_ref * synth.n_excitations_per_det(r.norb, r.nalpha, r.nalpha)
    assert count == {"hash": 83, "rank": 73, "bitstring": 44}
    assert 0.82 < share["hash"] / sum(share.values()) < 0.84


def _sys(norb=4):
    import synth
    h, eri, _ = synth.make_integrals(norb, 4, 1)
    return h, eri


@pytest.mark.parametrize("kw,match", [
    (dict(norb=0), "norb"), (dict(norb=129), "norb"), (dict(nalpha=5), "electron"),
    (dict(nbeta=-1), "electron")])
def test_create_rejects_bad_sizes(kw, match):
    import paper_1808_02049_amd as pt2
    args = dict(norb=4, nalpha=2, nbeta=2)
    args.update(kw)
    n = max(args["norb"], 1)
    h = np.eye(n)
    eri = np.zeros(n ** 4)
    o = pt2.default_options()
    ctx = C.c_void_p()
    rc = pt2._lib.pt2_create(h.ctypes.data_as(C.POINTER(C.c_double)),
                             eri.ctypes.data_as(C.POINTER(C.c_double)), args["norb"],
                             args["nalpha"], args["nbeta"], C.byref(o), C.byref(ctx))
    assert rc == pt2.PT2_E_INVALID
    assert match in pt2._lib.pt2_last_error().decode()


def test_create_rejects_asymmetric_integrals():
    import paper_1808_02049_amd as pt2
    h, eri = _sys()
    bad = eri.copy().reshape(4, 4, 4, 4)
    bad[0, 1, 2, 3] += 1e-6
    with pytest.raises(pt2.PT2Error) as e:
        pt2.Context(h, bad, 4, 2, 2)
    assert e.value.code == pt2.PT2_E_INVALID and "symmetric" in str(e.value)
    hb = h.copy()
    hb[0, 1] += 1e-3
    with pytest.raises(pt2.PT2Error) as e:
        pt2.Context(hb, eri, 4, 2, 2)
    assert e.value.code == pt2.PT2_E_INVALID


def test_bad_options_rejected():
    import paper_1808_02049_amd as pt2
    h, eri = _sys()
    with pytest.raises(pt2.PT2Error):
        pt2.Context(h, eri, 4, 2, 2, cutoff=-1.0)
    with pytest.raises(pt2.PT2Error):
        pt2.Context(h, eri, 4, 2, 2, log2_partitions=13)
    with pytest.raises(pt2.PT2Error):
        pt2.Context(h, eri, 4, 2, 2, compress_keys=2)
    with pytest.raises(pt2.PT2Error, match="hash_bits"):
        pt2.Context(h, eri, 4, 2, 2, hash_bits=65)
    with pytest.raises(pt2.PT2Error, match="hash_bits"):
        pt2.Context(h, eri, 4, 2, 2, hash_bits=-1)
    with pytest.raises(pt2.PT2Error, match="nalpha == nbeta"):
        pt2.Context(h, eri, 4, 2, 1, spin_flip=True)
    o = pt2.default_options()
    assert o.exclusion == 0
    o.exclusion = 2
    ctx = pt2._CTX()
    hh = np.ascontiguousarray(h, dtype=np.float64)
    ee = np.ascontiguousarray(eri, dtype=np.float64).reshape(-1)
    assert pt2._lib.pt2_create(hh.ctypes.data_as(pt2._f64p), ee.ctypes.data_as(pt2._f64p), 4, 2, 2,
                               pt2.C.byref(o), pt2.C.byref(ctx)) == pt2.PT2_E_INVALID
    o = pt2.default_options()
    o.precision = 3
    ctx = pt2._CTX()
    hh = np.ascontiguousarray(h, dtype=np.float64)
    ee = np.ascontiguousarray(eri, dtype=np.float64).reshape(-1)
    rc = pt2._lib.pt2_create(hh.ctypes.data_as(pt2._f64p), ee.ctypes.data_as(pt2._f64p), 4, 2, 2,
                             pt2.C.byref(o), pt2.C.byref(ctx))
    assert rc == pt2.PT2_E_INVALID
    o = pt2.default_options()
    o.spin_flip = 2
    ctx = pt2._CTX()
    rc = pt2._lib.pt2_create(hh.ctypes.data_as(pt2._f64p), ee.ctypes.data_as(pt2._f64p), 4, 2, 2,
                             pt2.C.byref(o), pt2.C.byref(ctx))
    assert rc == pt2.PT2_E_INVALID
    assert b"spin_flip" in pt2._lib.pt2_last_error()
    o = pt2.default_options()
    assert o.string_reuse == 1
    o.string_reuse = 3
    ctx = pt2._CTX()
    rc = pt2._lib.pt2_create(hh.ctypes.data_as(pt2._f64p), ee.ctypes.data_as(pt2._f64p), 4, 2, 2,
                             pt2.C.byref(o), pt2.C.byref(ctx))
    assert rc == pt2.PT2_E_INVALID
    assert b"string_reuse" in pt2._lib.pt2_last_error()


def test_evaluate_null_context_rejected():
    import paper_1808_02049_amd as pt2
    r = pt2.Result()
    r.struct_size = C.sizeof(pt2.Result)
    assert pt2._lib.pt2_evaluate(None, None, None, 0, 0.0, C.byref(r)) == pt2.PT2_E_INVALID
    r.struct_size = 3
    assert pt2._lib.pt2_poll(None, 1, C.byref(r)) == pt2.PT2_E_INVALID


def test_sort_records_argument_checks():
    import paper_1808_02049_amd as pt2
    k = np.zeros(4, dtype=np.uint64)
    p = np.zeros(4, dtype=np.float64)
    assert pt2._lib.pt2_sort_records(0, 5, 8, k.ctypes.data_as(C.POINTER(C.c_uint64)), p.ctypes.data, 8, 4) \
        == pt2.PT2_E_INVALID
    assert pt2._lib.pt2_sort_records(0, 1, 8, k.ctypes.data_as(C.POINTER(C.c_uint64)), p.ctypes.data, 2, 4) \
        == pt2.PT2_E_INVALID
    # n <= 1 is a no-op and needs no device
    assert pt2._lib.pt2_sort_records(0, 1, 8, k.ctypes.data_as(C.POINTER(C.c_uint64)), p.ctypes.data, 8, 1) \
        == pt2.PT2_OK


def test_no_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1808_02049_amd as pt2
    h, eri = _sys()
    with pytest.raises(pt2.PT2Error) as e:
        pt2.Context(h, eri, 4, 2, 2)
    assert e.value.code == pt2.PT2_E_DEVICE
