"""Packed FP32 hash records: the engine's 48-bit code of a record's parent
and flipped spin-orbitals (hash_pack / hash_unpack in csrc/pt2_internal.h)
must give back the auxiliary word exactly for every excitation kind, every
spatial orbital up to the largest packed norb, and parents up to the largest
packed index.  A host program built from the engine header with hipcc runs
the check (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1808_02049_amd", "csrc")

SRC = r"""
#include "pt2_internal.h"
#include <cstdio>
using namespace pt2;
static long bad = 0, ok = 0;
static void check(uint64_t aux, int norb)
{
    const uint64_t p = hash_pack(aux, norb);
    if (p >> 48) { bad++; return; }
    if (hash_unpack(p, norb) != aux) {
        if (bad++ < 5) printf("norb %d aux %llx -> %llx\n", norb, (unsigned long long)aux,
                              (unsigned long long)hash_unpack(p, norb));
    } else {
        ok++;
    }
}
static uint64_t word(uint64_t parent, uint32_t f0, uint32_t f1, uint32_t f2, uint32_t f3)
{
    return parent << 32 | (uint64_t)(f0 | f1 << 8 | f2 << 16) | (uint64_t)f3 << 24;
}
int main()
{
    const int norbs[] = {2, 3, 7, 40, 100, 126};
    const uint64_t parents[] = {0, 1, 77777, (1ull << 19) - 1};
    for (int norb : norbs)
        for (uint64_t par : parents) {
            const uint32_t n = (uint32_t)norb;
            for (uint32_t r = 0; r < n; r++)
                for (uint32_t a = 0; a < n; a++) {
                    if (r == a)
                        continue;
                    check(word(par, n + r, n + a, FLIP_NONE, FLIP_NONE), norb);  // alpha single
                    check(word(par, r, a, FLIP_NONE, FLIP_NONE), norb);          // beta single
                }
            // doubles: every quadruple for small norb, a stride through them otherwise
            const uint32_t step = n <= 7 ? 1 : 13;
            for (uint32_t r1 = 0; r1 < n; r1 += 1)
                for (uint32_t r2 = 0; r2 < n; r2 += step)
                    for (uint32_t a1 = 0; a1 < n; a1 += step)
                        for (uint32_t a2 = (r1 * 7 + r2) % step; a2 < n; a2 += step) {
                            check(word(par, n + r1, n + a1, r2, a2), norb);  // alpha-beta
                            if (r1 < r2 && a1 < a2) {
                                check(word(par, n + r1, n + r2, n + a1, n + a2), norb);  // alpha-alpha
                                check(word(par, r1, r2, a1, a2), norb);                  // beta-beta
                            }
                        }
        }
    printf("ok=%ld bad=%ld\n", ok, bad);
    return bad != 0;
}
"""


def test_hash_pack_round_trip(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    src = tmp_path / "pack.cpp"
    src.write_text(SRC)
    exe = tmp_path / "pack"
    r = subprocess.run([hipcc, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad=0" in out.stdout
