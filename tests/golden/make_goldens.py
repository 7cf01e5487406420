"""Write the stored FP64-oracle results that the GPU parity tests compare
against (calls only synth and oracle; test infrastructure).

Each case is an Epstein-Nesbet PT2 evaluation (the energy of Section II by
Algorithm 1, restricted to listed subsets of a 2^k hash split as in
Algorithm 2) of one of the synthetic workloads, on the stored inputs.  The
oracle runs it on this host with its compensated denominators; the energy
of each subset, the total, the counts and the key checksums are written to
``oracle_goldens.json`` with every float as a hex string, so the stored value
is the oracle's bit for bit.

Large cases are cut into several oracle calls of a few subsets each (the
oracle holds every record of the subsets it evaluates in host memory); the
calls' results are combined here in subset order.

Usage: python tests/golden/make_goldens.py [case ...] [--threads N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_goldens.json")

# name: (workload, number of leading references or None for all, log2 of the
# split, subsets evaluated (None: all), subsets per oracle call)
CASES = {
    # the whole of workload C2: every one of its 1,297,500,000 contributions
    "c2_full": ("c2", None, 5, None, 8),
    # the first 2,000 references of C3 (2,198,644,000 contributions)
    "c3_sample2000": ("c3", 2000, 6, None, 8),
    # eight subsets of the 4096-way split of the whole of C3
    "c3_parts12": ("c3", None, 12, [0, 777, 1365, 2048, 2730, 3001, 3500, 4095], 8),
    # the first 300 references of C5 (959,326,200 contributions)
    "c5_sample300": ("c5", 300, 5, None, 8),
    # the eight subsets 40..47 of the 4096-way split of the whole of C5, which
    # together are subset 5 of its 512-way split
    "c5_parts12": ("c5", None, 12, list(range(40, 48)), 2),
}


def load(name):
    w = synth.WORKLOADS[name]
    h, eri, rng = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(os.path.join(HERE, f"inputs_{name}.npz"))
    dets, e0 = f["dets"], float(f["e0"])
    c = f["c"] if "c" in f else synth.decaying_coefficients(w.n_ref, w.decay,
                                                            synth.draw_signs(rng, w.n_ref))
    return w, h, eri, dets, c, e0


def neumaier(values):
    s, comp = 0.0, 0.0
    for x in values:
        t = s + x
        comp += (s - t) + x if abs(s) >= abs(x) else (x - t) + s
        s = t
    return s + comp


def run_case(name, threads):
    wl, nref, log2p, parts, per_call = CASES[name]
    w, h, eri, dets, c, e0 = load(wl)
    if nref is not None:
        dets, c = dets[:nref], c[:nref]
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    plist = list(range(1 << log2p)) if parts is None else list(parts)
    t0 = time.time()
    e_parts, results = [], []
    for i in range(0, len(plist), per_call):
        chunk = plist[i:i + per_call]
        res, ep = O.pt2(dets, c, e0, log2p=log2p, parts=chunk, nthreads=threads)
        results.append(res)
        e_parts.extend(float(x) for x in ep)
        print(f"{name}: subsets {chunk[0]}..{chunk[-1]} done, {time.time() - t0:.0f} s", flush=True)
    tot = {k: int(sum(r[k] for r in results)) for k in
           ("n_contrib", "n_kept", "n_unique", "n_external", "n_in_ref_hit", "n_nonneg_denom")}
    kx, ks = 0, 0
    for r in results:
        kx ^= int(r["key_xor"])
        ks = (ks + int(r["key_sum"])) % (1 << 64)
    e_total = neumaier(e_parts)
    return {
        "workload": wl, "n_ref": int(len(dets)), "log2p": log2p, "parts": plist,
        "e0_hex": float(e0).hex(),
        "e_pt2": e_total, "e_pt2_hex": e_total.hex(),
        "e_parts_hex": [x.hex() for x in e_parts],
        "ref_cross_hex": float(sum(r["ref_cross"] for r in results)).hex(),
        "min_abs_denom_hex": float(min(r["min_abs_denom"] for r in results)).hex(),
        "key_xor": f"{kx:016x}", "key_sum": f"{ks:016x}",
        **tot,
        "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": threads,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    names = a.cases or list(CASES)
    for n in names:
        entry = run_case(n, a.threads)
        stored = json.load(open(OUT)) if os.path.exists(OUT) else {}
        stored[n] = entry
        with open(OUT, "w") as f:
            json.dump(stored, f, indent=1, sort_keys=True)
        print(json.dumps({k: entry[k] for k in ("workload", "n_ref", "e_pt2", "n_contrib",
                                                "n_external", "oracle_seconds")}), flush=True)


if __name__ == "__main__":
    main()
