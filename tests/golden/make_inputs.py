"""Write the stored inputs of the synthetic workloads (calls only synth and oracle).

For each workload the integrals and coefficient signs are regenerated from
the seed by ``synth``; what needs matrix elements is computed here by the
CPU oracle and stored:

* the reference determinants, in rank order: the ``n_ref`` lowest diagonal
  energies H_aa of the pool (HF plus excitations up to ``pool_rank``), HF
  forced to rank 0, ties broken by the bitstring;
* E0 = <c|H|c> (or, for an eigenvector reference, the lowest eigenvalue of
  H_RR together with its eigenvector c, sign fixed by c_HF > 0).

Usage: python tests/golden/make_inputs.py c1 c2
"""
from __future__ import annotations

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


def make(name: str, outdir: str = HERE) -> dict:
    w = synth.WORKLOADS[name]
    t0 = time.time()
    h, eri, rng = synth.make_integrals(w.norb, w.n_chol, w.seed)
    pool = synth.excitation_pool(w.norb, w.nalpha, w.nbeta, w.pool_rank)
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    energies = O.diag(pool)
    sel = synth.select_lowest(pool, energies, w.n_ref, force_first=0)
    dets = np.ascontiguousarray(pool[sel])
    out = {"dets": dets}
    if w.decay is None:
        H = O.hrr(dets)
        vals, vecs = np.linalg.eigh(H)
        c = vecs[:, 0] * (1.0 if vecs[0, 0] > 0 else -1.0)
        e0 = float(vals[0])
        out["c"] = c
    else:
        signs = synth.draw_signs(rng, w.n_ref)
        c = synth.decaying_coefficients(w.n_ref, w.decay, signs)
        e0 = float(O.expectation(dets, c))
    out["e0"] = np.float64(e0)
    np.savez_compressed(os.path.join(outdir, f"inputs_{name}.npz"), **out)
    meta = {"workload": name, "pool": int(len(pool)), "n_ref": int(w.n_ref), "e0": e0,
            "e0_hex": float(e0).hex(), "seconds": round(time.time() - t0, 1)}
    print(json.dumps(meta), flush=True)
    return meta


if __name__ == "__main__":
    names = sys.argv[1:] or ["c1", "c2"]
    summary_path = os.path.join(HERE, "inputs.json")
    summary = json.load(open(summary_path)) if os.path.exists(summary_path) else {}
    for n in names:
        summary[n] = make(n)
    with open(summary_path, "w") as f:
        json.dump(summary, f, indent=1, sort_keys=True)
