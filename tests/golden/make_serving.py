"""Write E0 = <c|H|c> of the 200 serving requests (calls only synth and oracle).

Each request's integrals, reference determinants (orbital-ladder rule) and
coefficients (+-exp(-0.002 rank), random signs, normalised) are regenerated
from its seed by synth; only E0 needs matrix elements and is stored here.

Usage: python tests/golden/make_serving.py
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = []
    t0 = time.time()
    for r in synth.serving_requests():
        h, eri, dets, c = synth.request_inputs(r)
        e0 = oracle.Oracle(h, eri, r.norb, r.nalpha, r.nalpha).expectation(dets, c)
        out.append({"index": r.index, "nalpha": r.nalpha, "norb": r.norb, "n_ref": r.n_ref,
                    "seed": r.seed, "e0": e0, "e0_hex": float(e0).hex()})
        if r.index % 20 == 0:
            print(r.index, round(time.time() - t0, 1), flush=True)
    with open(os.path.join(HERE, "serving_requests.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
