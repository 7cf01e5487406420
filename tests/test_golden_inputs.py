"""The stored inputs come from the committed generator: regenerating the
smallest workload (C1, its eigenvector reference) reproduces the stored file."""
import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_inputs_regenerate(tmp_path):
    spec = importlib.util.spec_from_file_location("make_inputs", os.path.join(HERE, "golden", "make_inputs.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    mk.make("c1", str(tmp_path))
    new = np.load(tmp_path / "inputs_c1.npz")
    old = np.load(os.path.join(HERE, "golden", "inputs_c1.npz"))
    assert np.array_equal(new["dets"], old["dets"])
    # an eigensolver may round differently elsewhere; the stored E0 and c are its output here
    np.testing.assert_allclose(new["e0"], old["e0"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(new["c"], old["c"], rtol=0, atol=1e-10)


def test_serving_e0_regenerates():
    """The stored E0 of the three smallest serving requests equals <c|H|c>
    recomputed from the request's seed, as the serving generator does."""
    import json
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import oracle
    import synth
    stored = {r["index"]: r["e0"] for r in json.load(open(os.path.join(HERE, "golden", "serving_requests.json")))}
    reqs = synth.serving_requests()
    reqs.sort(key=lambda r: r.n_ref * synth.n_excitations_per_det(r.norb, r.nalpha, r.nalpha))
    for r in reqs[:3]:
        h, eri, dets, c = synth.request_inputs(r)
        e0 = oracle.Oracle(h, eri, r.norb, r.nalpha, r.nalpha).expectation(dets, c)
        assert abs(e0 - stored[r.index]) <= 1e-12 * abs(stored[r.index]), (r.index, e0, stored[r.index])
