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

