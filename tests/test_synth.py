"""The seeded input generator: layout conventions and the integral recipe."""
import math

import numpy as np
import pytest

import synth


@pytest.mark.parametrize("norb", [1, 12, 32, 33, 40, 64, 76, 100, 128])
def test_pack_unpack_roundtrip(norb):
    rng = np.random.default_rng(norb)
    a = rng.random((20, norb)) < 0.3
    b = rng.random((20, norb)) < 0.4
    k = synth.pack_keys(a, b, norb)
    assert k.shape == (20, synth.key_words(norb))
    a2, b2 = synth.unpack_keys(k, norb)
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    # beta orbital p is bit p, alpha orbital p is bit norb + p
    for i in range(3):
        val = sum(int(k[i, w]) << (64 * w) for w in range(k.shape[1]))
        ref = sum(1 << int(p) for p in np.nonzero(b[i])[0]) + sum(1 << (norb + int(p)) for p in np.nonzero(a[i])[0])
        assert val == ref


def test_integrals_exactly_eightfold_symmetric():
    h, eri, _ = synth.make_integrals(9, 12, 5)
    g = eri.reshape(9, 9, 9, 9)
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(g, g.transpose(perm))
    np.testing.assert_allclose(np.diag(h), -2.0 + 0.25 * np.arange(9))


def test_integral_recipe_statistics():
    h, eri, _ = synth.make_integrals(40, 64, 1002)
    off = h[np.triu_indices(40, 1)]
    assert abs(off.std() - 0.05) < 0.005
    g = eri.reshape(40, 40, 40, 40)
    # (pp|pp) = sum_L (B^L_pp)^2 has mean L * 0.01
    assert abs(np.mean([g[p, p, p, p] for p in range(40)]) - 0.64) < 0.15


def test_pool_sizes():
    assert len(synth.excitation_pool(12, 4, 4, 2)) == 1425
    # rank-3 pool of (10a,10b)/40 by formula (enumerating it takes seconds)
    C = math.comb
    n = 1 + 2 * 10 * 30 + 2 * C(10, 2) * C(30, 2) + 300 * 300 \
        + 2 * C(10, 3) * C(30, 3) + 2 * C(10, 2) * C(30, 2) * 300
    assert n == 12_849_151


def test_pool_is_hf_first_and_distinct():
    pool = synth.excitation_pool(8, 3, 2, 2)
    assert np.array_equal(pool[0], synth.hf_key(8, 3, 2))
    assert len({tuple(r) for r in pool}) == len(pool)


def test_select_lowest_ties_by_key_and_forced_first():
    keys = np.array([[5], [3], [9], [1]], dtype=np.uint64)
    e = np.array([1.0, 0.5, 0.5, 2.0])
    assert list(synth.select_lowest(keys, e, 4, force_first=0)) == [0, 1, 2, 3]
    assert list(synth.select_lowest(keys, e, 3, force_first=None)) == [1, 2, 0]


def test_coefficients_normalised_with_hf_positive():
    rng = np.random.default_rng(0)
    s = synth.draw_signs(rng, 1000)
    c = synth.decaying_coefficients(1000, 0.002, s)
    assert abs(np.dot(c, c) - 1.0) < 1e-14 and c[0] > 0
    assert np.all(np.abs(np.diff(np.abs(c))) >= 0) or np.all(np.diff(np.abs(c)) <= 0)


def test_stored_inputs_regenerate():
    import os
    f = np.load(os.path.join(os.path.dirname(__file__), "golden", "inputs_c2.npz"))
    w = synth.WORKLOADS["c2"]
    assert f["dets"].shape == (w.n_ref, 2)
    a, b = synth.unpack_keys(f["dets"], w.norb)
    assert np.all(a.sum(1) == 10) and np.all(b.sum(1) == 10)
    assert np.array_equal(f["dets"][0], synth.hf_key(40, 10, 10))
    assert len({tuple(r) for r in f["dets"]}) == w.n_ref


def _brute_ladder(norb, na, nb):
    """Every determinant with its total orbital-index displacement (itertools)."""
    import itertools
    rows = []
    for oa in itertools.combinations(range(norb), na):
        for ob in itertools.combinations(range(norb), nb):
            e = sum(o - i for i, o in enumerate(oa)) + sum(o - i for i, o in enumerate(ob))
            A = np.zeros((1, norb), bool)
            B = np.zeros((1, norb), bool)
            A[0, list(oa)] = True
            B[0, list(ob)] = True
            rows.append((e, tuple(int(x) for x in synth.pack_keys(A, B, norb)[0][::-1])))
    rows.sort()
    return rows


@pytest.mark.parametrize("norb,na,nb,n_ref", [(8, 3, 3, 50), (9, 4, 2, 200), (7, 2, 2, 441), (10, 5, 5, 1)])
def test_ladder_references_match_brute_force(norb, na, nb, n_ref):
    got = synth.ladder_references(norb, na, nb, n_ref)
    want = _brute_ladder(norb, na, nb)[:n_ref]
    assert got.shape == (n_ref, synth.key_words(norb))
    assert [tuple(int(x) for x in r[::-1]) for r in got] == [k for _, k in want]
    assert np.array_equal(got[0], synth.hf_key(norb, na, nb))


def test_serving_requests_recipe():
    reqs = synth.serving_requests()
    assert len(reqs) == 200
    assert all(5 <= r.nalpha <= 12 for r in reqs)
    assert all(round(2.0 * 2 * r.nalpha) <= r.norb <= round(2.5 * 2 * r.nalpha) for r in reqs)
    assert all(1000 <= r.n_ref <= 50000 for r in reqs)
    t = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert 150 < t[-1] < 250      # 200 exponential gaps of mean 1 s
    assert synth.serving_requests(rate_per_s=2.0)[-1].arrival_s == pytest.approx(t[-1] / 2)


def test_stored_serving_e0_regenerates():
    """The stored E0 of the three smallest requests equals the oracle's
    <c|H|c> on the regenerated inputs (catches drift in the request recipe)."""
    import json
    import os
    import oracle
    stored = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                         "serving_requests.json")))
    reqs = synth.serving_requests()
    assert [(r.index, r.nalpha, r.norb, r.n_ref, r.seed) for r in reqs] == \
        [(s["index"], s["nalpha"], s["norb"], s["n_ref"], s["seed"]) for s in stored]
    for r in sorted(reqs, key=lambda r: r.n_ref)[:3]:
        h, eri, dets, c = synth.request_inputs(r)
        e0 = oracle.Oracle(h, eri, r.norb, r.nalpha, r.nalpha).expectation(dets, c)
        s = stored[r.index]
        assert abs(e0 - s["e0"]) <= 1e-12 * abs(s["e0"])
        assert float.fromhex(s["e0_hex"]) == s["e0"]


@pytest.mark.parametrize("norb,n_el,sign", [(10, 3, 1), (10, 3, -1), (40, 5, 1), (70, 4, -1)])
def test_swap_symmetric_references_are_closed(norb, n_el, sign):
    """Every determinant's alpha/beta swap is in the set, with coefficient
    sign * c, and the coefficients are normalised."""
    dets, c = synth.swap_symmetric_references(norb, n_el, 25, 3 + norb, sign)
    a, b = synth.unpack_keys(dets, norb)
    assert (a.sum(axis=1) == n_el).all() and (b.sum(axis=1) == n_el).all()
    index = {tuple(int(x) for x in k): i for i, k in enumerate(dets)}
    assert len(index) == len(dets)
    for i, k in enumerate(synth.pack_keys(b, a, norb)):
        j = index[tuple(int(x) for x in k)]
        assert c[j] == sign * c[i] or (i == j and sign > 0)
    assert np.linalg.norm(c) == pytest.approx(1.0, abs=1e-15)
