"""Parity of the HIP engine with the FP64 CPU oracle, through the C-ABI.

Keys and counts must match bit for bit; FP64 energies within 1e-9 Eh and
FP32-payload energies within 1e-6 Eh of the FP64 oracle (the stated bars);
per-term payloads within a few ulp.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def pt2():
    _need_gpu()
    import paper_1808_02049_amd as m
    return m


def load(name):
    w = synth.WORKLOADS[name]
    h, eri, rng = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(os.path.join(HERE, "golden", f"inputs_{name}.npz"))
    dets, e0 = f["dets"], float(f["e0"])
    if "c" in f:
        c = f["c"]
    else:
        c = synth.decaying_coefficients(w.n_ref, w.decay, synth.draw_signs(rng, w.n_ref))
    return w, h, eri, dets, c, e0


@pytest.fixture(scope="module")
def c1(pt2):
    w, h, eri, dets, c, e0 = load("c1")
    ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, timing=True)
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    ref, _ = O.pt2(dets, c, e0)
    yield dict(w=w, h=h, eri=eri, dets=dets, c=c, e0=e0, ctx=ctx, O=O, ref=ref)
    ctx.close()


COUNT_KEYS = ("n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum",
              "n_nonneg_denom")


def assert_matches(got, ref, tol=1e-9, cross_tol=1e-11):
    print(f"E gpu={got['e_pt2']:.15f} oracle={ref['e_pt2']:.15f} dE={got['e_pt2'] - ref['e_pt2']:.2e}",
          flush=True)
    assert abs(got["e_pt2"] - ref["e_pt2"]) <= tol
    for k in COUNT_KEYS:
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert got["ref_cross"] == pytest.approx(ref["ref_cross"], abs=cross_tol)
    if ref["n_external"]:
        assert got["min_abs_denom"] == pytest.approx(ref["min_abs_denom"], rel=1e-12)


def sort_by_key(dets):
    W = dets.shape[1]
    return np.lexsort(tuple(dets[:, w] for w in range(W)))


# ---------------------------------------------------------------------------
# C1: (4a,4b)/12, 200 reference determinants, eigenvector reference

def test_c1_energy_host_inputs(c1):
    got = c1["ctx"].evaluate(c1["dets"], c1["c"], c1["e0"])
    assert_matches(got, c1["ref"])
    assert got["n_contrib"] == 284_800 and got["n_partitions"] == 1


def test_c1_energy_device_inputs(c1):
    import torch
    d = torch.from_numpy(c1["dets"].view(np.int64)).cuda()
    cc = torch.from_numpy(c1["c"]).cuda()
    got = c1["ctx"].evaluate(d, cc, c1["e0"])
    assert_matches(got, c1["ref"])


def test_c1_generated_records_match_oracle(c1):
    order = sort_by_key(c1["dets"])
    dets, c = c1["dets"][order], c1["c"][order]
    gk, gv = c1["ctx"].dump_records(dets, c, sorted=False)
    ok, ov = c1["O"].emit(dets, c)
    assert gk.shape == ok.shape
    assert np.array_equal(gk, ok)
    np.testing.assert_allclose(gv, ov, rtol=0, atol=4 * np.finfo(float).eps * np.abs(ov).max())


def test_c1_sorted_records_are_stable_sort(c1):
    order = sort_by_key(c1["dets"])
    dets, c = c1["dets"][order], c1["c"][order]
    gk, gv = c1["ctx"].dump_records(dets, c, sorted=False)
    sk, sv = c1["ctx"].dump_records(dets, c, sorted=True)
    idx = np.lexsort(tuple(gk[:, w] for w in range(gk.shape[1])))  # stable
    assert np.array_equal(sk, gk[idx])
    assert np.array_equal(sv, gv[idx])


def test_c1_numerators_match_oracle(c1):
    gk, gn, gin = c1["ctx"].dump_numerators(c1["dets"], c1["c"])
    ok, on = c1["O"].numerators(c1["dets"], c1["c"])
    assert np.array_equal(gk, ok)
    np.testing.assert_allclose(gn, on, rtol=0, atol=1e-14)
    refset = {tuple(r) for r in c1["dets"]}
    assert np.array_equal(gin, np.array([tuple(k) in refset for k in ok]))


def test_c1_input_order_does_not_matter(c1):
    perm = np.random.default_rng(0).permutation(len(c1["dets"]))
    a = c1["ctx"].evaluate(c1["dets"], c1["c"], c1["e0"])
    b = c1["ctx"].evaluate(c1["dets"][perm], c1["c"][perm], c1["e0"])
    assert a["e_pt2"] == b["e_pt2"]


def test_c1_deterministic(c1):
    a = c1["ctx"].evaluate(c1["dets"], c1["c"], c1["e0"])
    b = c1["ctx"].evaluate(c1["dets"], c1["c"], c1["e0"])
    assert a["e_pt2"] == b["e_pt2"] and a["key_sum"] == b["key_sum"]


@pytest.mark.parametrize("log2p", [1, 3, 6])
def test_c1_forced_split(pt2, c1, log2p):
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, log2_partitions=log2p)
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    assert got["n_partitions"] == 1 << log2p
    assert_matches(got, c1["ref"])
    ctx.close()


def test_c1_bucket_tables_equal_built_buckets(pt2, c1):
    """Targeted generation and its count pass read the references' bucket
    tables, built once per call, unless those would take more than 1/32 of
    the budget; then each subset builds its own.  Both forms give the same
    records, so every result is bit-identical."""
    fields = ("e_pt2", "n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum",
              "n_partitions", "min_abs_denom", "ref_cross")
    res = []
    for budget in (0, 100_000):
        ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, log2_partitions=3, max_partition_bytes=budget)
        got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
        _, ep = ctx.evaluate_parts(c1["dets"], c1["c"], c1["e0"], 3, [6, 1, 3])
        res.append((got, ep))
        ctx.close()
    (a, ea), (b, eb) = res
    for k in fields:
        assert a[k] == b[k], (k, a[k], b[k])
    assert list(ea) == list(eb)
    assert_matches(a, c1["ref"])


def test_c1_small_budget_makes_planner_split(pt2, c1):
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, max_partition_bytes=2_000_000)
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    assert got["n_partitions"] > 1
    assert_matches(got, c1["ref"])
    ctx.close()


def test_c1_listed_subsets_match_oracle(c1):
    parts = [0, 5, 17, 31]
    got, ep = c1["ctx"].evaluate_parts(c1["dets"], c1["c"], c1["e0"], 5, parts)
    ref, rp = c1["O"].pt2(c1["dets"], c1["c"], c1["e0"], log2p=5, parts=parts)
    np.testing.assert_allclose(ep, rp, rtol=0, atol=1e-11)
    assert_matches(got, ref)


def test_c1_listed_subsets_any_order_and_no_repeats(pt2, c1):
    """Listed subsets in any order give the energies of those subsets (the
    count pass counts only the listed ones); a subset listed twice is
    rejected."""
    parts = [17, 0, 31, 5]
    got, ep = c1["ctx"].evaluate_parts(c1["dets"], c1["c"], c1["e0"], 5, parts)
    ref, rp = c1["O"].pt2(c1["dets"], c1["c"], c1["e0"], log2p=5, parts=parts)
    np.testing.assert_allclose(ep, rp, rtol=0, atol=1e-11)
    assert_matches(got, ref)
    with pytest.raises(pt2.PT2Error) as e:
        c1["ctx"].evaluate_parts(c1["dets"], c1["c"], c1["e0"], 5, [3, 9, 3])
    assert e.value.code == pt2.PT2_E_INVALID


def test_c1_fp32_payload_form(pt2, c1):
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, precision="fp32")
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    print("fp32 dE", got["e_pt2"] - c1["ref"]["e_pt2"], flush=True)
    assert abs(got["e_pt2"] - c1["ref"]["e_pt2"]) <= 1e-6
    for k in ("n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum"):
        assert got[k] == c1["ref"][k]
    ctx.close()


def test_c1_fp32_payload_records_are_rounded_fp64_terms(pt2, c1):
    """The FP32-payload form computes H_ai c_i in FP64 and rounds it once:
    every stored term is the oracle's term rounded to FP32 (within one FP32
    ulp, as the FP64 sums may differ in their last bits)."""
    order = sort_by_key(c1["dets"])
    dets, c = c1["dets"][order], c1["c"][order]
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, precision="fp32")
    gk, gv = ctx.dump_records(dets, c)
    ctx.close()
    ok, ov = c1["O"].emit(dets, c)
    assert np.array_equal(gk, ok)
    o32 = ov.astype(np.float32)
    assert np.all(gv.astype(np.float32) == gv)               # stored as FP32
    ulp = np.spacing(np.abs(o32)).astype(np.float64)
    assert np.all(np.abs(gv - o32.astype(np.float64)) <= ulp)
    assert np.mean(gv == o32.astype(np.float64)) > 0.99


def test_c1_fp32_arith_form(pt2, c1):
    """FP32 integrals and arithmetic: error bounded relative to E_PT2."""
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, precision="fp32-arith")
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    ctx.close()
    ref = c1["ref"]
    print("fp32-arith dE", got["e_pt2"] - ref["e_pt2"], flush=True)
    assert abs(got["e_pt2"] - ref["e_pt2"]) <= 1e-6 * abs(ref["e_pt2"])
    for k in ("n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum"):
        assert got[k] == ref[k]


def test_c1_subtraction_exclusion(pt2, c1):
    """C1's coefficients are an eigenvector of H in the reference space, so
    keeping the reference determinants and subtracting sum_i c_i^2 (E0 - H_ii)
    gives the same energy as excluding them by search."""
    for log2p, mode in ((-1, 0), (3, 0), (-1, 2), (2, 2)):
        ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, exclusion="subtract", log2_partitions=log2p,
                          compress_keys=mode)
        got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
        ctx.close()
        ref = c1["ref"]
        print("subtraction dE", got["e_pt2"] - ref["e_pt2"], flush=True)
        assert abs(got["e_pt2"] - ref["e_pt2"]) <= 1e-9
        assert got["n_in_ref_hit"] == 0 and got["n_unique"] == ref["n_unique"]
        assert got["n_external"] == ref["n_external"] + ref["n_in_ref_hit"]


def test_c1_cutoff(pt2, c1):
    k, v = c1["O"].emit(c1["dets"], c1["c"])
    cut = float(np.quantile(np.abs(v), 0.4))
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, cutoff=cut)
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    ref, _ = c1["O"].pt2(c1["dets"], c1["c"], c1["e0"], cutoff=cut)
    assert got["n_after_cutoff"] == ref["n_kept"]
    assert got["n_contrib"] == ref["n_contrib"]
    assert abs(got["e_pt2"] - ref["e_pt2"]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("log2p", [2, 5])
def test_c1_cutoff_with_split(pt2, c1, log2p):
    """Cutoff and a hash split together: counts come from the enumerating
    count pass (the cutoff needs every term's value), generation walks only
    each subset's terms."""
    k, v = c1["O"].emit(c1["dets"], c1["c"])
    cut = float(np.quantile(np.abs(v), 0.3))
    ctx = pt2.Context(c1["h"], c1["eri"], 12, 4, 4, cutoff=cut, log2_partitions=log2p)
    got = ctx.evaluate(c1["dets"], c1["c"], c1["e0"])
    ctx.close()
    ref, _ = c1["O"].pt2(c1["dets"], c1["c"], c1["e0"], cutoff=cut, log2p=log2p)
    assert got["n_partitions"] == 1 << log2p
    assert got["n_after_cutoff"] == ref["n_kept"] and got["n_contrib"] == ref["n_contrib"]
    assert abs(got["e_pt2"] - ref["e_pt2"]) <= 1e-9
    for key in ("n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum"):
        assert got[key] == ref[key]


# ---------------------------------------------------------------------------
# Word-straddling keys and every key width

@pytest.mark.parametrize("norb,na,nb,nref,log2p", [
    (6, 2, 2, 30, -1), (33, 3, 2, 25, -1), (40, 4, 4, 12, 2), (64, 3, 3, 10, -1),
    (65, 3, 2, 10, -1), (76, 4, 3, 6, 1), (100, 3, 3, 5, -1), (128, 2, 2, 5, -1), (9, 0, 3, 20, -1),
    (7, 4, 0, 15, -1)])
def test_random_systems_all_widths(pt2, norb, na, nb, nref, log2p):
    h, eri, _ = synth.make_integrals(norb, 6, 7000 + norb)
    dets = synth.random_determinants(norb, na, nb, nref, norb)
    c = np.random.default_rng(norb).normal(size=nref)
    O = oracle.Oracle(h, eri, norb, na, nb)
    e0 = float(O.diag(dets).min()) - 2.0
    ref, _ = O.pt2(dets, c, e0)
    ctx = pt2.Context(h, eri, norb, na, nb, log2_partitions=log2p)
    got = ctx.evaluate(dets, c, e0)
    assert_matches(got, ref)
    order = sort_by_key(dets)
    gk, gv = ctx.dump_records(dets[order], c[order])
    ok, ov = O.emit(dets[order], c[order])
    assert np.array_equal(gk, ok)
    np.testing.assert_allclose(gv, ov, rtol=0, atol=1e-14)
    ctx.close()


ALL_FIELDS = ("e_pt2", "n_contrib", "n_after_cutoff", "n_unique", "n_external", "n_in_ref_hit",
              "n_nonneg_denom", "key_xor", "key_sum", "ref_cross", "min_abs_denom")


@pytest.mark.parametrize("norb,na,nb,nref,log2p,prec", [
    (12, 4, 4, 40, -1, "fp64"), (20, 6, 3, 60, 3, "fp64"), (33, 3, 2, 25, -1, "fp32"),
    (40, 10, 10, 30, -1, "fp64"), (40, 4, 4, 50, 4, "fp32"), (64, 3, 3, 10, -1, "fp64"),
    (76, 5, 5, 12, 2, "fp64"), (100, 4, 3, 8, -1, "fp64"), (128, 3, 3, 6, 1, "fp64"),
    (9, 9, 0, 1, -1, "fp64"), (10, 0, 3, 20, -1, "fp64")])
def test_rank_keys_give_identical_results(pt2, norb, na, nb, nref, log2p, prec):
    """Terms keyed by the combinatorial rank of their determinant sort in the
    bitstring order, so every result equals the bitstring-keyed run bit for
    bit; both match the oracle."""
    h, eri, _ = synth.make_integrals(norb, 6, 8000 + norb)
    nref = min(nref, math.comb(norb, na) * math.comb(norb, nb))
    dets = synth.random_determinants(norb, na, nb, nref, norb + 1)
    c = np.random.default_rng(norb).normal(size=nref)
    c /= np.linalg.norm(c)
    O = oracle.Oracle(h, eri, norb, na, nb)
    # E0 below every diagonal element involved: no near-zero denominators,
    # whose conditioning would amplify last-bit differences of H_aa
    keys, _ = O.numerators(dets, c)
    e0 = float(np.concatenate([O.diag(keys), O.diag(dets)]).min()) - 1.0
    res = {}
    for mode in (0, 1):
        ctx = pt2.Context(h, eri, norb, na, nb, log2_partitions=log2p, precision=prec, compress_keys=mode)
        res[mode] = ctx.evaluate(dets, c, e0)
        ctx.close()
    print("key bits", res[0]["key_bits"], "->", res[1]["key_bits"], flush=True)
    assert res[0]["key_bits"] == 2 * norb
    assert res[1]["key_bits"] <= 2 * norb
    for k in ALL_FIELDS:
        assert res[0][k] == res[1][k], (k, res[0][k], res[1][k])
    ref, _ = O.pt2(dets, c, e0)
    if prec == "fp64":
        assert_matches(res[1], ref)
    else:  # FP32 terms: sum_i c_i N_i carries their rounding too
        assert_matches(res[1], ref, tol=1e-6, cross_tol=1e-7)


@pytest.mark.parametrize("log2p", [-1, 3])
def test_hash_compact_reference_table_is_exact(pt2, log2p):
    """Hash records rebuild each parent from the first sorted reference and
    its flips (every reference of C2 is within three excitations of it) or
    from its full bitstring: the same records, so every result field is
    bit-identical either way."""
    w, h, eri, dets, c, e0 = load("c2")
    dets, c = dets[:400], c[:400]
    res = []
    for compact in (True, False):
        ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, compress_keys=2, log2_partitions=log2p,
                          compact_refs=compact)
        res.append(ctx.evaluate(dets, c, e0))
        ctx.close()
    for k in ("e_pt2", "n_contrib", "n_unique", "n_external", "n_in_ref_hit", "n_nonneg_denom", "min_abs_denom",
              "ref_cross", "key_xor", "key_sum"):
        assert res[0][k] == res[1][k], (k, res[0][k], res[1][k])


@pytest.mark.parametrize("norb,na,nb,nref,log2p,prec,hash_bits", [
    (12, 4, 4, 40, -1, "fp64", 0), (12, 4, 4, 40, -1, "fp64", 10), (20, 6, 3, 60, 3, "fp64", 0),
    (20, 6, 3, 60, 2, "fp64", 12), (33, 3, 2, 25, -1, "fp32", 0), (40, 10, 10, 30, -1, "fp64", 16),
    (64, 3, 3, 10, 1, "fp64", 0), (76, 5, 5, 12, 2, "fp64", 0), (100, 4, 3, 8, -1, "fp64", 14),
    (127, 3, 3, 6, -1, "fp64", 0), (10, 0, 3, 20, -1, "fp64", 8)])
def test_hash_records_match(pt2, norb, na, nb, nref, log2p, prec, hash_bits):
    """Records keyed by the Zobrist hash (parent and flips carried along)
    give the bitstring-keyed counts and checksums exactly and the energy to
    rounding; truncated hashes force many collisions, which the single pass
    must separate exactly (every key set and count unchanged)."""
    h, eri, _ = synth.make_integrals(norb, 6, 9000 + norb)
    nref = min(nref, math.comb(norb, na) * math.comb(norb, nb))
    dets = synth.random_determinants(norb, na, nb, nref, norb + 2)
    c = np.random.default_rng(norb + 1).normal(size=nref)
    c /= np.linalg.norm(c)
    O = oracle.Oracle(h, eri, norb, na, nb)
    keys, _ = O.numerators(dets, c)
    e0 = float(np.concatenate([O.diag(keys), O.diag(dets)]).min()) - 1.0
    res = {}
    for mode in (0, 2):
        ctx = pt2.Context(h, eri, norb, na, nb, log2_partitions=log2p, precision=prec, compress_keys=mode,
                          hash_bits=hash_bits)
        res[mode] = ctx.evaluate(dets, c, e0)
        if mode == 2:  # collisions resolved the same way every time: bit-identical repeats
            again = ctx.evaluate(dets, c, e0)
            assert again["e_pt2"] == res[2]["e_pt2"] and again["ref_cross"] == res[2]["ref_cross"]
        ctx.close()
    print("key bits", res[0]["key_bits"], "->", res[2]["key_bits"], "passes", res[0]["n_sort_passes"], "->",
          res[2]["n_sort_passes"], flush=True)
    # hash bits: as given, or as few as keep the expected collisions small
    if hash_bits:
        assert res[2]["key_bits"] == min(hash_bits, 64)
    else:
        assert res[2]["key_bits"] in (32, 40, 48, 56, 64)
    for k in ("n_contrib", "n_after_cutoff", "n_unique", "n_external", "n_in_ref_hit", "n_nonneg_denom",
              "key_xor", "key_sum"):
        assert res[0][k] == res[2][k], (k, res[0][k], res[2][k])
    if prec == "fp64":
        assert res[2]["e_pt2"] == pytest.approx(res[0]["e_pt2"], rel=1e-12, abs=1e-12)
    # (FP32 payloads: hash records recompute the numerators of the terms their
    # rounding could move most from FP64 matrix elements, bitstring records
    # keep the rounded sum, so the two differ within the FP32 bar, checked
    # against the oracle below for both)
    assert res[2]["ref_cross"] == pytest.approx(res[0]["ref_cross"], rel=1e-12, abs=1e-14)
    ref, _ = O.pt2(dets, c, e0)
    if prec != "fp64":
        assert_matches(res[0], ref, tol=1e-6, cross_tol=1e-7)
        print("fp32 |dE| vs FP64 oracle: bitstring", abs(res[0]["e_pt2"] - ref["e_pt2"]), "hash",
              abs(res[2]["e_pt2"] - ref["e_pt2"]), flush=True)
    if prec == "fp64":
        assert_matches(res[2], ref)
    else:
        assert_matches(res[2], ref, tol=1e-6, cross_tol=1e-7)


def test_workspace_reuse_with_smaller_reference(pt2):
    """A context that evaluated a larger reference evaluates a smaller one
    (multi-word keys) correctly: buffers are reused with the right strides."""
    norb, na, nb = 40, 4, 4
    h, eri, _ = synth.make_integrals(norb, 6, 4040)
    dets = synth.random_determinants(norb, na, nb, 30, 4040)
    c = np.random.default_rng(4).normal(size=30)
    O = oracle.Oracle(h, eri, norb, na, nb)
    e0 = float(O.diag(dets).min()) - 2.0
    ctx = pt2.Context(h, eri, norb, na, nb)
    for m in (30, 7, 19, 1):
        ref, _ = O.pt2(dets[:m], c[:m], e0)
        assert_matches(ctx.evaluate(dets[:m], c[:m], e0), ref)
    ctx.close()


def test_full_fci_reference_gives_zero(pt2):
    norb, na, nb = 7, 3, 2
    h, eri, _ = synth.make_integrals(norb, 6, 5)
    B = oracle.Brute(h, eri, norb, na, nb)
    keys = B.keys_of(np.arange(B.dim()))
    c = np.random.default_rng(1).normal(size=len(keys))
    ctx = pt2.Context(h, eri, norb, na, nb)
    got = ctx.evaluate(keys, c, -10.0)
    assert got["e_pt2"] == 0.0 and got["n_external"] == 0
    assert got["n_in_ref_hit"] == len(keys)
    ctx.close()


def test_hf_only_and_empty_reference(pt2, c1):
    hf = synth.hf_key(12, 4, 4)[None]
    e0 = float(c1["O"].diag(hf)[0])
    got = c1["ctx"].evaluate(hf, [1.0], e0)
    ref, _ = c1["O"].pt2(hf, [1.0], e0)
    assert_matches(got, ref)
    assert got["n_unique"] == got["n_contrib"] == 1424
    empty = c1["ctx"].evaluate(np.zeros((0, 1), np.uint64), np.zeros(0), e0)
    assert empty["e_pt2"] == 0.0 and empty["n_contrib"] == 0


def test_invalid_references_rejected(pt2, c1):
    ctx = c1["ctx"]
    d = c1["dets"][:10].copy()
    with pytest.raises(pt2.PT2Error) as e:
        ctx.evaluate(np.concatenate([d, d[3:4]]), np.ones(11), -1.0)
    assert e.value.code == pt2.PT2_E_INVALID and "duplicate" in str(e.value)
    bad = d.copy()
    bad[0, 0] ^= np.uint64(1 << 11)  # flips one beta bit: wrong electron count
    with pytest.raises(pt2.PT2Error) as e:
        ctx.evaluate(bad, np.ones(10), -1.0)
    assert e.value.code == pt2.PT2_E_INVALID
    stray = d.copy()
    stray[0, 0] |= np.uint64(1 << 40)
    with pytest.raises(pt2.PT2Error) as e:
        ctx.evaluate(stray, np.ones(10), -1.0)
    assert e.value.code == pt2.PT2_E_INVALID
    # the context stays usable
    assert_matches(ctx.evaluate(c1["dets"], c1["c"], c1["e0"]), c1["ref"])


def spin_groups(dets, norb, spin, size=32):
    """Groups of at most `size` references sharing their alpha (spin 0) or beta
    (spin 1) string: the sum over distinct strings of ceil(count / size)."""
    counts = {}
    for row in dets:
        k = int.from_bytes(row.astype("<u8").tobytes(), "little")
        s = k >> norb if spin == 0 else k & ((1 << norb) - 1)
        counts[s] = counts.get(s, 0) + 1
    return sum((m + size - 1) // size for m in counts.values())


@pytest.mark.parametrize("norb,na,nb,n_alpha,per_alpha,prec", [
    (12, 4, 4, 3, 70, "fp64"), (40, 10, 10, 6, 45, "fp32"), (33, 5, 3, 4, 40, "fp32-arith"),
    (70, 4, 4, 3, 33, "fp64"), (8, 3, 2, 4, 28, "fp64")])
def test_string_reuse_gives_identical_results(pt2, norb, na, nb, n_alpha, per_alpha, prec):
    """References sharing alpha strings (in groups larger than the 32 a
    workgroup takes) and, the last case, beta strings: generating the same-spin
    doubles once per group of references sharing the spin string gives every
    result bit for bit as generating them per reference, with the group counts
    that the reference implies; the small cases also match the oracle."""
    rng = np.random.default_rng(norb * 100 + n_alpha)
    A, B, seen_a = [], [], set()
    while len(seen_a) < n_alpha:
        a = tuple(sorted(rng.choice(norb, na, replace=False)))
        if a in seen_a:
            continue
        seen_a.add(a)
        seen_b = set()
        while len(seen_b) < per_alpha:
            seen_b.add(tuple(sorted(rng.choice(norb, nb, replace=False))))
        for b in seen_b:
            ra, rb = np.zeros(norb, bool), np.zeros(norb, bool)
            ra[list(a)], rb[list(b)] = True, True
            A.append(ra)
            B.append(rb)
    dets = synth.pack_keys(np.array(A), np.array(B), norb)
    dets = dets[rng.permutation(len(dets))]
    c = rng.normal(size=len(dets))
    c /= np.linalg.norm(c)
    h, eri, _ = synth.make_integrals(norb, 6, 9100 + norb)
    O = oracle.Oracle(h, eri, norb, na, nb)
    e0 = float(O.diag(dets).min()) - 5.0
    res = {}
    for mode in (0, 1, 2):
        ctx = pt2.Context(h, eri, norb, na, nb, precision=prec, compress_keys=0, string_reuse=mode)
        res[mode] = ctx.evaluate(dets, c, e0)
        ctx.close()
    ga, gb = spin_groups(dets, norb, 0), spin_groups(dets, norb, 1)
    print("groups", res[2]["n_alpha_groups"], res[2]["n_beta_groups"], "expected", ga, gb, flush=True)
    assert (res[0]["n_alpha_groups"], res[0]["n_beta_groups"]) == (0, 0)
    assert (res[1]["n_alpha_groups"], res[1]["n_beta_groups"]) == (ga, 0)
    assert (res[2]["n_alpha_groups"], res[2]["n_beta_groups"]) == (ga, gb)
    for mode in (1, 2):
        for k in ALL_FIELDS:
            assert res[mode][k] == res[0][k], (mode, k, res[mode][k], res[0][k])
    if norb <= 12:
        ref, _ = O.pt2(dets, c, e0)
        assert_matches(res[2], ref)


# ---------------------------------------------------------------------------
# The radix sort on its own

@pytest.mark.parametrize("W,bits,n,pb,skew", [
    (1, 24, 1000, 8, False), (1, 64, 70_001, 4, False), (2, 80, 123_457, 8, True),
    (3, 152, 50_000, 8, False), (4, 200, 9_000, 4, True), (2, 72, 4096, 8, False),
    (2, 80, 4097, 8, True), (1, 8, 300_000, 8, True),
    # several chunks of 256 tiles: offsets within a chunk and across chunks
    (1, 16, 1_200_001, 8, True), (2, 80, 1_100_000, 4, True)])
def test_sort_records_matches_stable_sort(pt2, W, bits, n, pb, skew):
    rng = np.random.default_rng(W * 1000 + n)
    keys = rng.integers(0, 2 ** 63, size=(n, W), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(n, W), dtype=np.uint64)
    if skew:
        keys[rng.random(n) < 0.7] = keys[0]
        keys[:, 0] &= np.uint64(0xFF00FF00FFFF00FF)
    for w in range(W):
        top = bits - 64 * w
        if top <= 0:
            keys[:, w] = 0
        elif top < 64:
            keys[:, w] &= np.uint64((1 << top) - 1)
    pay = np.arange(n, dtype=np.float64 if pb == 8 else np.uint32)
    sk, sp = pt2.sort_records(keys.copy(), pay.copy(), bits)
    idx = np.lexsort(tuple(keys[:, w] for w in range(W)))
    assert np.array_equal(sk, keys[idx])
    assert np.array_equal(sp, pay[idx])


def test_sort_records_near_constant_digits(pt2):
    """Digits that take one value in all but a few records: most tiles hold a
    whole tile of one digit value, and that value's offsets within a chunk run
    up to the chunk's full length, over three chunks of tiles."""
    rng = np.random.default_rng(77)
    n = 1_500_000
    keys = np.full((n, 1), 0x5A5A, dtype=np.uint64)
    odd = rng.choice(n, size=12, replace=False)
    keys[odd, 0] = rng.integers(0, 1 << 16, size=12, dtype=np.uint64)
    pay = np.arange(n, dtype=np.float64)
    sk, sp = pt2.sort_records(keys.copy(), pay.copy(), 16)
    idx = np.argsort(keys[:, 0], kind="stable")
    assert np.array_equal(sk, keys[idx])
    assert np.array_equal(sp, pay[idx])


# ---------------------------------------------------------------------------
# C2 at full size: (10a,10b)/40, 10,000 references, 1.2975e9 terms

@pytest.fixture(scope="module")
def c2(pt2):
    w, h, eri, dets, c, e0 = load("c2")
    ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, timing=True)
    yield dict(w=w, h=h, eri=eri, dets=dets, c=c, e0=e0, ctx=ctx)
    ctx.close()


def test_c2_full_size_bench_configuration(c2):
    """The single-subset launch that the benchmark times, checked by properties
    that hold at any size: the closed-form count, the <c|H|c> identity built
    from the in-reference numerators, and the split-invariance of the total."""
    import torch
    d = torch.from_numpy(c2["dets"].view(np.int64)).cuda()
    cc = torch.from_numpy(c2["c"]).cuda()
    got = c2["ctx"].evaluate(d, cc, c2["e0"])
    print({k: got[k] for k in ("e_pt2", "n_contrib", "n_unique", "n_external", "n_in_ref_hit",
                               "ms_gen", "ms_sort", "ms_reduce", "ms_hist", "n_sort_passes")}, flush=True)
    assert got["n_contrib"] == 1_297_500_000 and got["n_partitions"] == 1
    O = oracle.Oracle(c2["h"], c2["eri"], 40, 10, 10)
    hii = O.diag(c2["dets"])
    assert got["ref_cross"] + float(np.sum(c2["c"] ** 2 * hii)) == pytest.approx(c2["e0"], abs=1e-9)
    assert got["n_unique"] == got["n_external"] + got["n_in_ref_hit"]
    c2["total"] = got


def test_c2_sampled_subsets_match_oracle(c2):
    parts = [0, 77, 511, 1023]
    got, ep = c2["ctx"].evaluate_parts(c2["dets"], c2["c"], c2["e0"], 10, parts)
    O = oracle.Oracle(c2["h"], c2["eri"], 40, 10, 10)
    ref, rp = O.pt2(c2["dets"], c2["c"], c2["e0"], log2p=10, parts=parts)
    print("subset energies", ep, rp, flush=True)
    np.testing.assert_allclose(ep, rp, rtol=0, atol=1e-9)
    assert_matches(got, ref)


def test_c2_split_total_equals_single_subset(c2):
    if "total" not in c2:
        pytest.skip("full-size run did not complete")
    import paper_1808_02049_amd as pt2
    ctx = pt2.Context(c2["h"], c2["eri"], 40, 10, 10, log2_partitions=3)
    got = ctx.evaluate(c2["dets"], c2["c"], c2["e0"])
    ctx.close()
    tot = c2["total"]
    assert got["e_pt2"] == pytest.approx(tot["e_pt2"], abs=1e-9)
    for k in ("n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum"):
        assert got[k] == tot[k]


@pytest.mark.parametrize("norb,n_el,nref,log2p,mode,prec,sign", [
    (10, 3, 30, -1, 0, "fp64", 1), (10, 3, 30, 2, 0, "fp64", -1), (36, 5, 40, -1, 1, "fp64", 1),
    (36, 5, 40, 3, 2, "fp64", 1), (40, 4, 30, -1, 2, "fp64", -1), (70, 4, 12, 1, 0, "fp64", 1),
    (12, 4, 50, -1, 0, "fp32", 1)])
def test_spin_flip_matches_full_sum(pt2, norb, n_el, nref, log2p, mode, prec, sign):
    """spin_flip on a swap-symmetric reference: only alpha >= beta determinants
    are generated and the alpha != beta terms count twice; the energy and the
    in-reference cross term equal the oracle's full sums, the structural count
    is unchanged, and about half the distinct determinants are visited."""
    h, eri, _ = synth.make_integrals(norb, 6, 5200 + norb)
    dets, c = synth.swap_symmetric_references(norb, n_el, nref, 41 + norb, sign)
    O = oracle.Oracle(h, eri, norb, n_el, n_el)
    keys, _ = O.numerators(dets, c)
    e0 = float(np.concatenate([O.diag(keys), O.diag(dets)]).min()) - 1.0
    ref, _ = O.pt2(dets, c, e0)
    ctx = pt2.Context(h, eri, norb, n_el, n_el, log2_partitions=log2p, precision=prec, compress_keys=mode,
                      spin_flip=True)
    got = ctx.evaluate(dets, c, e0)
    again = ctx.evaluate(dets, c, e0)
    ctx.close()
    print("spin flip", got["e_pt2"], ref["e_pt2"], got["e_pt2"] - ref["e_pt2"], got["n_unique"], ref["n_unique"],
          flush=True)
    tol = 1e-9 if prec == "fp64" else 1e-6
    assert abs(got["e_pt2"] - ref["e_pt2"]) <= tol * max(1.0, abs(ref["e_pt2"]))
    assert got["ref_cross"] == pytest.approx(ref["ref_cross"], abs=1e-11 if prec == "fp64" else 1e-7)
    assert got["n_contrib"] == ref["n_contrib"]
    assert ref["n_unique"] / 2 <= got["n_unique"] < ref["n_unique"] / 2 + ref["n_unique"] / 50 + 10
    assert again["e_pt2"] == got["e_pt2"]


def test_spin_flip_rejects_unsymmetric_input(pt2):
    """spin_flip needs nalpha == nbeta at creation, and at evaluation a
    reference closed under the swap with one sign relation throughout."""
    norb, n_el = 10, 3
    h, eri, _ = synth.make_integrals(norb, 6, 5210)
    with pytest.raises(pt2.PT2Error):
        pt2.Context(h, eri, norb, 3, 2, spin_flip=True)
    ctx = pt2.Context(h, eri, norb, n_el, n_el, spin_flip=True)
    dets, c = synth.swap_symmetric_references(norb, n_el, 20, 57)
    with pytest.raises(pt2.PT2Error):  # a partner missing
        ctx.evaluate(dets[1:], c[1:], -10.0)
    c2 = c.copy()
    a, b = synth.unpack_keys(dets, norb)
    sw = synth.pack_keys(b, a, norb)
    i = next(i for i in range(len(dets)) if not np.array_equal(sw[i], dets[i]))
    j = next(j for j in range(len(dets)) if np.array_equal(dets[j], sw[i]))
    c2[j] = -c2[i]  # one pair with the opposite sign relation
    with pytest.raises(pt2.PT2Error):
        ctx.evaluate(dets, c2, -10.0)
    got = ctx.evaluate(dets, c, -10.0)  # the context is still usable
    assert np.isfinite(got["e_pt2"])
    ctx.close()
