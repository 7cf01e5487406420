"""Pins of the FP64 CPU oracle against things other than itself.

Each test fixes part of the oracle by mathematics or by an independent
computation, so that a dropped term, a wrong sign or index, or a transposed
operand fails at least one of them:

* the literal operator-by-operator Hamiltonian (brute-force checker), itself
  pinned by textbook facts (one-electron spectrum = eig(h), a doubly occupied
  single orbital, invariance of the FCI energy under orbital rotations);
* a hand-worked two-orbital example;
* closed-form contribution counts;
* identities the paper states (duplicate removal for an eigenvector
  reference, Section V) and invariances of the Epstein-Nesbet sum.
"""
import numpy as np
import pytest

import oracle
import synth


def system(norb, na, nb, seed, nchol=8):
    h, eri, _ = synth.make_integrals(norb, nchol, seed)
    return h, eri


def all_dets(norb, na, nb):
    B = oracle.Brute(*system(norb, na, nb, 0), norb, na, nb)
    return B.keys_of(np.arange(B.dim()))


# --------------------------------------------------------------------------
# Pins of the brute-force checker (textbook facts)

def test_one_electron_spectrum_is_eig_h():
    norb = 5
    h, eri = system(norb, 1, 0, 11)
    B = oracle.Brute(h, eri, norb, 1, 0)
    H = B.dense()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(H)), np.sort(np.linalg.eigvalsh(h)),
                               atol=1e-13)


def test_doubly_occupied_single_orbital():
    h = np.array([[-1.25]])
    eri = np.array([0.7])
    B = oracle.Brute(h, eri, 1, 1, 1)
    assert B.dense()[0, 0] == pytest.approx(2 * -1.25 + 0.7, abs=1e-15)


def _rotate(h, eri, U):
    n = h.shape[0]
    g = eri.reshape(n, n, n, n)
    g = np.einsum("pa,qb,rc,sd,abcd->pqrs", U, U, U, U, g, optimize=True)
    return U @ h @ U.T, g.reshape(-1)


@pytest.mark.parametrize("norb,na,nb", [(4, 2, 1), (5, 2, 2), (4, 3, 0)])
def test_fci_energy_invariant_under_orbital_rotation(norb, na, nb):
    h, eri = system(norb, na, nb, 21)
    U, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(norb, norb)))
    h2, eri2 = _rotate(h, eri, U)
    e1 = np.linalg.eigvalsh(oracle.Brute(h, eri, norb, na, nb).dense())
    e2 = np.linalg.eigvalsh(oracle.Brute(h2, eri2, norb, na, nb).dense())
    np.testing.assert_allclose(e1, e2, atol=1e-11)


def test_brute_hamiltonian_is_symmetric():
    h, eri = system(6, 2, 2, 5)
    H = oracle.Brute(h, eri, 6, 2, 2).dense()
    np.testing.assert_allclose(H, H.T, atol=1e-14)


# --------------------------------------------------------------------------
# Hand-worked example: one alpha and one beta electron in two orbitals,
# reference = {HF}.  Slater-Condon by hand:
#   single (either spin):  F_01 = h01 + (01|00)          = 0.15
#   double (alpha and beta 0->1): (01|01)                = 0.15
#   H_00 = 2 h00 + (00|00) = -1.4 ; H_single = h00 + h11 + (00|11) = -1.1
#   H_double = 2 h11 + (11|11) = -0.5
#   E_PT2 = 2 * 0.15^2/(-0.3) + 0.15^2/(-0.9) = -0.175

def two_orbital_example():
    h = np.array([[-1.0, 0.1], [0.1, -0.5]])
    g = np.zeros((2, 2, 2, 2))
    vals = {(0, 0, 0, 0): 0.6, (1, 1, 1, 1): 0.5, (0, 0, 1, 1): 0.4, (0, 1, 0, 1): 0.15,
            (0, 0, 0, 1): 0.05, (0, 1, 1, 1): 0.03}
    for (p, q, r, s), v in vals.items():
        for a, b, c, d in {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                           (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}:
            g[a, b, c, d] = v
    return h, g.reshape(-1)


def test_hand_worked_two_orbital_example():
    h, eri = two_orbital_example()
    O = oracle.Oracle(h, eri, 2, 1, 1)
    hf = synth.hf_key(2, 1, 1)[None]
    assert O.diag(hf)[0] == pytest.approx(-1.4, abs=1e-15)
    res, _ = O.pt2(hf, [1.0], -1.4)
    assert res["e_pt2"] == pytest.approx(-0.175, abs=1e-15)
    assert res["n_contrib"] == 3 and res["n_external"] == 3
    B = oracle.Brute(h, eri, 2, 1, 1)
    e, n = B.pt2(hf, [1.0], -1.4)
    assert e == pytest.approx(-0.175, abs=1e-15)


# --------------------------------------------------------------------------
# Oracle against the brute-force checker

@pytest.mark.parametrize("norb,na,nb,nref,seed", [
    (6, 2, 2, 20, 1), (7, 3, 2, 40, 2), (5, 1, 0, 2, 3), (8, 3, 3, 60, 4), (7, 2, 3, 30, 5),
    (5, 2, 0, 3, 6), (6, 0, 2, 4, 7)])
def test_oracle_matches_brute_force_tiny(norb, na, nb, nref, seed):
    h, eri = system(norb, na, nb, seed)
    O = oracle.Oracle(h, eri, norb, na, nb)
    B = oracle.Brute(h, eri, norb, na, nb)
    rng = np.random.default_rng(seed)
    keys = B.keys_of(np.arange(B.dim()))
    pick = rng.choice(len(keys), size=min(nref, len(keys)), replace=False)
    R = keys[pick]
    c = rng.normal(size=len(R))
    c /= np.linalg.norm(c)
    e0 = float(rng.uniform(-30, -10))
    res, _ = O.pt2(R, c, e0)
    e_b, n_b = B.pt2(R, c, e0)
    assert res["e_pt2"] == pytest.approx(e_b, abs=1e-12)
    assert res["n_contrib"] == len(R) * synth.n_excitations_per_det(norb, na, nb)


def test_oracle_matches_dense_complement_formula():
    """PT2 = sum over the complement of (H_PR c)^2 / (E0 - H_aa) from a dense FCI H."""
    norb, na, nb = 6, 2, 2
    h, eri = system(norb, na, nb, 31)
    B = oracle.Brute(h, eri, norb, na, nb)
    H = B.dense()
    keys = B.keys_of(np.arange(B.dim()))
    R_idx = np.arange(0, B.dim(), 7)
    Hrr = H[np.ix_(R_idx, R_idx)]
    w, V = np.linalg.eigh(Hrr)
    c, e0 = V[:, 0], w[0]
    P_idx = np.setdiff1d(np.arange(B.dim()), R_idx)
    v = H[np.ix_(P_idx, R_idx)] @ c
    expect = float(np.sum(v ** 2 / (e0 - np.diag(H)[P_idx])))
    res, _ = oracle.Oracle(h, eri, norb, na, nb).pt2(keys[R_idx], c, e0)
    assert res["e_pt2"] == pytest.approx(expect, abs=1e-12)


def test_matrix_elements_match_brute_force():
    """Every emitted payload of a single reference equals <a|H|D> of the dense H."""
    norb, na, nb = 7, 3, 2
    h, eri = system(norb, na, nb, 41)
    O = oracle.Oracle(h, eri, norb, na, nb)
    B = oracle.Brute(h, eri, norb, na, nb)
    H = B.dense()
    keys = B.keys_of(np.arange(B.dim()))
    for j in np.random.default_rng(1).choice(len(keys), 12, replace=False):
        ek, ev = O.emit(keys[j][None], [1.0])
        idx = B.index_of(ek)
        np.testing.assert_allclose(ev, H[idx, j], atol=1e-13)
        # every determinant connected to D is emitted exactly once
        connected = np.nonzero(np.abs(H[:, j]) > 0)[0]
        connected = connected[connected != j]
        assert set(connected.tolist()) <= set(idx.tolist())
        assert len(set(idx.tolist())) == len(idx)
        # the general pairwise rule agrees too
        for i in idx[:40]:
            assert O.hij(keys[i], keys[j]) == pytest.approx(H[i, j], abs=1e-13)


def test_diagonal_matches_brute_force():
    norb, na, nb = 8, 3, 3
    h, eri = system(norb, na, nb, 51)
    O = oracle.Oracle(h, eri, norb, na, nb)
    B = oracle.Brute(h, eri, norb, na, nb)
    idx = np.random.default_rng(2).choice(B.dim(), 300, replace=False)
    np.testing.assert_allclose(O.diag(B.keys_of(idx)), B.diag(idx), atol=1e-12)


# --------------------------------------------------------------------------
# Workload C1: brute force over the 245,025-determinant FCI space

def load_c1():
    w = synth.WORKLOADS["c1"]
    h, eri, _ = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(synth_path("inputs_c1.npz"))
    return w, h, eri, f["dets"], f["c"], float(f["e0"])


def synth_path(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


def test_c1_oracle_matches_brute_force_fci():
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    B = oracle.Brute(h, eri, w.norb, w.nalpha, w.nbeta)
    assert B.dim() == 245_025
    res, _ = O.pt2(dets, c, e0)
    e_b, n_ext = B.pt2(dets, c, e0)
    assert res["e_pt2"] == pytest.approx(e_b, abs=1e-12)
    assert res["n_contrib"] == 284_800
    assert res["n_external"] >= n_ext  # brute force skips exact zeros only


def test_c1_reference_is_eigenvector_and_subtraction_identity():
    """Duplicate removal by subtraction (Section V) holds for an eigenvector:
    every in-reference numerator equals c_i (E0 - H_ii), so the in-reference
    PT2-like terms are c_i^2 (E0 - H_ii)."""
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    H = O.hrr(dets)
    np.testing.assert_allclose(H @ c, e0 * c, atol=1e-12)
    keys, nums = O.numerators(dets, c)
    haa = O.diag(keys)
    allterms = float(np.sum(nums ** 2 / (e0 - haa)))
    hii = O.diag(dets)
    res, _ = O.pt2(dets, c, e0)
    assert allterms - float(np.sum(c ** 2 * (e0 - hii))) == pytest.approx(res["e_pt2"], abs=1e-11)


def test_expectation_identity_from_in_reference_numerators():
    """sum_i c_i (N_i + H_ii c_i) = <c|H|c> for any coefficients."""
    w, h, eri, dets, _, _ = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    c = np.random.default_rng(5).normal(size=len(dets))
    c /= np.linalg.norm(c)
    res, _ = O.pt2(dets, c, -20.0)
    hii = O.diag(dets)
    H = O.hrr(dets)
    assert res["ref_cross"] + float(np.sum(c * c * hii)) == pytest.approx(float(c @ H @ c), abs=1e-12)


# --------------------------------------------------------------------------
# Special cases

@pytest.mark.parametrize("norb,na,nb", [(6, 2, 2), (8, 3, 3), (7, 3, 2)])
def test_full_fci_reference_gives_zero(norb, na, nb):
    h, eri = system(norb, na, nb, 61)
    keys = all_dets(norb, na, nb)
    c = np.random.default_rng(0).normal(size=len(keys))
    res, _ = oracle.Oracle(h, eri, norb, na, nb).pt2(keys, c, -5.0)
    assert res["e_pt2"] == 0.0
    assert res["n_external"] == 0


def test_hf_only_reference_closed_form():
    norb, na, nb = 8, 3, 3
    h, eri = system(norb, na, nb, 71)
    O = oracle.Oracle(h, eri, norb, na, nb)
    B = oracle.Brute(h, eri, norb, na, nb)
    hf = synth.hf_key(norb, na, nb)[None]
    H = B.dense()
    j = B.index_of(hf)[0]
    e0 = H[j, j]
    col = H[:, j].copy()
    col[j] = 0.0
    nz = np.nonzero(col)[0]
    expect = float(np.sum(col[nz] ** 2 / (e0 - np.diag(H)[nz])))
    res, _ = O.pt2(hf, [1.0], e0)
    assert res["e_pt2"] == pytest.approx(expect, abs=1e-13)
    assert res["n_unique"] == res["n_contrib"] == synth.n_excitations_per_det(norb, na, nb)


@pytest.mark.parametrize("norb,na,nb,expect", [
    (12, 4, 4, 1424), (40, 10, 10, 129_750), (76, 14, 14, 1_099_322), (100, 18, 18, 3_197_754)])
def test_closed_form_counts(norb, na, nb, expect):
    assert synth.n_excitations_per_det(norb, na, nb) == expect


def test_counts_equal_closed_form_enumeration():
    norb, na, nb = 9, 3, 2
    h, eri = system(norb, na, nb, 81)
    keys = all_dets(norb, na, nb)[:17]
    res, _ = oracle.Oracle(h, eri, norb, na, nb).pt2(keys, np.ones(17), -3.0)
    assert res["n_contrib"] == 17 * synth.n_excitations_per_det(norb, na, nb)
    # brute-force count of singles+doubles of one determinant
    occ = lambda k: set(np.nonzero(np.unpackbits(k.view(np.uint8), bitorder="little"))[0])
    o0 = occ(keys[0].copy())
    alld = all_dets(norb, na, nb)
    cnt = sum(1 for k in alld if 1 <= len(occ(k.copy()) - o0) <= 2)
    assert cnt == synth.n_excitations_per_det(norb, na, nb)


# --------------------------------------------------------------------------
# Invariances of the Epstein-Nesbet sum

def _perm_parity(seq):
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    return -1.0 if inv & 1 else 1.0


def test_invariant_under_orbital_relabelling():
    norb, na, nb = 7, 3, 2
    h, eri = system(norb, na, nb, 91)
    keys = all_dets(norb, na, nb)
    rng = np.random.default_rng(9)
    R = keys[rng.choice(len(keys), 50, replace=False)]
    c = rng.normal(size=50)
    e0 = float(oracle.Oracle(h, eri, norb, na, nb).diag(keys).min()) - 1.0
    ref, _ = oracle.Oracle(h, eri, norb, na, nb).pt2(R, c, e0)

    perm = rng.permutation(norb)
    h2 = np.empty_like(h)
    h2[np.ix_(perm, perm)] = h
    g = eri.reshape(norb, norb, norb, norb)
    g2 = np.empty_like(g)
    g2[np.ix_(perm, perm, perm, perm)] = g
    A, Bo = synth.unpack_keys(R, norb)
    A2 = np.zeros_like(A)
    B2 = np.zeros_like(Bo)
    c2 = c.copy()
    for i in range(len(R)):
        oa = np.nonzero(A[i])[0]
        ob = np.nonzero(Bo[i])[0]
        A2[i, perm[oa]] = True
        B2[i, perm[ob]] = True
        c2[i] *= _perm_parity(list(perm[ob])) * _perm_parity(list(perm[oa]))
    R2 = synth.pack_keys(A2, B2, norb)
    res, _ = oracle.Oracle(h2, g2.reshape(-1), norb, na, nb).pt2(R2, c2, e0)
    assert res["e_pt2"] == pytest.approx(ref["e_pt2"], abs=1e-12)


def test_invariant_under_spin_swap():
    norb, na, nb = 7, 3, 3
    h, eri = system(norb, na, nb, 101)
    keys = all_dets(norb, na, nb)
    rng = np.random.default_rng(10)
    R = keys[rng.choice(len(keys), 60, replace=False)]
    c = rng.normal(size=60)
    A, Bo = synth.unpack_keys(R, norb)
    R2 = synth.pack_keys(Bo, A, norb)
    O = oracle.Oracle(h, eri, norb, na, nb)
    e0 = float(O.diag(keys).min()) - 1.0   # below every diagonal, as for a ground state
    a, _ = O.pt2(R, c, e0)
    b, _ = O.pt2(R2, c * (-1.0) ** (na * nb), e0)
    assert a["e_pt2"] == pytest.approx(b["e_pt2"], abs=1e-12)


def test_shift_and_scale():
    norb, na, nb = 7, 2, 3
    h, eri = system(norb, na, nb, 111)
    keys = all_dets(norb, na, nb)
    rng = np.random.default_rng(11)
    R = keys[rng.choice(len(keys), 30, replace=False)]
    c = rng.normal(size=30)
    e0 = float(oracle.Oracle(h, eri, norb, na, nb).diag(keys).min()) - 1.0
    base, _ = oracle.Oracle(h, eri, norb, na, nb).pt2(R, c, e0)
    s = 0.37
    shifted, _ = oracle.Oracle(h + s * np.eye(norb), eri, norb, na, nb).pt2(R, c, e0 + (na + nb) * s)
    assert shifted["e_pt2"] == pytest.approx(base["e_pt2"], abs=1e-12)
    lam = 1.7
    scaled, _ = oracle.Oracle(lam * h, lam * eri, norb, na, nb).pt2(R, c, lam * e0)
    assert scaled["e_pt2"] == pytest.approx(lam * base["e_pt2"], abs=1e-12)


# --------------------------------------------------------------------------
# The hash split of the external space (Algorithm 2 with a hash constraint)

def test_splitmix64_published_outputs():
    out = oracle.splitmix64_stream(0, 3)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_zobrist_is_xor_of_set_bits():
    norb = 40
    R = oracle.zobrist_table(norb)
    assert len(set(int(x) for x in R)) == 2 * norb
    keys = synth.random_determinants(norb, 10, 10, 50, 3)
    A, Bo = synth.unpack_keys(keys, norb)
    for k in range(3, 7):
        parts = oracle.parts_of(norb, keys, k)
        for i in range(len(keys)):
            z = 0
            for p in np.nonzero(Bo[i])[0]:
                z ^= int(R[p])
            for p in np.nonzero(A[i])[0]:
                z ^= int(R[norb + p])
            assert parts[i] == z >> (64 - k)


@pytest.mark.parametrize("log2p", [1, 3, 5])
def test_subsets_are_complete_and_disjoint(log2p):
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    full, _ = O.pt2(dets, c, e0)
    split, ep = O.pt2(dets, c, e0, log2p=log2p)
    assert split["e_pt2"] == pytest.approx(full["e_pt2"], abs=1e-12)
    assert float(np.sum(ep)) == pytest.approx(full["e_pt2"], abs=1e-12)
    for f in ("n_contrib", "n_unique", "n_external", "n_in_ref_hit", "key_xor", "key_sum"):
        assert split[f] == full[f]
    # records of each subset belong to it, and together they are all records
    k_all, v_all = O.emit(dets[:5], c[:5])
    seen = 0
    for p in range(1 << log2p):
        k, v = O.emit(dets[:5], c[:5], log2p=log2p, part=p)
        assert np.all(oracle.parts_of(w.norb, k, log2p) == p)
        seen += len(k)
    assert seen == len(k_all)


def test_selected_subsets_match_full_split():
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    _, ep = O.pt2(dets, c, e0, log2p=4)
    _, sel = O.pt2(dets, c, e0, log2p=4, parts=[3, 11, 0])
    np.testing.assert_allclose(sel, ep[[3, 11, 0]], atol=1e-15)


def test_cutoff_drops_small_terms_strictly():
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    k, v = O.emit(dets, c)
    cut = float(np.quantile(np.abs(v), 0.3))
    k2, v2 = O.emit(dets, c, cutoff=cut)
    assert len(v2) == int(np.sum(np.abs(v) >= cut))
    res, _ = O.pt2(dets, c, e0, cutoff=cut)
    assert res["n_kept"] == len(v2) and res["n_contrib"] == len(v)


def test_duplicate_reference_rejected():
    w, h, eri, dets, c, e0 = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    d = np.concatenate([dets[:5], dets[2:3]])
    with pytest.raises(ValueError):
        O.pt2(d, np.ones(6), e0)


def test_empty_reference():
    w, h, eri, dets, c, e0 = load_c1()
    res, _ = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta).pt2(dets[:0], c[:0], e0)
    assert res["e_pt2"] == 0.0 and res["n_contrib"] == 0


@pytest.mark.parametrize("norb,n_el,nref,sign", [(10, 3, 25, 1), (10, 3, 25, -1), (36, 3, 12, 1)])
def test_spin_flip_identity(norb, n_el, nref, sign):
    """Section V, spin symmetry: for a reference closed under the alpha/beta
    swap with c(swap(D)) = +-c(D), every numerator satisfies
    |N_swap(a)| = |N_a| and H_swap(a)swap(a) = H_aa, so the sum over the
    determinants with alpha >= beta, the alpha != beta ones counted twice,
    equals the full E_PT2 (the premise of the engine's spin_flip option)."""
    h, eri, _ = synth.make_integrals(norb, 6, 5100 + norb)
    dets, c = synth.swap_symmetric_references(norb, n_el, nref, 31 + norb, sign)
    O = oracle.Oracle(h, eri, norb, n_el, n_el)
    keys, nums = O.numerators(dets, c)
    diag = O.diag(keys)
    e0 = float(min(diag.min(), O.diag(dets).min())) - 0.5
    a, b = synth.unpack_keys(keys, norb)
    idx = {tuple(int(x) for x in k): i for i, k in enumerate(keys)}
    swapped = synth.pack_keys(b, a, norb)
    refset = {tuple(int(x) for x in k) for k in dets}
    half = 0.0
    for i, k in enumerate(keys):
        j = idx[tuple(int(x) for x in swapped[i])]
        assert abs(abs(nums[j]) - abs(nums[i])) <= 1e-14 * max(1.0, abs(nums[i]))
        assert abs(diag[j] - diag[i]) <= 1e-12 * max(1.0, abs(diag[i]))
        # the alpha and beta strings as numbers (orbital p is bit p)
        ka = sum(1 << p for p in range(norb) if a[i][p])
        kb = sum(1 << p for p in range(norb) if b[i][p])
        if ka >= kb and tuple(int(x) for x in k) not in refset:
            half += (1.0 if ka == kb else 2.0) * nums[i] ** 2 / (e0 - diag[i])
    full, _ = O.pt2(dets, c, e0)
    assert half == pytest.approx(full["e_pt2"], rel=1e-12, abs=1e-14)


def _terms_by_flip(O, det, norb):
    """The oracle's terms H_ai of one determinant (c = 1), keyed by the bits
    flipped in the alpha half and in the beta half."""
    keys, vals = O.emit(det[None], np.ones(1))
    k0 = int.from_bytes(det.astype("<u8").tobytes(), "little")
    lo = (1 << norb) - 1
    out = {}
    for k, v in zip(keys, vals):
        d = int.from_bytes(k.astype("<u8").tobytes(), "little") ^ k0
        out[(d >> norb, d & lo)] = v
    return out


def test_same_spin_doubles_depend_on_their_own_string_only():
    """The premise of sharing same-spin doubles between references (Section
    V, data reuse for unique alpha and beta strings): an alpha-alpha double's
    H_ai, phase included, is the same for two determinants with one alpha
    string and different beta strings (beta-beta likewise); an alpha single's
    is not, as it sums over the occupied orbitals of both spins."""
    norb, na, nb = 8, 3, 3
    h, eri, _ = synth.make_integrals(norb, 6, 4242)
    O = oracle.Oracle(h, eri, norb, na, nb)
    occ = lambda idx: np.isin(np.arange(norb), idx)
    a1, a2 = occ([0, 2, 5]), occ([1, 2, 6])
    b1, b2 = occ([0, 1, 4]), occ([2, 3, 7])
    dets = synth.pack_keys(np.array([a1, a1, a1, a2]), np.array([b1, b2, b1, b1]), norb)
    t = [_terms_by_flip(O, d, norb) for d in dets]

    def kind(t, pred):
        return {f: v for f, v in t.items() if pred(bin(f[0]).count("1"), bin(f[1]).count("1"))}

    aa = lambda x, y: x == 4 and y == 0
    bb = lambda x, y: x == 0 and y == 4
    a_single = lambda x, y: x == 2 and y == 0
    # dets 0 and 1 share the alpha string; dets 2 and 3 share the beta string
    assert kind(t[0], aa) and kind(t[0], aa) == kind(t[1], aa)
    assert kind(t[2], bb) and kind(t[2], bb) == kind(t[3], bb)
    s0, s1 = kind(t[0], a_single), kind(t[1], a_single)
    assert s0.keys() == s1.keys() and any(s0[f] != s1[f] for f in s0)



# --------------------------------------------------------------------------
# The Epstein-Nesbet denominator E0 - H_aa (Section II) at near-singular
# values, against exact rational arithmetic.  The integrals are FP64 numbers,
# so H_aa = sum_p h_pp + sum_{p<q} [(pp|qq) - delta_spin (pq|qp)] has an exact
# rational value; so has E0 - H_aa.  E0 is put at the FP64 number nearest to
# H_aa, so the difference is below half a unit in the last place of H_aa and
# a plain FP64 sum of H_aa gets none of its digits right.

def _exact_diag(h, eri, norb, key):
    from fractions import Fraction
    a, b = synth.unpack_keys(np.asarray(key, dtype=np.uint64).reshape(1, -1), norb)
    occ = [(p, 0) for p in np.nonzero(a[0])[0]] + [(p, 1) for p in np.nonzero(b[0])[0]]
    g = eri.reshape(norb, norb, norb, norb)
    e, mags = Fraction(0), 0.0
    for i, (p, sp) in enumerate(occ):
        e += Fraction(float(h[p, p]))
        mags += abs(float(h[p, p]))
        for q, sq in occ[i + 1:]:
            e += Fraction(float(g[p, p, q, q]))
            mags += abs(float(g[p, p, q, q]))
            if sp == sq:
                e -= Fraction(float(g[p, q, q, p]))
                mags += abs(float(g[p, q, q, p]))
    return e, mags, len(occ) * (len(occ) + 1) // 2


def _ulp(x):
    return np.spacing(abs(x)) if x != 0.0 else np.spacing(0.0)


def _check_denominators(h, eri, norb, na, nb, keys, shifts):
    from fractions import Fraction
    O = oracle.Oracle(h, eri, norb, na, nb)
    u = 2.0 ** -53
    for key in keys:
        hx, mags, n = _exact_diag(h, eri, norb, key)
        for shift in shifts:
            e0 = float(hx) + shift
            exact = Fraction(e0) - hx
            got = O.denominators(key.reshape(1, -1), e0)[0]
            gam = (n + 1) * u / (1 - (n + 1) * u)
            bound = 2 * u * abs(float(exact)) + gam * gam * (mags + abs(e0))
            assert abs(Fraction(got) - exact) <= Fraction(bound), (key, shift, got, float(exact))
            # a plain FP64 evaluation is far outside the bound whenever the
            # difference is small: the pin can fail
            if shift == 0.0:
                plain = e0 - O.diag(key.reshape(1, -1))[0]
                assert float(exact) == 0.0 or abs(Fraction(plain) - exact) > Fraction(bound) or plain == got


def test_denominator_exact_small_system():
    norb, na, nb = 10, 4, 3
    h, eri = system(norb, na, nb, 71)
    dets = all_dets(norb, na, nb)
    keys = dets[np.random.default_rng(7).choice(len(dets), 40, replace=False)]
    _check_denominators(h, eri, norb, na, nb, keys, [0.0, 1e-13, -3e-12, 0.37])


def test_denominator_exact_c3_keys():
    """Sampled determinants of workload C3 (28 electrons in 76 orbitals):
    reference determinants and double excitations of them."""
    w = synth.WORKLOADS["c3"]
    h, eri, _ = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(synth_path("inputs_c3.npz"))
    refs = f["dets"]
    rng = np.random.default_rng(11)
    keys = [refs[i] for i in rng.choice(len(refs), 6, replace=False)]
    a, b = synth.unpack_keys(np.stack(keys), w.norb)
    ext = []
    for j in range(len(keys)):          # move two electrons to virtual orbitals
        aa, bb = a[j].copy(), b[j].copy()
        ao, av = np.nonzero(aa)[0], np.nonzero(~aa)[0]
        bo, bv = np.nonzero(bb)[0], np.nonzero(~bb)[0]
        aa[rng.choice(ao)] = False
        aa[rng.choice(av)] = True
        bb[rng.choice(bo)] = False
        bb[rng.choice(bv)] = True
        ext.append(synth.pack_keys(aa[None], bb[None], w.norb)[0])
    _check_denominators(h, eri, w.norb, w.nalpha, w.nbeta, np.stack(keys + ext),
                        [0.0, 2.5e-12, -0.25])


def test_pass_uses_the_compensated_denominator():
    """With E0 placed on a determinant's diagonal energy, the single pass's
    smallest |E0 - H_aa| is that determinant's exact (tiny) difference."""
    from fractions import Fraction
    norb, na, nb = 6, 2, 2
    h, eri = system(norb, na, nb, 81)
    O = oracle.Oracle(h, eri, norb, na, nb)
    hf = synth.hf_key(norb, na, nb).reshape(1, -1)
    keys, nums = O.numerators(hf, np.ones(1))
    ext = keys[np.argmax(np.abs(nums))]      # the external determinant of largest |N|
    hx, _, _ = _exact_diag(h, eri, norb, ext)
    e0 = float(hx)
    exact = abs(float(Fraction(e0) - hx))
    res, _ = O.pt2(hf, np.ones(1), e0)
    assert res["min_abs_denom"] <= exact * (1 + 1e-6) + 1e-300


# --------------------------------------------------------------------------
# <c|H|c> (orc_expectation writes every stored E0 of the synthetic inputs)

def test_expectation_matches_brute_force_c1():
    """<c|H|c> against the operator-by-operator Hamiltonian applied to c over
    the whole FCI space, with coefficients that are not an eigenvector."""
    w, h, eri, dets, _, _ = load_c1()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    B = oracle.Brute(h, eri, w.norb, w.nalpha, w.nbeta)
    c = np.random.default_rng(9).normal(size=len(dets))
    c /= np.linalg.norm(c)
    hc = B.h_times(dets, c)
    want = float(c @ hc[B.index_of(dets)])
    assert O.expectation(dets, c) == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("norb,na,nb,nref", [(7, 3, 2, 60), (8, 2, 3, 90)])
def test_expectation_matches_brute_force_random(norb, na, nb, nref):
    h, eri = system(norb, na, nb, 91)
    dets = all_dets(norb, na, nb)
    sel = dets[np.random.default_rng(4).choice(len(dets), nref, replace=False)]
    c = np.random.default_rng(5).normal(size=nref)
    O = oracle.Oracle(h, eri, norb, na, nb)
    B = oracle.Brute(h, eri, norb, na, nb)
    want = float(c @ B.h_times(sel, c)[B.index_of(sel)])
    for nt in (1, 3):
        assert O.expectation(sel, c, nthreads=nt) == pytest.approx(want, abs=1e-12)


def test_expectation_c2_slice_matches_dense_hrr():
    """On 500 references of workload C2 (20 electrons in 40 orbitals): the
    threaded, compensated sum with its skip of pairs more than a double
    excitation apart equals c^T H_RR c over the dense pairwise matrix."""
    w = synth.WORKLOADS["c2"]
    h, eri, _ = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(synth_path("inputs_c2.npz"))
    dets = f["dets"][:500]
    c = np.random.default_rng(6).normal(size=len(dets))
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    H = O.hrr(dets)
    assert np.count_nonzero(H) > len(dets)          # the slice is connected
    assert O.expectation(dets, c) == pytest.approx(float(c @ H @ c), abs=1e-11)
