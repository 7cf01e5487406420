"""Seeded synthetic inputs for the PT2 engine and its oracle.

This module draws random numbers and lays out bitstrings. It holds none of
the perturbation-theory arithmetic: no matrix elements, no diagonal energies,
no excitation phases. Both the HIP path and the CPU oracle read what it
produces, and neither imports the other.

Conventions shared by every consumer (the paper fixes only that alpha
orbitals are the most significant digits of a determinant bitstring, in the
triplet-constraint subsection of Section III):

* A determinant key is a 2*norb-bit integer stored as W = ceil(2*norb/64)
  little-endian uint64 words (word 0 least significant).
* Beta orbital p sits at bit p; alpha orbital p sits at bit norb + p.
* Integrals are real, in chemists' notation (pq|rs), stored row-major as
  eri[((p*n + q)*n + r)*n + s]; h is a symmetric norb x norb matrix.

Integral recipe (per workload): h_pp = -2.0 + 0.25 p, off-diagonal
h_pq ~ N(0, 0.05) (0.05 read as the standard deviation); eri = sum_L B^L (x) B^L
with symmetric B^L whose entries are N(0, 0.1). Draw order from
numpy's PCG64 ``default_rng(seed)``: the h upper triangle (row-major), then
each B^L's upper triangle including the diagonal (L-major), then the
coefficient signs.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "key_words", "pack_keys", "unpack_keys",
    "hf_key", "make_integrals", "excitation_pool", "decaying_coefficients",
    "draw_signs", "select_lowest", "random_determinants", "n_excitations_per_det",
    "swap_symmetric_references",
    "ladder_references", "Request", "serving_requests", "request_inputs",
]


@dataclass(frozen=True)
class Workload:
    """One synthetic system: sizes, seed and the reference-selection rule."""
    name: str
    norb: int
    nalpha: int
    nbeta: int
    n_chol: int
    n_ref: int
    seed: int
    pool_rank: int          # reference pool: HF plus excitations up to this rank
    decay: float | None     # c_i = +-exp(-decay*rank); None: eigenvector of H_RR
    notes: str = field(default="")


# The five workloads; the paper's molecular systems are not available, so
# these synthetic systems stand in for them by shape (electrons, orbitals,
# reference size and contribution count).
WORKLOADS = {
    "c1": Workload("c1", 12, 4, 4, 24, 200, 1001, 2, None,
                   "(4a,4b)/12, eigenvector reference; FCI space 245,025"),
    "c2": Workload("c2", 40, 10, 10, 64, 10_000, 1002, 3, 0.002,
                   "(10a,10b)/40, ~1.3e9 contributions, one partition"),
    "c3": Workload("c3", 76, 14, 14, 100, 100_000, 1003, 2, 3e-4,
                   "(14a,14b)/76, ~1.1e11 contributions, hash partitions"),
    "c5": Workload("c5", 100, 18, 18, 128, 300_000, 1005, 2, 1e-4,
                   "(18a,18b)/100, ~1e12 contributions"),
}


def key_words(norb: int) -> int:
    return (2 * norb + 63) // 64


def n_excitations_per_det(norb: int, na: int, nb: int) -> int:
    """Closed-form count of single plus double excitations of any determinant."""
    va, vb = norb - na, norb - nb
    c2 = lambda n: n * (n - 1) // 2
    return (na * va + nb * vb + c2(na) * c2(va) + c2(nb) * c2(vb)
            + na * va * nb * vb)


def pack_keys(alpha_occ: np.ndarray, beta_occ: np.ndarray, norb: int) -> np.ndarray:
    """Pack boolean occupations (n, norb) into keys (n, W) of uint64."""
    alpha_occ = np.asarray(alpha_occ, dtype=bool)
    beta_occ = np.asarray(beta_occ, dtype=bool)
    n = alpha_occ.shape[0]
    W = key_words(norb)
    bits = np.zeros((n, 64 * W), dtype=bool)
    bits[:, :norb] = beta_occ
    bits[:, norb:2 * norb] = alpha_occ
    packed = np.packbits(bits, axis=1, bitorder="little")
    return np.ascontiguousarray(packed).view("<u8").reshape(n, W).astype(np.uint64)


def unpack_keys(keys: np.ndarray, norb: int) -> tuple[np.ndarray, np.ndarray]:
    """Inverse of pack_keys: returns (alpha_occ, beta_occ) boolean arrays."""
    keys = np.ascontiguousarray(np.asarray(keys, dtype="<u8"))
    n, W = keys.shape
    bits = np.unpackbits(keys.view(np.uint8).reshape(n, 8 * W), axis=1,
                         bitorder="little").astype(bool)
    return bits[:, norb:2 * norb], bits[:, :norb]


def hf_key(norb: int, na: int, nb: int) -> np.ndarray:
    a = np.zeros((1, norb), bool)
    b = np.zeros((1, norb), bool)
    a[0, :na] = True
    b[0, :nb] = True
    return pack_keys(a, b, norb)[0]


def make_integrals(norb: int, n_chol: int, seed: int):
    """Draw (h, eri, rng) for one workload; eri is exactly 8-fold symmetric.

    Returns the generator so that later draws (coefficient signs) continue
    the same stream.
    """
    rng = np.random.default_rng(seed)
    h = np.diag(-2.0 + 0.25 * np.arange(norb, dtype=np.float64))
    iu = np.triu_indices(norb, k=1)
    off = rng.normal(0.0, 0.05, size=len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    # B^L on packed pairs p <= q, row-major over the upper triangle.
    iu0 = np.triu_indices(norb, k=0)
    npair = len(iu0[0])
    B = rng.normal(0.0, 0.1, size=(n_chol, npair))
    # M[P, Q] = sum_L B[L, P] B[L, Q]; take one triangle and mirror it so the
    # tensor is symmetric bit for bit under all eight index permutations.
    M = B.T @ B
    M = np.triu(M) + np.triu(M, 1).T
    pair = np.empty((norb, norb), dtype=np.int64)
    pair[iu0] = np.arange(npair)
    pair[(iu0[1], iu0[0])] = np.arange(npair)
    eri = M[pair[:, :, None, None], pair[None, None, :, :]]
    return h, np.ascontiguousarray(eri), rng


def _spin_configs(norb: int, n: int, k: int) -> np.ndarray:
    """All occupations of one spin with exactly k holes below n and k particles above."""
    out = []
    for holes in itertools.combinations(range(n), k):
        for parts in itertools.combinations(range(n, norb), k):
            occ = np.zeros(norb, bool)
            occ[:n] = True
            occ[list(holes)] = False
            occ[list(parts)] = True
            out.append(occ)
    if not out:
        return np.zeros((0, norb), bool)
    return np.array(out)


def excitation_pool(norb: int, na: int, nb: int, max_rank: int) -> np.ndarray:
    """HF plus every determinant whose total excitation rank is 1..max_rank.

    Order: by total rank, then alpha rank descending, then alpha configuration,
    then beta configuration. The result is a (n, W) uint64 key array with HF
    first.
    """
    pieces = []
    for rank in range(0, max_rank + 1):
        for ka in range(min(rank, na, norb - na), -1, -1):
            kb = rank - ka
            if kb > min(nb, norb - nb):
                continue
            A = _spin_configs(norb, na, ka)
            Bc = _spin_configs(norb, nb, kb)
            if len(A) == 0 or len(Bc) == 0:
                continue
            ia = np.repeat(np.arange(len(A)), len(Bc))
            ib = np.tile(np.arange(len(Bc)), len(A))
            # pack in slices to bound memory on the large pools
            step = 1 << 20
            for s in range(0, len(ia), step):
                pieces.append(pack_keys(A[ia[s:s + step]], Bc[ib[s:s + step]], norb))
    return np.concatenate(pieces, axis=0)


def select_lowest(keys: np.ndarray, energies: np.ndarray, n_ref: int,
                  force_first: int | None = 0) -> np.ndarray:
    """Indices of the n_ref lowest energies, ties broken by the key value.

    ``force_first`` (an index into keys) is placed at rank 0 regardless of its
    energy. The energies are supplied by the caller.
    """
    keys = np.asarray(keys)
    W = keys.shape[1]
    # lexsort: last key is primary -> energy, then key words most significant first
    order = np.lexsort(tuple(keys[:, w] for w in range(W)) + (energies,))
    if force_first is not None:
        order = np.concatenate([[force_first], order[order != force_first]])
    return order[:n_ref]


def draw_signs(rng: np.random.Generator, n: int) -> np.ndarray:
    """Random +-1 signs; the first (HF) sign is +1. Consumes n draws."""
    s = np.where(rng.integers(0, 2, size=n) == 0, 1.0, -1.0)
    s[0] = 1.0
    return s


def decaying_coefficients(n: int, decay: float, signs: np.ndarray) -> np.ndarray:
    """c_rank = sign * exp(-decay * rank), normalised to unit length."""
    c = signs[:n] * np.exp(-decay * np.arange(n, dtype=np.float64))
    return c / math.sqrt(float(np.dot(c, c)))


def swap_symmetric_references(norb: int, n_el: int, n: int, seed: int, sign: int = 1):
    """A reference closed under the alpha/beta swap (S_z = 0, n_el electrons of
    each spin): n random determinants, their swap partners added, and
    coefficients with c(swap(D)) = sign * c(D) (a determinant equal to its own
    swap gets 0 when sign is -1), normalised.  Returns (dets (m, W) uint64, c)."""
    base = random_determinants(norb, n_el, n_el, n, seed)
    a, b = unpack_keys(base, norb)
    both = np.concatenate([base, pack_keys(b, a, norb)])
    keys, inv = np.unique(both, axis=0, return_inverse=True)
    inv = np.asarray(inv).reshape(-1)
    rng = np.random.default_rng(seed + 1)
    c = np.zeros(len(keys))
    draw = rng.normal(size=n)
    for i in range(n):
        d, s_ = inv[i], inv[n + i]
        if d == s_:
            c[d] = draw[i] if sign > 0 else 0.0
        else:
            c[d] = draw[i]
            c[s_] = sign * draw[i]
    keep = c != 0.0
    keys, c = keys[keep], c[keep]
    return np.ascontiguousarray(keys), c / np.linalg.norm(c)


def random_determinants(norb: int, na: int, nb: int, n: int, seed: int) -> np.ndarray:
    """n distinct uniformly random determinants (for edge-case tests)."""
    rng = np.random.default_rng(seed)
    seen = set()
    rows = []
    while len(rows) < n:
        a = np.zeros(norb, bool)
        b = np.zeros(norb, bool)
        a[rng.choice(norb, na, replace=False)] = True
        b[rng.choice(norb, nb, replace=False)] = True
        k = pack_keys(a[None], b[None], norb)[0]
        t = tuple(int(x) for x in k)
        if t in seen:
            continue
        seen.add(t)
        rows.append(k)
    return np.array(rows, dtype=np.uint64).reshape(n, key_words(norb))


# ---------------------------------------------------------------------------
# Serving workload: 200 requests of different active spaces.

def _displacement_strings(norb: int, n: int, max_e: int):
    """Occupations of one spin whose orbital-index displacement from the
    lowest n orbitals, sum_i (o_i - i), is at most max_e; returns
    (list of occupied-index tuples, list of displacements)."""
    v = norb - n
    out, es = [], []

    def rec(i, lo, total, acc):
        if i == n:
            out.append(tuple(k + d for k, d in enumerate(acc)))
            es.append(total)
            return
        # displacements are non-decreasing and bounded by v
        for d in range(lo, v + 1):
            # the remaining n - i displacements are all >= d
            if total + d * (n - i) > max_e:
                break
            acc.append(d)
            rec(i + 1, d, total + d, acc)
            acc.pop()

    if n == 0:
        return [()], [0]
    rec(0, 0, 0, [])
    return out, es


def ladder_references(norb: int, na: int, nb: int, n_ref: int) -> np.ndarray:
    """The n_ref determinants lowest in orbital-ladder excitation energy: the
    total displacement of occupied orbital indices from the aufbau
    determinant (alpha plus beta), ties broken by the bitstring.  With the
    linear h_pp = -2 + 0.25 p of this recipe this is the one-body energy
    ordering; it uses orbital indices only, no integrals."""
    max_e = 0
    while True:
        sa, ea = _displacement_strings(norb, na, max_e)
        sb, eb = _displacement_strings(norb, nb, max_e)
        ea_arr, eb_arr = np.array(ea), np.array(eb)
        cnt = sum(int(np.sum(eb_arr <= max_e - e)) for e in ea)
        if cnt >= n_ref or max_e > 4 * norb:
            break
        max_e += 1
    ia, ib = np.nonzero(ea_arr[:, None] + eb_arr[None, :] <= max_e)
    SA = np.zeros((len(sa), norb), bool)
    SB = np.zeros((len(sb), norb), bool)
    for r, occ in enumerate(sa):
        SA[r, list(occ)] = True
    for r, occ in enumerate(sb):
        SB[r, list(occ)] = True
    keys = pack_keys(SA[ia], SB[ib], norb)
    energy = ea_arr[ia] + eb_arr[ib]
    W = keys.shape[1]
    order = np.lexsort(tuple(keys[:, w] for w in range(W)) + (energy,))
    return np.ascontiguousarray(keys[order[:n_ref]])


@dataclass(frozen=True)
class Request:
    index: int
    nalpha: int
    norb: int
    n_ref: int
    seed: int
    arrival_s: float


def serving_requests(count: int = 200, rate_per_s: float = 1.0) -> list[Request]:
    """Request parameters: electrons uniform on {10, 12, ..., 24} (equal alpha
    and beta), orbitals round(U[2.0, 2.5] * electrons), references
    round(exp U[ln 1e3, ln 5e4]), integral seed 4000 + j; Poisson arrivals of
    the given rate (exponential gaps from seed 4999; parameters from 4998)."""
    prm = np.random.default_rng(4998)
    arr = np.random.default_rng(4999)
    t, out = 0.0, []
    for j in range(count):
        ne = int(prm.integers(5, 13)) * 2
        norb = int(round(prm.uniform(2.0, 2.5) * ne))
        nref = int(round(math.exp(prm.uniform(math.log(1e3), math.log(5e4)))))
        t += float(arr.exponential(1.0 / rate_per_s))
        out.append(Request(j, ne // 2, norb, nref, 4000 + j, t))
    return out


def request_inputs(req: Request, n_chol: int = 64, decay: float = 0.002):
    """(h, eri, dets, c) of one serving request; E0 is stored separately."""
    h, eri, rng = make_integrals(req.norb, n_chol, req.seed)
    dets = ladder_references(req.norb, req.nalpha, req.nalpha, req.n_ref)
    c = decaying_coefficients(req.n_ref, decay, draw_signs(rng, req.n_ref))
    return h, eri, dets, c
