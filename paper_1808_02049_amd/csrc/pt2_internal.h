// Internal declarations shared by the HIP translation units of the PT2 engine.
// Nothing here is part of the C-ABI (include/pt2.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt2 {

constexpr int MAXW = 4;        // 2*norb <= 256 bits
// Payload modes (the values of pt2_options.precision)
constexpr int PM_FP64 = 0;          // FP64 integrals, arithmetic and payload
constexpr int PM_FP32_PAYLOAD = 1;  // FP64 arithmetic, payload rounded once to FP32
constexpr int PM_FP32_ARITH = 2;    // FP32 integrals, arithmetic and payload
constexpr int MAXORB = 128;
constexpr int SORT_THREADS = 256;
#ifndef PT2_XCD_TILES
#define PT2_XCD_TILES 1
#endif
#ifndef PT2_WIDE_PIPE
#define PT2_WIDE_PIPE 1
#endif
#ifndef PT2_SORT_ITEMS
#define PT2_SORT_ITEMS 8
#endif
constexpr int SORT_ITEMS = PT2_SORT_ITEMS;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;   // records per radix tile
// Records per thread for keys whose digits are uniform (hash records): every
// digit value takes a share of each tile, so longer tiles give longer runs.
constexpr int SORT_ITEMS_WIDE = 2 * SORT_ITEMS;
constexpr int SCAN_CHUNK = 256;                        // tiles per chunk of the offset scan
constexpr int RED_THREADS = 256;
constexpr int RED_ITEMS = 4;
constexpr int RED_TILE = RED_THREADS * RED_ITEMS;     // records per reduce tile
constexpr int RED_GRID = 4096;                        // fixed -> bit-reproducible sums
constexpr int RED_LDS_REFS = 64;                      // reference keys staged per tile
constexpr size_t RED_LDS_MAX = 64 * 1024;             // dynamic LDS of one single-pass workgroup
constexpr int GEN_THREADS = 256;
constexpr int REUSE_GROUP = 32;                      // references per workgroup of k_gen_spin
constexpr int64_t REUSE_CHUNK = 4096;                // same-spin doubles per workgroup of k_gen_spin

// Device-side error flags (bitmask in Flags::err).
enum : uint32_t {
    ERR_POPCOUNT = 1u,      // a reference has the wrong electron count
    ERR_STRAY_BITS = 2u,    // bits at or above 2*norb
    ERR_DUPLICATE = 4u,     // two equal reference determinants
    ERR_BOUNDS = 8u,        // a radix scatter destination fell outside the buffer
    ERR_SINGULAR = 16u,     // E0 - H_aa == 0 for an external determinant
    ERR_OVERFLOW = 32u,     // a compacted write ran past its planned range
    ERR_SWAP_MISSING = 64u, // spin flip: a reference's swap partner is absent or
                            // has a coefficient of another magnitude
    SWAP_SAME = 128u,       // spin flip: some c(swap(D)) == c(D) (not an error)
    SWAP_NEG = 256u         // spin flip: some c(swap(D)) == -c(D), D != swap(D)
};

struct Flags {
    uint32_t err;
    uint32_t pad;
};

// Compressed record keys.  Per spin, the occupied orbitals o_1 < ... < o_n
// of a string have the colex rank sum_i C(o_i, i) (the combinatorial number
// system), a bijection onto [0, C(norb, n)) that orders strings as their
// bitmasks do.  A record key (rank_alpha << bb) | rank_beta therefore sorts
// exactly as the determinant bitstring (alpha is the high part of both) in
// fewer bits: 60 instead of 80 for (10a,10b) in 40 orbitals.
struct KeyCodec {
    int hash;               // 1: records carry (Zobrist hash, parent and flips) instead (see below)
    int hpacked;            // 1: FP32 hash records packed into two 8-byte words (hash_pack)
    uint64_t hash_mask;     // bits of the hash stored: all 64, its top bits (fewer digit
                            // passes), or its low bits (tests that force collisions)
    int on;                 // 1: records carry rank keys
    int kw;                 // key words of a record (1 or 2)
    int ktop;               // bytes of the records' top key plane
    int kbits;              // key bits
    int bb;                 // bits of the beta rank
    int stride;             // row length of the binomial table
    const uint64_t *binom;  // C(x, j) at [x * stride + j], 0 <= x <= norb, 0 <= j < stride (device)
};

// Hash records.  A record holds the 64-bit Zobrist hash of its determinant
// (the sort key), an auxiliary word (parent index << 32 | four flipped
// spin-orbitals, one byte each, 0xFF unused) and the payload.  The sort takes
// 8 digit passes whatever norb is; the single pass rebuilds the bitstring from
// the parent and resolves the rare determinants whose hashes collide.
constexpr uint32_t FLIP_NONE = 0xFFu;

// Packed FP32 hash records, for norb <= HC_MAX_NORB and fewer than
// HC_MAX_REFS references, with at most HC_KEPT_BITS kept hash bits: the
// auxiliary word shrinks to 48 bits, parent << 29 | a 29-bit code of the
// flips, held in the free low 16 bits of the hash word and the high half of
// a second word whose low half is the FP32 payload.  16-byte records in two
// full 8-byte planes (a 4-byte plane would write half lines per bucket run).
// The code holds four 7-bit spatial orbitals and a bit: a same-spin double
// (bit 1) stores its removed r1 < r2 in that order for alpha and swapped for
// beta, then its added a1, a2; an alpha-beta double (bit 0) stores alpha r,
// a, then beta r, a; a single (bit 0) stores r, a, then 127 and 126 (alpha)
// or 127 (beta).
constexpr int HC_MAX_NORB = 126;
constexpr int64_t HC_MAX_REFS = (int64_t)1 << 19;
constexpr int HC_KEPT_BITS = 48;
constexpr int HC_CODE_BITS = 29;

__host__ __device__ inline uint64_t hash_pack(uint64_t aux, int norb)
{
    const uint32_t f0 = (uint32_t)aux & 255u, f1 = (uint32_t)(aux >> 8) & 255u;
    const uint32_t f2 = (uint32_t)(aux >> 16) & 255u, f3 = (uint32_t)(aux >> 24) & 255u;
    const uint32_t n = (uint32_t)norb;
    uint32_t x0, x1, x2, x3, bit = 0;
    if (f2 == FLIP_NONE) {
        const bool al = f0 >= n;
        const uint32_t off = al ? n : 0u;
        x0 = f0 - off, x1 = f1 - off, x2 = 127u, x3 = al ? 126u : 127u;
    } else if (f0 >= n && f2 < n) {
        x0 = f0 - n, x1 = f1 - n, x2 = f2, x3 = f3;
    } else {
        const bool al = f0 >= n;
        const uint32_t off = al ? n : 0u;
        bit = 1;
        x0 = al ? f0 - off : f1 - off, x1 = al ? f1 - off : f0 - off, x2 = f2 - off, x3 = f3 - off;
    }
    const uint64_t code = (uint64_t)(bit << 28 | x0 | x1 << 7 | x2 << 14 | x3 << 21);
    return (aux >> 32) << HC_CODE_BITS | code;
}

__host__ __device__ inline uint64_t hash_unpack(uint64_t a48, int norb)
{
    const uint32_t c = (uint32_t)(a48 & ((1ull << HC_CODE_BITS) - 1));
    const uint32_t x0 = c & 127u, x1 = (c >> 7) & 127u, x2 = (c >> 14) & 127u, x3 = (c >> 21) & 127u;
    const uint32_t n = (uint32_t)norb;
    uint32_t f0, f1, f2, f3;
    if (c >> 28) {
        if (x0 < x1)
            f0 = n + x0, f1 = n + x1, f2 = n + x2, f3 = n + x3;
        else
            f0 = x1, f1 = x0, f2 = x2, f3 = x3;
    } else if (x2 == 127u) {
        const uint32_t off = x3 == 126u ? n : 0u;
        f0 = off + x0, f1 = off + x1, f2 = FLIP_NONE, f3 = FLIP_NONE;
    } else {
        f0 = n + x0, f1 = n + x1, f2 = x2, f3 = x3;
    }
    return (a48 >> HC_CODE_BITS) << 32 | (uint64_t)(f0 | f1 << 8 | f2 << 16 | f3 << 24);
}

// Device view of the Hamiltonian (all pointers are device memory).
struct DevSys {
    int norb, na, nb, W;
    KeyCodec kc;
    const double *h;    // norb x norb
    const double *V;    // norb^4, (pq|rs) row-major
    const float *h32;   // FP32 copies (precision form), else null
    const float *V32;
    const double *T;    // packed upper-triangular spin-orbital pair table for the
                        // diagonal, row b1 at b1*nso - b1*(b1-1)/2 - b1, column b2 >= b1:
                        // T[b][b] = h_pp; T[b1][b2] = (pp|qq) - [same spin](pq|qp)
    const double *Tlo;  // the exact rounding error of each T entry (T + Tlo is exact)
    const double *A2;   // (ra|qb) - (rb|qa) for r < q, a < b at [pair(r, q) * npair + pair(a, b)],
                        // pair(i, j) = i (2 norb - i - 1) / 2 + j - i - 1, npair = norb (norb - 1) / 2
                        // (same-spin doubles: one read instead of two), or null
    const uint64_t *R;  // Zobrist words, one per bit (2 norb)
    int z2;             // spin flip: generate alpha >= beta only, weight alpha != beta by 2
};

// The anchor of the diagonals (Appendix, fast diagonal): one determinant A of
// the reference (the first in sorted order) whose energy and g vector
// g_x = h_x + sum_{c in A, c != x} T[x][c] are computed once per evaluation;
// every E0 - H_aa is then taken relative to A.  Pair energies T[x][y] with x
// or y in a spatial orbital occupied in A (the "hot" rows) are kept as the
// two integrals J = (pp|qq) and K = (pq|qp) so that the single pass holds
// them in LDS; other pairs come from the packed table DevSys::T.
constexpr int ANC_HOT_MAX = 2048;  // entries of the hot J (and K) rows
struct AnchorBlk {
    uint64_t bits[MAXW];
    double d0h, d0l;                     // E0 - E(A), double-double
    int nh;                              // hot spatial orbitals (0: no hot rows)
    int pad;
    int16_t hr[MAXORB];                  // hot row of a spatial orbital, -1 if none
    double gh[2 * MAXORB], gl[2 * MAXORB];  // g_x(A), double-double
    double Jh[ANC_HOT_MAX], Kh[ANC_HOT_MAX];  // row r (the r-th hot orbital p), column q: (pp|qq), (pq|qp)
};

// The alpha string (bits norb..2norb-1) and the beta string (bits 0..norb-1)
// of a bitstring, each as a 128-bit number (hi, lo); norb <= 127.
template <int W>
__host__ __device__ inline uint64_t bits64_at(const uint64_t (&k)[W], int start)
{
    const int w = start >> 6, sh = start & 63;
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < W; i++) {
        if (i == w)
            lo = k[i] >> sh;
        if (sh && i == w + 1)
            hi = k[i] << (64 - sh);
    }
    return lo | hi;
}

__host__ __device__ inline uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1); }

template <int W>
__host__ __device__ inline void spin_strings(const uint64_t (&k)[W], int norb, uint64_t &alo, uint64_t &ahi,
                                             uint64_t &blo, uint64_t &bhi)
{
    blo = bits64_at<W>(k, 0) & low_mask(norb);
    bhi = norb > 64 ? bits64_at<W>(k, 64) & low_mask(norb - 64) : 0ull;
    alo = bits64_at<W>(k, norb) & low_mask(norb);
    ahi = norb > 64 ? bits64_at<W>(k, norb + 64) & low_mask(norb - 64) : 0ull;
}

// alpha string >= beta string (the half the spin flip generates)
template <int W>
__host__ __device__ inline bool alpha_not_below_beta(const uint64_t (&k)[W], int norb)
{
    uint64_t alo, ahi, blo, bhi;
    spin_strings<W>(k, norb, alo, ahi, blo, bhi);
    return ahi != bhi ? ahi > bhi : alo >= blo;
}

// weight of a generated determinant's term under the spin flip: 2 when its
// swap partner is a different determinant (not generated), else 1
template <int W>
__host__ __device__ inline double swap_weight(const uint64_t (&k)[W], int norb)
{
    uint64_t alo, ahi, blo, bhi;
    spin_strings<W>(k, norb, alo, ahi, blo, bhi);
    return alo == blo && ahi == bhi ? 1.0 : 2.0;
}

// Structure-of-arrays record buffer: W key planes then one payload plane.
// Planes 0..W-2 hold uint64 words; the last key plane holds `topb`-byte
// elements (2, 4 or 8), wide enough for the key's top bits.
struct Planes {
    uint64_t *key[MAXW];
    void *pay;
    int topb;
};

// bytes of the last key plane for a 2*norb-bit key
inline int top_bytes(int norb)
{
    const int W = (2 * norb + 63) / 64;
    const int top_bits = 2 * norb - 64 * (W - 1);
    return top_bits <= 16 ? 2 : (top_bits <= 32 ? 4 : 8);
}

template <int W>
__device__ inline const void *plane_ptr(const Planes &p, int w)
{
    const void *r = p.key[0];
    if (W > 1 && w == 1)
        r = p.key[1];
    if (W > 2 && w == 2)
        r = p.key[2];
    if (W > 3 && w == 3)
        r = p.key[3];
    return r;
}

// word w of record i (the last plane widened from its element size)
template <int W>
__device__ inline uint64_t pl_get(const Planes &p, int w, int64_t i)
{
    const void *b = plane_ptr<W>(p, w);
    const int eb = w == W - 1 ? p.topb : 8;
    if (eb == 8)
        return ((const uint64_t *)b)[i];
    if (eb == 4)
        return ((const uint32_t *)b)[i];
    return ((const uint16_t *)b)[i];
}

template <int W>
__device__ inline void pl_put(const Planes &p, int w, int64_t i, uint64_t v)
{
    void *b = (void *)plane_ptr<W>(p, w);
    const int eb = w == W - 1 ? p.topb : 8;
    if (eb == 8)
        ((uint64_t *)b)[i] = v;
    else if (eb == 4)
        ((uint32_t *)b)[i] = (uint32_t)v;
    else
        ((uint16_t *)b)[i] = (uint16_t)v;
}

// Hash record i: its kept hash bits; its auxiliary word (parent << 32 | four
// flipped spin-orbitals) and its FP32 payload in either record form.
__device__ inline uint64_t hash_at(const KeyCodec &kc, const Planes &in, int64_t i)
{
    return in.key[0][i] & kc.hash_mask;
}
__device__ inline uint64_t aux_at(const KeyCodec &kc, int norb, const Planes &in, int64_t i)
{
    if (!kc.hpacked)
        return in.key[1][i];
    return hash_unpack((in.key[0][i] & 0xFFFFull) | (in.key[1][i] >> 32) << 16, norb);
}
__device__ inline float pay32_at(const KeyCodec &kc, const Planes &in, int64_t i)
{
    return kc.hpacked ? ((const float *)in.key[1])[2 * i] : ((const float *)in.pay)[i];
}
// Writes the hash and auxiliary words of hash record p (z: the full hash);
// the payload is written separately (store_pay).  nt: non-temporal stores
// (records read only by the next kernel).
__device__ inline void hash_put(const KeyCodec &kc, int norb, const Planes &out, int64_t p, uint64_t z, uint64_t aux,
                                bool nt)
{
    uint64_t k0 = z & kc.hash_mask;
    if (kc.hpacked) {
        const uint64_t a = hash_pack(aux, norb);
        k0 |= a & 0xFFFFull;
        const uint32_t hi = (uint32_t)(a >> 16);
        if (nt) {
            __builtin_nontemporal_store(k0, out.key[0] + p);
            __builtin_nontemporal_store(hi, (uint32_t *)out.key[1] + 2 * p + 1);
        } else {
            out.key[0][p] = k0;
            ((uint32_t *)out.key[1])[2 * p + 1] = hi;
        }
    } else if (nt) {
        __builtin_nontemporal_store(k0, out.key[0] + p);
        __builtin_nontemporal_store(aux, out.key[1] + p);
    } else {
        out.key[0][p] = k0;
        out.key[1][p] = aux;
    }
}

// Hash records: the collided segments (runs of one hash holding more than one
// determinant) a single-pass workgroup found.  Their last records' indices are
// listed in record order in the workgroup's region of a list buffer (from
// index first_tile * RED_TILE; it never holds more entries than records).
struct CollList {
    uint32_t n, pad;  // collided segments listed (their last records' indices, in record order,
                      // in the workgroup's region of the list buffer)
    int64_t lo, hi;   // the references whose hash lies in the workgroup's hash range
};

// Per-block partial of the single pass; summed in block order.
struct Partial {
    double e_sum, e_comp;     // Neumaier pair
    double ref_cross;
    double min_abs_denom;
    uint64_t n_unique, n_external, n_hit, n_nonneg;
    uint64_t key_xor, key_sum;
};

// Layout of one reference determinant's excitation space (closed form).
struct ExcLayout {
    int na, nb, va, vb;
    int64_t nSa, nSb, nDaa, nDbb, nDab;   // block sizes
    int64_t o1, o2, o3, o4, nper;         // block offsets; nper = total
    int nvpa, nvpb, nopa, nopb;           // virtual / occupied pair counts
    int rank = 0;                         // records carry rank keys (KeyCodec)
};

// ---- rank keys (see KeyCodec) ----
__host__ __device__ inline void rank_join(uint64_t ra, uint64_t rb, int bb, uint64_t &lo, uint64_t &hi)
{
    if (bb == 0) {
        lo = ra, hi = 0;
    } else if (bb == 64) {
        lo = rb, hi = ra;
    } else {
        lo = rb | (ra << bb), hi = ra >> (64 - bb);
    }
}

__host__ __device__ inline void rank_split(uint64_t lo, uint64_t hi, int bb, uint64_t &ra, uint64_t &rb)
{
    if (bb == 0) {
        ra = lo, rb = 0;
    } else if (bb == 64) {
        ra = hi, rb = lo;
    } else {
        rb = lo & ((1ull << bb) - 1), ra = (lo >> bb) | (hi << (64 - bb));
    }
}

// Rank of a spin string given as its ascending occupied list occ[0..n) with
// the entries at positions skip1, skip2 removed (-1: none) and the orbitals
// add1 < add2 inserted (-1: none), by merging the two sorted sequences.
__device__ inline uint64_t rank_edit(const uint8_t *occ, int n, int skip1, int skip2, int add1, int add2,
                                     const uint64_t *B, int stride)
{
    uint64_t r = 0;
    int pos = 1, i = 0;
    int ad = add1 >= 0 ? add1 : add2, ad2 = add1 >= 0 ? add2 : -1;
    while (true) {
        while (i < n && (i == skip1 || i == skip2))
            i++;
        const int x = i < n ? (int)occ[i] : 0x7fffffff;
        const int y = ad >= 0 ? ad : 0x7fffffff;
        if (x == 0x7fffffff && y == 0x7fffffff)
            break;
        if (x < y) {
            r += B[x * stride + pos];
            i++;
        } else {
            r += B[y * stride + pos];
            ad = ad2, ad2 = -1;
        }
        pos++;
    }
    return r;
}

// Set the bits of the spin string with rank r (n electrons) at bit offset off.
template <int WB>
__device__ inline void unrank_spin(uint64_t r, int n, int norb, int off, const uint64_t *B, int stride,
                                   uint64_t (&bits)[WB])
{
    int x = norb - 1;
    for (int j = n; j >= 1; j--) {
        while (B[x * stride + j] > r)
            x--;
        r -= B[x * stride + j];
        const int b = off + x;
#pragma unroll
        for (int w = 0; w < WB; w++)
            bits[w] |= (w == (b >> 6)) ? (1ull << (b & 63)) : 0ull;
        x--;
    }
}

// Bitstring of the determinant with rank key (lo, hi).
template <int WB>
__device__ inline void unrank_key(uint64_t lo, uint64_t hi, int norb, int na, int nb, int bb, const uint64_t *B,
                                  int stride, uint64_t (&bits)[WB])
{
    uint64_t ra, rb;
    rank_split(lo, hi, bb, ra, rb);
#pragma unroll
    for (int w = 0; w < WB; w++)
        bits[w] = 0;
    unrank_spin<WB>(ra, na, norb, norb, B, stride, bits);
    unrank_spin<WB>(rb, nb, norb, 0, B, stride, bits);
}

inline ExcLayout make_layout(int norb, int na, int nb)
{
    ExcLayout L;
    L.na = na, L.nb = nb, L.va = norb - na, L.vb = norb - nb;
    auto c2 = [](int64_t n) { return n * (n - 1) / 2; };
    L.nSa = (int64_t)na * L.va;
    L.nSb = (int64_t)nb * L.vb;
    L.nopa = (int)c2(na), L.nopb = (int)c2(nb), L.nvpa = (int)c2(L.va), L.nvpb = (int)c2(L.vb);
    L.nDaa = (int64_t)L.nopa * L.nvpa;
    L.nDbb = (int64_t)L.nopb * L.nvpb;
    L.nDab = L.nSa * L.nSb;
    L.o1 = L.nSa;
    L.o2 = L.o1 + L.nSb;
    L.o3 = L.o2 + L.nDaa;
    L.o4 = L.o3 + L.nDbb;
    L.nper = L.o4 + L.nDab;
    return L;
}

// Excitation-index chunk handled by one generation workgroup: a multiple of
// 16384 (or the whole determinant) such that the grid stays below
// max_chunks workgroups (and 2^32 work-items).
inline int64_t gen_chunk(const ExcLayout &L, int64_t nref, int64_t max_chunks)
{
    int64_t chunk = 16384;
    if (max_chunks > (int64_t)1 << 24)
        max_chunks = (int64_t)1 << 24;
    while (chunk < L.nper && nref * ((L.nper + chunk - 1) / chunk) > max_chunks)
        chunk *= 2;
    if (chunk > L.nper)
        chunk = L.nper > 0 ? L.nper : 1;
    return chunk;
}

inline int64_t gen_nchunks(const ExcLayout &L, int64_t nref, int64_t chunk)
{
    return nref * ((L.nper + chunk - 1) / chunk);
}

// ---- launch wrappers (runtime dispatch over W and payload precision) ----

// gen.hip
size_t gen_lds_bytes(const ExcLayout &L);
// Direct generation: every term of every reference, record index
// det*nper + k.  Requires no cutoff and a single subset.  skip_kinds = 1
// leaves the alpha-alpha doubles [o2, o3), 2 the same-spin doubles [o2, o4),
// to launch_gen_spin.
hipError_t launch_gen_direct(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                             int64_t chunk, int skip_kinds, Planes out, hipStream_t st);
// The same-spin doubles of spin sp (0: alpha-alpha, 1: beta-beta) of direct
// generation, computed once per group of references sharing that spin
// string: grp = ngrp (start, count) pairs into gidx, the member reference
// indices, count <= REUSE_GROUP.  Bitstring keys only.
bool spin_reuse_ok(const ExcLayout &L, int W);  // its LDS fits
hipError_t launch_gen_spin(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int sp, const uint32_t *grp,
                           const uint32_t *gidx, int64_t ngrp, Planes out, hipStream_t st);
// Count pass: cnt[p * nchunks + chunk] = kept terms of chunk in subset p.
hipError_t launch_count(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                        int64_t chunk, int log2p, double cutoff, uint32_t *cnt, int64_t nchunks, hipStream_t st);
// Targeted form of the two passes above for a 2^k split (k >= 1), one
// reference determinant per chunk (chunk = nper, nchunks = nref): the count
// needs cutoff 0; generation walks only the terms of the subset.
bool target_ok(const ExcLayout &L, int64_t nref, int log2p);
// launch_count_target_cut fits (its subset counts and map need LDS beyond
// the target layout)
bool count_cut_ok(const ExcLayout &L, int64_t nref, int log2p, int nparts);
size_t target_lds_bytes(const ExcLayout &L, int log2p);
// Counts of the listed subsets only: cnt[j * nref + det] for parts[j] (device
// list of nparts distinct subsets).
hipError_t launch_count_target(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                               const uint32_t *parts, int nparts, uint32_t *cnt, const uint16_t *bk, hipStream_t st);
// Bucket tables of every reference determinant for a 2^log2p split (u16
// words per determinant: gen_bucket_words), read by launch_count_target and
// launch_gen_target when passed (bk == nullptr: they build their own).
int64_t gen_bucket_words(const ExcLayout &L, int log2p);
// The same-spin integral differences of DevSys::A2 from the device integrals V.
hipError_t launch_build_a2(const double *V, int norb, double *A2, hipStream_t st);
bool gen_buckets_ok(const ExcLayout &L, int log2p);
hipError_t launch_gen_buckets(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                              uint16_t *bk, hipStream_t st);
// As launch_count_target, with a cutoff or the spin flip filter applied to
// the terms of the listed subsets (their bucket walks; pm sets the value's
// precision for the cutoff test).
hipError_t launch_count_target_cut(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                                   int log2p, const uint32_t *parts, int nparts, double cutoff, uint32_t *cnt,
                                   hipStream_t st);
hipError_t launch_gen_target(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                             int log2p, uint32_t part, double cutoff, const uint64_t *off, const uint64_t *tot,
                             Planes out, Flags *flags, const uint16_t *bk, hipStream_t st);
// Exclusive scan of cnt[p][*] into off[k][*] for each listed subset p = parts[k]
// (parts == nullptr: p = k); tot[k] = N of that subset.
hipError_t launch_chunk_scan(const uint32_t *cnt, int64_t nchunks, const uint32_t *parts, int nparts,
                             uint64_t *off, uint64_t *tot, hipStream_t st);
// Compacting generation of subset `part` (offsets from launch_chunk_scan).
hipError_t launch_gen_compact(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                              int64_t chunk, int log2p, uint32_t part, double cutoff, const uint64_t *off,
                              int64_t nchunks, uint64_t cap, Planes out, Flags *flags, hipStream_t st);

// sort.hip
// hist[d*256 + v] += count of digit value v at digit position d (d < ndig).
hipError_t launch_hist(int W, const Planes &in, int64_t n, int ndig, uint64_t *hist, hipStream_t st);
// bucket[d*256 + v] = exclusive scan of hist[d][*].
hipError_t launch_hist_scan(const uint64_t *hist, int ndig, uint64_t *bucket, hipStream_t st);
// One stable LSD digit pass: per-tile counts, offset scan, rank and scatter
// (in -> out by digit `dig`).  counts: ntiles*256 u16; csum:
// (nchunks+1)*256 u64; coff: nchunks*256 u64; rel: ntiles*256 u32 (offset within the chunk of
// SCAN_CHUNK tiles).  `mid` (optional) is recorded between the counting/scan
// kernels and the scatter.
hipError_t launch_radix_pass(int W, int pay_bytes, const Planes &in, const Planes &out, int64_t n, int dig,
                             const uint64_t *bucket, uint16_t *counts, uint64_t *csum, uint64_t *coff,
                             uint32_t *rel, Flags *flags, hipStream_t st, hipEvent_t mid,
                             int items = SORT_ITEMS);
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t st);
hipError_t launch_zero_u64(uint64_t *p, int64_t n, hipStream_t st);
// AoS dets + coeffs -> SoA planes, with input checks.
hipError_t launch_refs_split(int W, int norb, int na, int nb, const uint64_t *dets, const double *c,
                             int64_t n, Planes out, Flags *flags, hipStream_t st);
hipError_t launch_dup_check(int W, const Planes &sorted, int64_t n, Flags *flags, hipStream_t st);
// SoA planes -> AoS keys (for inspection)
hipError_t launch_planes_to_aos(int W, int pay_bytes, const Planes &in, int64_t n, uint64_t *keys,
                                double *pay, hipStream_t st);

// reduce.hip
// sorted: records with kw key words (rank keys when s.kc.on); refs: the
// reference keys in the same format, sorted.
// range: scratch of 2 int64 per tile of RED_TILE records.
// search == 0: no reference search (subtraction form of the exclusion).
hipError_t launch_reduce(const DevSys &s, int fp32, int kw, const Planes &sorted, int64_t n,
                         const Planes &refs, int64_t nref, double e0, const AnchorBlk *anc, int nh,
                         int64_t *range, int search, Partial *partials, Flags *flags, hipStream_t st);
// The anchor block of an evaluation from the sorted bitstring references
// (bits: W planes, nref of them) and E0; nh: the anchor's hot rows (read back
// by the host, it sizes the single pass's LDS).
hipError_t launch_anchor(const DevSys &s, const Planes &bits, int64_t nref, double e0, AnchorBlk *anc,
                         hipStream_t st);
// out->e_sum + e_comp = sum over the bitstring references of c_i^2 (E0 - H_ii)
// (partials: 256 entries of scratch).
hipError_t launch_ref_terms(const DevSys &s, const Planes &refs, int64_t n, double e0, Partial *partials,
                            Partial *out, hipStream_t st);
// Spin flip: check that every sorted reference's alpha/beta swap is present
// with a coefficient of equal magnitude (flags: ERR_SWAP_MISSING, SWAP_SAME,
// SWAP_NEG).
hipError_t launch_check_swap(const DevSys &s, const Planes &refs, int64_t n, Flags *flags, hipStream_t st);
// Rank keys of sorted bitstring references (planes of kw words + coefficients).
hipError_t launch_refs_rank(const DevSys &s, const Planes &bits, int64_t n, const Planes &out, hipStream_t st);
// Hash records: the references' hashes with their indices (planes: 1 key word
// with 8-byte top, u64 payload), sorted afterwards by hash; per reference
// E0 minus its energy (D0) and its g vector G (nref x 2 norb), double-double;
// the single pass.
hipError_t launch_refs_hash(const DevSys &s, const Planes &bits, int64_t n, const Planes &out, hipStream_t st);
// D0[p] = E0 - H_pp and G[p][x] (g_x, plus D0[p]/2 for x occupied in p) as
// double-double pairs (hi, lo).
hipError_t launch_parent_g(const DevSys &s, const Planes &bits, int64_t n, double e0, double *D0, double *G,
                           hipStream_t st);
// The references' bitstrings record by record, 2^ceil(log2 W) words each.
hipError_t launch_refs_aos(const DevSys &s, const Planes &bits, int64_t n, uint64_t *ra, hipStream_t st);
// pm: the payload mode (PM_*), which sets the FP32 rounding bound.
hipError_t launch_reduce_hash(const DevSys &s, int pm, const Planes &sorted, int64_t n, const Planes &bits,
                              const uint64_t *ra_full, const uint64_t *ra_ex, const uint32_t *ra_ex4,
                              const uint64_t *anc_bits,
                              const Planes &rh, int64_t nref, const double *D0, const double *G, double e0,
                              int search, Partial *partials, CollList *coll, int64_t *ctail, Flags *flags,
                              hipStream_t st);
// The references' flips relative to the first sorted reference (up to eight,
// one byte each, 0xFF unused) into ex (n words) and their first four into
// ex4 (n 32-bit words), that reference's words into anc_bits (MAXW words),
// and into *far (only raised) the most flips of a reference beyond four.
hipError_t launch_refs_ex(const DevSys &s, const Planes &bits, int64_t n, uint64_t *ex, uint32_t *ex4,
                          uint64_t *anc_bits, uint32_t *far, hipStream_t st);
// Sum RED_GRID partials in order into *out (device).
hipError_t launch_final(const Partial *partials, Partial *out, hipStream_t st);
// Inspection: unique keys and numerators (n_out on device).
hipError_t launch_numerators(int W, int fp32, const Planes &sorted, int64_t n, const Planes &refs,
                             int64_t nref, uint64_t *keys_aos, double *num, uint8_t *in_ref,
                             unsigned long long *n_out, int64_t cap, hipStream_t st);

}  // namespace pt2
