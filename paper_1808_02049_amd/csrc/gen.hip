// Excitation generation and Slater-Condon numerator terms (Algorithm 1,
// generation step: act with H on every reference determinant and store each
// connected determinant's bitstring with H_ai * c_i), plus the count pass
// that sizes every subset of the hash split (the work list of the
// parallelisation subsection of Section V).
//
// One workgroup handles a contiguous chunk of one reference determinant's
// excitation index space.  The index space of a determinant with n_s occupied
// and v_s virtual orbitals per spin s is laid out as
//   [alpha singles | beta singles | alpha-alpha doubles | beta-beta doubles |
//    alpha-beta doubles]
// and a term is decoded from its index arithmetically, so every term has a
// fixed position and the output needs no atomics.  Per-determinant tables
// (occupied/virtual lists, single-excitation phases, orbital pairs) live in
// LDS; integrals are read from HBM through the caches (the (ra|..) slice used
// by consecutive alpha-beta terms is contiguous).
//
// Matrix elements (real orbitals, chemists' notation), with ph(x->y) the
// parity of occupied same-spin orbitals strictly between x and y:
//   single r->a, spin s:  ph * [h_ra + sum_{j occ} (ra|jj) - sum_{j occ, spin s} (rj|ja)]
//   same-spin r<s->a<b:   ph(r->a) ph'(s->b) [(ra|sb) - (rb|sa)], ph' taken on the
//                         determinant after r->a
//   alpha r->a, beta s->b: ph_alpha(r->a) ph_beta(s->b) (ra|sb)
#include "pt2_internal.h"

namespace pt2 {
namespace {

struct GenHead {
    uint64_t key[MAXW];
    uint64_t z;
    uint64_t ra0, rb0;  // spin-string ranks of the determinant (rank keys only)
    double c;
    uint64_t R[2 * MAXORB];
    uint8_t occ[2][MAXORB];   // [spin][k]: spin 0 = alpha, 1 = beta
    uint8_t vir[2][MAXORB];
    uint64_t zw[GEN_THREADS / 64];  // per-wavefront parts of z while it is formed
};

struct GenLds {
    GenHead *head;
    int8_t *ph[2];      // [spin][occ_idx * v + vir_idx]
    uint16_t *op[2];    // occupied pairs (i | j << 8), i < j, indices into occ
    uint16_t *vp[2];    // virtual pairs, indices into vir
    uint64_t *sr[2];    // rank keys only: spin-string rank after each single, [occ_idx * v + vir_idx]
    // select by a runtime spin without indexing the pointer arrays (which
    // would force this struct out of registers)
    __device__ const int8_t *phs(int sp) const { return sp == 0 ? ph[0] : ph[1]; }
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// vp = false: no virtual-pair tables (the targeted kernels decode pair
// indices in closed form instead; the tables are the largest part of the
// layout, and LDS decides how many of those workgroups share a CU).
__host__ __device__ inline size_t lds_layout(const ExcLayout &L, size_t *o_ph0, size_t *o_ph1, size_t *o_op0,
                                             size_t *o_vp0, size_t *o_op1, size_t *o_vp1, size_t *o_sr = nullptr,
                                             bool vp = true)
{
    size_t o = align16(sizeof(GenHead));
    *o_ph0 = o;
    o = align16(o + (size_t)L.na * L.va);
    *o_ph1 = o;
    o = align16(o + (size_t)L.nb * L.vb);
    *o_op0 = o;
    o = align16(o + 2 * (size_t)L.nopa);
    *o_vp0 = o;
    o = align16(o + (vp ? 2 * (size_t)L.nvpa : 0));
    *o_op1 = o;
    o = align16(o + 2 * (size_t)L.nopb);
    *o_vp1 = o;
    o = align16(o + (vp ? 2 * (size_t)L.nvpb : 0));
    if (o_sr)
        *o_sr = o;
    if (L.rank)
        o = align16(o + 8 * (size_t)(L.nSa + L.nSb));
    return o;
}

__host__ __device__ inline size_t gen_lds_bytes_dev(const ExcLayout &L, bool vp = true)
{
    size_t a, b, c, d, e, f, r;
    return lds_layout(L, &a, &b, &c, &d, &e, &f, &r, vp);
}

__device__ inline GenLds carve(char *base, const ExcLayout &L, bool vp = true)
{
    size_t a, b, c, d, e, f, r;
    lds_layout(L, &a, &b, &c, &d, &e, &f, &r, vp);
    GenLds g;
    g.head = (GenHead *)base;
    g.ph[0] = (int8_t *)(base + a);
    g.ph[1] = (int8_t *)(base + b);
    g.op[0] = (uint16_t *)(base + c);
    g.vp[0] = vp ? (uint16_t *)(base + d) : nullptr;
    g.op[1] = (uint16_t *)(base + e);
    g.vp[1] = vp ? (uint16_t *)(base + f) : nullptr;
    g.sr[0] = (uint64_t *)(base + r);
    g.sr[1] = (uint64_t *)(base + r) + L.nSa;
    return g;
}

__device__ inline int get_bit(const uint64_t *k, int b) { return (int)((k[b >> 6] >> (b & 63)) & 1ull); }

// parity (as +1/-1) of set bits of the spin string strictly between orbitals x and y
__device__ inline int between_sign(const uint64_t *key, int norb, int spin, int x, int y)
{
    int lo = x < y ? x : y, hi = x < y ? y : x;
    int off = spin == 0 ? norb : 0;
    int cnt = 0;
    // bits (off+lo+1) .. (off+hi-1)
    int b0 = off + lo + 1, b1 = off + hi;  // half-open
    for (int w = b0 >> 6; w <= ((b1 - 1) >> 6) && b0 < b1; w++) {
        int s = w * 64;
        uint64_t m = ~0ull;
        if (b0 > s)
            m &= ~0ull << (b0 - s);
        if (b1 < s + 64)
            m &= (1ull << (b1 - s)) - 1ull;
        cnt += __popcll(key[w] & m);
    }
    return (cnt & 1) ? -1 : 1;
}

// pair index k of n items -> (i, j), i < j, lexicographic.  Row i starts at
// s(i) = i (2n - i - 1) / 2; i is the root estimate of s(i) = k, fixed up to
// the largest i with s(i) <= k.
__device__ inline void pair_decode(int k, int n, int &i, int &j)
{
    const float b = (float)(2 * n - 1);
    int r = (int)((b - sqrtf(b * b - 8.0f * (float)k)) * 0.5f);
    r = r < 0 ? 0 : (r > n - 2 ? n - 2 : r);
    while (r > 0 && r * (2 * n - r - 1) / 2 > k)
        r--;
    while (r + 1 <= n - 2 && (r + 1) * (2 * n - r - 2) / 2 <= k)
        r++;
    i = r;
    j = i + 1 + (k - r * (2 * n - r - 1) / 2);
}

template <int W>
__device__ void det_setup(const GenLds &g, const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t det,
                          bool ranks = true)
{
    GenHead *H = g.head;
    const int tid = threadIdx.x;
    if (tid < W)
        H->key[tid] = pl_get<W>(refs, tid, det);
    if (tid == 0)
        H->c = ((const double *)refs.pay)[det];
    for (int b = tid; b < 2 * s.norb; b += blockDim.x)
        H->R[b] = s.R[b];
    __syncthreads();
    {
        // occupied / virtual lists: thread b places spin-orbital b by the
        // count of occupied ones of its spin below it; the Zobrist hash is
        // the XOR of the occupied ones' words, reduced per wavefront
        uint64_t zx = 0;
        const int lane = tid & 63, wave = tid >> 6;
        for (int b = tid; b < 2 * s.norb; b += blockDim.x) {
            const int spin = b < s.norb ? 1 : 0, off = spin == 0 ? s.norb : 0, p = b - off;
            int below = 0;  // occupied spin-orbitals in [off, b)
            for (int w = off >> 6; w <= (b >> 6); w++) {
                uint64_t m = ~0ull;
                if (w == (off >> 6))
                    m &= ~0ull << (off & 63);
                if (w == (b >> 6))
                    m &= (b & 63) ? (~0ull >> (64 - (b & 63))) : 0ull;
                below += __popcll(H->key[w] & m);
            }
            if (get_bit(H->key, b)) {
                H->occ[spin][below] = (uint8_t)p;
                zx ^= H->R[b];
            } else {
                H->vir[spin][p - below] = (uint8_t)p;
            }
        }
        for (int o = 32; o >= 1; o >>= 1)
            zx ^= __shfl_xor(zx, o);
        if (lane == 0)
            H->zw[wave] = zx;
        __syncthreads();
        if (tid == 0) {
            uint64_t z = 0;
            for (int w = 0; w < GEN_THREADS / 64; w++)
                z ^= H->zw[w];
            H->z = z;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < L.na * L.va; idx += blockDim.x) {
        int oi = idx / L.va, vi = idx - oi * L.va;
        g.ph[0][idx] = (int8_t)between_sign(H->key, s.norb, 0, H->occ[0][oi], H->vir[0][vi]);
    }
    for (int idx = tid; idx < L.nb * L.vb; idx += blockDim.x) {
        int oi = idx / L.vb, vi = idx - oi * L.vb;
        g.ph[1][idx] = (int8_t)between_sign(H->key, s.norb, 1, H->occ[1][oi], H->vir[1][vi]);
    }
    for (int idx = tid; idx < L.nopa; idx += blockDim.x) {
        int i, j;
        pair_decode(idx, L.na, i, j);
        g.op[0][idx] = (uint16_t)(i | (j << 8));
    }
    for (int idx = tid; g.vp[0] && idx < L.nvpa; idx += blockDim.x) {
        int i, j;
        pair_decode(idx, L.va, i, j);
        g.vp[0][idx] = (uint16_t)(i | (j << 8));
    }
    for (int idx = tid; idx < L.nopb; idx += blockDim.x) {
        int i, j;
        pair_decode(idx, L.nb, i, j);
        g.op[1][idx] = (uint16_t)(i | (j << 8));
    }
    for (int idx = tid; g.vp[1] && idx < L.nvpb; idx += blockDim.x) {
        int i, j;
        pair_decode(idx, L.vb, i, j);
        g.vp[1][idx] = (uint16_t)(i | (j << 8));
    }
    if (ranks && s.kc.on && L.rank) {
        const uint64_t *B = s.kc.binom;
        const int st = s.kc.stride;
        if (tid == 0)
            H->ra0 = rank_edit(H->occ[0], L.na, -1, -1, -1, -1, B, st);
        else if (tid == 1)
            H->rb0 = rank_edit(H->occ[1], L.nb, -1, -1, -1, -1, B, st);
        for (int idx = tid; idx < L.nSa; idx += blockDim.x) {
            const int oi = idx / L.va, vi = idx - oi * L.va;
            g.sr[0][idx] = rank_edit(H->occ[0], L.na, oi, -1, H->vir[0][vi], -1, B, st);
        }
        for (int idx = tid; idx < L.nSb; idx += blockDim.x) {
            const int oi = idx / L.vb, vi = idx - oi * L.vb;
            g.sr[1][idx] = rank_edit(H->occ[1], L.nb, oi, -1, H->vir[1][vi], -1, B, st);
        }
    }
    __syncthreads();
}

// q = x / d for 0 <= x < 2^26, d >= 1, via a float reciprocal and exact fix-up
__device__ inline uint32_t udiv(uint32_t x, uint32_t d, float inv)
{
    uint32_t q = (uint32_t)((float)x * inv);
    while ((uint64_t)q * d > x)
        q--;
    while ((uint64_t)(q + 1) * d <= x)
        q++;
    return q;
}

// A decoded excitation: kind 0/1 single alpha/beta, 2/3 double alpha-alpha /
// beta-beta, 4 alpha-beta; indices into the occupied / virtual lists.
struct Exc {
    int kind;
    int oi, vi, oj, vj;   // (oi -> vi) and, for doubles, (oj -> vj)
};

struct DivConsts {
    float inv_va, inv_vb, inv_nvpa, inv_nvpb, inv_nSb;
};

// Virtual pair q of spin sp (i | j << 8, indices into the virtual list):
// from the LDS table, or decoded when the layout has none.
__device__ inline uint16_t vpair(const GenLds &g, const ExcLayout &L, int sp, int q)
{
    const uint16_t *t = sp == 0 ? g.vp[0] : g.vp[1];
    if (t)
        return t[q];
    int i, j;
    pair_decode(q, sp == 0 ? L.va : L.vb, i, j);
    return (uint16_t)(i | (j << 8));
}

__device__ inline Exc decode(const GenLds &g, const ExcLayout &L, const DivConsts &D, int64_t k)
{
    Exc e;
    if (k < L.o1) {
        uint32_t x = (uint32_t)k;
        e.kind = 0;
        e.oi = (int)udiv(x, L.va, D.inv_va);
        e.vi = (int)(x - (uint32_t)e.oi * L.va);
    } else if (k < L.o2) {
        uint32_t x = (uint32_t)(k - L.o1);
        e.kind = 1;
        e.oi = (int)udiv(x, L.vb, D.inv_vb);
        e.vi = (int)(x - (uint32_t)e.oi * L.vb);
    } else if (k < L.o3) {
        uint32_t x = (uint32_t)(k - L.o2);
        uint32_t pi = udiv(x, L.nvpa, D.inv_nvpa), qi = x - pi * L.nvpa;
        uint16_t op = g.op[0][pi], vp = vpair(g, L, 0, (int)qi);
        e.kind = 2;
        e.oi = op & 255, e.oj = op >> 8, e.vi = vp & 255, e.vj = vp >> 8;
    } else if (k < L.o4) {
        uint32_t x = (uint32_t)(k - L.o3);
        uint32_t pi = udiv(x, L.nvpb, D.inv_nvpb), qi = x - pi * L.nvpb;
        uint16_t op = g.op[1][pi], vp = vpair(g, L, 1, (int)qi);
        e.kind = 3;
        e.oi = op & 255, e.oj = op >> 8, e.vi = vp & 255, e.vj = vp >> 8;
    } else {
        uint32_t x = (uint32_t)(k - L.o4);
        uint32_t ra = udiv(x, (uint32_t)L.nSb, D.inv_nSb), sb = x - ra * (uint32_t)L.nSb;
        e.kind = 4;
        e.oi = (int)udiv(ra, L.va, D.inv_va);
        e.vi = (int)(ra - (uint32_t)e.oi * L.va);
        e.oj = (int)udiv(sb, L.vb, D.inv_vb);
        e.vj = (int)(sb - (uint32_t)e.oj * L.vb);
    }
    return e;
}

template <int W>
__device__ inline void flip(uint64_t (&k)[W], int bit)
{
#pragma unroll
    for (int w = 0; w < W; w++)
        k[w] ^= ((bit >> 6) == w) ? (1ull << (bit & 63)) : 0ull;
}

// Bits flipped by an excitation (spin-orbital indices) -> key and Zobrist hash.
template <int W>
__device__ inline void flip_hash(const GenHead *H, uint64_t (&key)[W], uint64_t &z, int bit)
{
    flip<W>(key, bit);
    z ^= H->R[bit];
}

template <int W>
__device__ inline void exc_key(const GenLds &g, int norb, const Exc &e, uint64_t (&key)[W], uint64_t &z)
{
    const GenHead *H = g.head;
#pragma unroll
    for (int w = 0; w < W; w++)
        key[w] = H->key[w];
    z = H->z;
    if (e.kind == 0 || e.kind == 1) {
        const int off = e.kind == 0 ? norb : 0, sp = e.kind;
        flip_hash<W>(H, key, z, off + H->occ[sp][e.oi]);
        flip_hash<W>(H, key, z, off + H->vir[sp][e.vi]);
    } else if (e.kind == 2 || e.kind == 3) {
        const int sp = e.kind - 2, off = sp == 0 ? norb : 0;
        flip_hash<W>(H, key, z, off + H->occ[sp][e.oi]);
        flip_hash<W>(H, key, z, off + H->occ[sp][e.oj]);
        flip_hash<W>(H, key, z, off + H->vir[sp][e.vi]);
        flip_hash<W>(H, key, z, off + H->vir[sp][e.vj]);
    } else {
        flip_hash<W>(H, key, z, norb + H->occ[0][e.oi]);
        flip_hash<W>(H, key, z, norb + H->vir[0][e.vi]);
        flip_hash<W>(H, key, z, H->occ[1][e.oj]);
        flip_hash<W>(H, key, z, H->vir[1][e.vj]);
    }
}

__device__ inline int64_t eidx(int n, int p, int q, int r, int t)
{
    return (((int64_t)p * n + q) * n + r) * n + t;
}

// H_ai (without c_i) in the working precision F (double or float).
template <typename F>
__device__ inline F exc_value(const GenLds &g, const DevSys &s, const ExcLayout &L, const Exc &e,
                              const F *V, const F *h)
{
    const GenHead *H = g.head;
    const int n = s.norb;
    if (e.kind <= 1) {
        int sp = e.kind;
        int r = H->occ[sp][e.oi], a = H->vir[sp][e.vi];
        int vcount = sp == 0 ? L.va : L.vb;
        F f = h[r * n + a];
        const F *Vra = V + eidx(n, r, a, 0, 0);
        for (int t = 0; t < 2; t++) {
            int no = t == 0 ? L.na : L.nb;
            for (int jj = 0; jj < no; jj++) {
                int j = H->occ[t][jj];
                f += Vra[j * n + j];
                if (t == sp)
                    f -= V[eidx(n, r, j, j, a)];
            }
        }
        return (F)g.phs(sp)[e.oi * vcount + e.vi] * f;
    }
    if (e.kind <= 3) {
        int sp = e.kind - 2;
        int vcount = sp == 0 ? L.va : L.vb;
        int r = H->occ[sp][e.oi], q = H->occ[sp][e.oj];
        int a = H->vir[sp][e.vi], b = H->vir[sp][e.vj];
        const int8_t *pt = g.phs(sp);
        int ph1 = pt[e.oi * vcount + e.vi];
        int ph2 = pt[e.oj * vcount + e.vj];
        int lo = q < b ? q : b, hi = q < b ? b : q;
        if (r > lo && r < hi)
            ph2 = -ph2;
        if (a > lo && a < hi)
            ph2 = -ph2;
        F v;
        if constexpr (sizeof(F) == 8) {
            if (s.A2) {
                // the same difference, formed once per context (r < q, a < b)
                const size_t np = (size_t)n * (n - 1) / 2;
                v = s.A2[(size_t)(r * (2 * n - r - 1) / 2 + q - r - 1) * np + (size_t)(a * (2 * n - a - 1) / 2 + b - a - 1)];
            } else {
                v = V[eidx(n, r, a, q, b)] - V[eidx(n, r, b, q, a)];
            }
        } else {
            v = V[eidx(n, r, a, q, b)] - V[eidx(n, r, b, q, a)];
        }
        return (F)(ph1 * ph2) * v;
    }
    int r = H->occ[0][e.oi], a = H->vir[0][e.vi];
    int q = H->occ[1][e.oj], b = H->vir[1][e.vj];
    int ph = g.ph[0][e.oi * L.va + e.vi] * g.ph[1][e.oj * L.vb + e.vj];
    return (F)ph * V[eidx(n, r, a, q, b)];
}

__device__ inline DivConsts div_consts(const ExcLayout &L)
{
    DivConsts D;
    D.inv_va = L.va ? 1.0f / (float)L.va : 0.f;
    D.inv_vb = L.vb ? 1.0f / (float)L.vb : 0.f;
    D.inv_nvpa = L.nvpa ? 1.0f / (float)L.nvpa : 0.f;
    D.inv_nvpb = L.nvpb ? 1.0f / (float)L.nvpb : 0.f;
    D.inv_nSb = L.nSb ? 1.0f / (float)L.nSb : 0.f;
    return D;
}

template <int W>
__device__ inline void store_keys(const Planes &out, int64_t pos, const uint64_t (&key)[W])
{
#pragma unroll
    for (int w = 0; w < W; w++)
        pl_put<W>(out, w, pos, key[w]);
}

__device__ inline void put_top(void *plane, int topb, int64_t i, uint64_t v)
{
    if (topb == 8)
        ((uint64_t *)plane)[i] = v;
    else if (topb == 4)
        ((uint32_t *)plane)[i] = (uint32_t)v;
    else
        ((uint16_t *)plane)[i] = (uint16_t)v;
}

// hash_put for payload mode PM: FP64 records are never packed, so their
// kernels carry no packed branch.
template <int PM>
__device__ inline void put_hash_rec(const DevSys &s, const Planes &out, int64_t p, uint64_t z, uint64_t aux, bool nt)
{
    if (PM == PM_FP64) {
        KeyCodec kc = s.kc;
        kc.hpacked = 0;
        hash_put(kc, s.norb, out, p, z, aux, nt);
    } else {
        hash_put(s.kc, s.norb, out, p, z, aux, nt);
    }
}

// Record key of an excitation: its bitstring, or its rank key (KeyCodec).
// Singles and alpha-beta doubles take their spin-string ranks from the
// per-determinant tables; same-spin doubles rank the edited string.
template <int W, int PM>
__device__ inline void store_rec_key(const GenLds &g, const DevSys &s, const ExcLayout &L, const Exc &e,
                                     const uint64_t (&key)[W], uint64_t z, int64_t det, const Planes &out,
                                     int64_t pos)
{
    if (s.kc.hash) {
        const GenHead *H = g.head;
        const int n = s.norb;
        uint32_t f0, f1, f2 = FLIP_NONE, f3 = FLIP_NONE;
        if (e.kind <= 1) {
            const int off = e.kind == 0 ? n : 0;
            f0 = off + H->occ[e.kind][e.oi], f1 = off + H->vir[e.kind][e.vi];
        } else if (e.kind <= 3) {
            const int sp = e.kind - 2, off = sp == 0 ? n : 0;
            f0 = off + H->occ[sp][e.oi], f1 = off + H->occ[sp][e.oj];
            f2 = off + H->vir[sp][e.vi], f3 = off + H->vir[sp][e.vj];
        } else {
            f0 = n + H->occ[0][e.oi], f1 = n + H->vir[0][e.vi];
            f2 = H->occ[1][e.oj], f3 = H->vir[1][e.vj];
        }
        put_hash_rec<PM>(s, out, pos, z, ((uint64_t)det << 32) | (f0 | (f1 << 8) | (f2 << 16) | (f3 << 24)), false);
        return;
    }
    if (!s.kc.on) {
        store_keys<W>(out, pos, key);
        return;
    }
    const GenHead *H = g.head;
    const uint64_t *B = s.kc.binom;
    const int st = s.kc.stride;
    uint64_t ra = H->ra0, rb = H->rb0;
    if (e.kind == 0) {
        ra = g.sr[0][e.oi * L.va + e.vi];
    } else if (e.kind == 1) {
        rb = g.sr[1][e.oi * L.vb + e.vi];
    } else if (e.kind == 2) {
        ra = rank_edit(H->occ[0], L.na, e.oi, e.oj, H->vir[0][e.vi], H->vir[0][e.vj], B, st);
    } else if (e.kind == 3) {
        rb = rank_edit(H->occ[1], L.nb, e.oi, e.oj, H->vir[1][e.vi], H->vir[1][e.vj], B, st);
    } else {
        ra = g.sr[0][e.oi * L.va + e.vi];
        rb = g.sr[1][e.oj * L.vb + e.vj];
    }
    uint64_t lo, hi;
    rank_join(ra, rb, s.kc.bb, lo, hi);
    if (s.kc.kw == 1) {
        put_top(out.key[0], out.topb, pos, lo);
    } else {
        out.key[0][pos] = lo;
        put_top(out.key[1], out.topb, pos, hi);
    }
}

// The hash record words of an excitation without its bitstring: the Zobrist
// hash z of the excited determinant and the flipped spin-orbitals (one byte
// each, FLIP_NONE unused), as store_rec_key writes them.
__device__ inline void exc_flips(const GenLds &g, int norb, const Exc &e, uint64_t &z, uint32_t &fl)
{
    const GenHead *H = g.head;
    uint32_t f0, f1, f2 = FLIP_NONE, f3 = FLIP_NONE;
    if (e.kind <= 1) {
        const int off = e.kind == 0 ? norb : 0;
        f0 = off + H->occ[e.kind][e.oi], f1 = off + H->vir[e.kind][e.vi];
        z = H->z ^ H->R[f0] ^ H->R[f1];
    } else {
        if (e.kind <= 3) {
            const int sp = e.kind - 2, off = sp == 0 ? norb : 0;
            f0 = off + H->occ[sp][e.oi], f1 = off + H->occ[sp][e.oj];
            f2 = off + H->vir[sp][e.vi], f3 = off + H->vir[sp][e.vj];
        } else {
            f0 = norb + H->occ[0][e.oi], f1 = norb + H->vir[0][e.vi];
            f2 = H->occ[1][e.oj], f3 = H->vir[1][e.vj];
        }
        z = H->z ^ H->R[f0] ^ H->R[f1] ^ H->R[f2] ^ H->R[f3];
    }
    fl = f0 | (f1 << 8) | (f2 << 16) | (f3 << 24);
}

// The payload H_ai * c_i: FP64; FP64 arithmetic rounded once to FP32; or
// FP32 integrals and arithmetic.
// (FP32 payloads of packed hash records go to the low half of the second word.)
template <int PM>
__device__ inline void store_pay(const GenLds &g, const DevSys &s, const ExcLayout &L, const Exc &e, double c,
                                 const Planes &out, int64_t i)
{
    if (PM == PM_FP64) {
        ((double *)out.pay)[i] = exc_value<double>(g, s, L, e, s.V, s.h) * c;
        return;
    }
    float *dst = s.kc.hpacked ? (float *)out.key[1] + 2 * i : (float *)out.pay + i;
    if (PM == PM_FP32_PAYLOAD)
        *dst = (float)(exc_value<double>(g, s, L, e, s.V, s.h) * c);
    else
        *dst = exc_value<float>(g, s, L, e, s.V32, s.h32) * (float)c;
}

// store_pay with a non-temporal store
template <int PM>
__device__ inline void store_pay_stream(const GenLds &g, const DevSys &s, const ExcLayout &L, const Exc &e, double c,
                                        const Planes &out, int64_t i)
{
    if (PM == PM_FP64) {
        __builtin_nontemporal_store(exc_value<double>(g, s, L, e, s.V, s.h) * c, (double *)out.pay + i);
        return;
    }
    float *dst = s.kc.hpacked ? (float *)out.key[1] + 2 * i : (float *)out.pay + i;
    if (PM == PM_FP32_PAYLOAD)
        __builtin_nontemporal_store((float)(exc_value<double>(g, s, L, e, s.V, s.h) * c), dst);
    else
        __builtin_nontemporal_store(exc_value<float>(g, s, L, e, s.V32, s.h32) * (float)c, dst);
}

// ---------------------------------------------------------------------------
// Every term of every reference determinant, at its place in the reference's
// block of nper records.  skip_kinds = 1 leaves the alpha-alpha doubles
// [o2, o3), 2 all same-spin doubles [o2, o4), to k_gen_spin, which shares them
// between references of one spin string.
template <int W, int PM>
__global__ __launch_bounds__(GEN_THREADS) void k_gen_direct(DevSys s, ExcLayout L, const Planes refs, int64_t nref, int64_t chunk,
                                                            int cpd, int skip_kinds, Planes out)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L);
    const int64_t det = blockIdx.x / cpd;
    const int64_t ch = blockIdx.x - det * cpd;
    det_setup<W>(g, s, L, refs, det);
    const DivConsts D = div_consts(L);
    const int64_t skip = (skip_kinds >= 1 ? L.nDaa : 0) + (skip_kinds == 2 ? L.nDbb : 0);
    const int64_t lo = ch * chunk;
    const int64_t hi = lo + chunk < L.nper - skip ? lo + chunk : L.nper - skip;
    const int64_t base = det * L.nper;
    const double c = g.head->c;
    for (int64_t kr = lo + threadIdx.x; kr < hi; kr += GEN_THREADS) {
        const int64_t k = kr < L.o2 ? kr : kr + skip;
        Exc e = decode(g, L, D, k);
        uint64_t key[W], z;
        exc_key<W>(g, s.norb, e, key, z);
        store_rec_key<W, PM>(g, s, L, e, key, z, det, out, base + k);
        store_pay<PM>(g, s, L, e, c, out, base + k);
    }
}

// Same-spin doubles shared by the references of one spin string (Section V,
// data reuse for unique alpha and beta strings).  An alpha-alpha double, its
// matrix element and its phase depend on the alpha string alone (beta-beta:
// the beta string), so a workgroup takes a group of at most REUSE_GROUP
// references that share that string and a chunk of their index space of that
// kind, computes each term once and writes it for every reference of the
// group: the record keeps the reference's other string and is scaled by its
// coefficient.  Records land where k_gen_direct puts them, with the same
// values (bitstring keys only).  grp holds (start, count) pairs into gidx,
// the reference indices of the groups one after another.
template <int W, int PM, int SP>
__global__ __launch_bounds__(GEN_THREADS) void k_gen_spin(DevSys s, ExcLayout L, const Planes refs,
                                                          const uint32_t *grp, const uint32_t *gidx, int64_t achunk,
                                                          int cpa, Planes out)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L);
    uint64_t *s_key = (uint64_t *)(lds + gen_lds_bytes_dev(L));  // [REUSE_GROUP][W]
    double *s_c = (double *)(s_key + REUSE_GROUP * W);            // [REUSE_GROUP]
    int64_t *s_det = (int64_t *)(s_c + REUSE_GROUP);              // [REUSE_GROUP]
    const int64_t gi = blockIdx.x / cpa;
    const int64_t ch = blockIdx.x - gi * cpa;
    const uint32_t *members = gidx + grp[2 * gi];
    const int m = (int)grp[2 * gi + 1];
    det_setup<W>(g, s, L, refs, members[0], false);
    for (int i = threadIdx.x; i < m; i += GEN_THREADS) {
        const int64_t d = members[i];
#pragma unroll
        for (int w = 0; w < W; w++)
            s_key[i * W + w] = pl_get<W>(refs, w, d);
        s_c[i] = ((const double *)refs.pay)[d];
        s_det[i] = d;
    }
    __syncthreads();
    const DivConsts D = div_consts(L);
    const GenHead *H = g.head;
    const int n = s.norb, off = SP == 0 ? n : 0;
    const int64_t o0 = SP == 0 ? L.o2 : L.o3, nk = SP == 0 ? L.nDaa : L.nDbb;
    const int64_t lo = ch * achunk;
    const int64_t hi = lo + achunk < nk ? lo + achunk : nk;
    for (int64_t x = lo + threadIdx.x; x < hi; x += GEN_THREADS) {
        const Exc e = decode(g, L, D, o0 + x);
        uint64_t fm[W];
#pragma unroll
        for (int w = 0; w < W; w++)
            fm[w] = 0;
        flip<W>(fm, off + H->occ[SP][e.oi]);
        flip<W>(fm, off + H->occ[SP][e.oj]);
        flip<W>(fm, off + H->vir[SP][e.vi]);
        flip<W>(fm, off + H->vir[SP][e.vj]);
        double vd = 0.0;
        float vf = 0.f;
        if (PM == PM_FP32_ARITH)
            vf = exc_value<float>(g, s, L, e, s.V32, s.h32);
        else
            vd = exc_value<double>(g, s, L, e, s.V, s.h);
        for (int r = 0; r < m; r++) {
            const int64_t pos = s_det[r] * L.nper + o0 + x;
            uint64_t key[W];
#pragma unroll
            for (int w = 0; w < W; w++)
                key[w] = s_key[r * W + w] ^ fm[w];
            store_keys<W>(out, pos, key);
            const double c = s_c[r];
            if (PM == PM_FP64)
                ((double *)out.pay)[pos] = vd * c;
            else if (PM == PM_FP32_PAYLOAD)
                ((float *)out.pay)[pos] = (float)(vd * c);
            else
                ((float *)out.pay)[pos] = vf * (float)c;
        }
    }
}

// The cutoff test in the precision the term is computed in (FP32 only when
// the integrals and the arithmetic are FP32).
template <int W, int PM>
__device__ inline bool keep_term(const GenLds &g, const DevSys &s, const ExcLayout &L, const Exc &e,
                                 double cutoff, const uint64_t (&key)[W])
{
    if (s.z2 && !alpha_not_below_beta<W>(key, s.norb))
        return false;  // the swap partner stands for it
    if (cutoff <= 0.0)
        return true;
    if (PM == PM_FP32_ARITH) {
        float v = exc_value<float>(g, s, L, e, s.V32, s.h32) * (float)g.head->c;
        return fabsf(v) >= (float)cutoff;
    }
    double v = exc_value<double>(g, s, L, e, s.V, s.h) * g.head->c;
    return fabs(v) >= cutoff;
}

__device__ inline uint32_t part_of(uint64_t z, int log2p) { return log2p == 0 ? 0u : (uint32_t)(z >> (64 - log2p)); }

template <int W, int PM>
__global__ __launch_bounds__(GEN_THREADS) void k_count(DevSys s, ExcLayout L, const Planes refs, int64_t nref, int64_t chunk,
                                                       int cpd, int log2p, double cutoff, uint32_t *cnt,
                                                       int64_t nchunks)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L);
    size_t a, b, c2, d, e2, f;
    uint32_t *hist = (uint32_t *)(lds + lds_layout(L, &a, &b, &c2, &d, &e2, &f));
    const int P = 1 << log2p;
    for (int p = threadIdx.x; p < P; p += GEN_THREADS)
        hist[p] = 0;
    const int64_t det = blockIdx.x / cpd;
    const int64_t ch = blockIdx.x - det * cpd;
    det_setup<W>(g, s, L, refs, det, false);
    const DivConsts D = div_consts(L);
    const int64_t lo = ch * chunk;
    const int64_t hi = lo + chunk < L.nper ? lo + chunk : L.nper;
    for (int64_t k = lo + threadIdx.x; k < hi; k += GEN_THREADS) {
        Exc e = decode(g, L, D, k);
        uint64_t key[W], z;
        exc_key<W>(g, s.norb, e, key, z);
        if (keep_term<W, PM>(g, s, L, e, cutoff, key))
            atomicAdd(&hist[part_of(z, log2p)], 1u);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += GEN_THREADS)
        cnt[(int64_t)p * nchunks + blockIdx.x] = hist[p];
}

template <int W, int PM>
__global__ __launch_bounds__(GEN_THREADS) void k_gen_compact(DevSys s, ExcLayout L, const Planes refs, int64_t nref, int64_t chunk,
                                                             int cpd, int log2p, uint32_t part, double cutoff,
                                                             const uint64_t *off, uint64_t cap, Planes out,
                                                             Flags *flags)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L);
    size_t a, b, c2, d, e2, f;
    uint32_t *wtot = (uint32_t *)(lds + lds_layout(L, &a, &b, &c2, &d, &e2, &f));
    const int64_t det = blockIdx.x / cpd;
    const int64_t ch = blockIdx.x - det * cpd;
    det_setup<W>(g, s, L, refs, det);
    const DivConsts D = div_consts(L);
    const int64_t lo = ch * chunk;
    const int64_t hi = lo + chunk < L.nper ? lo + chunk : L.nper;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t pos = off[blockIdx.x];
    const double c = g.head->c;
    for (int64_t k0 = lo; k0 < hi; k0 += GEN_THREADS) {
        const int64_t k = k0 + threadIdx.x;
        bool keep = false;
        Exc e;
        uint64_t key[W], z = 0;
        if (k < hi) {
            e = decode(g, L, D, k);
            exc_key<W>(g, s.norb, e, key, z);
            keep = part_of(z, log2p) == part && keep_term<W, PM>(g, s, L, e, cutoff, key);
        }
        uint64_t m = __ballot(keep);
        if (lane == 0)
            wtot[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t woff = 0, btot = 0;
        for (int w = 0; w < GEN_THREADS / 64; w++) {
            uint32_t t = wtot[w];
            woff += w < wave ? t : 0u;
            btot += t;
        }
        if (keep) {
            uint64_t p = pos + woff + (uint64_t)__popcll(m & lt);
            if (p < cap) {
                store_rec_key<W, PM>(g, s, L, e, key, z, det, out, (int64_t)p);
                store_pay<PM>(g, s, L, e, c, out, (int64_t)p);
            } else {
                atomicOr(&flags->err, ERR_OVERFLOW);
            }
        }
        pos += btot;
        __syncthreads();
    }
}

// Exclusive scan over chunks of one subset's counts; one workgroup per subset.
__global__ __launch_bounds__(1024) void k_chunk_scan(const uint32_t *cnt, int64_t nchunks, const uint32_t *parts,
                                                     uint64_t *off, uint64_t *tot)
{
    __shared__ uint64_t sh[1024];
    const uint32_t p = parts ? parts[blockIdx.x] : blockIdx.x;
    const uint32_t *src = cnt + (int64_t)p * nchunks;
    uint64_t *dst = off + (int64_t)blockIdx.x * nchunks;
    uint64_t carry = 0;
    for (int64_t b = 0; b < nchunks; b += 1024) {
        int64_t i = b + threadIdx.x;
        uint64_t v = i < nchunks ? src[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunks)
            dst[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        tot[blockIdx.x] = carry;
}

// ---------------------------------------------------------------------------
// Targeted counting and generation for a 2^k hash split (one workgroup per
// reference determinant).
//
// The subset of a candidate is top_k(z), z = z(D) ^ (table words of the
// flipped spin-orbitals), and top_k is XOR-linear.  Doubles split into an
// outer and an inner part whose words combine by XOR:
//   same-spin doubles:  outer = occupied pair (r, s), inner = virtual pair (a, b)
//   alpha-beta doubles: outer = alpha single r -> a, inner = beta single s -> b
// so the inner parts completing outer part o into subset p are exactly those
// with top_k(h_inner) == p ^ top_k(z(D) ^ h_outer(o)).  The inner parts are
// bucketed by top_k(h_inner) in LDS, each bucket in ascending index order,
// and only the matching bucket of every outer part is walked: the work per
// subset is the subset's own terms instead of every candidate.  Singles are
// few and are filtered.

struct Tgt {
    uint32_t *bstart;  // [B + 1] bucket counts; after filling, bstart[b] = end of bucket b
    uint32_t *hist;    // [B] counts of the listed subsets (count pass only; aliases blist..pre)
    uint16_t *pmap;    // [B] position of a subset in the list, 0xFFFF if unlisted (count pass)
    uint16_t *plist;   // [B] the listed subsets (count pass)
    uint16_t *blist;   // [max inner] inner indices grouped by bucket
    uint16_t *tgt;     // [max outer] matching bucket of each outer part
    uint32_t *pre;     // [max outer + 1] prefix of matching inner counts
    uint32_t *wsum;    // [GEN_THREADS / 64]
};

__host__ __device__ inline void tgt_sizes(const ExcLayout &L, int *max_in, int *max_out)
{
    int a = L.nvpa > L.nvpb ? L.nvpa : L.nvpb;
    *max_in = a > (int)L.nSb ? a : (int)L.nSb;
    int b = L.nopa > L.nopb ? L.nopa : L.nopb;
    *max_out = b > (int)L.nSa ? b : (int)L.nSa;
}

__host__ __device__ inline size_t tgt_lds_layout(const ExcLayout &L, int log2p, size_t *o)
{
    int mi, mo;
    tgt_sizes(L, &mi, &mo);
    const size_t B = (size_t)1 << log2p;
    size_t x = 0;
    o[0] = x, x = align16(x + 4 * (B + 1));
    o[5] = x, x = align16(x + 4 * (GEN_THREADS / 64));
    const size_t rest = x;
    o[2] = x, x = align16(x + 2 * (size_t)(mi > 0 ? mi : 1));
    o[3] = x, x = align16(x + 2 * (size_t)(mo > 0 ? mo : 1));
    o[4] = x, x = align16(x + 4 * ((size_t)mo + 1));
    // the count pass keeps its subset counts, the subset list and its
    // inverse where generation keeps its lists
    o[1] = rest;
    o[6] = align16(rest + 4 * B);
    o[7] = align16(o[6] + 2 * B);
    const size_t xc = align16(o[7] + 2 * B);
    return x > xc ? x : xc;
}

__device__ inline Tgt carve_tgt(char *base, const ExcLayout &L, int log2p)
{
    size_t o[8];
    tgt_lds_layout(L, log2p, o);
    Tgt t;
    t.pmap = (uint16_t *)(base + o[6]);
    t.plist = (uint16_t *)(base + o[7]);
    t.bstart = (uint32_t *)(base + o[0]);
    t.hist = (uint32_t *)(base + o[1]);
    t.blist = (uint16_t *)(base + o[2]);
    t.tgt = (uint16_t *)(base + o[3]);
    t.pre = (uint32_t *)(base + o[4]);
    t.wsum = (uint32_t *)(base + o[5]);
    return t;
}

__device__ inline uint32_t top_bits(uint64_t z, int log2p) { return (uint32_t)(z >> (64 - log2p)); }

// first slot of bucket b once the buckets are filled
__device__ inline uint32_t bucket_lo(const Tgt &t, int b) { return b ? t.bstart[b - 1] : 0u; }

// In-place exclusive scan of a[0..n) (block-wide); returns the total.
__device__ uint32_t block_scan_excl(uint32_t *a, int n, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + GEN_THREADS - 1) / GEN_THREADS;
    const int lo = tid * per, hi = lo + per < n ? lo + per : n;
    uint32_t loc = 0;
    for (int i = lo; i < hi; i++)
        loc += a[i];
    uint32_t x = loc;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
    for (int w = 0; w < GEN_THREADS / 64; w++) {
        const uint32_t t = wsum[w];
        wpre += w < wave ? t : 0u;
        tot += t;
    }
    uint32_t run = wpre + x - loc;
    for (int i = lo; i < hi; i++) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return tot;
}

// Exclusive prefix of one value per thread over the block (thread order);
// tot gets the block's total.  wsum: GEN_THREADS / 64 words of scratch.
__device__ uint32_t block_excl_one(uint32_t v, uint32_t *wsum, uint32_t &tot)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    __syncthreads();
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    uint32_t wpre = 0;
    tot = 0;
    for (int w = 0; w < GEN_THREADS / 64; w++) {
        const uint32_t t = wsum[w];
        wpre += w < wave ? t : 0u;
        tot += t;
    }
    __syncthreads();
    return wpre + x - v;
}

// Hash words of the inner / outer parts (kind 2, 3: spin sp; kind 4: alpha-beta).
__device__ inline uint64_t inner_hash(const GenLds &g, const ExcLayout &L, int norb, int kind, int q)
{
    const GenHead *H = g.head;
    if (kind == 4) {
        const int oj = q / L.vb, vj = q - oj * L.vb;
        return H->R[H->occ[1][oj]] ^ H->R[H->vir[1][vj]];
    }
    const int sp = kind - 2, off = sp == 0 ? norb : 0;
    const uint16_t vp = vpair(g, L, sp, q);
    return H->R[off + H->vir[sp][vp & 255]] ^ H->R[off + H->vir[sp][vp >> 8]];
}

__device__ inline uint64_t outer_hash(const GenLds &g, const ExcLayout &L, int norb, int kind, int o)
{
    const GenHead *H = g.head;
    if (kind == 4) {
        const int oi = o / L.va, vi = o - oi * L.va;
        return H->R[norb + H->occ[0][oi]] ^ H->R[norb + H->vir[0][vi]];
    }
    const int sp = kind - 2, off = sp == 0 ? norb : 0;
    const uint16_t op = sp == 0 ? g.op[0][o] : g.op[1][o];
    return H->R[off + H->occ[sp][op & 255]] ^ H->R[off + H->occ[sp][op >> 8]];
}

__device__ inline int n_inner(const ExcLayout &L, int kind) { return kind == 2 ? L.nvpa : kind == 3 ? L.nvpb : (int)L.nSb; }
__device__ inline int n_outer(const ExcLayout &L, int kind) { return kind == 2 ? L.nopa : kind == 3 ? L.nopb : (int)L.nSa; }

// Bucket counts (and, if fill, the bucket lists in ascending index order) of
// the inner parts of one kind.
__device__ void build_buckets(const GenLds &g, const Tgt &t, const ExcLayout &L, int norb, int kind, int log2p,
                              bool fill)
{
    const int tid = threadIdx.x, B = 1 << log2p, ni = n_inner(L, kind);
    for (int b = tid; b <= B; b += GEN_THREADS)
        t.bstart[b] = 0;
    __syncthreads();
    for (int q = tid; q < ni; q += GEN_THREADS)
        atomicAdd(&t.bstart[top_bits(inner_hash(g, L, norb, kind, q), log2p)], 1u);
    __syncthreads();
    if (!fill)
        return;
    block_scan_excl(t.bstart, B + 1, t.wsum);
    // filling advances every start to its bucket's end
    for (int q = tid; q < ni; q += GEN_THREADS) {
        const uint32_t slot = atomicAdd(&t.bstart[top_bits(inner_hash(g, L, norb, kind, q), log2p)], 1u);
        t.blist[slot] = (uint16_t)q;
    }
    __syncthreads();
    // the fill order above is arbitrary: sort every bucket (they are small)
    for (int b = tid; b < B; b += GEN_THREADS) {
        const uint32_t lo = bucket_lo(t, b), hi = t.bstart[b];
        for (uint32_t i = lo + 1; i < hi; i++) {
            const uint16_t v = t.blist[i];
            uint32_t j = i;
            while (j > lo && t.blist[j - 1] > v) {
                t.blist[j] = t.blist[j - 1];
                j--;
            }
            t.blist[j] = v;
        }
    }
    __syncthreads();
}

// Layout of one determinant's bucket table (u16 words): for kinds 2, 3 and 4
// in turn, the B bucket ends, then the kind's inner indices bucket by bucket
// in ascending order (what build_buckets leaves in LDS).
__host__ __device__ inline int64_t bucket_kind_off(const ExcLayout &L, int log2p, int kind)
{
    const int64_t B = (int64_t)1 << log2p;
    return kind == 2 ? 0 : kind == 3 ? B + L.nvpa : 2 * B + L.nvpa + L.nvpb;
}
__host__ __device__ inline int64_t bucket_table_words(const ExcLayout &L, int log2p)
{
    const int64_t w = bucket_kind_off(L, log2p, 4) + ((int64_t)1 << log2p) + L.nSb;
    return (w + 7) & ~(int64_t)7;
}

// The state build_buckets(fill = true) leaves, read from a determinant's
// bucket table (src: that kind's part); with lists = false only the ends.
__device__ void load_buckets(const Tgt &t, const ExcLayout &L, int kind, int log2p, const uint16_t *src, bool lists)
{
    const int tid = threadIdx.x, B = 1 << log2p, ni = n_inner(L, kind);
    for (int b = tid; b < B; b += GEN_THREADS)
        t.bstart[b] = src[b];
    if (tid == 0)
        t.bstart[B] = (uint32_t)ni;
    if (lists)
        for (int q = tid; q < ni; q += GEN_THREADS)
            t.blist[q] = src[B + q];
    __syncthreads();
}

__device__ inline Exc make_exc(const GenLds &g, const ExcLayout &L, const DivConsts &D, int kind, int o, int q)
{
    Exc e;
    e.kind = kind;
    if (kind == 4) {
        e.oi = (int)udiv((uint32_t)o, (uint32_t)L.va, D.inv_va), e.vi = o - e.oi * L.va;
        e.oj = (int)udiv((uint32_t)q, (uint32_t)L.vb, D.inv_vb), e.vj = q - e.oj * L.vb;
    } else {
        const int sp = kind - 2;
        const uint16_t op = sp == 0 ? g.op[0][o] : g.op[1][o];
        const uint16_t vp = vpair(g, L, sp, q);
        e.oi = op & 255, e.oj = op >> 8, e.vi = vp & 255, e.vj = vp >> 8;
    }
    return e;
}

// One block-wide step of compacted emission: threads with have == true hold
// a candidate; kept ones are written at consecutive positions from pos.
template <int W, int PM>
__device__ inline void emit_step(const GenLds &g, const DevSys &s, const ExcLayout &L, bool have, const Exc &e,
                                 bool filter, int log2p, uint32_t part, double cutoff, uint64_t &pos,
                                 uint64_t end, const Planes &out, Flags *flags, uint32_t *wtot, bool &bad,
                                 int64_t det)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t key[W], z = 0;
    bool keep = false;
    if (have) {
        exc_key<W>(g, s.norb, e, key, z);
        const bool in = part_of(z, log2p) == part;
        if (!in && !filter)
            bad = true;  // a walked candidate outside the subset: bucketing is inconsistent
        keep = in && keep_term<W, PM>(g, s, L, e, cutoff, key);
    }
    const uint64_t m = __ballot(keep);
    if (lane == 0)
        wtot[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t woff = 0, btot = 0;
    for (int w = 0; w < GEN_THREADS / 64; w++) {
        const uint32_t t = wtot[w];
        woff += w < wave ? t : 0u;
        btot += t;
    }
    if (keep) {
        const uint64_t p = pos + woff + (uint64_t)__popcll(m & lt);
        if (p < end) {
            store_rec_key<W, PM>(g, s, L, e, key, z, det, out, (int64_t)p);
            store_pay<PM>(g, s, L, e, g.head->c, out, (int64_t)p);
        } else {
            atomicOr(&flags->err, ERR_OVERFLOW);
        }
    }
    pos += btot;
    __syncthreads();
}

template <int W, int PM>
__global__ __launch_bounds__(GEN_THREADS) __attribute__((amdgpu_waves_per_eu(5))) void k_gen_target(DevSys s, ExcLayout L, const Planes refs, int64_t nref,
                                                            int log2p, uint32_t part, double cutoff,
                                                            const uint64_t *off, const uint64_t *tot, Planes out,
                                                            Flags *flags, const uint16_t *bk)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L, false);
    Tgt t = carve_tgt(lds + gen_lds_bytes_dev(L, false), L, log2p);
    const int64_t det = blockIdx.x;
    const int tid = threadIdx.x;
    det_setup<W>(g, s, L, refs, det);
    const DivConsts D = div_consts(L);
    uint64_t pos = off[det];
    const uint64_t end = det + 1 < nref ? off[det + 1] : *tot;
    const uint64_t zp = g.head->z;
    bool bad = false;
    // doubles: alpha-alpha, beta-beta, alpha-beta; without a cutoff or the
    // spin flip every candidate the bucket walk visits is kept
    const bool direct = cutoff <= 0.0 && !s.z2;
    // singles: filtered by their subset
    if (direct) {
        // each thread takes a contiguous range of single-excitation indices
        // and writes those in the subset after the earlier threads' ones:
        // index order, as the filtered path below
        const int64_t per = (L.o2 + GEN_THREADS - 1) / GEN_THREADS;
        const int64_t k0 = (int64_t)tid * per, k1 = k0 + per < L.o2 ? k0 + per : L.o2;
        uint32_t mine = 0;
        for (int64_t k = k0; k < k1; k++) {
            uint64_t z;
            uint32_t fl;
            exc_flips(g, s.norb, decode(g, L, D, k), z, fl);
            mine += part_of(z, log2p) == part ? 1u : 0u;
        }
        uint32_t tot_s;
        uint64_t p = pos + block_excl_one(mine, t.wsum, tot_s);
        for (int64_t k = k0; k < k1; k++) {
            const Exc e = decode(g, L, D, k);
            uint64_t z;
            uint32_t fl;
            exc_flips(g, s.norb, e, z, fl);
            if (part_of(z, log2p) != part)
                continue;
            if (p < end) {
                if (s.kc.hash) {
                    put_hash_rec<PM>(s, out, (int64_t)p, z, ((uint64_t)det << 32) | fl, false);
                } else {
                    uint64_t key[W], zk;
                    exc_key<W>(g, s.norb, e, key, zk);
                    store_rec_key<W, PM>(g, s, L, e, key, zk, det, out, (int64_t)p);
                }
                store_pay<PM>(g, s, L, e, g.head->c, out, (int64_t)p);
            } else {
                atomicOr(&flags->err, ERR_OVERFLOW);
            }
            p++;
        }
        pos += tot_s;
    } else {
        for (int64_t k0 = 0; k0 < L.o2; k0 += GEN_THREADS) {
            const int64_t k = k0 + tid;
            Exc e;
            const bool have = k < L.o2;
            if (have)
                e = decode(g, L, D, k);
            emit_step<W, PM>(g, s, L, have, e, true, log2p, part, cutoff, pos, end, out, flags, t.wsum, bad, det);
        }
    }
    for (int kind = 2; kind <= 4; kind++) {
        const int no = n_outer(L, kind);
        if (no == 0 || n_inner(L, kind) == 0)
            continue;
        if (bk)
            load_buckets(t, L, kind, log2p, bk + det * bucket_table_words(L, log2p) + bucket_kind_off(L, log2p, kind),
                         true);
        else
            build_buckets(g, t, L, s.norb, kind, log2p, true);
        for (int o = tid; o < no; o += GEN_THREADS) {
            const uint32_t b = part ^ top_bits(zp ^ outer_hash(g, L, s.norb, kind, o), log2p);
            t.tgt[o] = (uint16_t)b;
            t.pre[o] = t.bstart[b] - bucket_lo(t, b);
        }
        if (tid == 0)
            t.pre[no] = 0;
        __syncthreads();
        const uint32_t T = block_scan_excl(t.pre, no + 1, t.wsum);
        for (uint32_t f0 = 0; f0 < T; f0 += GEN_THREADS) {
            const uint32_t f = f0 + tid;
            const bool have = f < T;
            Exc e;
            if (have) {
                // outer part: the last o with pre[o] <= f
                int lo = 0, hi = no;  // pre[lo] <= f < pre[hi] (pre[no] = T)
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (t.pre[mid] <= f)
                        lo = mid;
                    else
                        hi = mid;
                }
                const int q = t.blist[bucket_lo(t, t.tgt[lo]) + (f - t.pre[lo])];
                e = make_exc(g, L, D, kind, lo, q);
            }
            if (direct && s.kc.hash) {
                // hash records: no bitstring is formed
                if (have) {
                    uint64_t z;
                    uint32_t fl;
                    exc_flips(g, s.norb, e, z, fl);
                    if (part_of(z, log2p) != part)
                        bad = true;  // bucketing is inconsistent
                    const uint64_t p = pos + f;
                    if (p < end) {
                        // records are written once and read by the next
                        // kernel: non-temporal stores keep the L2 for the
                        // integrals the terms gather
                        put_hash_rec<PM>(s, out, (int64_t)p, z, ((uint64_t)det << 32) | fl, true);
                        store_pay_stream<PM>(g, s, L, e, g.head->c, out, (int64_t)p);
                    } else {
                        atomicOr(&flags->err, ERR_OVERFLOW);
                    }
                }
            } else if (direct) {
                // every walked candidate is kept: its slot is its walk index
                if (have) {
                    uint64_t key[W], z;
                    exc_key<W>(g, s.norb, e, key, z);
                    if (part_of(z, log2p) != part)
                        bad = true;  // bucketing is inconsistent
                    const uint64_t p = pos + f;
                    if (p < end) {
                        store_rec_key<W, PM>(g, s, L, e, key, z, det, out, (int64_t)p);
                        store_pay<PM>(g, s, L, e, g.head->c, out, (int64_t)p);
                    } else {
                        atomicOr(&flags->err, ERR_OVERFLOW);
                    }
                }
            } else {
                emit_step<W, PM>(g, s, L, have, e, false, log2p, part, cutoff, pos, end, out, flags, t.wsum, bad,
                                 det);
            }
        }
        if (direct)
            pos += T;
        __syncthreads();
    }
    if (bad || (tid == 0 && pos != end))
        atomicOr(&flags->err, ERR_OVERFLOW);
}

// Counts of the listed subsets parts[0..nparts) of every reference
// determinant (cutoff 0): cnt[j * nref + det] for the j-th listed subset.
template <int W>
__global__ __launch_bounds__(GEN_THREADS) void k_count_target(DevSys s, ExcLayout L, const Planes refs, int64_t nref,
                                                              int log2p, const uint32_t *parts, int nparts,
                                                              uint32_t *cnt, const uint16_t *bk)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L, false);
    Tgt t = carve_tgt(lds + gen_lds_bytes_dev(L, false), L, log2p);
    const int64_t det = blockIdx.x;
    const int tid = threadIdx.x, B = 1 << log2p;
    uint32_t *hist = t.hist;  // [nparts]
    det_setup<W>(g, s, L, refs, det, false);
    const DivConsts D = div_consts(L);
    const uint64_t zp = g.head->z;
    for (int b = tid; b < B; b += GEN_THREADS) {
        hist[b] = 0;
        t.pmap[b] = 0xFFFFu;
    }
    __syncthreads();
    for (int j = tid; j < nparts; j += GEN_THREADS) {
        t.plist[j] = (uint16_t)parts[j];
        t.pmap[parts[j]] = (uint16_t)j;
    }
    __syncthreads();
    for (int64_t k = tid; k < L.o2; k += GEN_THREADS) {
        const Exc e = decode(g, L, D, k);
        uint64_t key[W], z;
        exc_key<W>(g, s.norb, e, key, z);
        const uint32_t j = t.pmap[top_bits(z, log2p)];
        if (j != 0xFFFFu)
            atomicAdd(&hist[j], 1u);
    }
    for (int kind = 2; kind <= 4; kind++) {
        const int no = n_outer(L, kind), ni = n_inner(L, kind);
        if (no == 0 || ni == 0)
            continue;
        if (B <= ni) {
            // bucket counts, then every (outer part, listed subset) pair: the
            // inner parts completing o into subset p are the bucket
            // p ^ top(z(D) ^ h_o)
            if (bk)
                load_buckets(t, L, kind, log2p,
                             bk + det * bucket_table_words(L, log2p) + bucket_kind_off(L, log2p, kind), false);
            else
                build_buckets(g, t, L, s.norb, kind, log2p, false);
            const uint32_t np = (uint32_t)no * (uint32_t)nparts;
            for (uint32_t x = tid; x < np; x += GEN_THREADS) {
                const uint32_t o = x / (uint32_t)nparts, j = x - o * (uint32_t)nparts;
                const uint32_t b = t.plist[j] ^ top_bits(zp ^ outer_hash(g, L, s.norb, kind, (int)o), log2p);
                // loaded tables hold bucket ends, built ones counts
                const uint32_t c = bk ? t.bstart[b] - bucket_lo(t, (int)b) : t.bstart[b];
                if (c)
                    atomicAdd(&hist[j], c);
            }
        } else {
            // fewer inner parts than subsets: every pair
            const int64_t np = (int64_t)no * ni;
            for (int64_t x = tid; x < np; x += GEN_THREADS) {
                const int o = (int)(x / ni), q = (int)(x - (int64_t)o * ni);
                const uint64_t z = zp ^ outer_hash(g, L, s.norb, kind, o) ^ inner_hash(g, L, s.norb, kind, q);
                const uint32_t j = t.pmap[top_bits(z, log2p)];
                if (j != 0xFFFFu)
                    atomicAdd(&hist[j], 1u);
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int j = tid; j < nparts; j += GEN_THREADS)
        cnt[(int64_t)j * nref + det] = hist[j];
}

// The bucket table of every reference determinant (layout at
// bucket_table_words), written once per evaluation call: the buckets depend
// on the determinant and the split, not on the subset, so each subset's
// generation and the count pass load them instead of building them.
template <int W>
__global__ __launch_bounds__(GEN_THREADS) void k_gen_buckets(DevSys s, ExcLayout L, const Planes refs, int64_t nref,
                                                             int log2p, uint16_t *bk)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L, false);
    Tgt t = carve_tgt(lds + gen_lds_bytes_dev(L, false), L, log2p);
    const int64_t det = blockIdx.x;
    const int tid = threadIdx.x, B = 1 << log2p;
    det_setup<W>(g, s, L, refs, det, false);
    uint16_t *dst0 = bk + det * bucket_table_words(L, log2p);
    for (int kind = 2; kind <= 4; kind++) {
        const int ni = n_inner(L, kind);
        uint16_t *dst = dst0 + bucket_kind_off(L, log2p, kind);
        if (n_outer(L, kind) == 0 || ni == 0) {
            for (int b = tid; b < B; b += GEN_THREADS)
                dst[b] = 0;
            continue;
        }
        build_buckets(g, t, L, s.norb, kind, log2p, true);
        for (int b = tid; b < B; b += GEN_THREADS)
            dst[b] = (uint16_t)t.bstart[b];
        for (int q = tid; q < ni; q += GEN_THREADS)
            dst[B + q] = t.blist[q];
        __syncthreads();  // the next kind's buckets reuse the arrays
    }
}

// Counts of the listed subsets with a cutoff (or the spin flip filter): the
// bucket walk of k_gen_target for each listed subset, counting the walked
// terms that are kept, so a call costs its own subsets' terms, not an
// enumeration of every candidate.  cnt[j * nref + det] as k_count_target.
// The walk needs generation's bucket lists, which occupy the region where the
// bucketed count keeps its counts and subset map, so this kernel keeps them
// in LDS of their own after the target layout (count_cut_lds_extra bytes):
// the counts of the listed subsets, then the map from subset to list position.
__host__ __device__ inline size_t count_cut_lds_extra(int log2p, int nparts)
{
    return align16((size_t)4 * nparts) + align16((size_t)2 << log2p);
}

template <int W, int PM>
__global__ __launch_bounds__(GEN_THREADS) void k_count_target_cut(DevSys s, ExcLayout L, const Planes refs,
                                                                  int64_t nref, int log2p, const uint32_t *parts,
                                                                  int nparts, double cutoff, uint32_t *cnt)
{
    extern __shared__ __align__(16) char lds[];
    GenLds g = carve(lds, L, false);
    Tgt t = carve_tgt(lds + gen_lds_bytes_dev(L, false), L, log2p);
    size_t o[8];
    char *extra = lds + gen_lds_bytes_dev(L, false) + tgt_lds_layout(L, log2p, o);
    uint32_t *ccount = (uint32_t *)extra;                                     // [nparts]
    uint16_t *cmap = (uint16_t *)(extra + align16((size_t)4 * nparts));      // [B]
    const int64_t det = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, B = 1 << log2p;
    __shared__ uint32_t s_cnt[GEN_THREADS / 64];
    det_setup<W>(g, s, L, refs, det);
    const DivConsts D = div_consts(L);
    const uint64_t zp = g.head->z;
    for (int b = tid; b < B; b += GEN_THREADS)
        cmap[b] = 0xFFFFu;
    for (int j = tid; j < nparts; j += GEN_THREADS)
        ccount[j] = 0;
    __syncthreads();
    for (int j = tid; j < nparts; j += GEN_THREADS)
        cmap[parts[j]] = (uint16_t)j;
    __syncthreads();
    // the singles of all listed subsets in one enumeration (a few per subset)
    for (int64_t k = tid; k < L.o2; k += GEN_THREADS) {
        const Exc e = decode(g, L, D, k);
        uint64_t key[W], z;
        exc_key<W>(g, s.norb, e, key, z);
        const uint32_t j = cmap[top_bits(z, log2p)];
        if (j != 0xFFFFu && keep_term<W, PM>(g, s, L, e, cutoff, key))
            atomicAdd(&ccount[j], 1u);
    }
    // the doubles, subset by subset, by block sums
    for (int kind = 2; kind <= 4; kind++) {
        const int no = n_outer(L, kind);
        if (no == 0 || n_inner(L, kind) == 0)
            continue;
        build_buckets(g, t, L, s.norb, kind, log2p, true);
        for (int j = 0; j < nparts; j++) {
            const uint32_t part = parts[j];
            for (int o = tid; o < no; o += GEN_THREADS) {
                const uint32_t b = part ^ top_bits(zp ^ outer_hash(g, L, s.norb, kind, o), log2p);
                t.tgt[o] = (uint16_t)b;
                t.pre[o] = t.bstart[b] - bucket_lo(t, b);
            }
            if (tid == 0)
                t.pre[no] = 0;
            __syncthreads();
            const uint32_t T = block_scan_excl(t.pre, no + 1, t.wsum);
            uint32_t kept = 0;
            for (uint32_t f = tid; f < T; f += GEN_THREADS) {
                int lo = 0, hi = no;  // pre[lo] <= f < pre[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (t.pre[mid] <= f)
                        lo = mid;
                    else
                        hi = mid;
                }
                const int q = t.blist[bucket_lo(t, t.tgt[lo]) + (f - t.pre[lo])];
                const Exc e = make_exc(g, L, D, kind, lo, q);
                uint64_t key[W], z;
                exc_key<W>(g, s.norb, e, key, z);
                kept += keep_term<W, PM>(g, s, L, e, cutoff, key) ? 1u : 0u;
            }
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1)
                kept += __shfl_xor(kept, sh);
            if (lane == 0)
                s_cnt[wave] = kept;
            __syncthreads();
            if (tid == 0) {
                uint32_t x = 0;
                for (int w = 0; w < GEN_THREADS / 64; w++)
                    x += s_cnt[w];
                ccount[j] += x;
            }
            // t.pre, t.tgt and s_cnt are rewritten for the next subset
            __syncthreads();
        }
    }
    __syncthreads();
    for (int j = tid; j < nparts; j += GEN_THREADS)
        cnt[(int64_t)j * nref + det] = ccount[j];
}

// Rank keys of the sorted bitstring references, same order, with their
// coefficients (the single pass matches records against these).
template <int W>
__global__ void k_refs_rank(DevSys s, Planes bits, int64_t n, Planes out)
{
    const uint64_t *B = s.kc.binom;
    const int st = s.kc.stride;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t ra = 0, rb = 0;
        int pa = 1, pb = 1;
#pragma unroll
        for (int w = 0; w < W; w++) {
            uint64_t m = pl_get<W>(bits, w, i);
            while (m) {
                const int b = w * 64 + __builtin_ctzll(m);
                m &= m - 1;
                if (b < s.norb)
                    rb += B[b * st + (pb++)];
                else
                    ra += B[(b - s.norb) * st + (pa++)];
            }
        }
        uint64_t lo, hi;
        rank_join(ra, rb, s.kc.bb, lo, hi);
        if (s.kc.kw == 1) {
            put_top(out.key[0], out.topb, i, lo);
        } else {
            out.key[0][i] = lo;
            put_top(out.key[1], out.topb, i, hi);
        }
        ((double *)out.pay)[i] = ((const double *)bits.pay)[i];
    }
}

template <int W, int PM>
hipError_t gen_direct_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int64_t chunk,
                        int skip_kinds, Planes out, hipStream_t st)
{
    const int64_t nred = L.nper - (skip_kinds >= 1 ? L.nDaa : 0) - (skip_kinds == 2 ? L.nDbb : 0);
    int cpd = (int)((nred + chunk - 1) / chunk);
    int64_t blocks = nref * cpd;
    if (blocks == 0 || nred == 0)
        return hipSuccess;
    if (blocks > 0x7FFFFFFFll)
        return hipErrorInvalidValue;
    size_t lds = gen_lds_bytes(L);
    hipLaunchKernelGGL((k_gen_direct<W, PM>), dim3((unsigned)blocks), dim3(GEN_THREADS), lds, st, s, L, refs, nref,
                       chunk, cpd, skip_kinds, out);
    return hipGetLastError();
}

template <int W, int PM>
hipError_t gen_spin_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int sp, const uint32_t *grp,
                      const uint32_t *gidx, int64_t ngrp, Planes out, hipStream_t st)
{
    const int64_t nk = sp == 0 ? L.nDaa : L.nDbb;
    if (ngrp == 0 || nk == 0)
        return hipSuccess;
    const int64_t achunk = REUSE_CHUNK;
    const int cpa = (int)((nk + achunk - 1) / achunk);
    const int64_t blocks = ngrp * cpa;
    if (blocks > 0x7FFFFFFFll)
        return hipErrorInvalidValue;
    const size_t lds = gen_lds_bytes(L) + (size_t)REUSE_GROUP * (W * 8 + 16);
    if (sp == 0)
        hipLaunchKernelGGL((k_gen_spin<W, PM, 0>), dim3((unsigned)blocks), dim3(GEN_THREADS), lds, st, s, L, refs,
                           grp, gidx, achunk, cpa, out);
    else
        hipLaunchKernelGGL((k_gen_spin<W, PM, 1>), dim3((unsigned)blocks), dim3(GEN_THREADS), lds, st, s, L, refs,
                           grp, gidx, achunk, cpa, out);
    return hipGetLastError();
}

}  // namespace

size_t gen_lds_bytes(const ExcLayout &L)
{
    size_t a, b, c, d, e, f;
    return lds_layout(L, &a, &b, &c, &d, &e, &f);
}

size_t target_lds_bytes(const ExcLayout &L, int log2p)
{
    size_t o[8];
    return gen_lds_bytes_dev(L, false) + tgt_lds_layout(L, log2p, o);
}

bool spin_reuse_ok(const ExcLayout &L, int W)
{
    return gen_lds_bytes(L) + (size_t)REUSE_GROUP * (W * 8 + 16) <= 65536;
}

bool count_cut_ok(const ExcLayout &L, int64_t nref, int log2p, int nparts)
{
    return target_ok(L, nref, log2p) && target_lds_bytes(L, log2p) + count_cut_lds_extra(log2p, nparts) <= 65536;
}

bool target_ok(const ExcLayout &L, int64_t nref, int log2p)
{
    return log2p >= 1 && log2p <= 12 && target_lds_bytes(L, log2p) <= 65536 &&
           ((int64_t)1 << log2p) * nref <= ((int64_t)1 << 30);
}

#define PT2_DISPATCH(W_, PM_, CALL)                                                                    \
    switch ((W_) * 3 + (PM_)) {                                                                        \
    case 3: return CALL(1, 0);                                                                         \
    case 4: return CALL(1, 1);                                                                         \
    case 5: return CALL(1, 2);                                                                         \
    case 6: return CALL(2, 0);                                                                         \
    case 7: return CALL(2, 1);                                                                         \
    case 8: return CALL(2, 2);                                                                         \
    case 9: return CALL(3, 0);                                                                         \
    case 10: return CALL(3, 1);                                                                        \
    case 11: return CALL(3, 2);                                                                        \
    case 12: return CALL(4, 0);                                                                        \
    case 13: return CALL(4, 1);                                                                        \
    case 14: return CALL(4, 2);                                                                        \
    default: return hipErrorInvalidValue;                                                              \
    }

hipError_t launch_gen_direct(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref, int64_t chunk,
                             int skip_kinds, Planes out, hipStream_t st)
{
#define CALL(W, F) gen_direct_t<W, F>(s, L, refs, nref, chunk, skip_kinds, out, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

hipError_t launch_gen_spin(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int sp, const uint32_t *grp,
                           const uint32_t *gidx, int64_t ngrp, Planes out, hipStream_t st)
{
#define CALL(W, F) gen_spin_t<W, F>(s, L, refs, sp, grp, gidx, ngrp, out, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

namespace {
template <int W, int PM>
hipError_t count_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref,
                   int64_t chunk, int log2p, double cutoff, uint32_t *cnt, int64_t nchunks, hipStream_t st)
{
    int cpd = (int)((L.nper + chunk - 1) / chunk);
    if (nchunks != nref * cpd)
        return hipErrorInvalidValue;
    if (nchunks == 0)
        return hipSuccess;
    size_t lds = gen_lds_bytes(L) + sizeof(uint32_t) * ((size_t)1 << log2p);
    hipLaunchKernelGGL((k_count<W, PM>), dim3((unsigned)nchunks), dim3(GEN_THREADS), lds, st, s, L, refs,
                       nref, chunk, cpd, log2p, cutoff, cnt, nchunks);
    return hipGetLastError();
}

template <int W, int PM>
hipError_t gen_compact_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int64_t chunk, int log2p, uint32_t part, double cutoff, const uint64_t *off,
                         int64_t nchunks, uint64_t cap, Planes out, Flags *flags, hipStream_t st)
{
    int cpd = (int)((L.nper + chunk - 1) / chunk);
    if (nchunks != nref * cpd)
        return hipErrorInvalidValue;
    if (nchunks == 0)
        return hipSuccess;
    size_t lds = gen_lds_bytes(L) + sizeof(uint32_t) * (GEN_THREADS / 64);
    hipLaunchKernelGGL((k_gen_compact<W, PM>), dim3((unsigned)nchunks), dim3(GEN_THREADS), lds, st, s, L, refs, nref, chunk, cpd, log2p, part, cutoff, off, cap, out, flags);
    return hipGetLastError();
}
template <int W>
hipError_t count_target_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                          const uint32_t *parts, int nparts, uint32_t *cnt, const uint16_t *bk, hipStream_t st)
{
    if (nref == 0 || nparts == 0)
        return hipSuccess;
    const size_t lds = target_lds_bytes(L, log2p);
    hipLaunchKernelGGL((k_count_target<W>), dim3((unsigned)nref), dim3(GEN_THREADS), lds, st, s, L, refs, nref,
                       log2p, parts, nparts, cnt, bk);
    return hipGetLastError();
}
template <int W>
hipError_t gen_buckets_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                         uint16_t *bk, hipStream_t st)
{
    if (nref == 0)
        return hipSuccess;
    const size_t lds = target_lds_bytes(L, log2p);
    hipLaunchKernelGGL((k_gen_buckets<W>), dim3((unsigned)nref), dim3(GEN_THREADS), lds, st, s, L, refs, nref,
                       log2p, bk);
    return hipGetLastError();
}

template <int W, int PM>
hipError_t gen_target_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                        uint32_t part, double cutoff, const uint64_t *off, const uint64_t *tot, Planes out,
                        Flags *flags, const uint16_t *bk, hipStream_t st)
{
    if (nref == 0)
        return hipSuccess;
    const size_t lds = target_lds_bytes(L, log2p);
    hipLaunchKernelGGL((k_gen_target<W, PM>), dim3((unsigned)nref), dim3(GEN_THREADS), lds, st, s, L, refs, nref,
                       log2p, part, cutoff, off, tot, out, flags, bk);
    return hipGetLastError();
}
template <int W, int PM>
hipError_t count_target_cut_t(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                              const uint32_t *parts, int nparts, double cutoff, uint32_t *cnt, hipStream_t st)
{
    if (nref == 0 || nparts == 0)
        return hipSuccess;
    if (!count_cut_ok(L, nref, log2p, nparts))
        return hipErrorInvalidValue;
    const size_t lds = target_lds_bytes(L, log2p) + count_cut_lds_extra(log2p, nparts);
    hipLaunchKernelGGL((k_count_target_cut<W, PM>), dim3((unsigned)nref), dim3(GEN_THREADS), lds, st, s, L, refs,
                       nref, log2p, parts, nparts, cutoff, cnt);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_count(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref, int64_t chunk, int log2p, double cutoff, uint32_t *cnt, int64_t nchunks,
                        hipStream_t st)
{
#define CALL(W, F) count_t<W, F>(s, L, refs, nref, chunk, log2p, cutoff, cnt, nchunks, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

hipError_t launch_gen_compact(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref, int64_t chunk, int log2p, uint32_t part,
                              double cutoff, const uint64_t *off, int64_t nchunks, uint64_t cap, Planes out,
                              Flags *flags, hipStream_t st)
{
#define CALL(W, F) \
    gen_compact_t<W, F>(s, L, refs, nref, chunk, log2p, part, cutoff, off, nchunks, cap, out, flags, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

hipError_t launch_count_target(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                               const uint32_t *parts, int nparts, uint32_t *cnt, const uint16_t *bk, hipStream_t st)
{
    if (!target_ok(L, nref, log2p))
        return hipErrorInvalidValue;
    switch (s.W) {
    case 1: return count_target_t<1>(s, L, refs, nref, log2p, parts, nparts, cnt, bk, st);
    case 2: return count_target_t<2>(s, L, refs, nref, log2p, parts, nparts, cnt, bk, st);
    case 3: return count_target_t<3>(s, L, refs, nref, log2p, parts, nparts, cnt, bk, st);
    case 4: return count_target_t<4>(s, L, refs, nref, log2p, parts, nparts, cnt, bk, st);
    default: return hipErrorInvalidValue;
    }
}

int64_t gen_bucket_words(const ExcLayout &L, int log2p) { return bucket_table_words(L, log2p); }

// A2[pair(r, q) * npair + pair(a, b)] = (ra|qb) - (rb|qa) for r < q, a < b
// (the FP64 subtraction the terms would make).
__global__ __launch_bounds__(256) void k_build_a2(const double *V, int n, double *A2)
{
    const int64_t np = (int64_t)n * (n - 1) / 2;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < np * np;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = x / np, v = x - u * np;
        int r, q, a, b;
        pair_decode((int)u, n, r, q);
        pair_decode((int)v, n, a, b);
        A2[x] = V[eidx(n, r, a, q, b)] - V[eidx(n, r, b, q, a)];
    }
}

hipError_t launch_build_a2(const double *V, int norb, double *A2, hipStream_t st)
{
    const int64_t np = (int64_t)norb * (norb - 1) / 2;
    if (np <= 0)
        return hipSuccess;
    const int64_t blocks = (np * np + 255) / 256;
    hipLaunchKernelGGL(k_build_a2, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, st, V, norb, A2);
    return hipGetLastError();
}

bool gen_buckets_ok(const ExcLayout &L, int log2p)
{
    // u16 ends and indices
    return L.nvpa <= 65535 && L.nvpb <= 65535 && L.nSb <= 65535 && log2p <= 12;
}

hipError_t launch_gen_buckets(const DevSys &s, const ExcLayout &L, const Planes &refs, int64_t nref, int log2p,
                              uint16_t *bk, hipStream_t st)
{
    if (!gen_buckets_ok(L, log2p))
        return hipErrorInvalidValue;
    switch (s.W) {
    case 1: return gen_buckets_t<1>(s, L, refs, nref, log2p, bk, st);
    case 2: return gen_buckets_t<2>(s, L, refs, nref, log2p, bk, st);
    case 3: return gen_buckets_t<3>(s, L, refs, nref, log2p, bk, st);
    case 4: return gen_buckets_t<4>(s, L, refs, nref, log2p, bk, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_count_target_cut(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                                   int log2p, const uint32_t *parts, int nparts, double cutoff, uint32_t *cnt,
                                   hipStream_t st)
{
    if (!target_ok(L, nref, log2p))
        return hipErrorInvalidValue;
#define CALL(W, F) count_target_cut_t<W, F>(s, L, refs, nref, log2p, parts, nparts, cutoff, cnt, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

hipError_t launch_gen_target(const DevSys &s, const ExcLayout &L, int pm, const Planes &refs, int64_t nref,
                             int log2p, uint32_t part, double cutoff, const uint64_t *off, const uint64_t *tot,
                             Planes out, Flags *flags, const uint16_t *bk, hipStream_t st)
{
    if (!target_ok(L, nref, log2p))
        return hipErrorInvalidValue;
#define CALL(W, F) gen_target_t<W, F>(s, L, refs, nref, log2p, part, cutoff, off, tot, out, flags, bk, st)
    PT2_DISPATCH(s.W, pm, CALL)
#undef CALL
}

hipError_t launch_refs_rank(const DevSys &s, const Planes &bits, int64_t n, const Planes &out, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_refs_rank<1>), g, b, 0, st, s, bits, n, out); break;
    case 2: hipLaunchKernelGGL((k_refs_rank<2>), g, b, 0, st, s, bits, n, out); break;
    case 3: hipLaunchKernelGGL((k_refs_rank<3>), g, b, 0, st, s, bits, n, out); break;
    case 4: hipLaunchKernelGGL((k_refs_rank<4>), g, b, 0, st, s, bits, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_chunk_scan(const uint32_t *cnt, int64_t nchunks, const uint32_t *parts, int nparts, uint64_t *off,
                             uint64_t *tot, hipStream_t st)
{
    if (nparts == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_chunk_scan, dim3(nparts), dim3(1024), 0, st, cnt, nchunks, parts, off, tot);
    return hipGetLastError();
}

}  // namespace pt2
