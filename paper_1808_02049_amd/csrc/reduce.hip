// Single pass over the sorted records (Algorithm 1, final step): form the
// numerator N_a of every distinct bitstring a, drop a if it is in the
// reference, otherwise add N_a^2 / (E0 - H_aa) to the energy (the
// Epstein-Nesbet equation of Section II; Algorithm 1 prints the term without
// the square, read here as the square of the summed numerator).
//
// Reference membership is decided by binary search (the direct check of the
// duplicate-removal subsection of Section V), but per distinct bitstring and
// against only the few reference bitstrings that fall inside the tile's key
// range, staged in LDS: the sorted records and the sorted reference list are
// merged tile by tile.  H_aa comes from a spin-orbital pair table (packed
// upper triangle, in LDS when it fits), sum over occupied pairs b1 <= b2 of
// T[b1][b2], taken relative to an anchor determinant.
//
// The denominator E0 - H_aa is formed in double-double arithmetic: E0 and
// H_aa are of order 10^2 Eh while their difference can be 10^-6 Eh or less,
// and such a determinant's term moves by its own size for every relative
// change of the difference.  Every summand is an exact FP64 number (the pair
// table carries each entry's rounding error beside it), the anchor's g vector
// and E0 - E(anchor) are double-double, and the per-key combination adds the
// pairs with the two-sum error-free transformation, so the difference is
// exact to a few units in its own last place.
//
// A fixed grid of RED_GRID workgroups takes contiguous ranges of tiles; a
// workgroup owns the segments whose first record lies in its tiles, follows a
// segment past a tile end with one wavefront, queues the segment ends of a
// tile in LDS and evaluates them round-robin over its threads, keeping a
// Neumaier-compensated sum.  Partials are combined in workgroup order, so the
// energy is bit-reproducible.
#include "pt2_internal.h"

namespace pt2 {
namespace {

template <int W>
__device__ inline int key_cmp(const uint64_t (&a)[W], const uint64_t (&b)[W])
{
#pragma unroll
    for (int w = W - 1; w >= 0; w--) {
        if (a[w] < b[w])
            return -1;
        if (a[w] > b[w])
            return 1;
    }
    return 0;
}

template <int W>
__device__ inline bool key_eq(const uint64_t (&a)[W], const uint64_t (&b)[W])
{
    bool e = true;
#pragma unroll
    for (int w = 0; w < W; w++)
        e = e && a[w] == b[w];
    return e;
}

template <int W>
__device__ inline void load_key(const Planes &p, int64_t i, uint64_t (&k)[W])
{
#pragma unroll
    for (int w = 0; w < W; w++)
        k[w] = pl_get<W>(p, w, i);
}

template <int PB>
__device__ inline double load_pay(const Planes &p, int64_t i)
{
    if (PB == 8)
        return ((const double *)p.pay)[i];
    return (double)((const float *)p.pay)[i];
}

// Hash and auxiliary words of hash record i: FP64 records are never packed,
// so their kernels read the words as stored.
template <int PB>
__device__ inline uint64_t rec_hash(const KeyCodec &kc, const Planes &in, int64_t i)
{
    return PB == 8 ? in.key[0][i] : hash_at(kc, in, i);
}
template <int PB>
__device__ inline uint64_t rec_aux(const KeyCodec &kc, int norb, const Planes &in, int64_t i)
{
    return PB == 8 ? in.key[1][i] : aux_at(kc, norb, in, i);
}

// Payload of hash record i (FP32 payloads may be packed; see hash_put).
template <int PB>
__device__ inline double hpay_at(const KeyCodec &kc, const Planes &in, int64_t i)
{
    if (PB == 8)
        return ((const double *)in.pay)[i];
    return (double)pay32_at(kc, in, i);
}

// first index in [lo, hi) whose reference key is >= k (upper == false) or > k
template <int W>
__device__ int64_t ref_bound(const Planes &refs, int64_t lo, int64_t hi, const uint64_t (&k)[W], bool upper)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        uint64_t r[W];
        load_key<W>(refs, mid, r);
        int c = key_cmp<W>(r, k);
        if (c < 0 || (upper && c == 0))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ inline uint64_t splitmix_step(uint64_t st)
{
    uint64_t z = st + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int W>
__device__ inline uint64_t key_mix(const uint64_t (&k)[W])
{
    uint64_t acc = 0x243F6A8885A308D3ull;
#pragma unroll
    for (int w = 0; w < W; w++)
        acc = splitmix_step(k[w] ^ acc);
    return acc;
}

// Packed upper-triangular pair table of the spin-orbitals (b1 <= b2): the row
// of b1 starts at tri_row(b1) and is indexed by b2.
__host__ __device__ inline int tri_row(int b1, int nso) { return b1 * nso - (b1 * (b1 - 1)) / 2 - b1; }

// Double-double accumulator: the exact value is hi + lo.  Knuth's two-sum
// gives the exact rounding error of each addition.
struct DD {
    double hi, lo;
};

__device__ inline double two_sum(double a, double b, double &err)
{
    const double s = a + b;
    const double bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

// x += (vh + vl)
__device__ inline void dd_add(DD &x, double vh, double vl)
{
    double e;
    x.hi = two_sum(x.hi, vh, e);
    x.lo += e + vl;
}

__device__ inline DD dd_sum(const DD &x, const DD &y)
{
    DD r = x;
    dd_add(r, y.hi, y.lo);
    return r;
}

__device__ inline double tri_at(const double *Tp, int nso, int b1, int b2)
{
    const int lo = b1 < b2 ? b1 : b2, hi = b1 < b2 ? b2 : b1;
    return Tp[tri_row(lo, nso) + hi];
}

// x += sign * T[b1][b2] (both parts; the low part is zero for pairs of
// opposite spin and for the diagonal, so it is read only for same-spin pairs)
__device__ inline void dd_add_pair(DD &x, const double *Tp, const double *Tl, int nso, int b1, int b2, double sign)
{
    const int lo = b1 < b2 ? b1 : b2, hi = b1 < b2 ? b2 : b1;
    const int at = tri_row(lo, nso) + hi;
    const bool same = (lo < nso / 2) == (hi < nso / 2) && lo != hi;
    dd_add(x, sign * Tp[at], same ? sign * Tl[at] : 0.0);
}

// E0 - H_aa from scratch: E0 minus every occupied pair b1 <= b2 of T, in
// double-double.
template <int W>
__device__ inline double den_scratch(const double *Tp, const double *Tl, int nso, const uint64_t (&k)[W], double e0)
{
    DD d = {e0, 0.0};
#pragma unroll
    for (int w1 = 0; w1 < W; w1++) {
        uint64_t m1 = k[w1];
        while (m1) {
            const int b1 = w1 * 64 + __builtin_ctzll(m1);
            m1 &= m1 - 1;
            dd_add(d, -Tp[tri_row(b1, nso) + b1], 0.0);
            uint64_t m2 = m1;
            while (m2) {
                dd_add_pair(d, Tp, Tl, nso, b1, w1 * 64 + __builtin_ctzll(m2), -1.0);
                m2 &= m2 - 1;
            }
#pragma unroll
            for (int w2 = w1 + 1; w2 < W; w2++) {
                uint64_t m3 = k[w2];
                while (m3) {
                    dd_add_pair(d, Tp, Tl, nso, b1, w2 * 64 + __builtin_ctzll(m3), -1.0);
                    m3 &= m3 - 1;
                }
            }
        }
    }
    return d.hi + d.lo;
}

// The anchor block staged in LDS (the parts an evaluation uses).
struct AncView {
    const uint64_t *bits;       // MAXW words
    DD d0;                      // E0 - E(A)
    const int16_t *hr;          // norb entries
    const double *gh, *gl;      // nso entries each
    const double *Jh, *Kh;      // nh x norb each
};

__host__ __device__ inline size_t anc_lds_bytes(int norb, int nh)
{
    return (size_t)MAXW * 8 + (((size_t)norb * 2 + 15) & ~(size_t)15) + (size_t)norb * 32 +
           (size_t)nh * norb * 16;
}

// Copy the anchor block into dyn (anc_lds_bytes bytes, 16-byte aligned) with
// all threads; the caller synchronises before use.
__device__ inline AncView stage_anchor(const AnchorBlk *g, char *dyn, int norb, int nh, int nthreads)
{
    const int tid = threadIdx.x, nso = 2 * norb;
    AncView v;
    uint64_t *bits = (uint64_t *)dyn;
    int16_t *hr = (int16_t *)(dyn + MAXW * 8);
    double *gh = (double *)(dyn + MAXW * 8 + (((size_t)norb * 2 + 15) & ~(size_t)15));
    double *gl = gh + nso;
    double *Jh = gl + nso;
    double *Kh = Jh + (size_t)nh * norb;
    if (tid < MAXW)
        bits[tid] = g->bits[tid];
    for (int i = tid; i < norb; i += nthreads)
        hr[i] = g->hr[i];
    for (int i = tid; i < nso; i += nthreads) {
        gh[i] = g->gh[i];
        gl[i] = g->gl[i];
    }
    for (int i = tid; i < nh * norb; i += nthreads) {
        Jh[i] = g->Jh[i];
        Kh[i] = g->Kh[i];
    }
    v.bits = bits, v.hr = hr, v.gh = gh, v.gl = gl, v.Jh = Jh, v.Kh = Kh;
    v.d0.hi = g->d0h, v.d0.lo = g->d0l;
    return v;
}

// x += sign * T[x1][x2] (x1 != x2): from the hot J and K rows when either
// spatial orbital is occupied in the anchor (a same-spin pair adds J and -K,
// each exact), else from the packed table.
__device__ inline void dd_add_t(DD &x, const AncView &a, const double *Tp, const double *Tl, int norb, int x1, int x2,
                                double sign)
{
    const int p = x1 < norb ? x1 : x1 - norb, q = x2 < norb ? x2 : x2 - norb;
    int r = a.hr[p], c = q;
    if (r < 0)
        r = a.hr[q], c = p;
    if (r >= 0) {
        const int at = r * norb + c;
        dd_add(x, sign * a.Jh[at], 0.0);
        if ((x1 < norb) == (x2 < norb))
            dd_add(x, -sign * a.Kh[at], 0.0);
    } else {
        dd_add_pair(x, Tp, Tl, 2 * norb, x1, x2, sign);
    }
}

// E0 - H_aa relative to the anchor A, given d0 = E0 - E(A) and
// g_x = h_x + sum_{c in A, c != x} T[x][c] (both double-double): with R the
// spin-orbitals removed from A and P those added,
//   H = E(A) - sum_R g_r + sum_P g_a + sum_{r<r' in R} T + sum_{a<a' in P} T
//       - sum_{a in P, r in R} T[a][r],
// so E0 - H = d0 + sum_R g_r - sum_P g_a - sum_RR T - sum_PP T + sum_PR T.
// Falls back to the from-scratch sum when the difference is large.
template <int W>
__device__ inline double den_anchor(const AncView &an, const double *Tp, const double *Tl, int norb, int nel,
                                    const uint64_t (&k)[W], double e0)
{
    uint64_t rm[W], ad[W];
    int m = 0;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const uint64_t d = k[w] ^ an.bits[w];
        rm[w] = d & an.bits[w];
        ad[w] = d & k[w];
        m += __popcll(ad[w]);
    }
    if (2 * m * m + m >= (nel * nel) / 2)
        return den_scratch<W>(Tp, Tl, 2 * norb, k, e0);
    DD d = an.d0;
#pragma unroll
    for (int w1 = 0; w1 < W; w1++) {
        uint64_t x = rm[w1];
        while (x) {
            const int r = w1 * 64 + __builtin_ctzll(x);
            x &= x - 1;
            dd_add(d, an.gh[r], an.gl[r]);
            uint64_t y = x;  // r < r' within R
            while (y) {
                dd_add_t(d, an, Tp, Tl, norb, r, w1 * 64 + __builtin_ctzll(y), -1.0);
                y &= y - 1;
            }
#pragma unroll
            for (int w2 = w1 + 1; w2 < W; w2++) {
                uint64_t z = rm[w2];
                while (z) {
                    dd_add_t(d, an, Tp, Tl, norb, r, w2 * 64 + __builtin_ctzll(z), -1.0);
                    z &= z - 1;
                }
            }
#pragma unroll
            for (int w2 = 0; w2 < W; w2++) {
                uint64_t z = ad[w2];  // cross pairs with P
                while (z) {
                    dd_add_t(d, an, Tp, Tl, norb, r, w2 * 64 + __builtin_ctzll(z), 1.0);
                    z &= z - 1;
                }
            }
        }
    }
#pragma unroll
    for (int w1 = 0; w1 < W; w1++) {
        uint64_t x = ad[w1];
        while (x) {
            const int a = w1 * 64 + __builtin_ctzll(x);
            x &= x - 1;
            dd_add(d, -an.gh[a], -an.gl[a]);
            uint64_t y = x;
            while (y) {
                dd_add_t(d, an, Tp, Tl, norb, a, w1 * 64 + __builtin_ctzll(y), -1.0);
                y &= y - 1;
            }
#pragma unroll
            for (int w2 = w1 + 1; w2 < W; w2++) {
                uint64_t z = ad[w2];
                while (z) {
                    dd_add_t(d, an, Tp, Tl, norb, a, w2 * 64 + __builtin_ctzll(z), -1.0);
                    z &= z - 1;
                }
            }
        }
    }
    return d.hi + d.lo;
}

__device__ inline void neumaier(double &sum, double &comp, double x)
{
    double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

struct Acc {
    double e_sum, e_comp, ref_cross, min_abs;
    uint64_t n_unique, n_ext, n_hit, n_nonneg, kx, ks;
    uint32_t singular;
};

__device__ inline void acc_init(Acc &a)
{
    a.e_sum = a.e_comp = a.ref_cross = 0.0;
    a.min_abs = __builtin_inf();
    a.n_unique = a.n_ext = a.n_hit = a.n_nonneg = a.kx = a.ks = 0;
    a.singular = 0;
}

struct RefSlice {
    int64_t lo, hi;  // global range of reference keys inside the tile's key range
    int staged;      // 1 if [lo, hi) is staged in LDS
};

// One distinct bitstring with its numerator: exclusion test, then the term.
// k is the record key (W words); the diagonal and the checksum use the
// bitstring (WB words), which is k itself or, for rank keys, unranked from it.
template <int W, int WB, bool RK>
__device__ inline void process_segment(const DevSys &s, const double *Tp, const double *Tl, const AncView &an,
                                       const Planes &refs,
                                       const RefSlice &rs, const uint64_t *s_rk, const double *s_rc, double e0,
                                       const uint64_t (&k)[W], double num, Acc &a, const uint64_t *binom,
                                       bool search)
{
    a.n_unique++;
    // spin flip: the weight of a generated determinant (2 unless alpha == beta)
    auto weight = [&]() -> double {
        if (!s.z2)
            return 1.0;
        uint64_t kw[WB];
        if constexpr (RK) {
            unrank_key<WB>(k[0], W > 1 ? k[W > 1 ? 1 : 0] : 0ull, s.norb, s.na, s.nb, s.kc.bb, binom,
                           s.kc.stride, kw);
        } else {
#pragma unroll
            for (int w = 0; w < WB; w++)
                kw[w] = k[w < W ? w : 0];
        }
        return swap_weight<WB>(kw, s.norb);
    };
    if (!search) {
        // reference determinants stay in; their terms are subtracted afterwards
    } else if (rs.staged) {
        int lo = 0, hi = (int)(rs.hi - rs.lo);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            uint64_t r[W];
#pragma unroll
            for (int w = 0; w < W; w++)
                r[w] = s_rk[w * RED_LDS_REFS + mid];
            const int c = key_cmp<W>(r, k);
            if (c == 0) {
                a.n_hit++;
                a.ref_cross += weight() * (s_rc[mid] * num);
                return;
            }
            if (c < 0)
                lo = mid + 1;
            else
                hi = mid;
        }
    } else {
        const int64_t i = ref_bound<W>(refs, rs.lo, rs.hi, k, false);
        if (i < rs.hi) {
            uint64_t r[W];
            load_key<W>(refs, i, r);
            if (key_eq<W>(r, k)) {
                a.n_hit++;
                a.ref_cross += weight() * (((const double *)refs.pay)[i] * num);
                return;
            }
        }
    }
    uint64_t kb[WB];
    if constexpr (RK) {
        unrank_key<WB>(k[0], W > 1 ? k[W > 1 ? 1 : 0] : 0ull, s.norb, s.na, s.nb, s.kc.bb, binom, s.kc.stride, kb);
    } else {
#pragma unroll
        for (int w = 0; w < WB; w++)
            kb[w] = k[w < W ? w : 0];
    }
    const double den = den_anchor<WB>(an, Tp, Tl, s.norb, s.na + s.nb, kb, e0);
    a.n_ext++;
    const double ad = fabs(den);
    a.min_abs = ad < a.min_abs ? ad : a.min_abs;
    if (den >= 0.0)
        a.n_nonneg++;
    if (den == 0.0)
        a.singular = 1;
    else
        neumaier(a.e_sum, a.e_comp, (s.z2 ? swap_weight<WB>(kb, s.norb) : 1.0) * (num * num / den));
    const uint64_t m = key_mix<WB>(kb);
    a.kx ^= m;
    a.ks += m;
}

// Wavefront scan: first index >= from whose reference key is > k (strict) or
// >= k (!strict).  All 64 lanes of the wavefront call it with equal arguments.
template <int W>
__device__ inline int64_t ref_advance(const Planes &refs, int64_t nref, int64_t from, const uint64_t (&k)[W],
                                      bool strict)
{
    const int lane = threadIdx.x & 63;
    int64_t cur = from;
    while (cur < nref) {
        const int64_t i = cur + lane;
        bool before = false;
        if (i < nref) {
            uint64_t r[W];
            load_key<W>(refs, i, r);
            const int c = key_cmp<W>(r, k);
            before = strict ? c <= 0 : c < 0;
        }
        const uint64_t m = __ballot(before);  // a prefix of the lanes: references are sorted
        if (m == ~0ull) {
            cur += 64;
            continue;
        }
        cur += __builtin_ctzll(~m);
        break;
    }
    return cur < nref ? cur : nref;
}


constexpr int RED_Q = RED_TILE + 1;  // segment ends of one tile plus a continuation

// Reference range of every tile: [lo, hi) holds the reference keys between
// the tile's first and last record keys (one thread per tile, ahead of the
// single pass, so that no workgroup waits on a search between its tiles).
template <int W>
__global__ void k_tile_refs(Planes in, int64_t n, Planes refs, int64_t nref, int64_t *range)
{
    const int64_t ntiles = (n + RED_TILE - 1) / RED_TILE;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t base = t * RED_TILE;
        const int64_t tend = base + RED_TILE < n ? base + RED_TILE : n;
        uint64_t kf[W], kl[W];
        load_key<W>(in, base, kf);
        load_key<W>(in, tend - 1, kl);
        const int64_t lo = ref_bound<W>(refs, 0, nref, kf, false);
        range[2 * t] = lo;
        range[2 * t + 1] = ref_bound<W>(refs, lo, nref, kl, true);
    }
}

// Partial sums of one workgroup, combined in a fixed order.
__device__ inline void partial_merge(Partial &x, const Partial &y)
{
    double sum = x.e_sum, comp = x.e_comp + y.e_comp;
    neumaier(sum, comp, y.e_sum);
    x.e_sum = sum, x.e_comp = comp;
    x.ref_cross += y.ref_cross;
    x.min_abs_denom = y.min_abs_denom < x.min_abs_denom ? y.min_abs_denom : x.min_abs_denom;
    x.n_unique += y.n_unique, x.n_external += y.n_external, x.n_hit += y.n_hit;
    x.n_nonneg += y.n_nonneg, x.key_xor ^= y.key_xor, x.key_sum += y.key_sum;
}

__device__ inline Partial acc_partial(const Acc &a)
{
    Partial me;
    me.e_sum = a.e_sum, me.e_comp = a.e_comp, me.ref_cross = a.ref_cross, me.min_abs_denom = a.min_abs;
    me.n_unique = a.n_unique, me.n_external = a.n_ext, me.n_hit = a.n_hit, me.n_nonneg = a.n_nonneg;
    me.key_xor = a.kx, me.key_sum = a.ks;
    return me;
}

// Each workgroup takes a contiguous range of tiles.
template <int W, int PB, int WB, bool RK>
__global__ __launch_bounds__(RED_THREADS) void k_reduce(DevSys s, Planes in, int64_t n, Planes refs, int64_t nref,
                                                        double e0, const AnchorBlk *anc, int nh, int64_t tiles_per_block,
                                                        size_t q_bytes, const int64_t *range, int search,
                                                        Partial *partials, Flags *flags)
{
    extern __shared__ __align__(16) char dyn[];
    __shared__ uint8_t s_f[RED_THREADS / 64];
    __shared__ double s_v[RED_THREADS / 64];
    __shared__ uint32_t s_cnt[RED_THREADS / 64];
    __shared__ uint64_t s_rk[W * RED_LDS_REFS];
    __shared__ double s_rc[RED_LDS_REFS];
    __shared__ uint64_t s_ck[W];
    __shared__ double s_cv;
    __shared__ int64_t s_lo, s_hi;
    __shared__ int s_cflag;
    __shared__ Partial s_wp[RED_THREADS / 64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // queue of owned segment ends: the numerator and the record's index in
    // its tile (the key is read back from the tile, which is in the caches)
    double *q_num = (double *)dyn;                            // [RED_Q]
    uint32_t *q_idx = (uint32_t *)(dyn + (size_t)RED_Q * 8);  // [RED_Q]
    // the evaluation's anchor after the queue region, then the binomial
    // table for unranking rank keys
    const AncView an = stage_anchor(anc, dyn + q_bytes, s.norb, nh, RED_THREADS);
    const double *Tp = s.T;
    const double *Tl = s.Tlo;
    uint64_t *binom = nullptr;
    if constexpr (RK) {
        binom = (uint64_t *)(dyn + q_bytes + anc_lds_bytes(s.norb, nh));
        const int nb = (s.norb + 1) * s.kc.stride;
        for (int i = tid; i < nb; i += RED_THREADS)
            binom[i] = s.kc.binom[i];
    }
    // the staged tables are read by every thread from here on
    __syncthreads();
    Acc a;
    acc_init(a);

    const int64_t ntiles = (n + RED_TILE - 1) / RED_TILE;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_block;
    const int64_t t_end = t_begin + tiles_per_block < ntiles ? t_begin + tiles_per_block : ntiles;
    for (int64_t tile = t_begin; tile < t_end; tile++) {
        const int64_t base = tile * RED_TILE;
        const int64_t tend = base + RED_TILE < n ? base + RED_TILE : n;
        const int64_t r0 = base + (int64_t)tid * RED_ITEMS;
        uint64_t k[RED_ITEMS][W];
        double p[RED_ITEMS];
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            if (idx < tend) {
                load_key<W>(in, idx, k[j]);
                p[j] = load_pay<PB>(in, idx);
            } else {
#pragma unroll
                for (int w = 0; w < W; w++)
                    k[j][w] = 0;
                p[j] = 0.0;
            }
        }
        uint64_t kp[W], kn[W];
        const bool has_prev = r0 > 0 && r0 < tend;
        const bool has_next = r0 + RED_ITEMS < n;
        if (has_prev)
            load_key<W>(in, r0 - 1, kp);
        if (has_next)
            load_key<W>(in, r0 + RED_ITEMS, kn);
        if (tid == 0) {
            s_lo = range[2 * tile];
            s_hi = range[2 * tile + 1];
            s_cflag = 0;
        }
        __syncthreads();
        RefSlice rs;
        rs.lo = s_lo, rs.hi = s_hi;
        rs.staged = search && (rs.hi - rs.lo) <= RED_LDS_REFS;
        if (rs.staged)
            for (int i = tid; i < (int)(rs.hi - rs.lo); i += RED_THREADS) {
#pragma unroll
                for (int w = 0; w < W; w++)
                    s_rk[w * RED_LDS_REFS + i] = pl_get<W>(refs, w, rs.lo + i);
                s_rc[i] = ((const double *)refs.pay)[rs.lo + i];
            }


        double run[RED_ITEMS];
        bool hh[RED_ITEMS], tl[RED_ITEMS];
        double sacc = 0.0;
        bool any = false;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool valid = idx < tend;
            bool head;
            if (j == 0)
                head = idx == 0 || !has_prev || !key_eq<W>(k[0], kp);
            else
                head = !key_eq<W>(k[j], k[j - 1]);
            head = head && valid;
            bool tail;
            if (j == RED_ITEMS - 1)
                tail = !has_next || !key_eq<W>(k[j], kn);
            else
                tail = idx + 1 >= n || !key_eq<W>(k[j], k[j + 1]);
            tl[j] = tail && valid;
            if (valid) {
                sacc = head ? p[j] : sacc + p[j];
                any = any || head;
            }
            run[j] = sacc;
            hh[j] = any;
        }
        // block exclusive segmented scan of (any, sacc) over threads: inclusive
        // scan within each wavefront by shuffles, then the earlier wavefronts'
        // totals; the operator is (f1,v1).(f2,v2) = (f1|f2, f2 ? v2 : v1+v2)
        bool fi = any;
        double vi = sacc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int fo = __shfl_up((int)fi, o);
            const double vo = __shfl_up(vi, o);
            if (lane >= o) {
                vi = fi ? vi : vo + vi;
                fi = fi || fo;
            }
        }
        if (lane == 63) {
            s_f[wave] = fi ? 1 : 0;
            s_v[wave] = vi;
        }
        // exclusive value within the wavefront
        int fx = __shfl_up((int)fi, 1);
        double vx = __shfl_up(vi, 1);
        if (lane == 0) {
            fx = 0;
            vx = 0.0;
        }
        __syncthreads();
        // prefix of the earlier wavefronts, combined in order
        bool fw = false;
        double vw = 0.0;
        for (int w = 0; w < wave; w++) {
            const bool f2 = s_f[w] != 0;
            vw = f2 ? s_v[w] : vw + s_v[w];
            fw = fw || f2;
        }
        const bool cf = fx ? true : fw;
        const double cv = fx ? vx : vw + vx;

        // owned segment ends of this thread go to the queue in record order
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool owned = idx < tend && (hh[j] || cf);
            if (owned && tl[j])
                mine++;
            if (owned && !tl[j] && idx == tend - 1) {
                // the segment continues past the tile end
#pragma unroll
                for (int w = 0; w < W; w++)
                    s_ck[w] = k[j][w];
                s_cv = hh[j] ? run[j] : cv + run[j];
                s_cflag = 1;
            }
        }
        uint32_t x = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o)
                x += y;
        }
        if (lane == 63)
            s_cnt[wave] = x;
        __syncthreads();
        uint32_t pre = 0, qtot = 0;
#pragma unroll
        for (int w = 0; w < RED_THREADS / 64; w++) {
            const uint32_t t = s_cnt[w];
            pre += w < wave ? t : 0u;
            qtot += t;
        }
        uint32_t slot = pre + x - mine;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool owned = idx < tend && (hh[j] || cf);
            if (owned && tl[j]) {
                q_idx[slot] = (uint32_t)(idx - base);
                q_num[slot] = hh[j] ? run[j] : cv + run[j];
                slot++;
            }
        }
        const int cflag = s_cflag;
        if (cflag && tid < 64) {
            // wave 0 follows the continuing segment into the following records
            uint64_t ck[W];
#pragma unroll
            for (int w = 0; w < W; w++)
                ck[w] = s_ck[w];
            double total = 0.0;
            int64_t pos = tend;
            while (true) {
                const int64_t idx = pos + lane;
                bool eq = false;
                double v = 0.0;
                if (idx < n) {
                    uint64_t kk[W];
                    load_key<W>(in, idx, kk);
                    eq = key_eq<W>(kk, ck);
                    if (eq)
                        v = load_pay<PB>(in, idx);
                }
                const uint64_t m = __ballot(eq);
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1)
                    v += __shfl_down(v, o);
                total += v;  // lane 0 holds the sum of this step
                if (m != ~0ull)
                    break;
                pos += 64;
            }
            if (lane == 0) {
                q_idx[qtot] = (uint32_t)(tend - 1 - base);  // a record of that segment
                q_num[qtot] = s_cv + total;
            }
        }
        __syncthreads();
        const int qn = (int)qtot + cflag;
        for (int e = tid; e < qn; e += RED_THREADS) {
            uint64_t kk[W];
            load_key<W>(in, base + q_idx[e], kk);
            process_segment<W, WB, RK>(s, Tp, Tl, an, refs, rs, s_rk, s_rc, e0, kk, q_num[e], a, binom,
                                       search != 0);
        }
        __syncthreads();
    }

    // block reduction of the accumulators in a fixed order: a shuffle tree
    // within each wavefront, then the wavefronts in order
    if (a.singular)
        atomicOr(&flags->err, ERR_SINGULAR);
    Partial me;
    me.e_sum = a.e_sum, me.e_comp = a.e_comp, me.ref_cross = a.ref_cross, me.min_abs_denom = a.min_abs;
    me.n_unique = a.n_unique, me.n_external = a.n_ext, me.n_hit = a.n_hit, me.n_nonneg = a.n_nonneg;
    me.key_xor = a.kx, me.key_sum = a.ks;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        Partial y;
        y.e_sum = __shfl_down(me.e_sum, o);
        y.e_comp = __shfl_down(me.e_comp, o);
        y.ref_cross = __shfl_down(me.ref_cross, o);
        y.min_abs_denom = __shfl_down(me.min_abs_denom, o);
        y.n_unique = __shfl_down(me.n_unique, o);
        y.n_external = __shfl_down(me.n_external, o);
        y.n_hit = __shfl_down(me.n_hit, o);
        y.n_nonneg = __shfl_down(me.n_nonneg, o);
        y.key_xor = __shfl_down(me.key_xor, o);
        y.key_sum = __shfl_down(me.key_sum, o);
        if (lane < o) {
            double sum = me.e_sum, comp = me.e_comp + y.e_comp;
            neumaier(sum, comp, y.e_sum);
            me.e_sum = sum, me.e_comp = comp;
            me.ref_cross += y.ref_cross;
            me.min_abs_denom = y.min_abs_denom < me.min_abs_denom ? y.min_abs_denom : me.min_abs_denom;
            me.n_unique += y.n_unique, me.n_external += y.n_external, me.n_hit += y.n_hit;
            me.n_nonneg += y.n_nonneg, me.key_xor ^= y.key_xor, me.key_sum += y.key_sum;
        }
    }
    if (lane == 0)
        s_wp[wave] = me;
    __syncthreads();
    if (tid == 0) {
        Partial x2 = s_wp[0];
        for (int w = 1; w < RED_THREADS / 64; w++) {
            const Partial y = s_wp[w];
            double sum = x2.e_sum, comp = x2.e_comp + y.e_comp;
            neumaier(sum, comp, y.e_sum);
            x2.e_sum = sum, x2.e_comp = comp;
            x2.ref_cross += y.ref_cross;
            x2.min_abs_denom = y.min_abs_denom < x2.min_abs_denom ? y.min_abs_denom : x2.min_abs_denom;
            x2.n_unique += y.n_unique, x2.n_external += y.n_external, x2.n_hit += y.n_hit;
            x2.n_nonneg += y.n_nonneg, x2.key_xor ^= y.key_xor, x2.key_sum += y.key_sum;
        }
        partials[blockIdx.x] = x2;
    }
}

// sum over the reference of c_i^2 (E0 - H_ii), per block (subtraction form
// of the exclusion); H_ii from scratch, FP64
template <int W>
__global__ __launch_bounds__(256) void k_ref_terms(DevSys s, Planes refs, int64_t n, double e0, Partial *partials)
{
    __shared__ double s_s[256], s_c[256];
    double sum = 0.0, comp = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        uint64_t k[W];
        load_key<W>(refs, i, k);
        const double ci = ((const double *)refs.pay)[i];
        neumaier(sum, comp, ci * ci * den_scratch<W>(s.T, s.Tlo, 2 * s.norb, k, e0));
    }
    s_s[threadIdx.x] = sum;
    s_c[threadIdx.x] = comp;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            double a = s_s[threadIdx.x], ca = s_c[threadIdx.x] + s_c[threadIdx.x + o];
            neumaier(a, ca, s_s[threadIdx.x + o]);
            s_s[threadIdx.x] = a;
            s_c[threadIdx.x] = ca;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Partial p;
        p.e_sum = s_s[0], p.e_comp = s_c[0], p.ref_cross = 0.0, p.min_abs_denom = __builtin_inf();
        p.n_unique = p.n_external = p.n_hit = p.n_nonneg = p.key_xor = p.key_sum = 0;
        partials[blockIdx.x] = p;
    }
}

// The anchor block of an evaluation: A is the first sorted reference (an
// empty determinant when there is none, for which the same formulas hold).
// One workgroup: the hot rows (J and K of the spatial orbitals occupied in A
// in either spin, if they fit), g_x(A) for every spin-orbital x (one thread
// per x) and E0 - E(A), where E(A) is half the sum over occupied x of
// h_x + g_x (every pair is counted from both ends), all double-double.
template <int WB>
__global__ __launch_bounds__(256) void k_anchor(DevSys s, Planes bits, int64_t nref, double e0, AnchorBlk *out)
{
    __shared__ uint64_t s_k[MAXW];
    __shared__ int16_t s_hr[MAXORB];
    __shared__ int s_nh;
    __shared__ double s_row[256 / 64], s_rowl[256 / 64];
    const int norb = s.norb, nso = 2 * norb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < MAXW)
        s_k[tid] = tid < WB && nref > 0 ? pl_get<WB>(bits, tid, 0) : 0ull;
    __syncthreads();
    if (tid == 0) {
        int nh = 0;
        for (int p = 0; p < norb; p++) {
            const int b = p + norb;
            const bool occ = ((s_k[p >> 6] >> (p & 63)) & 1ull) || ((s_k[b >> 6] >> (b & 63)) & 1ull);
            s_hr[p] = occ ? (int16_t)nh++ : (int16_t)-1;
        }
        if (nh * norb > ANC_HOT_MAX) {
            for (int p = 0; p < norb; p++)
                s_hr[p] = -1;
            nh = 0;
        }
        s_nh = nh;
    }
    __syncthreads();
    if (tid < MAXW)
        out->bits[tid] = s_k[tid];
    for (int p = tid; p < MAXORB; p += 256)
        out->hr[p] = p < norb ? s_hr[p] : (int16_t)-1;
    if (tid == 0)
        out->nh = s_nh;
    const int64_t n = norb;
    for (int x = tid; x < norb * norb; x += 256) {
        const int p = x / norb, q = x - p * norb, r = s_hr[p];
        if (r >= 0) {
            out->Jh[r * norb + q] = s.V[((p * n + p) * n + q) * n + q];
            out->Kh[r * norb + q] = s.V[((p * n + q) * n + q) * n + p];
        }
    }
    DD ex = {0.0, 0.0};
    if (tid < nso) {
        const int bx = tid;
        const bool occ = (s_k[bx >> 6] >> (bx & 63)) & 1ull;
        const double hx = s.T[tri_row(bx, nso) + bx];
        DD gx = {hx, 0.0};
#pragma unroll
        for (int w = 0; w < MAXW; w++) {
            uint64_t m = s_k[w];
            while (m) {
                const int c = w * 64 + __builtin_ctzll(m);
                m &= m - 1;
                if (c != bx)
                    dd_add_pair(gx, s.T, s.Tlo, nso, bx, c, 1.0);
            }
        }
        out->gh[bx] = gx.hi;
        out->gl[bx] = gx.lo;
        if (occ) {
            ex = gx;
            dd_add(ex, hx, 0.0);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const DD y = {__shfl_down(ex.hi, o), __shfl_down(ex.lo, o)};
        ex = dd_sum(ex, y);
    }
    if (lane == 0) {
        s_row[wave] = ex.hi;
        s_rowl[wave] = ex.lo;
    }
    __syncthreads();
    if (tid == 0) {
        DD e2 = {0.0, 0.0};
        for (int w = 0; w < 256 / 64; w++)
            dd_add(e2, s_row[w], s_rowl[w]);
        DD d = {e0, 0.0};
        dd_add(d, -0.5 * e2.hi, -0.5 * e2.lo);
        out->d0h = d.hi;
        out->d0l = d.lo;
    }
}

// ---------------------------------------------------------------------------
// Hash records (KeyCodec::hash): the records are sorted by the 64-bit Zobrist
// hash of their determinant, so equal determinants are adjacent, but
// neighbouring determinants are unrelated.  H_aa is therefore taken relative
// to each record's parent (the anchored form with the parent as anchor,
// which is the fast diagonal of the Appendix), and the bitstring is rebuilt
// from the parent and the four flipped spin-orbitals.

// Zobrist hash of every (bitstring-sorted) reference, with its index.
template <int WB>
__global__ void k_refs_hash(DevSys s, Planes bits, int64_t n, Planes out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = 0;
#pragma unroll
        for (int w = 0; w < WB; w++) {
            uint64_t m = pl_get<WB>(bits, w, i);
            while (m) {
                z ^= s.R[w * 64 + __builtin_ctzll(m)];
                m &= m - 1;
            }
        }
        out.key[0][i] = z & s.kc.hash_mask;
        ((uint64_t *)out.pay)[i] = (uint64_t)i;
    }
}

// Per reference p, double-double: D0[p] = E0 - H_pp (at 2p, 2p+1) and
// g[p][x] = h_x + sum_{c in p, c != x} T[x][c] for every spin-orbital x (at
// 2(p nso + x), +1), one workgroup per reference, one thread per x.  The
// energy is half the sum over occupied x of h_x + g_x (every pair is counted
// from both ends).
template <int WB>
__global__ __launch_bounds__(256) void k_parent_g(DevSys s, Planes bits, int64_t n, double e0, double *D0, double *G)
{
    __shared__ uint64_t s_k[WB];
    __shared__ double s_row[256 / 64], s_rowl[256 / 64];
    __shared__ double s_d0[2];
    const int nso = 2 * s.norb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t p = blockIdx.x; p < n; p += gridDim.x) {
        if (tid < WB)
            s_k[tid] = pl_get<WB>(bits, tid, p);
        __syncthreads();
        DD ex = {0.0, 0.0};
        DD gx = {0.0, 0.0};
        bool occ = false;
        if (tid < nso) {
            const int bx = tid;
            occ = (s_k[bx >> 6] >> (bx & 63)) & 1ull;
            const double hx = s.T[tri_row(bx, nso) + bx];
            gx = {hx, 0.0};
#pragma unroll
            for (int w = 0; w < WB; w++) {
                uint64_t m = s_k[w];
                while (m) {
                    const int c = w * 64 + __builtin_ctzll(m);
                    m &= m - 1;
                    if (c != bx)
                        dd_add_pair(gx, s.T, s.Tlo, nso, bx, c, 1.0);
                }
            }
            if (!occ) {
                G[2 * (p * nso + bx)] = gx.hi;
                G[2 * (p * nso + bx) + 1] = gx.lo;
            } else {
                ex = gx;
                dd_add(ex, hx, 0.0);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const DD y = {__shfl_down(ex.hi, o), __shfl_down(ex.lo, o)};
            ex = dd_sum(ex, y);
        }
        if (lane == 0) {
            s_row[wave] = ex.hi;
            s_rowl[wave] = ex.lo;
        }
        __syncthreads();
        if (tid == 0) {
            DD e2 = {0.0, 0.0};
            for (int w = 0; w < 256 / 64; w++)
                dd_add(e2, s_row[w], s_rowl[w]);
            DD d = {e0, 0.0};
            dd_add(d, -0.5 * e2.hi, -0.5 * e2.lo);
            D0[2 * p] = d.hi;
            D0[2 * p + 1] = d.lo;
            s_d0[0] = d.hi, s_d0[1] = d.lo;
        }
        __syncthreads();
        if (occ) {
            // occupied entries carry half of D0 (den_parent)
            dd_add(gx, 0.5 * s_d0[0], 0.5 * s_d0[1]);
            G[2 * (p * nso + tid)] = gx.hi;
            G[2 * (p * nso + tid) + 1] = gx.lo;
        }
        __syncthreads();
    }
}

// The references' bitstrings record by record (stride ref_stride<WB>() words,
// a power of two), so that rebuilding a record from its parent reads one
// cache line instead of one per key plane.
template <int WB>
__host__ __device__ constexpr int ref_stride()
{
    return WB == 3 ? 4 : WB;
}

template <int WB>
__global__ void k_refs_aos(Planes bits, int64_t n, uint64_t *ra)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int w = 0; w < ref_stride<WB>(); w++)
            ra[i * ref_stride<WB>() + w] = w < WB ? pl_get<WB>(bits, w, i) : 0ull;
}

// Where a single pass finds a parent's bitstring: the record-by-record table
// above, or, when every reference is within four excitations of the anchor A
// (the first sorted reference), the anchor's bitstring with up to eight
// flipped spin-orbitals per reference (one byte each, 0xFF unused): 8 B per
// reference instead of 32, a table that stays in the L2 cache while records
// stream past it.
struct RefTab {
    const uint64_t *full;  // ref_stride words per reference
    const uint64_t *ex;    // flips relative to the anchor (up to eight), or null
    const uint32_t *ex4;   // the same when every reference is within four flips (half the bytes), or null
    uint64_t a[MAXW];      // the anchor's bitstring
};

template <int WB>
__device__ inline void ref_bits(const RefTab &t, int64_t p, uint64_t (&k)[WB])
{
    if (t.ex4) {
        const uint32_t e = t.ex4[p];
#pragma unroll
        for (int w = 0; w < WB; w++)
            k[w] = t.a[w];
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const uint32_t b = (e >> (8 * f)) & 0xFFu;
            if (b != FLIP_NONE) {
#pragma unroll
                for (int w = 0; w < WB; w++)
                    k[w] ^= (w == (int)(b >> 6)) ? (1ull << (b & 63)) : 0ull;
            }
        }
        return;
    }
    if (t.ex) {
        const uint64_t e = t.ex[p];
#pragma unroll
        for (int w = 0; w < WB; w++)
            k[w] = t.a[w];
#pragma unroll
        for (int f = 0; f < 8; f++) {
            const uint32_t b = (uint32_t)(e >> (8 * f)) & 0xFFu;
            if (b != FLIP_NONE) {
#pragma unroll
                for (int w = 0; w < WB; w++)
                    k[w] ^= (w == (int)(b >> 6)) ? (1ull << (b & 63)) : 0ull;
            }
        }
        return;
    }
    const uint64_t *r = t.full + p * ref_stride<WB>();
    if constexpr (WB == 2 || WB == 4) {
        const ulonglong2 *r2 = (const ulonglong2 *)r;
#pragma unroll
        for (int w = 0; w < WB; w += 2) {
            const ulonglong2 v = r2[w / 2];
            k[w] = v.x, k[w + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int w = 0; w < WB; w++)
            k[w] = r[w];
    }
}

// The compact table: every reference's flips relative to the anchor (the
// first of the sorted bitstrings); *far gets 1 if some reference differs
// from the anchor in more than eight spin-orbitals; the anchor's words go to
// anc_bits.
template <int WB>
__global__ void k_refs_ex(Planes bits, int64_t n, uint64_t *ex, uint32_t *ex4, uint64_t *anc_bits, uint32_t *far)
{
    uint64_t a[WB];
#pragma unroll
    for (int w = 0; w < WB; w++)
        a[w] = pl_get<WB>(bits, w, 0);
    if (blockIdx.x == 0 && threadIdx.x < MAXW)
        anc_bits[threadIdx.x] = threadIdx.x < WB ? a[threadIdx.x] : 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t e = ~0ull;
        int nf = 0;
#pragma unroll
        for (int w = 0; w < WB; w++) {
            uint64_t d = pl_get<WB>(bits, w, i) ^ a[w];
            while (d) {
                const int b = w * 64 + __builtin_ctzll(d);
                d &= d - 1;
                if (nf < 8)
                    e = (e & ~(0xFFull << (8 * nf))) | ((uint64_t)b << (8 * nf));
                nf++;
            }
        }
        if (nf > 4)
            atomicMax(far, (uint32_t)nf);
        ex[i] = e;
        ex4[i] = (uint32_t)e;
    }
}

// Bitstring of a hash record: its parent's bitstring with the flips applied.
template <int WB>
__device__ inline void hash_key(const RefTab &ra, uint64_t aux, uint64_t (&k)[WB])
{
    const int64_t p = (int64_t)(aux >> 32);
    ref_bits<WB>(ra, p, k);
#pragma unroll
    for (int f = 0; f < 4; f++) {
        const uint32_t b = (uint32_t)(aux >> (8 * f)) & 0xFFu;
        if (b != FLIP_NONE) {
#pragma unroll
            for (int w = 0; w < WB; w++)
                k[w] ^= (w == (int)(b >> 6)) ? (1ull << (b & 63)) : 0ull;
        }
    }
}

// E0 - H_aa relative to the parent p (at most two spin-orbitals removed and
// two added), double-double:
//   D0[p] + sum_R g_r - sum_A g_a - sum_{r<r'} T - sum_{a<a'} T + sum_{a,r} T.
template <int WB>
__device__ inline double den_parent(const double *Tp, const double *Tl, int nso, const uint64_t (&k)[WB],
                                    const RefTab &ra, int64_t p, const double *G, const double *D0)
{
    int rm[2], ad[2], nr = 0, na = 0;
    uint64_t pk[WB];
    ref_bits<WB>(ra, p, pk);
#pragma unroll
    for (int w = 0; w < WB; w++) {
        const uint64_t pw = pk[w];
        uint64_t d = k[w] ^ pw;
        while (d) {
            const int b = w * 64 + __builtin_ctzll(d);
            d &= d - 1;
            if ((pw >> (b & 63)) & 1ull) {
                if (nr < 2)
                    rm[nr] = b;
                nr++;
            } else {
                if (na < 2)
                    ad[na] = b;
                na++;
            }
        }
    }
    // G holds g_x + D0/2 for the parent's occupied x (k_parent_g), so a
    // double's two removed orbitals bring D0 = E0 - E(parent) with them; a
    // single reads the other half
    const double2 *g = (const double2 *)G + p * nso;
    DD d = {0.0, 0.0};
    if (nr < 2) {
        const double2 d0 = ((const double2 *)D0)[p];
        d.hi = nr == 1 ? 0.5 * d0.x : d0.x, d.lo = nr == 1 ? 0.5 * d0.y : d0.y;
    }
    for (int i = 0; i < nr && i < 2; i++) {
        const double2 v = g[rm[i]];
        dd_add(d, v.x, v.y);
    }
    for (int i = 0; i < na && i < 2; i++) {
        const double2 v = g[ad[i]];
        dd_add(d, -v.x, -v.y);
    }
    if (nr == 2)
        dd_add_pair(d, Tp, Tl, nso, rm[0], rm[1], -1.0);
    if (na == 2)
        dd_add_pair(d, Tp, Tl, nso, ad[0], ad[1], -1.0);
    for (int i = 0; i < nr && i < 2; i++)
        for (int j = 0; j < na && j < 2; j++)
            dd_add_pair(d, Tp, Tl, nso, ad[j], rm[i], 1.0);
    return d.hi + d.lo;
}

constexpr int HR_REFS = 256;  // reference hashes staged per workgroup

__device__ inline int64_t eri_at(int n, int p, int q, int r, int t)
{
    return (((int64_t)p * n + q) * n + r) * n + t;
}

template <int WB>
__device__ inline bool bit_set(const uint64_t (&k)[WB], int b)
{
    uint64_t w = k[0];
#pragma unroll
    for (int i = 1; i < WB; i++)
        w = (b >> 6) == i ? k[i] : w;
    return (w >> (b & 63)) & 1ull;
}

// (-1)^(occupied orbitals of spin sp strictly between orbitals x and y)
template <int WB>
__device__ inline int spin_phase(const uint64_t (&k)[WB], int norb, int sp, int x, int y)
{
    const int off = sp == 0 ? norb : 0, lo = (x < y ? x : y) + off + 1, hi = (x < y ? y : x) + off;
    int cnt = 0;
#pragma unroll
    for (int w = 0; w < WB; w++) {
        const int s0 = w * 64;
        uint64_t m = ~0ull;
        if (lo > s0)
            m = lo - s0 >= 64 ? 0ull : m & (~0ull << (lo - s0));
        if (hi < s0 + 64)
            m = hi <= s0 ? 0ull : m & ((1ull << (hi - s0)) - 1ull);
        cnt += __popcll(k[w] & m);
    }
    return (cnt & 1) ? -1 : 1;
}

// H_ai c_i of one hash record in FP64, from its parent's bitstring and the
// flipped spin-orbitals, by the Slater-Condon rules with the operations in
// the order FP64 generation uses (so the value is that record's FP64
// payload bit for bit):
//   single r->a:        ph * [h_ra + sum_{j occ} (ra|jj) - sum_{j occ, same spin} (rj|ja)]
//   same-spin r<q->a<b: ph(r->a) ph(q->b after r->a) [(ra|qb) - (rb|qa)]
//   alpha r->a, beta q->b: ph_alpha ph_beta (ra|qb)
template <int WB>
__device__ inline double rec_value64(const DevSys &s, const RefTab &ra, const double *coef, uint64_t aux)
{
    const int64_t p = (int64_t)(aux >> 32);
    uint64_t pk[WB];
    ref_bits<WB>(ra, p, pk);
    const int n = s.norb;
    const int f0 = (int)(aux & 0xFFu), f1 = (int)((aux >> 8) & 0xFFu);
    const int f2 = (int)((aux >> 16) & 0xFFu), f3 = (int)((aux >> 24) & 0xFFu);
    double v;
    if (f2 == (int)FLIP_NONE) {
        const int sp = f0 >= n ? 0 : 1, off = sp == 0 ? n : 0;
        const int r = f0 - off, a = f1 - off;
        double f = s.h[r * n + a];
        const double *Vra = s.V + eri_at(n, r, a, 0, 0);
        for (int t = 0; t < 2; t++) {
            const int o2 = t == 0 ? n : 0;
            for (int j = 0; j < n; j++) {
                if (!bit_set<WB>(pk, o2 + j))
                    continue;
                f += Vra[j * n + j];
                if (t == sp)
                    f -= s.V[eri_at(n, r, j, j, a)];
            }
        }
        v = (double)spin_phase<WB>(pk, n, sp, r, a) * f;
    } else if (bit_set<WB>(pk, f1)) {
        const int sp = f0 >= n ? 0 : 1, off = sp == 0 ? n : 0;
        const int r = f0 - off, q = f1 - off, a = f2 - off, b = f3 - off;
        const int ph1 = spin_phase<WB>(pk, n, sp, r, a);
        int ph2 = spin_phase<WB>(pk, n, sp, q, b);
        const int lo = q < b ? q : b, hi = q < b ? b : q;
        if (r > lo && r < hi)
            ph2 = -ph2;
        if (a > lo && a < hi)
            ph2 = -ph2;
        const double d = s.V[eri_at(n, r, a, q, b)] - s.V[eri_at(n, r, b, q, a)];
        v = (double)(ph1 * ph2) * d;
    } else {
        const int r = f0 - n, a = f1 - n, q = f2, b = f3;
        const int ph = spin_phase<WB>(pk, n, 0, r, a) * spin_phase<WB>(pk, n, 1, q, b);
        v = (double)ph * s.V[eri_at(n, r, a, q, b)];
    }
    return v * coef[p];
}

// FP32 payloads: a term whose numerator's storage rounding could move it by
// more than REFINE_TOL gets its numerator again as the FP64 sum of its
// records' FP64 payloads.  The rounding moves N by at most eps * sum |p_i|,
// so the term by about 2 |N/d| eps sum |p_i|; the sum of |p_i| is read only
// when |N/d| exceeds REFINE_RATIO.  The single pass lists such segments with
// the collided ones; the second kernel sums their records' FP64 values.
constexpr double REFINE_RATIO = 1e-3;
constexpr double REFINE_TOL = 1e-11;

__device__ inline bool refine_needed(const DevSys &s, const Planes &in, uint64_t h, int64_t tail, double num,
                                     double den, double eps)
{
    int64_t head = tail;
    double absum = fabs((double)pay32_at(s.kc, in, tail));
    while (head > 0 && hash_at(s.kc, in, head - 1) == h) {
        head--;
        absum += fabs((double)pay32_at(s.kc, in, head));
    }
    return 2.0 * fabs(num / den) * absum * eps > REFINE_TOL;
}

// One distinct determinant of a hash segment: exclusion, then the term.
// tail: index of the segment's last record, for the FP32 refinement check (a
// segment that needs it sets *defer and adds nothing: the second kernel takes
// it); tail < 0: the numerator is already FP64.
template <int WB, int PB>
__device__ inline void hash_key_term(const DevSys &s, const Planes &in, const Planes &bits, const RefTab &ra,
                                     const Planes &rh, int64_t lo, int64_t hi, const uint64_t *s_rh, const int64_t *s_ri,
                                     bool staged, uint64_t h, const uint64_t (&k)[WB], int64_t parent, int64_t tail,
                                     double num, const double *D0, const double *G, Acc &a, bool search, double eps,
                                     int *defer = nullptr)
{
    a.n_unique++;
    if (!search)
        lo = hi = 0;  // subtraction form: references stay in
    // references with hash h: a few at most
    int64_t j0 = lo, j1 = hi;
    {
        int64_t l = lo, r = hi;  // first index with hash >= h
        while (l < r) {
            const int64_t m = l + (r - l) / 2;
            const uint64_t hm = staged ? s_rh[m - lo] : rh.key[0][m];
            if (hm < h)
                l = m + 1;
            else
                r = m;
        }
        j0 = l;
        j1 = hi;
    }
    for (int64_t j = j0; j < j1; j++) {
        const uint64_t hj = staged ? s_rh[j - lo] : rh.key[0][j];
        if (hj != h)
            break;
        const int64_t idx = staged ? s_ri[j - lo] : (int64_t)((const uint64_t *)rh.pay)[j];
        uint64_t rk[WB];
        ref_bits<WB>(ra, idx, rk);
        bool eq = true;
#pragma unroll
        for (int w = 0; w < WB; w++)
            eq = eq && rk[w] == k[w];
        if (eq) {
            a.n_hit++;
            a.ref_cross += (s.z2 ? swap_weight<WB>(k, s.norb) : 1.0) * (((const double *)bits.pay)[idx] * num);
            return;
        }
    }
    const double den = den_parent<WB>(s.T, s.Tlo, 2 * s.norb, k, ra, parent, G, D0);
    if constexpr (PB == 4) {
        if (tail >= 0 && den != 0.0 && fabs(num / den) > REFINE_RATIO && refine_needed(s, in, h, tail, num, den, eps)) {
            a.n_unique--;  // counted again by the second kernel
            *defer = 1;
            return;
        }
    }
    a.n_ext++;
    const double ad = fabs(den);
    a.min_abs = ad < a.min_abs ? ad : a.min_abs;
    if (den >= 0.0)
        a.n_nonneg++;
    if (den == 0.0)
        a.singular = 1;
    else
        neumaier(a.e_sum, a.e_comp, (s.z2 ? swap_weight<WB>(k, s.norb) : 1.0) * (num * num / den));
    const uint64_t m = key_mix<WB>(k);
    a.kx ^= m;
    a.ks += m;
}

// Tree sum of the workgroup's per-thread partials (s_p holds RED_THREADS).
__device__ inline void block_partial(Partial *s_p)
{
    const int tid = threadIdx.x;
    __syncthreads();
    for (int o = RED_THREADS / 2; o >= 1; o >>= 1) {
        if (tid < o) {
            Partial x = s_p[tid];
            partial_merge(x, s_p[tid + o]);
            s_p[tid] = x;
        }
        __syncthreads();
    }
}

// Single pass over hash records.  A fixed grid of workgroups takes
// contiguous ranges of RED_TILE-record tiles; a tile owns the segments (runs
// of equal hash) whose first record lies in it.  Every thread loads its
// RED_ITEMS records and rebuilds their bitstrings at once (the parent reads
// are independent), marks segment heads and tails and the records whose
// bitstring differs from the previous record of their segment, and a
// segmented scan over the tile carries each segment's sum, its first record's
// parent word and whether it holds more than one determinant.  The owned
// segment ends are queued in LDS and processed by all threads.  A segment
// that runs past the tile end is followed by wave 0.  Segments holding more
// than one determinant (a hash collision) are left to k_reduce_hash_coll and
// the workgroup marks itself in coll[].
struct HashScan {
    int f;       // a segment head was seen
    double v;    // sum since the last head
    uint64_t a;  // parent word of the last head
    int c;       // the segment since the last head holds two determinants
};

__device__ inline HashScan hscan_op(const HashScan &x, const HashScan &y)
{
    HashScan r;
    r.f = x.f | y.f;
    r.v = y.f ? y.v : x.v + y.v;
    r.a = y.f ? y.a : x.a;
    r.c = y.f ? y.c : (x.c | y.c);
    return r;
}

template <int WB>
__device__ inline bool bits_eq(const uint64_t (&x)[WB], const uint64_t (&y)[WB])
{
    bool e = true;
#pragma unroll
    for (int w = 0; w < WB; w++)
        e = e && x[w] == y[w];
    return e;
}

template <int WB, int PB>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_hash(DevSys s, Planes in, int64_t n, Planes bits,
                                                             RefTab ra, Planes rh,
                                                             int64_t nref, const double *D0, const double *G,
                                                             int64_t tiles_per_block, int search, double eps,
                                                             Partial *partials, CollList *coll, int64_t *ctail,
                                                             Flags *flags)
{
    // queue of owned segment ends (hash, parent word, sum, collided, index of
    // the last record relative to the tile); the block's partials reuse it at
    // the end
    constexpr size_t QB = (size_t)RED_Q * (8 + 8 + 8 + 4 + 4);
    constexpr size_t LB = QB > sizeof(Partial) * RED_THREADS ? QB : sizeof(Partial) * RED_THREADS;
    __shared__ __align__(16) char s_q[LB];
    uint64_t *q_h = (uint64_t *)s_q;
    uint64_t *q_a = q_h + RED_Q;
    double *q_v = (double *)(q_a + RED_Q);
    int *q_c = (int *)(q_v + RED_Q);
    uint32_t *q_t = (uint32_t *)(q_c + RED_Q);
    __shared__ uint64_t s_rh[HR_REFS];
    __shared__ int64_t s_ri[HR_REFS];
    __shared__ int64_t s_lo, s_hi;
    __shared__ HashScan s_w[RED_THREADS / 64];
    __shared__ uint32_t s_cnt[RED_THREADS / 64];
    __shared__ HashScan s_cont;
    __shared__ uint64_t s_ch;
    __shared__ int s_cflag;
    __shared__ int s_tcoll;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ntiles = (n + RED_TILE - 1) / RED_TILE;
    const int64_t t_begin = (int64_t)blockIdx.x * tiles_per_block;
    const int64_t t_end = t_begin + tiles_per_block < ntiles ? t_begin + tiles_per_block : ntiles;
    Acc a;
    acc_init(a);
    // the workgroup's collided segments, listed by wave 0 in record order
    int64_t *my_tail = ctail + t_begin * RED_TILE;
    uint32_t ncoll = 0;
    // references whose hash lies in the workgroup's hash range, staged in LDS
    // when few
    int64_t lo = 0, hi = 0;
    bool staged = false;
    if (t_begin < t_end) {
        if (tid == 0) {
            const int64_t b0 = t_begin * RED_TILE, b1 = t_end * RED_TILE < n ? t_end * RED_TILE : n;
            const uint64_t h0 = rec_hash<PB>(s.kc, in, b0), h1 = rec_hash<PB>(s.kc, in, b1 - 1);
            int64_t l = 0, r = nref;
            while (l < r) {
                const int64_t m = l + (r - l) / 2;
                if (rh.key[0][m] < h0)
                    l = m + 1;
                else
                    r = m;
            }
            s_lo = l;
            r = nref;
            while (l < r) {
                const int64_t m = l + (r - l) / 2;
                if (rh.key[0][m] <= h1)
                    l = m + 1;
                else
                    r = m;
            }
            s_hi = l;
        }
        __syncthreads();
        lo = s_lo, hi = s_hi;
        staged = hi - lo <= HR_REFS;
        if (staged)
            for (int64_t j = tid; j < hi - lo; j += RED_THREADS) {
                s_rh[j] = rh.key[0][lo + j];
                s_ri[j] = (int64_t)((const uint64_t *)rh.pay)[lo + j];
            }
    }
    for (int64_t tile = t_begin; tile < t_end; tile++) {
        const int64_t base = tile * RED_TILE;
        const int64_t tend = base + RED_TILE < n ? base + RED_TILE : n;
        if (tid == 0)
            s_cflag = 0, s_tcoll = 0;
        const int64_t r0 = base + (int64_t)tid * RED_ITEMS;
        uint64_t h[RED_ITEMS], ax[RED_ITEMS], kb[RED_ITEMS][WB];
        double p[RED_ITEMS];
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool valid = idx < tend;
            h[j] = valid ? rec_hash<PB>(s.kc, in, idx) : 0ull;
            ax[j] = valid ? rec_aux<PB>(s.kc, s.norb, in, idx) : 0ull;
            p[j] = valid ? hpay_at<PB>(s.kc, in, idx) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            if (r0 + j < tend)
                hash_key<WB>(ra, ax[j], kb[j]);
            else
#pragma unroll
                for (int w = 0; w < WB; w++)
                    kb[j][w] = 0;
        }
        // the previous record (the last of the previous lane, or loaded) and
        // the next record's hash
        uint64_t hprev = 0, kprev[WB];
#pragma unroll
        for (int w = 0; w < WB; w++)
            kprev[w] = __shfl_up(kb[RED_ITEMS - 1][w], 1);
        hprev = __shfl_up(h[RED_ITEMS - 1], 1);
        const bool has_prev = r0 > 0 && r0 < tend;
        if (lane == 0 && has_prev) {
            hprev = rec_hash<PB>(s.kc, in, r0 - 1);
            if (r0 > base)
                hash_key<WB>(ra, rec_aux<PB>(s.kc, s.norb, in, r0 - 1), kprev);
        }
        const uint64_t hnext = r0 + RED_ITEMS < n ? rec_hash<PB>(s.kc, in, r0 + RED_ITEMS) : 0ull;
        const bool has_next = r0 + RED_ITEMS < n;

        double run[RED_ITEMS];
        uint64_t rha[RED_ITEMS];
        int rc[RED_ITEMS];
        bool hh[RED_ITEMS], tl[RED_ITEMS];
        HashScan me;
        me.f = 0, me.v = 0.0, me.a = 0, me.c = 0;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool valid = idx < tend;
            bool head, differs;
            if (j == 0) {
                head = idx == 0 || !has_prev || h[0] != hprev;
                differs = !head && r0 > base && !bits_eq<WB>(kb[0], kprev);
            } else {
                head = h[j] != h[j - 1];
                differs = !head && !bits_eq<WB>(kb[j], kb[j - 1]);
            }
            head = head && valid;
            bool tail;
            if (j == RED_ITEMS - 1)
                tail = !has_next || h[j] != hnext;
            else
                tail = idx + 1 >= n || h[j] != h[j + 1];
            tl[j] = tail && valid;
            if (valid) {
                if (head) {
                    me.f = 1, me.v = p[j], me.a = ax[j], me.c = 0;
                } else {
                    me.v += p[j];
                    me.c |= differs ? 1 : 0;
                }
            }
            run[j] = me.v, rha[j] = me.a, rc[j] = me.c;
            hh[j] = me.f != 0;
        }
        // inclusive scan within the wavefront, then the earlier wavefronts
        HashScan x = me;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            HashScan y;
            y.f = __shfl_up(x.f, o);
            y.v = __shfl_up(x.v, o);
            y.a = __shfl_up(x.a, o);
            y.c = __shfl_up(x.c, o);
            if (lane >= o)
                x = hscan_op(y, x);
        }
        if (lane == 63)
            s_w[wave] = x;
        HashScan ex;  // exclusive within the wavefront
        ex.f = __shfl_up(x.f, 1);
        ex.v = __shfl_up(x.v, 1);
        ex.a = __shfl_up(x.a, 1);
        ex.c = __shfl_up(x.c, 1);
        if (lane == 0)
            ex.f = 0, ex.v = 0.0, ex.a = 0, ex.c = 0;
        __syncthreads();
        HashScan cw;
        cw.f = 0, cw.v = 0.0, cw.a = 0, cw.c = 0;
        for (int w = 0; w < wave; w++)
            cw = hscan_op(cw, s_w[w]);
        const HashScan carry = hscan_op(cw, ex);

        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool owned = idx < tend && (hh[j] || carry.f);
            if (owned && tl[j])
                mine++;
            if (owned && !tl[j] && idx == tend - 1) {
                // the segment continues past the tile end
                s_ch = h[j];
                s_cont.f = 1;
                s_cont.v = hh[j] ? run[j] : carry.v + run[j];
                s_cont.a = hh[j] ? rha[j] : carry.a;
                s_cont.c = hh[j] ? rc[j] : (carry.c | rc[j]);
                s_cflag = 1;
            }
        }
        uint32_t xs = mine;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(xs, o);
            if (lane >= o)
                xs += y;
        }
        if (lane == 63)
            s_cnt[wave] = xs;
        __syncthreads();
        uint32_t pre = 0, qtot = 0;
#pragma unroll
        for (int w = 0; w < RED_THREADS / 64; w++) {
            const uint32_t t = s_cnt[w];
            pre += w < wave ? t : 0u;
            qtot += t;
        }
        uint32_t slot = pre + xs - mine;
#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            const bool owned = idx < tend && (hh[j] || carry.f);
            if (owned && tl[j]) {
                q_h[slot] = h[j];
                q_v[slot] = hh[j] ? run[j] : carry.v + run[j];
                q_a[slot] = hh[j] ? rha[j] : carry.a;
                q_c[slot] = hh[j] ? rc[j] : (carry.c | rc[j]);
                q_t[slot] = (uint32_t)(idx - base);
                if (q_c[slot])
                    s_tcoll = 1;
                slot++;
            }
        }
        const int cflag = s_cflag;
        if (cflag && tid < 64) {
            // wave 0 follows the continuing segment into the following records
            const uint64_t ch = s_ch;
            uint64_t k0[WB];
            hash_key<WB>(ra, s_cont.a, k0);
            double total = 0.0;
            int col = 0;
            int64_t pos = tend;
            while (true) {
                const int64_t idx = pos + lane;
                bool eq = false;
                double v = 0.0;
                if (idx < n && rec_hash<PB>(s.kc, in, idx) == ch) {
                    eq = true;
                    v = hpay_at<PB>(s.kc, in, idx);
                    uint64_t kk[WB];
                    hash_key<WB>(ra, rec_aux<PB>(s.kc, s.norb, in, idx), kk);
                    col |= bits_eq<WB>(kk, k0) ? 0 : 1;
                }
                const uint64_t m = __ballot(eq);
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    v += __shfl_down(v, o);
                    col |= __shfl_down(col, o);
                }
                total += v;  // lane 0 holds the sum of this step
                if (m != ~0ull) {
                    pos += __builtin_ctzll(~m);  // equal records are a prefix of the lanes
                    break;
                }
                pos += 64;
            }
            if (lane == 0) {
                q_h[qtot] = ch;
                q_v[qtot] = s_cont.v + total;
                q_a[qtot] = s_cont.a;
                // the tile part compared neighbours, the continuation compares
                // with the segment's first record
                q_c[qtot] = s_cont.c | col;
                q_t[qtot] = (uint32_t)(pos - 1 - base);
                if (q_c[qtot])
                    s_tcoll = 1;
            }
        }
        __syncthreads();
        const int qn = (int)qtot + cflag;
        for (int e = tid; e < qn; e += RED_THREADS) {
            if (q_c[e])
                continue;
            uint64_t k0[WB];
            const uint64_t aux = q_a[e];
            hash_key<WB>(ra, aux, k0);
            hash_key_term<WB, PB>(s, in, bits, ra, rh, lo, hi, s_rh, s_ri, staged, q_h[e], k0, (int64_t)(aux >> 32),
                                  base + (int64_t)q_t[e], q_v[e], D0, G, a, search != 0, eps, &q_c[e]);
            if (PB == 4 && q_c[e])
                s_tcoll = 1;
        }
        __syncthreads();
        if (s_tcoll && wave == 0) {
            // collided segments (and, with FP32 payloads, those to refine) are
            // left to k_reduce_hash_coll: wave 0 lists them in queue (record)
            // order
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            for (int e0 = 0; e0 < qn; e0 += 64) {
                const int e = e0 + lane;
                const bool c = e < qn && q_c[e] != 0;
                const uint64_t m = __ballot(c);
                if (c)
                    my_tail[ncoll + (uint32_t)__popcll(m & lt)] = base + (int64_t)q_t[e];
                ncoll += (uint32_t)__popcll(m);
            }
        }
        __syncthreads();
    }
    Partial *s_p = (Partial *)s_q;
    s_p[tid] = acc_partial(a);
    if (a.singular)
        atomicOr(&flags->err, ERR_SINGULAR);
    block_partial(s_p);
    if (tid == 0) {
        partials[blockIdx.x] = s_p[0];
        CollList cl;
        cl.n = ncoll;  // wave 0's count (lane 0 holds it)
        cl.pad = 0;
        // (from LDS: holding lo and hi in registers to here costs occupancy)
        cl.lo = t_begin < t_end ? s_lo : 0;
        cl.hi = t_begin < t_end ? s_hi : 0;
        coll[blockIdx.x] = cl;
    }
}

// Records [i, e) are one collided segment (one hash, several determinants):
// each distinct determinant, taken at its first record, gets the sum of its
// records' payloads (with FP32 payloads, of their FP64 values) and its term.
// One thread; references searched over [lo, hi).
template <int WB, int PB>
__device__ inline void coll_segment(const DevSys &s, const Planes &in, const Planes &bits, const RefTab &ra,
                                    const Planes &rh, int64_t lo, int64_t hi, const double *D0, const double *G,
                                    int64_t i, int64_t e, Acc &a, bool search)
{
    const uint64_t h = rec_hash<PB>(s.kc, in, i);
    for (int64_t x = i; x < e; x++) {
        uint64_t kx[WB];
        const uint64_t ax = rec_aux<PB>(s.kc, s.norb, in, x);
        hash_key<WB>(ra, ax, kx);
        bool seen = false;
        for (int64_t y = i; y < x && !seen; y++) {
            uint64_t ky[WB];
            hash_key<WB>(ra, rec_aux<PB>(s.kc, s.norb, in, y), ky);
            seen = bits_eq<WB>(ky, kx);
        }
        if (seen)
            continue;
        double nx = 0.0;
        for (int64_t y = x; y < e; y++) {
            uint64_t ky[WB];
            const uint64_t ay = rec_aux<PB>(s.kc, s.norb, in, y);
            hash_key<WB>(ra, ay, ky);
            if (bits_eq<WB>(ky, kx))
                nx += PB == 4 ? rec_value64<WB>(s, ra, (const double *)bits.pay, ay) : hpay_at<PB>(s.kc, in, y);
        }
        hash_key_term<WB, PB>(s, in, bits, ra, rh, lo, hi, nullptr, nullptr, false, h, kx, (int64_t)(ax >> 32), -1,
                              nx, D0, G, a, search, 0.0);
    }
}

// Distinct determinants one wavefront tracks in a collided segment.
constexpr int COLL_DETS = 8;

// One collided segment [i, e) split by one wavefront, 64 records at a time
// (record c + lane): each lane rebuilds its record's bitstring and matches it
// against the determinants met so far (kept in LDS, in order of first
// appearance; a record matching none opens the next); each lane keeps one sum
// per determinant over its records.  At the end the sums are reduced over the
// wavefront and lane 0 adds each determinant's term.  A segment with more
// than COLL_DETS determinants (only with hashes truncated far below 64 bits)
// is split by lane 0 alone.
template <int WB, int PB>
__device__ inline void coll_segment_wave(const DevSys &s, const Planes &in, const Planes &bits, const RefTab &ra,
                                         const Planes &rh, int64_t lo, int64_t hi, const double *D0,
                                         const double *G, int64_t i, int64_t e, uint64_t *s_dk, uint64_t *s_dax,
                                         Acc &a, bool search)
{
    const int lane = threadIdx.x & 63;
    double dv[COLL_DETS];
#pragma unroll
    for (int d = 0; d < COLL_DETS; d++)
        dv[d] = 0.0;
    int nd = 0;
    bool over = false;
    for (int64_t c0 = i; c0 < e && !over; c0 += 64) {
        const int64_t x = c0 + lane;
        const bool valid = x < e;
        uint64_t k[WB], ax = 0ull;
        double v = 0.0;
        if (valid) {
            ax = rec_aux<PB>(s.kc, s.norb, in, x);
            hash_key<WB>(ra, ax, k);
            v = PB == 4 ? rec_value64<WB>(s, ra, (const double *)bits.pay, ax) : hpay_at<PB>(s.kc, in, x);
        } else {
#pragma unroll
            for (int w = 0; w < WB; w++)
                k[w] = 0ull;
        }
        int my = -1;
        for (int d = 0; d < nd; d++) {
            bool eq = true;
#pragma unroll
            for (int w = 0; w < WB; w++)
                eq = eq && s_dk[d * WB + w] == k[w];
            my = (my < 0 && eq) ? d : my;
        }
        uint64_t un = __ballot(valid && my < 0);
        while (un) {
            if (nd == COLL_DETS) {
                over = true;
                break;
            }
            const int l = __builtin_ctzll(un);
            uint64_t kx[WB];
#pragma unroll
            for (int w = 0; w < WB; w++)
                kx[w] = __shfl(k[w], l);
            const uint64_t axl = __shfl(ax, l);
            if (lane == 0) {
#pragma unroll
                for (int w = 0; w < WB; w++)
                    s_dk[nd * WB + w] = kx[w];
                s_dax[nd] = axl;
            }
            if (valid && my < 0 && bits_eq<WB>(k, kx))
                my = nd;
            nd++;
            un = __ballot(valid && my < 0);
        }
        // lane 0's LDS writes stay ahead of the other lanes' later reads
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int d = 0; d < COLL_DETS; d++)
            dv[d] += my == d ? v : 0.0;
    }
    if (over) {
        if (lane == 0)
            coll_segment<WB, PB>(s, in, bits, ra, rh, lo, hi, D0, G, i, e, a, search);
        return;
    }
    const uint64_t h = rec_hash<PB>(s.kc, in, i);
#pragma unroll
    for (int d = 0; d < COLL_DETS; d++) {
        if (d >= nd)
            break;
        double nx = dv[d];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            nx += __shfl_down(nx, o);
        if (lane == 0) {
            uint64_t kx[WB];
#pragma unroll
            for (int w = 0; w < WB; w++)
                kx[w] = s_dk[d * WB + w];
            hash_key_term<WB, PB>(s, in, bits, ra, rh, lo, hi, nullptr, nullptr, false, h, kx,
                                  (int64_t)(s_dax[d] >> 32), -1, nx, D0, G, a, search, 0.0);
        }
    }
}

// The collided segments k_reduce_hash listed, per workgroup, in record
// order: entry e on wavefront e mod 4 (so the sums are reproducible), each
// walked back to its first record and split by determinant.  The
// workgroup's partial is merged into the one k_reduce_hash wrote.
// Workgroups with none return at once.
template <int WB, int PB>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_hash_coll(DevSys s, Planes in, int64_t n, Planes bits,
                                                                  RefTab ra, Planes rh, const double *D0,
                                                                  const double *G, int64_t tiles_per_block,
                                                                  int search, Partial *partials,
                                                                  const CollList *coll, const int64_t *ctail,
                                                                  Flags *flags)
{
    __shared__ Partial s_p[RED_THREADS];
    __shared__ uint64_t s_dk[RED_THREADS / 64][COLL_DETS * WB];
    __shared__ uint64_t s_dax[RED_THREADS / 64][COLL_DETS];
    const CollList cl = coll[blockIdx.x];
    if (cl.n == 0)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t *my_tail = ctail + (int64_t)blockIdx.x * tiles_per_block * RED_TILE;
    Acc a;
    acc_init(a);
    for (uint32_t e = wave; e < cl.n; e += RED_THREADS / 64) {
        const int64_t t = my_tail[e];
        const uint64_t h = rec_hash<PB>(s.kc, in, t);
        // the segment's first record: 64 records back at a time
        int64_t b = t;
        while (true) {
            const int64_t y = b - 1 - lane;
            const bool same = y >= 0 && rec_hash<PB>(s.kc, in, y) == h;
            const uint64_t m = __ballot(same);  // a prefix of the lanes
            if (m != ~0ull) {
                b -= __builtin_ctzll(~m);
                break;
            }
            b -= 64;
        }
        coll_segment_wave<WB, PB>(s, in, bits, ra, rh, cl.lo, cl.hi, D0, G, b, t + 1, s_dk[wave], s_dax[wave], a,
                                  search != 0);
    }
    s_p[tid] = acc_partial(a);
    if (a.singular)
        atomicOr(&flags->err, ERR_SINGULAR);
    block_partial(s_p);
    if (tid == 0) {
        Partial x = partials[blockIdx.x];
        partial_merge(x, s_p[0]);
        partials[blockIdx.x] = x;
    }
}

__global__ __launch_bounds__(256) void k_final(const Partial *partials, int np, Partial *out)
{
    __shared__ Partial s_p[256];
    const int tid = threadIdx.x;
    Partial x;
    x.e_sum = x.e_comp = x.ref_cross = 0.0;
    x.min_abs_denom = __builtin_inf();
    x.n_unique = x.n_external = x.n_hit = x.n_nonneg = x.key_xor = x.key_sum = 0;
    for (int i = tid; i < np; i += 256) {
        const Partial y = partials[i];
        double sum = x.e_sum, comp = x.e_comp + y.e_comp;
        neumaier(sum, comp, y.e_sum);
        x.e_sum = sum, x.e_comp = comp;
        x.ref_cross += y.ref_cross;
        x.min_abs_denom = y.min_abs_denom < x.min_abs_denom ? y.min_abs_denom : x.min_abs_denom;
        x.n_unique += y.n_unique, x.n_external += y.n_external, x.n_hit += y.n_hit;
        x.n_nonneg += y.n_nonneg, x.key_xor ^= y.key_xor, x.key_sum += y.key_sum;
    }
    s_p[tid] = x;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) {
            Partial a = s_p[tid], y = s_p[tid + o];
            double sum = a.e_sum, comp = a.e_comp + y.e_comp;
            neumaier(sum, comp, y.e_sum);
            a.e_sum = sum, a.e_comp = comp;
            a.ref_cross += y.ref_cross;
            a.min_abs_denom = y.min_abs_denom < a.min_abs_denom ? y.min_abs_denom : a.min_abs_denom;
            a.n_unique += y.n_unique, a.n_external += y.n_external, a.n_hit += y.n_hit;
            a.n_nonneg += y.n_nonneg, a.key_xor ^= y.key_xor, a.key_sum += y.key_sum;
            s_p[tid] = a;
        }
        __syncthreads();
    }
    if (tid == 0)
        *out = s_p[0];
}

// Inspection: one thread per segment head walks its segment (small inputs only).
template <int W, int PB>
__global__ void k_numerators(Planes in, int64_t n, Planes refs, int64_t nref, uint64_t *keys_aos, double *num,
                             uint8_t *in_ref, unsigned long long *n_out, int64_t cap)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k[W];
        load_key<W>(in, i, k);
        if (i > 0) {
            uint64_t kp[W];
            load_key<W>(in, i - 1, kp);
            if (key_eq<W>(k, kp))
                continue;
        }
        double v = 0.0;
        int64_t j = i;
        while (j < n) {
            uint64_t kk[W];
            load_key<W>(in, j, kk);
            if (!key_eq<W>(kk, k))
                break;
            v += load_pay<PB>(in, j);
            j++;
        }
        const int64_t r = ref_bound<W>(refs, 0, nref, k, false);
        bool hit = false;
        if (r < nref) {
            uint64_t rk[W];
            load_key<W>(refs, r, rk);
            hit = key_eq<W>(rk, k);
        }
        const unsigned long long slot = atomicAdd(n_out, 1ull);
        if ((int64_t)slot < cap) {
#pragma unroll
            for (int w = 0; w < W; w++)
                keys_aos[slot * W + w] = k[w];
            num[slot] = v;
            in_ref[slot] = hit ? 1 : 0;
        }
    }
}

}  // namespace

// Workgroups of a single pass that take tiles: the largest whole number of
// rounds of the workgroups that fit on the device at once, at most RED_GRID
// (the rest of the fixed grid writes empty partials).  Equal work per
// workgroup then leaves no partly filled last round.
static int64_t red_workers(const void *kernel, size_t dyn)
{
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, RED_THREADS, dyn) != hipSuccess || nb <= 0 ||
        cus <= 0) {
        (void)hipGetLastError();
        return RED_GRID;
    }
    const int64_t resident = (int64_t)nb * cus;
    return resident >= RED_GRID ? RED_GRID : (RED_GRID / resident) * resident;
}

hipError_t launch_reduce(const DevSys &s, int fp32, int kw, const Planes &sorted, int64_t n, const Planes &refs,
                         int64_t nref, double e0, const AnchorBlk *anc, int nh, int64_t *range, int search,
                         Partial *partials, Flags *flags, hipStream_t st)
{
    const int64_t ntiles = (n + RED_TILE - 1) / RED_TILE;
    const bool rk = s.kc.on != 0;
    size_t q_bytes = (size_t)RED_Q * (8 + 4);
    q_bytes = (q_bytes + 15) & ~(size_t)15;
    const size_t binom_bytes = rk ? (size_t)(s.norb + 1) * s.kc.stride * 8 : 0;
    const size_t dyn = q_bytes + anc_lds_bytes(s.norb, nh) + binom_bytes;
    if (dyn > RED_LDS_MAX)
        return hipErrorInvalidValue;
    if (ntiles > 0 && search) {
        const int64_t gt = (ntiles + 255) / 256;
        dim3 gg((unsigned)(gt < 4096 ? gt : 4096)), bb(256);
        switch (kw) {
        case 1: hipLaunchKernelGGL((k_tile_refs<1>), gg, bb, 0, st, sorted, n, refs, nref, range); break;
        case 2: hipLaunchKernelGGL((k_tile_refs<2>), gg, bb, 0, st, sorted, n, refs, nref, range); break;
        case 3: hipLaunchKernelGGL((k_tile_refs<3>), gg, bb, 0, st, sorted, n, refs, nref, range); break;
        case 4: hipLaunchKernelGGL((k_tile_refs<4>), gg, bb, 0, st, sorted, n, refs, nref, range); break;
        default: return hipErrorInvalidValue;
        }
    }
    dim3 g(RED_GRID), b(RED_THREADS);
#define RD(WW, PB, WBB, RKK)                                                                                   \
    do {                                                                                                       \
        const int64_t ge = red_workers((const void *)&k_reduce<WW, PB, WBB, RKK>, dyn);                         \
        const int64_t per = (ntiles + ge - 1) / ge;                                                            \
        hipLaunchKernelGGL((k_reduce<WW, PB, WBB, RKK>), g, b, dyn, st, s, sorted, n, refs, nref, e0, anc, nh,    \
                           per, q_bytes, range, search, partials, flags);                                       \
    } while (0)
#define RD2(WW, WBB, RKK)      \
    do {                       \
        if (fp32)              \
            RD(WW, 4, WBB, RKK); \
        else                   \
            RD(WW, 8, WBB, RKK); \
    } while (0)
    if (!rk) {
        if (kw != s.W)
            return hipErrorInvalidValue;
        switch (kw) {
        case 1: RD2(1, 1, false); break;
        case 2: RD2(2, 2, false); break;
        case 3: RD2(3, 3, false); break;
        case 4: RD2(4, 4, false); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (kw * 8 + s.W) {
        case 8 + 1: RD2(1, 1, true); break;
        case 8 + 2: RD2(1, 2, true); break;
        case 8 + 3: RD2(1, 3, true); break;
        case 8 + 4: RD2(1, 4, true); break;
        case 16 + 2: RD2(2, 2, true); break;
        case 16 + 3: RD2(2, 3, true); break;
        case 16 + 4: RD2(2, 4, true); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef RD2
#undef RD
    return hipGetLastError();
}

hipError_t launch_ref_terms(const DevSys &s, const Planes &refs, int64_t n, double e0, Partial *partials,
                            Partial *out, hipStream_t st)
{
    dim3 g(256), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_ref_terms<1>), g, b, 0, st, s, refs, n, e0, partials); break;
    case 2: hipLaunchKernelGGL((k_ref_terms<2>), g, b, 0, st, s, refs, n, e0, partials); break;
    case 3: hipLaunchKernelGGL((k_ref_terms<3>), g, b, 0, st, s, refs, n, e0, partials); break;
    case 4: hipLaunchKernelGGL((k_ref_terms<4>), g, b, 0, st, s, refs, n, e0, partials); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, 256, out);
    return hipGetLastError();
}

// Spin flip: each sorted reference's alpha/beta swap must be present with a
// coefficient of equal magnitude; the signs must agree for all references or
// be opposite for all (an eigenfunction of the swap).
template <int W>
__global__ void k_check_swap(DevSys s, Planes refs, int64_t n, Flags *flags)
{
    const int norb = s.norb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k[W], sw[W];
        load_key<W>(refs, i, k);
        uint64_t alo, ahi, blo, bhi;
        spin_strings<W>(k, norb, alo, ahi, blo, bhi);
        // swapped: beta part <- alpha string, alpha part <- beta string
#pragma unroll
        for (int w = 0; w < W; w++)
            sw[w] = 0;
        auto put = [&](int start, uint64_t v, int len) {
            for (int b = 0; b < len; b++)
                if ((v >> b) & 1ull) {
                    const int bit = start + b;
#pragma unroll
                    for (int w = 0; w < W; w++)
                        sw[w] |= (w == (bit >> 6)) ? (1ull << (bit & 63)) : 0ull;
                }
        };
        const int l0 = norb < 64 ? norb : 64;
        put(0, alo, l0);
        put(64, ahi, norb - l0);
        put(norb, blo, l0);
        put(norb + 64, bhi, norb - l0);
        const int64_t j = ref_bound<W>(refs, 0, n, sw, false);
        uint64_t r[W];
        bool found = false;
        if (j < n) {
            load_key<W>(refs, j, r);
            found = key_eq<W>(r, sw);
        }
        const double ci = ((const double *)refs.pay)[i];
        const double cj = found ? ((const double *)refs.pay)[j] : 0.0;
        if (!found || fabs(ci) != fabs(cj))
            atomicOr(&flags->err, ERR_SWAP_MISSING);
        else if (ci == cj)
            atomicOr(&flags->err, SWAP_SAME);
        else
            atomicOr(&flags->err, SWAP_NEG);
    }
}

hipError_t launch_check_swap(const DevSys &s, const Planes &refs, int64_t n, Flags *flags, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_check_swap<1>), g, b, 0, st, s, refs, n, flags); break;
    case 2: hipLaunchKernelGGL((k_check_swap<2>), g, b, 0, st, s, refs, n, flags); break;
    case 3: hipLaunchKernelGGL((k_check_swap<3>), g, b, 0, st, s, refs, n, flags); break;
    case 4: hipLaunchKernelGGL((k_check_swap<4>), g, b, 0, st, s, refs, n, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_refs_hash(const DevSys &s, const Planes &bits, int64_t n, const Planes &out, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_refs_hash<1>), g, b, 0, st, s, bits, n, out); break;
    case 2: hipLaunchKernelGGL((k_refs_hash<2>), g, b, 0, st, s, bits, n, out); break;
    case 3: hipLaunchKernelGGL((k_refs_hash<3>), g, b, 0, st, s, bits, n, out); break;
    case 4: hipLaunchKernelGGL((k_refs_hash<4>), g, b, 0, st, s, bits, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_refs_aos(const DevSys &s, const Planes &bits, int64_t n, uint64_t *ra, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_refs_aos<1>), g, b, 0, st, bits, n, ra); break;
    case 2: hipLaunchKernelGGL((k_refs_aos<2>), g, b, 0, st, bits, n, ra); break;
    case 3: hipLaunchKernelGGL((k_refs_aos<3>), g, b, 0, st, bits, n, ra); break;
    case 4: hipLaunchKernelGGL((k_refs_aos<4>), g, b, 0, st, bits, n, ra); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_anchor(const DevSys &s, const Planes &bits, int64_t nref, double e0, AnchorBlk *anc,
                         hipStream_t st)
{
    if (2 * s.norb > 256)
        return hipErrorInvalidValue;
    dim3 g(1), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_anchor<1>), g, b, 0, st, s, bits, nref, e0, anc); break;
    case 2: hipLaunchKernelGGL((k_anchor<2>), g, b, 0, st, s, bits, nref, e0, anc); break;
    case 3: hipLaunchKernelGGL((k_anchor<3>), g, b, 0, st, s, bits, nref, e0, anc); break;
    case 4: hipLaunchKernelGGL((k_anchor<4>), g, b, 0, st, s, bits, nref, e0, anc); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_parent_g(const DevSys &s, const Planes &bits, int64_t n, double e0, double *D0, double *G,
                           hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    if (2 * s.norb > 256)
        return hipErrorInvalidValue;
    dim3 g((unsigned)(n < 65536 ? n : 65536)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_parent_g<1>), g, b, 0, st, s, bits, n, e0, D0, G); break;
    case 2: hipLaunchKernelGGL((k_parent_g<2>), g, b, 0, st, s, bits, n, e0, D0, G); break;
    case 3: hipLaunchKernelGGL((k_parent_g<3>), g, b, 0, st, s, bits, n, e0, D0, G); break;
    case 4: hipLaunchKernelGGL((k_parent_g<4>), g, b, 0, st, s, bits, n, e0, D0, G); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_refs_ex(const DevSys &s, const Planes &bits, int64_t n, uint64_t *ex, uint32_t *ex4,
                          uint64_t *anc_bits, uint32_t *far, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
    switch (s.W) {
    case 1: hipLaunchKernelGGL((k_refs_ex<1>), g, b, 0, st, bits, n, ex, ex4, anc_bits, far); break;
    case 2: hipLaunchKernelGGL((k_refs_ex<2>), g, b, 0, st, bits, n, ex, ex4, anc_bits, far); break;
    case 3: hipLaunchKernelGGL((k_refs_ex<3>), g, b, 0, st, bits, n, ex, ex4, anc_bits, far); break;
    case 4: hipLaunchKernelGGL((k_refs_ex<4>), g, b, 0, st, bits, n, ex, ex4, anc_bits, far); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_hash(const DevSys &s, int pm, const Planes &sorted, int64_t n, const Planes &bits,
                              const uint64_t *ra_full, const uint64_t *ra_ex, const uint32_t *ra_ex4,
                              const uint64_t *anc_bits,
                              const Planes &rh, int64_t nref, const double *D0, const double *G, double e0,
                              int search, Partial *partials, CollList *coll, int64_t *ctail, Flags *flags,
                              hipStream_t st)
{
    RefTab ra;
    ra.full = ra_full;
    ra.ex = ra_ex;
    ra.ex4 = ra_ex4;
    for (int w = 0; w < MAXW; w++)
        ra.a[w] = ra_ex || ra_ex4 ? anc_bits[w] : 0ull;
    (void)e0;  // carried by D0
    // relative rounding of a stored FP32 payload: once (FP64 arithmetic), or
    // FP32 integrals and arithmetic (a looser bound)
    const double eps = pm == PM_FP32_ARITH ? std::ldexp(1.0, -20) : std::ldexp(1.0, -24);
    const bool fp32 = pm != PM_FP64;
    const int64_t ntiles = (n + RED_TILE - 1) / RED_TILE;
    dim3 g(RED_GRID), b(RED_THREADS);
#define RH(WB, PB)                                                                                                 \
    do {                                                                                                           \
        const int64_t ge = red_workers((const void *)&k_reduce_hash<WB, PB>, 0);                                    \
        const int64_t per = (ntiles + ge - 1) / ge;                                                                \
        hipLaunchKernelGGL((k_reduce_hash<WB, PB>), g, b, 0, st, s, sorted, n, bits, ra, rh, nref, D0, G, per,         \
                           search, eps, partials, coll, ctail, flags);                                             \
        hipLaunchKernelGGL((k_reduce_hash_coll<WB, PB>), g, b, 0, st, s, sorted, n, bits, ra, rh, D0, G, per, search, \
                           partials, coll, ctail, flags);                                                          \
    } while (0)
    switch (s.W * 2 + (fp32 ? 0 : 1)) {
    case 2: RH(1, 4); break;
    case 3: RH(1, 8); break;
    case 4: RH(2, 4); break;
    case 5: RH(2, 8); break;
    case 6: RH(3, 4); break;
    case 7: RH(3, 8); break;
    case 8: RH(4, 4); break;
    case 9: RH(4, 8); break;
    default: return hipErrorInvalidValue;
    }
#undef RH
    return hipGetLastError();
}

hipError_t launch_final(const Partial *partials, Partial *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, RED_GRID, out);
    return hipGetLastError();
}

hipError_t launch_numerators(int W, int fp32, const Planes &sorted, int64_t n, const Planes &refs, int64_t nref,
                             uint64_t *keys_aos, double *num, uint8_t *in_ref, unsigned long long *n_out, int64_t cap,
                             hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    int64_t gg = (n + 255) / 256;
    dim3 g((unsigned)(gg < 4096 ? gg : 4096)), b(256);
#define NM(WW, PB) \
    hipLaunchKernelGGL((k_numerators<WW, PB>), g, b, 0, st, sorted, n, refs, nref, keys_aos, num, in_ref, n_out, cap)
    switch (W * 2 + (fp32 ? 0 : 1)) {
    case 2: NM(1, 4); break;
    case 3: NM(1, 8); break;
    case 4: NM(2, 4); break;
    case 5: NM(2, 8); break;
    case 6: NM(3, 4); break;
    case 7: NM(3, 8); break;
    case 8: NM(4, 4); break;
    case 9: NM(4, 8); break;
    default: return hipErrorInvalidValue;
    }
#undef NM
    return hipGetLastError();
}

}  // namespace pt2
