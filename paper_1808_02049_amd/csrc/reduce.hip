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
// merged tile by tile.  H_aa is evaluated from scratch from a spin-orbital pair
// table, sum over occupied pairs b1 <= b2 of T[b1][b2].
//
// A fixed grid of RED_GRID workgroups strides over tiles; each workgroup owns
// the segments whose first record lies in its tile, follows a segment past
// the tile end with one wavefront, and keeps a Neumaier-compensated sum.
// Partials are combined in workgroup order, so the energy is bit-reproducible.
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
        k[w] = p.key[w][i];
}

template <int PB>
__device__ inline double load_pay(const Planes &p, int64_t i)
{
    if (PB == 8)
        return ((const double *)p.pay)[i];
    return (double)((const float *)p.pay)[i];
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

// H_aa = sum over occupied spin-orbital pairs b1 <= b2 of T[b1][b2]
template <int W>
__device__ inline double diag_energy(const double *T, int nso, const uint64_t (&k)[W])
{
    double e = 0.0;
#pragma unroll
    for (int w1 = 0; w1 < W; w1++) {
        uint64_t m1 = k[w1];
        while (m1) {
            const int b1 = w1 * 64 + __builtin_ctzll(m1);
            m1 &= m1 - 1;
            const double *row = T + (int64_t)b1 * nso;
            double acc = row[b1];
            uint64_t m2 = m1;
            while (m2) {
                acc += row[w1 * 64 + __builtin_ctzll(m2)];
                m2 &= m2 - 1;
            }
#pragma unroll
            for (int w2 = w1 + 1; w2 < W; w2++) {
                uint64_t m3 = k[w2];
                while (m3) {
                    acc += row[w2 * 64 + __builtin_ctzll(m3)];
                    m3 &= m3 - 1;
                }
            }
            e += acc;
        }
    }
    return e;
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

template <int W>
__device__ inline void process_segment(const DevSys &s, const Planes &refs, const RefSlice &rs, const uint64_t *s_rk,
                                       const double *s_rc, double e0, const uint64_t (&k)[W], double num, Acc &a)
{
    a.n_unique++;
    int64_t hit = -1;
    if (rs.staged) {
        int lo = 0, hi = (int)(rs.hi - rs.lo);
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            uint64_t r[W];
#pragma unroll
            for (int w = 0; w < W; w++)
                r[w] = s_rk[w * RED_LDS_REFS + mid];
            int c = key_cmp<W>(r, k);
            if (c == 0) {
                hit = mid;
                break;
            }
            if (c < 0)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (hit >= 0) {
            a.n_hit++;
            a.ref_cross += s_rc[hit] * num;
            return;
        }
    } else {
        int64_t i = ref_bound<W>(refs, rs.lo, rs.hi, k, false);
        if (i < rs.hi) {
            uint64_t r[W];
            load_key<W>(refs, i, r);
            if (key_eq<W>(r, k)) {
                a.n_hit++;
                a.ref_cross += ((const double *)refs.pay)[i] * num;
                return;
            }
        }
    }
    const double haa = diag_energy<W>(s.T, 2 * s.norb, k);
    const double den = e0 - haa;
    a.n_ext++;
    const double ad = fabs(den);
    a.min_abs = ad < a.min_abs ? ad : a.min_abs;
    if (den >= 0.0)
        a.n_nonneg++;
    if (den == 0.0)
        a.singular = 1;
    else
        neumaier(a.e_sum, a.e_comp, num * num / den);
    const uint64_t m = key_mix<W>(k);
    a.kx ^= m;
    a.ks += m;
}

template <int W, int PB>
__global__ __launch_bounds__(RED_THREADS) void k_reduce(DevSys s, Planes in, int64_t n, Planes refs, int64_t nref,
                                                        double e0, Partial *partials, Flags *flags)
{
    __shared__ uint8_t s_f[RED_THREADS];
    __shared__ double s_v[RED_THREADS];
    __shared__ uint64_t s_rk[W * RED_LDS_REFS];
    __shared__ double s_rc[RED_LDS_REFS];
    __shared__ int64_t s_lo, s_hi;
    __shared__ uint64_t s_ck[W];
    __shared__ double s_cv;
    __shared__ int s_cflag;

    const int tid = threadIdx.x, lane = tid & 63;
    Acc a;
    acc_init(a);

    for (int64_t tile = blockIdx.x; tile * RED_TILE < n; tile += gridDim.x) {
        const int64_t base = tile * RED_TILE;
        const int64_t tend = base + RED_TILE < n ? base + RED_TILE : n;
        if (tid == 0) {
            uint64_t kf[W], kl[W];
            load_key<W>(in, base, kf);
            load_key<W>(in, tend - 1, kl);
            s_lo = ref_bound<W>(refs, 0, nref, kf, false);
            s_hi = ref_bound<W>(refs, s_lo, nref, kl, true);
            s_cflag = 0;
        }
        __syncthreads();
        RefSlice rs;
        rs.lo = s_lo, rs.hi = s_hi;
        rs.staged = (rs.hi - rs.lo) <= RED_LDS_REFS;
        if (rs.staged)
            for (int i = tid; i < (int)(rs.hi - rs.lo); i += RED_THREADS) {
#pragma unroll
                for (int w = 0; w < W; w++)
                    s_rk[w * RED_LDS_REFS + i] = refs.key[w][rs.lo + i];
                s_rc[i] = ((const double *)refs.pay)[rs.lo + i];
            }

        // my records
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
        // block exclusive segmented scan of (any, sacc) over threads
        s_f[tid] = any ? 1 : 0;
        s_v[tid] = sacc;
        __syncthreads();
        for (int o = 1; o < RED_THREADS; o <<= 1) {
            uint8_t f2 = 0;
            double v2 = 0.0;
            if (tid >= o) {
                f2 = s_f[tid - o];
                v2 = s_v[tid - o];
            }
            __syncthreads();
            if (tid >= o) {
                // combine (earlier = f2,v2) with (later = current)
                const uint8_t fc = s_f[tid];
                const double vc = s_v[tid];
                s_v[tid] = fc ? vc : v2 + vc;
                s_f[tid] = fc | f2;
            }
            __syncthreads();
        }
        const bool cf = tid > 0 ? s_f[tid - 1] != 0 : false;
        const double cv = tid > 0 ? s_v[tid - 1] : 0.0;
        __syncthreads();

#pragma unroll
        for (int j = 0; j < RED_ITEMS; j++) {
            const int64_t idx = r0 + j;
            if (idx >= tend)
                continue;
            const bool owned = hh[j] || cf;
            if (!owned)
                continue;
            const double val = hh[j] ? run[j] : cv + run[j];
            if (tl[j]) {
                process_segment<W>(s, refs, rs, s_rk, s_rc, e0, k[j], val, a);
            } else if (idx == tend - 1) {
                // the segment continues into the next tile
#pragma unroll
                for (int w = 0; w < W; w++)
                    s_ck[w] = k[j][w];
                s_cv = val;
                s_cflag = 1;
            }
        }
        __syncthreads();
        if (s_cflag && tid < 64) {
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
                // fixed-order tree sum over the wavefront
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1)
                    v += __shfl_down(v, o);
                total += v;  // lane 0 holds the step sum
                if (m != ~0ull)
                    break;
                pos += 64;
            }
            if (lane == 0)
                process_segment<W>(s, refs, rs, s_rk, s_rc, e0, ck, s_cv + total, a);
        }
        __syncthreads();
    }

    // block reduction of the accumulators (fixed tree)
    __shared__ Partial s_p[RED_THREADS];
    Partial me;
    me.e_sum = a.e_sum, me.e_comp = a.e_comp, me.ref_cross = a.ref_cross, me.min_abs_denom = a.min_abs;
    me.n_unique = a.n_unique, me.n_external = a.n_ext, me.n_hit = a.n_hit, me.n_nonneg = a.n_nonneg;
    me.key_xor = a.kx, me.key_sum = a.ks;
    s_p[tid] = me;
    if (a.singular)
        atomicOr(&flags->err, ERR_SINGULAR);
    __syncthreads();
    for (int o = RED_THREADS / 2; o >= 1; o >>= 1) {
        if (tid < o) {
            Partial x = s_p[tid], y = s_p[tid + o];
            double sum = x.e_sum, comp = x.e_comp + y.e_comp;
            neumaier(sum, comp, y.e_sum);
            x.e_sum = sum, x.e_comp = comp;
            x.ref_cross += y.ref_cross;
            x.min_abs_denom = y.min_abs_denom < x.min_abs_denom ? y.min_abs_denom : x.min_abs_denom;
            x.n_unique += y.n_unique, x.n_external += y.n_external, x.n_hit += y.n_hit;
            x.n_nonneg += y.n_nonneg, x.key_xor ^= y.key_xor, x.key_sum += y.key_sum;
            s_p[tid] = x;
        }
        __syncthreads();
    }
    if (tid == 0)
        partials[blockIdx.x] = s_p[0];
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

hipError_t launch_reduce(const DevSys &s, int fp32, const Planes &sorted, int64_t n, const Planes &refs, int64_t nref,
                         double e0, Partial *partials, Flags *flags, hipStream_t st)
{
    dim3 g(RED_GRID), b(RED_THREADS);
#define RD(WW, PB) hipLaunchKernelGGL((k_reduce<WW, PB>), g, b, 0, st, s, sorted, n, refs, nref, e0, partials, flags)
    switch (s.W * 2 + (fp32 ? 0 : 1)) {
    case 2: RD(1, 4); break;
    case 3: RD(1, 8); break;
    case 4: RD(2, 4); break;
    case 5: RD(2, 8); break;
    case 6: RD(3, 4); break;
    case 7: RD(3, 8); break;
    case 8: RD(4, 4); break;
    case 9: RD(4, 8); break;
    default: return hipErrorInvalidValue;
    }
#undef RD
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
