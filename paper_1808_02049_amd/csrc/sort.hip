// Stable LSD radix sort of the numerator records by determinant bitstring
// (Algorithm 1, sort step; the paper sorts on the CPU or offloads to a GPU
// library, Section V).  Records are structure-of-arrays: W uint64 key planes
// and one payload plane (FP64 or FP32 bits).
//
// Each 8-bit digit is one pass of three steps (reduce-then-scan):
//   1. k_tile_count: every tile of SORT_TILE records counts its digits (one
//      read of the plane holding the digit, LDS histograms per wavefront);
//   2. k_tile_offsets / k_chunk_scan / k_chunk_start: exclusive scan of the
//      counts over tiles, per digit value: the offset of every tile within
//      its chunk of SCAN_CHUNK tiles (u32; counts are u16, a tile holding at
//      most 4096 records, so the per-tile arrays move 6 B per digit value,
//      not 12) with the chunk's totals, then of every chunk from the digit's
//      bucket start (u64; one workgroup per digit value);
//   3. k_scatter: every tile ranks its records by digit with wavefront
//      ballots (stable), stages each plane through LDS in digit order and
//      writes it out in runs of consecutive addresses.
// Tiles never wait for each other.  (A single-kernel "onesweep" pass with
// decoupled look-back was measured slower on MI355X: its status words must be
// read coherently across the eight XCDs' L2 caches, and the look-back took
// about 40% of the pass.)
// Digit histograms of all positions are computed up front in one read of the
// key planes; they give the bucket starts, and a digit whose histogram has a
// single nonzero bin is skipped.  (Hash records skip them: their varying
// digits are known, and each pass takes its bucket starts from its own
// totals.)
#include "pt2_internal.h"

namespace pt2 {
namespace {

// Exclusive scan of one value per thread over a 256-thread block.
__device__ inline uint32_t block_excl_scan256(uint32_t v, uint32_t *sh4, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        sh4[wave] = x;
    __syncthreads();
    uint32_t pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        uint32_t t = sh4[w];
        pre += w < wave ? t : 0u;
        total += t;
    }
    __syncthreads();
    return pre + x - v;
}

// ---------------------------------------------------------------------------
// N consecutive keys of plane w from record r0 (0 past n), in 16-byte loads
// when all N exist: plane bases are 256-byte aligned and r0 is a multiple of N.
template <int W, int N>
__device__ inline void load_keys_run(const Planes &in, int w, int64_t r0, int64_t n, uint64_t (&v)[N])
{
    static_assert(N % 8 == 0, "8 two-byte keys per 16-byte load");
    if (r0 + N <= n) {
        const int eb = w == W - 1 ? in.topb : 8;
        const char *b = (const char *)plane_ptr<W>(in, w) + r0 * eb;
        if (eb == 8) {
#pragma unroll
            for (int j = 0; j < N; j += 2) {
                const ulonglong2 x = ((const ulonglong2 *)b)[j / 2];
                v[j] = x.x, v[j + 1] = x.y;
            }
        } else if (eb == 4) {
#pragma unroll
            for (int j = 0; j < N; j += 4) {
                const uint4 x = ((const uint4 *)b)[j / 4];
                v[j] = x.x, v[j + 1] = x.y, v[j + 2] = x.z, v[j + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < N; j += 8) {
                const uint4 x = ((const uint4 *)b)[j / 8];
                const uint32_t u[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int q = 0; q < 4; q++)
                    v[j + 2 * q] = u[q] & 0xFFFFu, v[j + 2 * q + 1] = u[q] >> 16;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; j++)
            v[j] = r0 + j < n ? pl_get<W>(in, w, r0 + j) : 0ull;
    }
}

// Digit counts of N consecutive keys into an LDS histogram.  Most lanes of a
// wavefront usually see the same digit value, and LDS atomics from many lanes
// on one address serialise.  So the keys equal to a wavefront-wide reference
// value (the digit of the first active lane's first key) are counted in a
// register and added by one lane; runs of other values are merged per thread
// and added one atomic per run.  All lanes of the wavefront must call this.
// (The all-digits histogram pass keeps plain run merging: there the wavefront
// sums of ten digit positions cost more than the conflicts they remove.)
template <int N>
__device__ inline void count_digits(const uint64_t (&v)[N], int shift, int64_t r0, int64_t n, uint32_t *h)
{
    const uint32_t ref = __builtin_amdgcn_readfirstlane((uint32_t)(v[0] >> shift) & 255u);
    uint32_t nref = 0, last = 0xFFFFFFFFu, cnt = 0;
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (r0 + j < n) {
            const uint32_t d = (uint32_t)(v[j] >> shift) & 255u;
            if (d == ref) {
                nref++;
            } else if (d == last) {
                cnt++;
            } else {
                if (cnt)
                    atomicAdd(&h[last], cnt);
                last = d;
                cnt = 1;
            }
        }
    }
    if (cnt)
        atomicAdd(&h[last], cnt);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        nref += __shfl_xor(nref, o);
    if ((threadIdx.x & 63) == 0 && nref)
        atomicAdd(&h[ref], nref);
}

// Digit histograms of every digit position (one read of the key planes).
template <int W>
__global__ __launch_bounds__(256) void k_hist(Planes in, int64_t n, int ndig, unsigned long long *hist)
{
    __shared__ uint32_t h[32 * 256];
    for (int i = threadIdx.x; i < ndig * 256; i += 256)
        h[i] = 0;
    __syncthreads();
    constexpr int RI = 16;
    for (int64_t t0 = (int64_t)blockIdx.x * 256 * RI; t0 < n; t0 += (int64_t)gridDim.x * 256 * RI) {
        const int64_t r0 = t0 + (int64_t)threadIdx.x * RI;
#pragma unroll
        for (int w = 0; w < W; w++) {
            uint64_t v[RI];
            load_keys_run<W, RI>(in, w, r0, n, v);
#pragma unroll
            for (int dd = 0; dd < 8; dd++) {
                const int d = w * 8 + dd;
                if (d >= ndig)
                    break;
                uint32_t last = 0xFFFFFFFFu, cnt = 0;
#pragma unroll
                for (int j = 0; j < RI; j++) {
                    if (r0 + j < n) {
                        uint32_t dv = (uint32_t)(v[j] >> (8 * dd)) & 255u;
                        if (dv == last) {
                            cnt++;
                        } else {
                            if (cnt)
                                atomicAdd(&h[d * 256 + last], cnt);
                            last = dv;
                            cnt = 1;
                        }
                    }
                }
                if (cnt)
                    atomicAdd(&h[d * 256 + last], cnt);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ndig * 256; i += 256)
        if (h[i])
            atomicAdd(&hist[i], (unsigned long long)h[i]);
}

__global__ __launch_bounds__(256) void k_hist_scan(const unsigned long long *hist, uint64_t *bucket)
{
    __shared__ uint64_t sh[256];
    const int d = blockIdx.x;
    uint64_t v = hist[d * 256 + threadIdx.x];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    bucket[d * 256 + threadIdx.x] = sh[threadIdx.x] - v;
}

// ---------------------------------------------------------------------------
// Step 1: digit counts of every tile (counts[tile * 256 + digit]).  Each
// thread reads SORT_ITEMS consecutive records and counts their digits into its
// wavefront's LDS histogram.
template <int W, int IT>
__global__ __launch_bounds__(SORT_THREADS) void k_tile_count(Planes in, int64_t n, int dig, uint16_t *counts)
{
    constexpr int TILE = SORT_THREADS * IT;
    static_assert(TILE <= 65535, "tile counts are u16");
    __shared__ uint32_t h[SORT_THREADS / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < (SORT_THREADS / 64) * 256; i += SORT_THREADS)
        (&h[0][0])[i] = 0;
    __syncthreads();
    const int word = dig >> 3, shift = (dig & 7) * 8;
    const int64_t r0 = (int64_t)blockIdx.x * TILE + (int64_t)tid * IT;
    uint64_t v[IT];
    load_keys_run<W, IT>(in, word, r0, n, v);
    count_digits<IT>(v, shift, r0, n, h[wave]);
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < SORT_THREADS / 64; w++)
        t += h[w][tid];
    counts[(int64_t)blockIdx.x * 256 + tid] = (uint16_t)t;
}

// Step 2a: per chunk of SCAN_CHUNK tiles, the offset of each tile's first
// record of each digit from its chunk's (the record goes to
// coff[chunk][digit] + rel[tile][digit]), and the chunk's count of each digit.
__global__ __launch_bounds__(256) void k_tile_offsets(const uint16_t *counts, int64_t ntiles, uint32_t *rel,
                                                      uint64_t *csum)
{
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_CHUNK;
    const int64_t t1 = t0 + SCAN_CHUNK < ntiles ? t0 + SCAN_CHUNK : ntiles;
    uint32_t run = 0;
    for (int64_t t = t0; t < t1; t++) {
        rel[t * 256 + threadIdx.x] = run;
        run += counts[t * 256 + threadIdx.x];
    }
    csum[(int64_t)blockIdx.x * 256 + threadIdx.x] = run;
}

static_assert((int64_t)SCAN_CHUNK * SORT_THREADS * SORT_ITEMS_WIDE <= 0xFFFFFFFFll, "in-chunk offsets are u32");

// Exclusive prefix of s[0..256) in place (thread 0; the values are few), the
// total returned to thread 0.
__device__ inline uint64_t excl256_serial(uint64_t *s)
{
    uint64_t run = 0;
    for (int v = 0; v < 256; v++) {
        const uint64_t x = s[v];
        s[v] = run;
        run += x;
    }
    return run;
}

// Step 2b: one workgroup per digit value: the exclusive scan of that digit's
// chunk counts over the chunks (each thread a contiguous range of chunks), and
// the digit's total in tot[digit].
__global__ __launch_bounds__(256) void k_chunk_scan(const uint64_t *csum, int64_t nchunks, uint64_t *coff,
                                                    uint64_t *tot)
{
    __shared__ uint64_t s_part[256];
    const int v = blockIdx.x, tid = threadIdx.x;
    const int64_t per = (nchunks + 255) / 256;
    const int64_t c0 = (int64_t)tid * per < nchunks ? (int64_t)tid * per : nchunks;
    const int64_t c1 = c0 + per < nchunks ? c0 + per : nchunks;
    uint64_t sum = 0;
    for (int64_t c = c0; c < c1; c++)
        sum += csum[c * 256 + v];
    s_part[tid] = sum;
    __syncthreads();
    if (tid == 0)
        tot[v] = excl256_serial(s_part);
    __syncthreads();
    uint64_t run = s_part[tid];
    for (int64_t c = c0; c < c1; c++) {
        const uint64_t x = csum[c * 256 + v];
        coff[c * 256 + v] = run;
        run += x;
    }
}

// Step 2c: each digit's bucket start added to its chunk offsets: from the
// all-digit histograms, or, when bucket is null, the exclusive scan over
// digit values of the totals.
__global__ __launch_bounds__(256) void k_chunk_start(uint64_t *coff, int64_t nchunks, const uint64_t *bucket,
                                                     const uint64_t *tot)
{
    __shared__ uint64_t s_start[256];
    const int tid = threadIdx.x;
    s_start[tid] = bucket ? bucket[tid] : tot[tid];
    __syncthreads();
    if (!bucket && tid == 0)
        (void)excl256_serial(s_start);
    __syncthreads();
    const uint64_t st = s_start[tid];
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        coff[c * 256 + tid] += st;
}

// Step 3: rank and scatter one tile.
template <int W, int PB, int IT>
__global__ __launch_bounds__(SORT_THREADS) void k_scatter(Planes in, Planes out, int64_t n, int dig,
                                                          const uint64_t *coff, const uint32_t *rel, Flags *flags)
{
    __shared__ uint32_t s_wc[4][256];
    __shared__ uint32_t s_tstart[256];
    __shared__ int64_t s_gbase[256];
    __shared__ uint32_t s_sc[4];
    constexpr int TILE = SORT_THREADS * IT;
    __shared__ uint64_t s_stage[TILE];
    __shared__ uint8_t s_dig[TILE];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int i = tid; i < 4 * 256; i += SORT_THREADS)
        (&s_wc[0][0])[i] = 0;
#if PT2_XCD_TILES
    // Workgroups are dealt to the 8 XCDs in turn; give each XCD a contiguous
    // range of tiles, so that the runs consecutive tiles write into a bucket
    // meet in one L2.  A bijection of [0, ntiles) for any ntiles.
    const int64_t nt = gridDim.x, q = nt >> 3, r = nt & 7;
    const int64_t x = blockIdx.x & 7, i = blockIdx.x >> 3;
    const int64_t tile = x * q + (x < r ? x : r) + i;
#else
    const int64_t tile = blockIdx.x;
#endif
    const int64_t base = tile * TILE;
    const int word = dig >> 3, shift = (dig & 7) * 8;
    const uint64_t my_off = coff[(tile / SCAN_CHUNK) * 256 + tid] + rel[tile * 256 + tid];

    uint64_t kw[IT];
    uint32_t rank[IT];
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const int64_t idx = base + (int64_t)wave * 64 * IT + j * 64 + lane;
        kw[j] = idx < n ? pl_get<W>(in, word, idx) : 0ull;
    }
    __syncthreads();
    // rank within the wave: peers = lanes with the same digit (stable)
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const int64_t idx = base + (int64_t)wave * 64 * IT + j * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = (uint32_t)(kw[j] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        rank[j] = 0;
        if (valid) {
            const uint32_t cnt = s_wc[wave][d];
            rank[j] = cnt + below;
            if (below == 0)
                s_wc[wave][d] = cnt + (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    {
        const int d = tid;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            const uint32_t c = s_wc[w][d];
            s_wc[w][d] = tot;
            tot += c;
        }
        uint32_t tile_total;
        s_tstart[d] = block_excl_scan256(tot, s_sc, tile_total);
        s_gbase[d] = (int64_t)my_off - (int64_t)s_tstart[d];
    }
    __syncthreads();

    uint32_t lpos[IT];
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const uint32_t d = (uint32_t)(kw[j] >> shift) & 255u;
        lpos[j] = s_tstart[d] + s_wc[wave][d] + rank[j];
    }
    const int64_t rem = n - base;
    const int tile_n = rem < TILE ? (int)rem : TILE;

    // plane w of the tile's records, in input order (the digit plane is
    // already in registers)
    auto load_plane = [&](int w, uint64_t(&v)[IT]) {
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int64_t idx = base + (int64_t)wave * 64 * IT + j * 64 + lane;
            uint64_t x = 0;
            if (w == word)
                x = kw[j];
            else if (idx < n)
                x = w < W ? pl_get<W>(in, w, idx)
                          : (PB == 8 ? ((const uint64_t *)in.pay)[idx]
                                     : (uint64_t)((const uint32_t *)in.pay)[idx]);
            v[j] = x;
        }
    };
    // narrow tiles keep the next plane's loads in flight while one plane is
    // staged; wide tiles load each plane when it is staged (registers).
    // PB == 0: no payload plane (packed records).
    constexpr bool PIPE = IT <= SORT_ITEMS || PT2_WIDE_PIPE;
    constexpr int NPL = W + (PB ? 1 : 0);
    uint64_t cur[IT];
    if constexpr (PIPE)
        load_plane(0, cur);

#pragma unroll
    for (int w = 0; w < NPL; w++) {
        uint64_t nxt[IT];
        if constexpr (PIPE) {
            if (w + 1 < NPL)
                load_plane(w + 1, nxt);
        } else {
            load_plane(w, cur);
        }
        uint64_t(&cv)[IT] = cur;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int64_t idx = base + (int64_t)wave * 64 * IT + j * 64 + lane;
            if (idx < n) {
                s_stage[lpos[j]] = cv[j];
                if (w == 0)
                    s_dig[lpos[j]] = (uint8_t)((kw[j] >> shift) & 255u);
            }
        }
        __syncthreads();
        for (int q = tid; q < tile_n; q += SORT_THREADS) {
            const int64_t dst = s_gbase[s_dig[q]] + q;
            if ((uint64_t)dst >= (uint64_t)n) {
                atomicOr(&flags->err, ERR_BOUNDS);
                continue;
            }
            const uint64_t v = s_stage[q];
            if (w < W)
                pl_put<W>(out, w, dst, v);
            else if (PB == 8)
                ((uint64_t *)out.pay)[dst] = v;
            else
                ((uint32_t *)out.pay)[dst] = (uint32_t)v;
        }
        __syncthreads();
        if (PIPE && w + 1 < NPL) {
#pragma unroll
            for (int j = 0; j < IT; j++)
                cur[j] = nxt[j];
        }
    }
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero_u64(uint64_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int W>
__global__ void k_refs_split(int norb, int na, int nb, const uint64_t *dets, const double *c, int64_t n, Planes out,
                             Flags *flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int pa = 0, pb = 0;
        bool stray = false;
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint64_t v = dets[i * W + w];
            pl_put<W>(out, w, i, v);
            for (int b = 0; b < 64; b++) {
                const int bit = w * 64 + b;
                if (!((v >> b) & 1ull))
                    continue;
                if (bit < norb)
                    pb++;
                else if (bit < 2 * norb)
                    pa++;
                else
                    stray = true;
            }
        }
        ((double *)out.pay)[i] = c[i];
        if (pa != na || pb != nb)
            atomicOr(&flags->err, ERR_POPCOUNT);
        if (stray)
            atomicOr(&flags->err, ERR_STRAY_BITS);
    }
}

template <int W>
__global__ void k_dup_check(Planes sorted, int64_t n, Flags *flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool eq = true;
#pragma unroll
        for (int w = 0; w < W; w++)
            eq = eq && pl_get<W>(sorted, w, i) == pl_get<W>(sorted, w, i - 1);
        if (eq)
            atomicOr(&flags->err, ERR_DUPLICATE);
    }
}

template <int W>
__global__ void k_planes_to_aos(Planes in, int pay_bytes, int64_t n, uint64_t *keys, double *pay)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int w = 0; w < W; w++)
            keys[i * W + w] = pl_get<W>(in, w, i);
        if (pay)
            pay[i] = pay_bytes == 8 ? ((const double *)in.pay)[i] : (double)((const float *)in.pay)[i];
    }
}

inline unsigned grid_for(int64_t n, int threads, unsigned cap)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1)
        g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace

hipError_t launch_hist(int W, const Planes &in, int64_t n, int ndig, uint64_t *hist, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    if (ndig > 32 || ndig > 8 * W)
        return hipErrorInvalidValue;
    unsigned g = grid_for(n, 256 * 16, 1024);
    unsigned long long *h = (unsigned long long *)hist;
    switch (W) {
    case 1: hipLaunchKernelGGL((k_hist<1>), dim3(g), dim3(256), 0, st, in, n, ndig, h); break;
    case 2: hipLaunchKernelGGL((k_hist<2>), dim3(g), dim3(256), 0, st, in, n, ndig, h); break;
    case 3: hipLaunchKernelGGL((k_hist<3>), dim3(g), dim3(256), 0, st, in, n, ndig, h); break;
    case 4: hipLaunchKernelGGL((k_hist<4>), dim3(g), dim3(256), 0, st, in, n, ndig, h); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_hist_scan(const uint64_t *hist, int ndig, uint64_t *bucket, hipStream_t st)
{
    hipLaunchKernelGGL(k_hist_scan, dim3(ndig), dim3(256), 0, st, (const unsigned long long *)hist, bucket);
    return hipGetLastError();
}

hipError_t launch_radix_pass(int W, int pay_bytes, const Planes &in, const Planes &out, int64_t n, int dig,
                             const uint64_t *bucket, uint16_t *counts, uint64_t *csum, uint64_t *coff,
                             uint32_t *rel, Flags *flags, hipStream_t st, hipEvent_t mid, int items)
{
    if (n <= 0)
        return hipSuccess;
    if (items != SORT_ITEMS && items != SORT_ITEMS_WIDE)
        return hipErrorInvalidValue;
    const int64_t tile = (int64_t)SORT_THREADS * items;
    const int64_t ntiles = (n + tile - 1) / tile;
    const int64_t nchunks = (ntiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (ntiles > 0x7FFFFFFFll)
        return hipErrorInvalidValue;
    dim3 g((unsigned)ntiles), b(SORT_THREADS);
#define TC(WW, IT) hipLaunchKernelGGL((k_tile_count<WW, IT>), g, b, 0, st, in, n, dig, counts)
    switch (W * 2 + (items == SORT_ITEMS ? 0 : 1)) {
    case 2: TC(1, SORT_ITEMS); break;
    case 3: TC(1, SORT_ITEMS_WIDE); break;
    case 4: TC(2, SORT_ITEMS); break;
    case 5: TC(2, SORT_ITEMS_WIDE); break;
    case 6: TC(3, SORT_ITEMS); break;
    case 7: TC(3, SORT_ITEMS_WIDE); break;
    case 8: TC(4, SORT_ITEMS); break;
    case 9: TC(4, SORT_ITEMS_WIDE); break;
    default: return hipErrorInvalidValue;
    }
#undef TC
    // csum holds nchunks + 1 rows: the last takes the digits' totals
    uint64_t *tot = csum + nchunks * 256;
    hipLaunchKernelGGL(k_tile_offsets, dim3((unsigned)nchunks), dim3(256), 0, st, counts, ntiles, rel, csum);
    hipLaunchKernelGGL(k_chunk_scan, dim3(256), dim3(256), 0, st, csum, nchunks, coff, tot);
    hipLaunchKernelGGL(k_chunk_start, dim3((unsigned)(nchunks < 1024 ? nchunks : 1024)), dim3(256), 0, st, coff,
                       nchunks, bucket, tot);
    if (mid)
        (void)hipEventRecord(mid, st);
#define SC(WW, PB)                                                                                            \
    do {                                                                                                      \
        if (items == SORT_ITEMS)                                                                              \
            hipLaunchKernelGGL((k_scatter<WW, PB, SORT_ITEMS>), g, b, 0, st, in, out, n, dig, coff, rel, flags);      \
        else                                                                                                  \
            hipLaunchKernelGGL((k_scatter<WW, PB, SORT_ITEMS_WIDE>), g, b, 0, st, in, out, n, dig, coff, rel, flags); \
    } while (0)
    if (pay_bytes == 0) {
        // packed hash records: two 8-byte key planes, wide tiles
        if (W != 2 || items != SORT_ITEMS_WIDE)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_scatter<2, 0, SORT_ITEMS_WIDE>), g, b, 0, st, in, out, n, dig, coff, rel, flags);
        return hipGetLastError();
    }
    switch (W * 2 + (pay_bytes == 8 ? 1 : 0)) {
    case 2: SC(1, 4); break;
    case 3: SC(1, 8); break;
    case 4: SC(2, 4); break;
    case 5: SC(2, 8); break;
    case 6: SC(3, 4); break;
    case 7: SC(3, 8); break;
    case 8: SC(4, 4); break;
    case 9: SC(4, 8); break;
    default: return hipErrorInvalidValue;
    }
#undef SC
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t *p, int64_t n, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_refs_split(int W, int norb, int na, int nb, const uint64_t *dets, const double *c, int64_t n,
                             Planes out, Flags *flags, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    dim3 g(grid_for(n, 256, 4096)), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_refs_split<1>), g, b, 0, st, norb, na, nb, dets, c, n, out, flags); break;
    case 2: hipLaunchKernelGGL((k_refs_split<2>), g, b, 0, st, norb, na, nb, dets, c, n, out, flags); break;
    case 3: hipLaunchKernelGGL((k_refs_split<3>), g, b, 0, st, norb, na, nb, dets, c, n, out, flags); break;
    case 4: hipLaunchKernelGGL((k_refs_split<4>), g, b, 0, st, norb, na, nb, dets, c, n, out, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dup_check(int W, const Planes &sorted, int64_t n, Flags *flags, hipStream_t st)
{
    if (n <= 1)
        return hipSuccess;
    dim3 g(grid_for(n, 256, 4096)), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_dup_check<1>), g, b, 0, st, sorted, n, flags); break;
    case 2: hipLaunchKernelGGL((k_dup_check<2>), g, b, 0, st, sorted, n, flags); break;
    case 3: hipLaunchKernelGGL((k_dup_check<3>), g, b, 0, st, sorted, n, flags); break;
    case 4: hipLaunchKernelGGL((k_dup_check<4>), g, b, 0, st, sorted, n, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_planes_to_aos(int W, int pay_bytes, const Planes &in, int64_t n, uint64_t *keys, double *pay,
                                hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    dim3 g(grid_for(n, 256, 4096)), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_planes_to_aos<1>), g, b, 0, st, in, pay_bytes, n, keys, pay); break;
    case 2: hipLaunchKernelGGL((k_planes_to_aos<2>), g, b, 0, st, in, pay_bytes, n, keys, pay); break;
    case 3: hipLaunchKernelGGL((k_planes_to_aos<3>), g, b, 0, st, in, pay_bytes, n, keys, pay); break;
    case 4: hipLaunchKernelGGL((k_planes_to_aos<4>), g, b, 0, st, in, pay_bytes, n, keys, pay); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pt2
