// Stable LSD radix sort of the numerator records by determinant bitstring
// (Algorithm 1, sort step; the paper sorts on the CPU or offloads to a GPU
// library, Section V).  Records are structure-of-arrays: W uint64 key planes
// and one payload plane (FP64 or FP32 bits).
//
// Each 8-bit digit is one "onesweep" pass (Adinets and Merrill, 2022): a tile
// of SORT_TILE records takes its tile index from an atomic counter, ranks its
// records by digit inside the tile with wavefront ballots, publishes its
// per-digit counts, and resolves its global offsets by decoupled look-back
// over the tiles before it.  Records are then staged through LDS in digit
// order so that each plane is written in runs of consecutive addresses.
// Digit histograms of all positions are computed up front in one read of the
// key planes; a digit whose histogram has a single nonzero bin is skipped.
#include "pt2_internal.h"

namespace pt2 {
namespace {

constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_INC = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 46) - 1;
constexpr uint32_t SPIN_MAX = 1u << 24;
constexpr int LB_WIN = 16;  // predecessors examined per look-back step

__device__ inline uint64_t st_pack(uint64_t flag, uint32_t epoch, uint64_t v)
{
    return flag | ((uint64_t)(epoch & 0xFFFFu) << 46) | (v & ST_VAL);
}

__device__ inline uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__device__ inline const uint64_t *plane_c(const Planes &p, int w)
{
    const uint64_t *r = p.key[0];
    if (W > 1 && w == 1)
        r = p.key[1];
    if (W > 2 && w == 2)
        r = p.key[2];
    if (W > 3 && w == 3)
        r = p.key[3];
    return r;
}

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
            const uint64_t *src = plane_c<W>(in, w);
#pragma unroll
            for (int j = 0; j < RI; j++)
                v[j] = r0 + j < n ? src[r0 + j] : 0;
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
// One onesweep digit pass.
template <int W, int PB>
__global__ __launch_bounds__(SORT_THREADS) void k_onesweep(Planes in, Planes out, int64_t n, int dig,
                                                           const uint64_t *bucket, uint64_t *status,
                                                           uint32_t *tile_ctr, uint32_t epoch, Flags *flags)
{
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wc[4][256];
    __shared__ uint32_t s_tstart[256];
    __shared__ int64_t s_gbase[256];
    __shared__ uint32_t s_sc[4];
    __shared__ uint64_t s_stage[SORT_TILE];
    __shared__ uint8_t s_dig[SORT_TILE];
    __shared__ int s_fail;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (tid == 0) {
        s_tile = atomicAdd(tile_ctr, 1u);
        s_fail = 0;
    }
    for (int i = tid; i < 4 * 256; i += SORT_THREADS)
        (&s_wc[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * SORT_TILE;
    const int word = dig >> 3, shift = (dig & 7) * 8;
    const uint64_t *src = plane_c<W>(in, word);

    uint64_t kw[SORT_ITEMS];
    uint32_t rank[SORT_ITEMS];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        const int64_t idx = base + (int64_t)wave * 64 * SORT_ITEMS + j * 64 + lane;
        kw[j] = idx < n ? src[idx] : 0ull;
    }
    // rank within the wave: peers = lanes with the same digit
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        const int64_t idx = base + (int64_t)wave * 64 * SORT_ITEMS + j * 64 + lane;
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

    // thread = digit: wave offsets, tile totals, look-back
    {
        const int d = tid;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            uint32_t c = s_wc[w][d];
            s_wc[w][d] = tot;
            tot += c;
        }
        uint64_t *my = status + (int64_t)tile * 256 + d;
        st_agent(my, st_pack(tile == 0 ? ST_INC : ST_AGG, epoch, tot));
        uint32_t tile_total;
        s_tstart[d] = block_excl_scan256(tot, s_sc, tile_total);
        int64_t excl = 0;
        if (tile > 0) {
            // windowed look-back: LB_WIN predecessors' status words are read at
            // once; AGG values are summed newest to oldest until an INC is found
            int64_t p = (int64_t)tile - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                uint64_t v[LB_WIN];
#pragma unroll
                for (int i = 0; i < LB_WIN; i++)
                    v[i] = p - i >= 0 ? ld_agent(status + (p - i) * 256 + d) : 0ull;
                int used = 0;
#pragma unroll
                for (int i = 0; i < LB_WIN; i++) {
                    if (done || used != i)
                        continue;
                    const uint64_t flag = v[i] & (3ull << 62);
                    const uint32_t ep = (uint32_t)(v[i] >> 46) & 0xFFFFu;
                    if (flag == 0 || ep != (epoch & 0xFFFFu))
                        continue;  // not yet published: stop consuming here
                    excl += (int64_t)(v[i] & ST_VAL);
                    used = i + 1;
                    if (flag == ST_INC)
                        done = true;
                }
                if (done)
                    break;
                p -= used;
                if (p < 0) {
                    atomicOr(&flags->err, ERR_LOOKBACK);
                    s_fail = 1;
                    break;
                }
                if (used == 0) {
                    if (++spins > SPIN_MAX) {
                        atomicOr(&flags->err, ERR_LOOKBACK);
                        s_fail = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            st_agent(my, st_pack(ST_INC, epoch, (uint64_t)excl + tot));
        }
        s_gbase[d] = (int64_t)bucket[d] + excl - (int64_t)s_tstart[d];
    }
    __syncthreads();

    uint32_t lpos[SORT_ITEMS];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        const uint32_t d = (uint32_t)(kw[j] >> shift) & 255u;
        lpos[j] = s_tstart[d] + s_wc[wave][d] + rank[j];
    }
    const int64_t rem = n - base;
    const int tile_n = rem < SORT_TILE ? (int)rem : SORT_TILE;
    if (s_fail)
        return;  // offsets are unknown: write nothing (the host reports the error)

    // scatter every plane through LDS
#pragma unroll
    for (int w = 0; w < W + 1; w++) {
#pragma unroll
        for (int j = 0; j < SORT_ITEMS; j++) {
            const int64_t idx = base + (int64_t)wave * 64 * SORT_ITEMS + j * 64 + lane;
            if (idx < n) {
                uint64_t v;
                if (w == word)
                    v = kw[j];
                else if (w < W)
                    v = plane_c<W>(in, w)[idx];
                else
                    v = PB == 8 ? ((const uint64_t *)in.pay)[idx] : (uint64_t)((const uint32_t *)in.pay)[idx];
                s_stage[lpos[j]] = v;
                if (w == 0)
                    s_dig[lpos[j]] = (uint8_t)((kw[j] >> shift) & 255u);
            }
        }
        __syncthreads();
        for (int q = tid; q < tile_n; q += SORT_THREADS) {
            const int64_t dst = s_gbase[s_dig[q]] + q;
            if ((uint64_t)dst >= (uint64_t)n) {
                atomicOr(&flags->err, ERR_LOOKBACK);
                continue;
            }
            const uint64_t v = s_stage[q];
            if (w < W)
                out.key[w][dst] = v;
            else if (PB == 8)
                ((uint64_t *)out.pay)[dst] = v;
            else
                ((uint32_t *)out.pay)[dst] = (uint32_t)v;
        }
        __syncthreads();
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
            out.key[w][i] = v;
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
            eq = eq && sorted.key[w][i] == sorted.key[w][i - 1];
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
            keys[i * W + w] = in.key[w][i];
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

hipError_t launch_onesweep(int W, int pay_bytes, const Planes &in, const Planes &out, int64_t n, int dig,
                           const uint64_t *bucket, uint64_t *status, uint32_t *tile_ctr, uint32_t epoch,
                           Flags *flags, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (tiles > 0xFFFFFFFFll)
        return hipErrorInvalidValue;
    dim3 g((unsigned)tiles), b(SORT_THREADS);
#define OS(WW, PB) hipLaunchKernelGGL((k_onesweep<WW, PB>), g, b, 0, st, in, out, n, dig, bucket, status, tile_ctr, \
                                      epoch, flags)
    const int key = W * 2 + (pay_bytes == 8 ? 1 : 0);
    switch (key) {
    case 2: OS(1, 4); break;
    case 3: OS(1, 8); break;
    case 4: OS(2, 4); break;
    case 5: OS(2, 8); break;
    case 6: OS(3, 4); break;
    case 7: OS(3, 8); break;
    case 8: OS(4, 4); break;
    case 9: OS(4, 8); break;
    default: return hipErrorInvalidValue;
    }
#undef OS
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
