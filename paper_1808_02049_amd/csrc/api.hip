// Host runtime of the PT2 engine: the C-ABI of include/pt2.h.
//
// A context holds one Hamiltonian resident in HBM.  An evaluation
//   1. copies / checks the reference determinants and sorts them (the sorted
//      list is what the single pass merges against);
//   2. plans the split of the external space (Algorithm 2): the record buffers
//      of one subset, two ping-pong copies of W key planes and a payload plane,
//      must fit the device budget; a count pass (the work list of Section V)
//      gives each subset's exact size when the split has more than one subset
//      or a cutoff drops terms;
//   3. per subset: generation -> LSD radix sort -> single pass;
//   4. sums the subsets in index order.
// The serving form queues requests from any context into one scheduler whose
// worker threads each own a stream and a workspace; a request starts when a
// worker is free and its projected record bytes fit the remaining budget.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pt2_internal.h"
#include "../../include/pt2.h"

#define PT2_API extern "C" __attribute__((visibility("default")))

using namespace pt2;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(PT2_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

uint64_t splitmix_next(uint64_t &st)
{
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// device memory through the optional hook

// A bump arena over a fixed device region: buffers are carved in order and
// never freed one by one (the whole arena is dropped after the call).
struct BumpArena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};

struct Alloc {
    void *(*fa)(size_t, void *) = nullptr;
    void (*ff)(void *, size_t, void *) = nullptr;
    void *user = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;  // non-null: stream-ordered allocation on this stream
    BumpArena *arena = nullptr;    // non-null: carve from this region, allocate nothing
    bool same_source(const Alloc &o) const { return fa == o.fa && ff == o.ff && user == o.user; }
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;  // a slice of the serving arena: never freed, only dropped
};

int buf_alloc(const Alloc &A, Buf &b, size_t bytes)
{
    b.p = nullptr;
    b.bytes = 0;
    if (bytes == 0)
        return PT2_OK;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (A.arena) {
        if (bytes > A.arena->cap - A.arena->used)
            return fail(PT2_E_NOMEM, "the evaluation needs more than the %zu MiB static scratch (%zu MiB in use, "
                                     "%zu more requested)",
                        A.arena->cap >> 20, A.arena->used >> 20, bytes >> 20);
        b.p = A.arena->base + A.arena->used;
        b.bytes = bytes;
        A.arena->used += bytes;
        return PT2_OK;
    }
    if (A.fa) {
        p = A.fa(bytes, A.user);
        if (!p)
            return fail(PT2_E_NOMEM, "allocator hook failed for %zu bytes", bytes);
    } else {
        hipError_t e = A.stream ? hipMallocAsync(&p, bytes, A.stream) : hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(PT2_E_NOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
    }
    b.p = p;
    b.bytes = bytes;
    return PT2_OK;
}

void buf_free(const Alloc &A, Buf &b)
{
    if (b.p && !b.borrowed && !A.arena) {
        if (A.ff) {
            // an external allocator may hand the block out at once: let every
            // queued kernel that might still use it finish first
            (void)hipDeviceSynchronize();
            A.ff(b.p, b.bytes, A.user);
        } else if (A.stream) {
            (void)hipFreeAsync(b.p, A.stream);
        } else {
            (void)hipFree(b.p);
        }
    }
    b.p = nullptr;
    b.bytes = 0;
    b.borrowed = false;
}

int buf_ensure(const Alloc &A, Buf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p)
        return PT2_OK;
    buf_free(A, b);
    return buf_alloc(A, b, bytes);
}

// ---------------------------------------------------------------------------
// per-stream workspace

constexpr int MAX_DIG = 32;
constexpr int MAX_LOG2P = 12;  // the count pass keeps one LDS counter per subset
constexpr int MAX_PASS_CTR = 64;

struct Small {  // one device block for small control data
    Flags flags;
    uint32_t tile_ctr[MAX_PASS_CTR];
    uint64_t hist[MAX_DIG * 256];
    uint64_t bucket[MAX_DIG * 256];
    Partial partials[RED_GRID];
    CollList coll[RED_GRID];  // hash records: collided segments per single-pass workgroup
    Partial result;
    unsigned long long n_out;
    AnchorBlk anc;            // the anchor of the diagonals (one evaluation)
    uint32_t ref_far;         // hash records: most flips of a reference from the first, when beyond four
    uint32_t pad2;
};

struct Workspace {
    Alloc A;
    Buf dets, coef;          // device copies of host inputs
    Buf refA, refB;          // reference planes (W keys + FP64 coefficient)
    Buf refK;                // the references' rank keys (same order) when records carry them
    Buf tref;                // reference range of every single-pass tile
    Buf refH0, refH1;        // hash records: reference hashes with indices (sort ping-pong)
    Buf hp, gv;              // hash records: E0 - energy and g vector of every reference (double-double)
    Buf refX;                // hash records: reference bitstrings record by record
    Buf refE;                // hash records: references as flips relative to the first (compact)
    Buf recA, recB;          // record planes
    int64_t rec_cap = 0;
    int rec_W = 0, rec_pb = 0, rec_topb = 0;
    Buf counts, csum, coff, offs;  // per-tile digit counts (u16), chunk offsets (u64), in-chunk offsets (u32)
    int64_t scan_tiles = 0;
    Buf small;
    Buf cnt, off, tot, parts_dev;
    Buf bkt;                 // targeted generation: every reference's bucket table for the call's split
    Buf agrp;                              // groups of references sharing a spin string (spin_groups)
    std::vector<uint64_t> agrp_keys;       // host copy of the sorted reference keys, for grouping
    std::vector<uint32_t> agrp_host;       // source of the last upload of agrp
    int64_t agrp_ngrp = 0;                 // alpha plus beta groups in agrp
    Small *host_small = nullptr;  // pinned mirror
    bool own_host_small = true;   // false: static host storage (allocation-free evaluation)
    std::vector<hipEvent_t> evpool;
    size_t ev_used = 0;
    hipStream_t zero_stream = nullptr;  // allocation-free evaluation: the stream that clears `small`

    ~Workspace() { release(); }

    void release()
    {
        buf_free(A, dets), buf_free(A, coef), buf_free(A, refA), buf_free(A, refB), buf_free(A, refK);
        buf_free(A, tref), buf_free(A, refH0), buf_free(A, refH1), buf_free(A, hp), buf_free(A, gv), buf_free(A, refX), buf_free(A, refE);
        buf_free(A, recA), buf_free(A, recB), buf_free(A, small);
        buf_free(A, counts), buf_free(A, csum), buf_free(A, coff), buf_free(A, offs);
        buf_free(A, cnt), buf_free(A, off), buf_free(A, tot), buf_free(A, parts_dev), buf_free(A, agrp);
        buf_free(A, bkt);
        rec_cap = scan_tiles = 0;
        if (host_small && own_host_small)
            (void)hipHostFree(host_small);
        host_small = nullptr;
        for (auto e : evpool)
            (void)hipEventDestroy(e);
        evpool.clear();
    }

    size_t record_bytes() const { return recA.bytes + recB.bytes + counts.bytes + offs.bytes; }

    Small *dsmall() { return (Small *)small.p; }

    hipEvent_t event()
    {
        if (ev_used == evpool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess)
                return nullptr;
            evpool.push_back(e);
        }
        return evpool[ev_used++];
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// W-1 uint64 planes, then the last key plane of topb-byte elements, then the
// payload plane; every plane starts on a 256-byte boundary.
Planes planes_of(const Buf &b, int W, int64_t cap, int pb, int topb)
{
    Planes p;
    char *base = (char *)b.p;
    size_t o = 0;
    for (int w = 0; w < MAXW; w++) {
        p.key[w] = nullptr;
        if (w < W) {
            p.key[w] = (uint64_t *)(base + o);
            o += align256((size_t)cap * (w == W - 1 ? topb : 8));
        }
    }
    p.pay = base + o;
    p.topb = topb;
    (void)pb;
    return p;
}

size_t planes_bytes(int W, int64_t cap, int pb, int topb)
{
    return align256((size_t)cap * 8) * (W - 1) + align256((size_t)cap * topb) + align256((size_t)cap * pb);
}

// bytes of one record: W-1 full key words, the narrow top word, the payload
double record_bytes(int W, int pb, int topb) { return 8.0 * (W - 1) + topb + pb; }

}  // namespace

// ---------------------------------------------------------------------------
// context

struct pt2_ctx {
    pt2_options opt;
    int norb, na, nb, W;
    int topb;  // bytes of the last key plane of a record
    Alloc A;
    Buf h, V, h32, V32, T, Tlo, R, binom, A2;
    DevSys sys;
    ExcLayout L;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    std::mutex mu;  // serialises pt2_evaluate* on this context
    Workspace ws;
    int inflight = 0;  // serving requests not yet polled out (guarded by the scheduler lock)
};

namespace {

struct Timing {
    bool on = false;
    struct Ev {
        hipEvent_t a, b;
        int kind;  // 0 gen, 1 radix scatter, 2 reduce, 3 hist/other, 4 radix count+scan
    };
    std::vector<Ev> evs;
};

int timed_begin(Workspace &ws, Timing &t, hipStream_t st, hipEvent_t &a)
{
    a = nullptr;
    if (!t.on)
        return PT2_OK;
    a = ws.event();
    if (!a)
        return fail(PT2_E_DEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(a, st));
    return PT2_OK;
}

int timed_end(Workspace &ws, Timing &t, hipStream_t st, hipEvent_t a, int kind)
{
    if (!t.on)
        return PT2_OK;
    hipEvent_t b = ws.event();
    if (!b)
        return fail(PT2_E_DEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(b, st));
    t.evs.push_back({a, b, kind});
    return PT2_OK;
}

int ensure_small(Workspace &ws)
{
    if (!ws.small.p) {
        int rc = buf_alloc(ws.A, ws.small, sizeof(Small));
        if (rc)
            return rc;
        // cleared in the order of the stream that allocated it: a block of the
        // stream-ordered pool may have been freed by another stream whose
        // earlier kernels still use it, which only that stream waits for
        static_assert(sizeof(Small) % 8 == 0, "Small is cleared in 8-byte words");
        if (ws.A.stream)
            HIPCHK(launch_zero_u64((uint64_t *)ws.small.p, (int64_t)(sizeof(Small) / 8), ws.A.stream));
        else if (ws.A.arena)  // cleared on the evaluation's stream (ensure_small's caller passes it)
            HIPCHK(launch_zero_u64((uint64_t *)ws.small.p, (int64_t)(sizeof(Small) / 8), ws.zero_stream));
        else
            HIPCHK(hipMemset(ws.small.p, 0, sizeof(Small)));
    }
    if (!ws.host_small)
        HIPCHK(hipHostMalloc((void **)&ws.host_small, sizeof(Small), hipHostMallocDefault));
    return PT2_OK;
}

int ensure_scan(Workspace &ws, int64_t n)
{
    int64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (tiles < 1)
        tiles = 1;
    if (ws.scan_tiles < tiles) {
        buf_free(ws.A, ws.counts), buf_free(ws.A, ws.csum), buf_free(ws.A, ws.coff), buf_free(ws.A, ws.offs);
        ws.scan_tiles = 0;
        const int64_t chunks = (tiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
        int rc;
        if ((rc = buf_alloc(ws.A, ws.counts, (size_t)tiles * 256 * 2)) ||
            (rc = buf_alloc(ws.A, ws.offs, (size_t)tiles * 256 * 4)) ||
            (rc = buf_alloc(ws.A, ws.csum, (size_t)(chunks + 1) * 256 * 8)) ||
            (rc = buf_alloc(ws.A, ws.coff, (size_t)chunks * 256 * 8)))
            return rc;
        ws.scan_tiles = tiles;
    }
    return PT2_OK;
}

// Record and scan buffers of a request whose largest subset holds cap records
// (what ensure_records and ensure_scan allocate), as one slice.
size_t slice_bytes(int W, int pb, int topb, int64_t cap)
{
    const int64_t tiles = std::max<int64_t>(1, (cap + SORT_TILE - 1) / SORT_TILE);
    const int64_t chunks = (tiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return 2 * planes_bytes(W, cap, pb, topb) + align256((size_t)tiles * 256 * 2) +
           align256((size_t)tiles * 256 * 4) + align256((size_t)(chunks + 1) * 256 * 8) +
           align256((size_t)chunks * 256 * 8);
}

// Point a workspace's record and scan buffers into a slice of slice_bytes().
void carve_slice(Workspace &ws, char *p, int W, int pb, int topb, int64_t cap)
{
    const int64_t tiles = std::max<int64_t>(1, (cap + SORT_TILE - 1) / SORT_TILE);
    const int64_t chunks = (tiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    auto take = [&](Buf &b, size_t bytes) {
        buf_free(ws.A, b);
        b.p = p, b.bytes = bytes, b.borrowed = true;
        p += bytes;
    };
    take(ws.recA, planes_bytes(W, cap, pb, topb));
    take(ws.recB, planes_bytes(W, cap, pb, topb));
    take(ws.counts, align256((size_t)tiles * 256 * 2));
    take(ws.offs, align256((size_t)tiles * 256 * 4));
    take(ws.csum, align256((size_t)(chunks + 1) * 256 * 8));  // the last row: the digits' totals
    take(ws.coff, align256((size_t)chunks * 256 * 8));
    ws.rec_cap = cap, ws.rec_W = W, ws.rec_pb = pb, ws.rec_topb = topb;
    ws.scan_tiles = tiles;
}

// Stable LSD sort of n records held in *src (ping-pong with *dst) on key bits
// [0, nbits).  On return *src holds the sorted records.
// digits: when nonzero, the bit mask of the digit positions to sort (the
// others are known to hold one value): no all-digit histogram pass, and each
// pass takes its bucket starts from its own tile counts.
int radix_sort(Workspace &ws, int W, int pb, Planes &src, Planes &dst, int64_t n, int nbits, hipStream_t st,
               Timing &tm, uint32_t *passes_out, double *bytes_out, int items = SORT_ITEMS, uint32_t digits = 0)
{
    if (n <= 1)
        return PT2_OK;
    const int ndig = (nbits + 7) / 8;
    if (ndig > MAX_DIG)
        return fail(PT2_E_INVALID, "key too long");
    int rc = ensure_scan(ws, n);
    if (rc)
        return rc;
    Small *ds = ws.dsmall();
    if (!digits) {
        hipEvent_t a;
        if ((rc = timed_begin(ws, tm, st, a)))
            return rc;
        HIPCHK(launch_zero_u64(ds->hist, ndig * 256, st));
        HIPCHK(launch_hist(W, src, n, ndig, ds->hist, st));
        HIPCHK(launch_hist_scan(ds->hist, ndig, ds->bucket, st));
        HIPCHK(hipMemcpyAsync(ws.host_small->hist, ds->hist, sizeof(uint64_t) * ndig * 256, hipMemcpyDeviceToHost,
                              st));
        if ((rc = timed_end(ws, tm, st, a, 3)))
            return rc;
        HIPCHK(hipStreamSynchronize(st));
    }
    for (int d = 0; d < ndig; d++) {
        if (digits) {
            if (!((digits >> d) & 1u))
                continue;
        } else {
            const uint64_t *h = ws.host_small->hist + d * 256;
            bool trivial = false;
            for (int v = 0; v < 256; v++)
                if (h[v] == (uint64_t)n)
                    trivial = true;
            if (trivial)
                continue;
        }
        hipEvent_t pa, mid = nullptr;
        if ((rc = timed_begin(ws, tm, st, pa)))
            return rc;
        if (tm.on && !(mid = ws.event()))
            return fail(PT2_E_DEVICE, "hipEventCreate failed");
        HIPCHK(launch_radix_pass(W, pb, src, dst, n, d, digits ? nullptr : ds->bucket + d * 256, (uint16_t *)ws.counts.p,
                                 (uint64_t *)ws.csum.p, (uint64_t *)ws.coff.p, (uint32_t *)ws.offs.p, &ds->flags,
                                 st, mid, items));
        if (tm.on) {
            if ((rc = timed_end(ws, tm, st, mid, 1)))
                return rc;
            tm.evs.push_back({pa, mid, 4});
        }
        std::swap(src, dst);
        if (passes_out)
            (*passes_out)++;
        if (bytes_out)
            *bytes_out += 2.0 * (double)n * record_bytes(W, pb, src.topb) +
                          (double)n * ((d >> 3) == W - 1 ? src.topb : 8);
    }
    return PT2_OK;
}

// Upload (if host), check and sort the reference list.  On success refs holds
// the sorted reference planes (keys + FP64 coefficients).
int prepare_refs(pt2_ctx *c, Workspace &ws, const uint64_t *dets, const double *coeffs, int64_t n, bool host,
                 hipStream_t st, Timing &tm, Planes &refs)
{
    const int W = c->W;
    int rc;
    if ((rc = ensure_small(ws)))
        return rc;
    if (host) {
        if ((rc = buf_ensure(ws.A, ws.dets, (size_t)n * W * 8)) || (rc = buf_ensure(ws.A, ws.coef, (size_t)n * 8)))
            return rc;
        HIPCHK(hipMemcpyAsync(ws.dets.p, dets, (size_t)n * W * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ws.coef.p, coeffs, (size_t)n * 8, hipMemcpyHostToDevice, st));
        dets = (const uint64_t *)ws.dets.p;
        coeffs = (const double *)ws.coef.p;
    }
    // sized in bytes: a workspace serves contexts of different key widths
    if ((rc = buf_ensure(ws.A, ws.refA, planes_bytes(W, n, 8, 8))) ||
        (rc = buf_ensure(ws.A, ws.refB, planes_bytes(W, n, 8, 8))))
        return rc;
    Small *ds = ws.dsmall();
    HIPCHK(launch_zero_u32(&ds->flags.err, 2, st));
    // plane stride = n: the generation kernel indexes reference planes by nref
    Planes ra = planes_of(ws.refA, W, n, 8, 8), rb = planes_of(ws.refB, W, n, 8, 8);
    HIPCHK(launch_refs_split(W, c->norb, c->na, c->nb, dets, coeffs, n, ra, &ds->flags, st));
    Timing none;
    if ((rc = radix_sort(ws, W, 8, ra, rb, n, 2 * c->norb, st, none, nullptr, nullptr)))
        return rc;
    HIPCHK(launch_dup_check(W, ra, n, &ds->flags, st));
    HIPCHK(hipMemcpyAsync(&ws.host_small->flags, &ds->flags, sizeof(Flags), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint32_t err = ws.host_small->flags.err;
    if (err & ERR_POPCOUNT)
        return fail(PT2_E_INVALID, "a reference determinant does not have %d alpha and %d beta electrons", c->na,
                    c->nb);
    if (err & ERR_STRAY_BITS)
        return fail(PT2_E_INVALID, "a reference determinant has bits at or above 2*norb");
    if (err & ERR_DUPLICATE)
        return fail(PT2_E_INVALID, "duplicate reference determinants");
    if (err & ERR_BOUNDS)
        return fail(PT2_E_DEVICE, "radix scatter destination out of range");
    refs = ra;
    (void)tm;
    return PT2_OK;
}

int ensure_records(Workspace &ws, int W, int pb, int topb, int64_t cap)
{
    if (ws.rec_cap >= cap && ws.rec_W == W && ws.rec_pb == pb && ws.rec_topb == topb)
        return PT2_OK;
    buf_free(ws.A, ws.recA), buf_free(ws.A, ws.recB);
    ws.rec_cap = 0;
    int rc;
    if ((rc = buf_alloc(ws.A, ws.recA, planes_bytes(W, cap, pb, topb))) ||
        (rc = buf_alloc(ws.A, ws.recB, planes_bytes(W, cap, pb, topb)))) {
        buf_free(ws.A, ws.recA), buf_free(ws.A, ws.recB);
        return rc;
    }
    ws.rec_cap = cap, ws.rec_W = W, ws.rec_pb = pb, ws.rec_topb = topb;
    return PT2_OK;
}

// projected device bytes for one subset of n records
// (two record buffers, plus per-tile counts and offsets: 6 B per digit value
// per tile of SORT_TILE records)
double subset_bytes(int W, int pb, int topb, double n)
{
    return n * (2.0 * record_bytes(W, pb, topb) + 6.0 * 256.0 / SORT_TILE) + 65536.0;
}

struct Plan {
    int log2p = 0;
    bool compact = false;
    bool target = false;  // targeted count/generation, one determinant per chunk
    int64_t chunk = 0, nchunks = 0;
    std::vector<uint32_t> parts;
    std::vector<uint64_t> sizes;  // records per listed subset
    std::vector<uint64_t> structural;  // structural candidates per listed subset
    uint64_t cap_hint = 0;  // record capacity for any subset of the split (0: the listed ones' largest)
    const uint16_t *bk = nullptr;  // bucket tables of the targeted generation (null: built per subset)
};

struct Job {
    const uint64_t *dets;
    const double *coeffs;
    int64_t n;
    bool host;
    double e0;
    int forced_log2p;              // -1 planner
    bool live_budget = false;      // plan against free memory now, not at creation
    double plan_budget = 0.0;      // > 0: plan against this many bytes
    const uint32_t *parts = nullptr;
    int nparts = 0;
    double *e_parts = nullptr;
    // inspection
    int dump = 0;                  // 1 records (generation order), 2 records sorted, 3 numerators
    uint64_t *keys_out = nullptr;
    double *vals_out = nullptr;
    uint8_t *inref_out = nullptr;
    int64_t cap = 0;
    int64_t *n_out = nullptr;
};

// Key format of the stored terms of one job: rank keys when the context
// enables them (not for the inspection dumps, which return bitstrings).
struct RecLayout {
    int W, topb, bits;
    bool rank;    // rank keys
    bool hash;    // hash records: (hash, parent and flips, payload), sorted on the hash
    int pb;       // bytes of the payload plane (0: packed into the key words)
    bool packed;  // FP32 hash records packed into two 8-byte words (hash_pack)
};

// nref: references of the job (packed hash records hold parents below
// HC_MAX_REFS)
RecLayout rec_layout(const pt2_ctx *c, bool dump, int64_t nref)
{
    const int pb = c->opt.precision != PT2_FP64 ? 4 : 8;
    if (c->sys.kc.hash && !dump) {
        if (pb == 4 && c->opt.hash_bits == 0 && c->norb <= HC_MAX_NORB && nref <= HC_MAX_REFS)
            return {2, 8, 64, false, true, 0, true};
        return {2, 8, 64, false, true, pb, false};
    }
    if (c->sys.kc.on && !dump)
        return {c->sys.kc.kw, c->sys.kc.ktop, c->sys.kc.kbits, true, false, pb, false};
    return {c->W, c->topb, 2 * c->norb, false, false, pb, false};
}

int count_pass(pt2_ctx *c, const DevSys &sys, const ExcLayout &L, Workspace &ws, const Planes &refs, int64_t nref,
               Plan &P, double cutoff, hipStream_t st, std::vector<uint64_t> &tot_out)
{
    int rc;
    const int Pn = 1 << P.log2p;
    const int pm = c->opt.precision;
    // the bucketed count takes only the listed subsets (with a cutoff or the
    // spin flip: their bucket walks with the filter); without bucketing, the
    // enumerating count takes every subset
    const bool listed = P.target && ((cutoff <= 0.0 && !sys.z2) ||
                                     count_cut_ok(L, nref, P.log2p, (int)P.parts.size()));
    const size_t ncols = listed ? P.parts.size() : (size_t)Pn;
    if ((rc = buf_ensure(ws.A, ws.cnt, (size_t)P.nchunks * ncols * 4)))
        return rc;
    if ((rc = buf_ensure(ws.A, ws.off, (size_t)P.nchunks * P.parts.size() * 8)) ||
        (rc = buf_ensure(ws.A, ws.tot, P.parts.size() * 8)) ||
        (rc = buf_ensure(ws.A, ws.parts_dev, P.parts.size() * 4)))
        return rc;
    HIPCHK(hipMemcpyAsync(ws.parts_dev.p, P.parts.data(), P.parts.size() * 4, hipMemcpyHostToDevice, st));
    if (listed && cutoff <= 0.0 && !sys.z2)
        HIPCHK(launch_count_target(sys, L, refs, nref, P.log2p, (const uint32_t *)ws.parts_dev.p,
                                   (int)P.parts.size(), (uint32_t *)ws.cnt.p, P.bk, st));
    else if (listed)
        HIPCHK(launch_count_target_cut(sys, L, pm, refs, nref, P.log2p, (const uint32_t *)ws.parts_dev.p,
                                       (int)P.parts.size(), cutoff, (uint32_t *)ws.cnt.p, st));
    else
        HIPCHK(launch_count(sys, L, pm, refs, nref, P.chunk, P.log2p, cutoff, (uint32_t *)ws.cnt.p, P.nchunks, st));
    HIPCHK(launch_chunk_scan((const uint32_t *)ws.cnt.p, P.nchunks, listed ? nullptr : (const uint32_t *)ws.parts_dev.p,
                             (int)P.parts.size(), (uint64_t *)ws.off.p, (uint64_t *)ws.tot.p, st));
    tot_out.assign(P.parts.size(), 0);
    HIPCHK(hipMemcpyAsync(tot_out.data(), ws.tot.p, P.parts.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PT2_OK;
}

double serving_device_budget(int dev);

int plan_job(pt2_ctx *c, const DevSys &sys, const ExcLayout &L, const RecLayout &RL, Workspace &ws,
             const Planes &refs, int64_t nref, const Job &J, hipStream_t st, Plan &P)
{
    const int W = RL.W;
    const int pb = RL.pb;
    const double total = (double)nref * (double)L.nper;
    uint64_t budget = J.plan_budget > 0.0 ? (uint64_t)J.plan_budget : c->budget;
    if (!c->opt.device_budget_bytes && J.live_budget) {
        // without an explicit budget: the budget the scheduler plans served
        // requests against (80% of what was free when the device was first
        // used), so that a request evaluated alone takes the plan, and with it
        // the summation order, it takes when served; unless less is free now
        // (80% of the free memory plus the record buffers this workspace
        // already holds, which are reused)
        budget = (uint64_t)serving_device_budget(c->opt.device);
        size_t freeb = 0, totalb = 0;
        if (hipMemGetInfo(&freeb, &totalb) == hipSuccess)
            budget = std::min<uint64_t>(budget, (uint64_t)(0.8 * ((double)freeb + (double)ws.record_bytes())));
    }
    const double cap_bytes =
        (double)(c->opt.max_partition_bytes && c->opt.max_partition_bytes < budget ? c->opt.max_partition_bytes
                                                                                  : budget);
    const double cutoff = c->opt.cutoff;
    int k;
    if (J.forced_log2p >= 0)
        k = J.forced_log2p;
    else if (c->opt.log2_partitions >= 0)
        k = c->opt.log2_partitions;
    else {
        k = 0;
        while (k < MAX_LOG2P && subset_bytes(W, pb, RL.topb, total / (double)(1 << k) * 1.02 + 4096.0) > cap_bytes)
            k++;
    }
    for (int attempt = 0; attempt < 4; attempt++) {
        if (k > MAX_LOG2P)
            return fail(PT2_E_NOMEM, "no split of at most 2^%d subsets fits the device budget", MAX_LOG2P);
        P.log2p = k;
        // a cutoff or the spin flip filter terms: counted by enumeration
        const bool filtered = cutoff > 0.0 || sys.z2;
        P.compact = k > 0 || filtered;
        P.parts.clear();
        if (J.parts) {
            for (int i = 0; i < J.nparts; i++) {
                if (J.parts[i] >= (1u << k))
                    return fail(PT2_E_INVALID, "subset index %u out of range", J.parts[i]);
                P.parts.push_back(J.parts[i]);
            }
            std::vector<uint32_t> u(P.parts);
            std::sort(u.begin(), u.end());
            if (std::adjacent_find(u.begin(), u.end()) != u.end())
                return fail(PT2_E_INVALID, "subset %u is listed twice", *std::adjacent_find(u.begin(), u.end()));
        } else {
            for (uint32_t p = 0; p < (1u << k); p++)
                P.parts.push_back(p);
        }
        if (!P.compact) {
            P.chunk = gen_chunk(L, nref, (int64_t)1 << 23);
            P.nchunks = gen_nchunks(L, nref, P.chunk);
            P.sizes.assign(1, (uint64_t)nref * (uint64_t)L.nper);
            P.structural = P.sizes;
            return PT2_OK;
        }
        P.target = target_ok(L, nref, k);
        P.bk = nullptr;
        if (P.target) {
            P.chunk = std::max<int64_t>(L.nper, 1);
            P.nchunks = nref;
            // the references' bucket tables, built once for the call's
            // subsets, when they take at most 1/32 of the budget (the record
            // buffers are planned against the rest); not from the static
            // scratch of the allocation-free entry point
            const double bk_bytes = (double)nref * (double)gen_bucket_words(L, k) * 2.0;
            if (!ws.A.arena && gen_buckets_ok(L, k) && bk_bytes <= cap_bytes / 32.0) {
                int rc0;
                if ((rc0 = buf_ensure(ws.A, ws.bkt, (size_t)bk_bytes)))
                    return rc0;
                HIPCHK(launch_gen_buckets(sys, L, refs, nref, k, (uint16_t *)ws.bkt.p, st));
                P.bk = (const uint16_t *)ws.bkt.p;
            }
        } else {
            const int64_t max_chunks =
                std::max<int64_t>(1, std::min<int64_t>((int64_t)1 << 23, ((int64_t)1 << 27) >> k));
            P.chunk = gen_chunk(L, nref, max_chunks);
            P.nchunks = gen_nchunks(L, nref, P.chunk);
        }
        int rc;
        std::vector<uint64_t> tot;
        if (filtered) {
            // structural count: every term, no cutoff, no spin flip filter
            DevSys s0 = sys;
            s0.z2 = 0;
            if ((rc = count_pass(c, s0, L, ws, refs, nref, P, 0.0, st, tot)))
                return rc;
            P.structural = tot;
        }
        if ((rc = count_pass(c, sys, L, ws, refs, nref, P, cutoff, st, tot)))
            return rc;
        P.sizes = tot;
        if (!filtered)
            P.structural = tot;
        uint64_t mx = 0;
        for (auto t : tot)
            mx = std::max(mx, t);
        if (subset_bytes(W, pb, RL.topb, (double)mx) <= cap_bytes || J.forced_log2p >= 0 || c->opt.log2_partitions >= 0) {
            // record buffers sized for the split's expected subset (as the
            // planner projects it), so that later calls listing other
            // subsets of the same split reuse them instead of growing them
            const double want = total / (double)(1 << k) * 1.02 + 4096.0;
            if ((double)mx < want && subset_bytes(W, pb, RL.topb, want) <= cap_bytes)
                P.cap_hint = (uint64_t)want;
            return PT2_OK;
        }
        k++;
    }
    return fail(PT2_E_NOMEM, "planner could not fit a subset into the device budget");
}

void fill_result(pt2_result *out, const Partial &p)
{
    out->e_pt2 = p.e_sum + p.e_comp;
    out->n_unique = p.n_unique;
    out->n_external = p.n_external;
    out->n_in_ref_hit = p.n_hit;
    out->min_abs_denom = p.min_abs_denom;
    out->n_nonneg_denom = p.n_nonneg;
    out->ref_cross = p.ref_cross;
    out->key_xor = p.key_xor;
    out->key_sum = p.key_sum;
}

// Groups of at most REUSE_GROUP references that share their alpha string
// (bits [norb, 2 norb) of the key; consecutive in the sorted reference) and
// if beta, groups that share their beta string (bits [0, norb); from a stable
// sort of the reference by beta string), for k_gen_spin.  Uploaded to ws.agrp
// as u32: the nga alpha (start, count) pairs, the ngb beta pairs, then the
// alpha and the beta member lists (n indices each) that the starts point into.
int spin_groups(Workspace &ws, const Planes &refs, int W, int norb, int64_t n, bool beta, hipStream_t st,
                int64_t &nga, int64_t &ngb)
{
    nga = ngb = 0;
    if (n <= 0 || n > 0x7FFFFFFFll)
        return PT2_OK;
    ws.agrp_keys.resize((size_t)n * W);
    for (int w = 0; w < W; w++)
        HIPCHK(hipMemcpyAsync(ws.agrp_keys.data() + (size_t)w * n, refs.key[w], (size_t)n * 8,
                              hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    uint64_t am[MAXW] = {}, bm[MAXW] = {};
    for (int b = 0; b < 2 * norb; b++)
        (b < norb ? bm : am)[b >> 6] |= 1ull << (b & 63);
    const uint64_t *K = ws.agrp_keys.data();
    auto word = [&](int64_t i, int w) { return K[(size_t)w * n + i]; };
    auto same = [&](int64_t i, int64_t j, const uint64_t *mask) {
        for (int w = 0; w < W; w++)
            if ((word(i, w) ^ word(j, w)) & mask[w])
                return false;
        return true;
    };
    std::vector<uint32_t> ia((size_t)n), ib;
    for (int64_t i = 0; i < n; i++)
        ia[(size_t)i] = (uint32_t)i;
    if (beta)
        ib = ia;
    std::stable_sort(ib.begin(), ib.end(), [&](uint32_t x, uint32_t y) {
        for (int w = W - 1; w >= 0; w--) {
            const uint64_t a = word(x, w) & bm[w], b = word(y, w) & bm[w];
            if (a != b)
                return a < b;
        }
        return false;
    });
    std::vector<uint32_t> ga, gb;
    auto cut = [&](const std::vector<uint32_t> &ord, const uint64_t *mask, std::vector<uint32_t> &grp) {
        int64_t first = 0;
        for (int64_t i = 1; i <= n; i++) {
            if (i < n && i - first < REUSE_GROUP && same(ord[(size_t)i], ord[(size_t)first], mask))
                continue;
            grp.push_back((uint32_t)first);
            grp.push_back((uint32_t)(i - first));
            first = i;
        }
    };
    cut(ia, am, ga);
    if (beta)
        cut(ib, bm, gb);
    nga = (int64_t)ga.size() / 2, ngb = (int64_t)gb.size() / 2;
    ws.agrp_ngrp = nga + ngb;
    ws.agrp_host = ga;
    ws.agrp_host.insert(ws.agrp_host.end(), gb.begin(), gb.end());
    ws.agrp_host.insert(ws.agrp_host.end(), ia.begin(), ia.end());
    ws.agrp_host.insert(ws.agrp_host.end(), ib.begin(), ib.end());
    int rc;
    if ((rc = buf_ensure(ws.A, ws.agrp, ws.agrp_host.size() * 4)))
        return rc;
    HIPCHK(hipMemcpyAsync(ws.agrp.p, ws.agrp_host.data(), ws.agrp_host.size() * 4, hipMemcpyHostToDevice, st));
    return PT2_OK;
}

int run_job(pt2_ctx *c, Workspace &ws, hipStream_t st, const Job &J, pt2_result *out)
{
    const double t0 = now_ms();
    const RecLayout RL = rec_layout(c, J.dump != 0, J.n);
    const int W = RL.W;  // key words of a stored term
    const bool subtract = c->opt.exclusion == PT2_EXCLUDE_SUBTRACT && !J.dump;
    DevSys sys = c->sys;
    ExcLayout L = c->L;
    if (!RL.rank)
        sys.kc.on = 0, L.rank = 0;
    if (!RL.hash)
        sys.kc.hash = 0;
    sys.kc.hpacked = RL.packed ? 1 : 0;
    const int pm = c->opt.precision;
    const int fp32 = pm != PT2_FP64;  // FP32 payloads
    const int pb = RL.pb;             // bytes of the payload plane
    int rc;
    Timing tm;
    tm.on = c->opt.timing != 0 && !ws.A.arena;  // no events are created without allocation
    ws.ev_used = 0;
    pt2_result res;
    memset(&res, 0, sizeof res);
    res.struct_size = sizeof(pt2_result);
    res.min_abs_denom = __builtin_inf();
    if (J.n == 0) {
        if (J.e_parts)
            for (int i = 0; i < J.nparts; i++)
                J.e_parts[i] = 0.0;
        if (J.n_out)
            *J.n_out = 0;
        res.ms_total = now_ms() - t0;
        memcpy(out, &res, sizeof res);
        return PT2_OK;
    }
    Planes refs;
    if ((rc = prepare_refs(c, ws, J.dets, J.coeffs, J.n, J.host, st, tm, refs)))
        return rc;
    if (sys.z2) {
        // the spin flip is exact only for a reference closed under the swap
        Small *d0 = ws.dsmall();
        HIPCHK(launch_zero_u32(&d0->flags.err, 2, st));
        HIPCHK(launch_check_swap(sys, refs, J.n, &d0->flags, st));
        HIPCHK(hipMemcpyAsync(&ws.host_small->flags, &d0->flags, sizeof(Flags), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const uint32_t f = ws.host_small->flags.err;
        if ((f & ERR_SWAP_MISSING) || ((f & SWAP_SAME) && (f & SWAP_NEG)))
            return fail(PT2_E_INVALID, "spin_flip needs a reference closed under the alpha/beta swap, with "
                                       "c(swap(D)) = c(D) for all D or -c(D) for all D");
        HIPCHK(launch_zero_u32(&d0->flags.err, 2, st));
    }
    // the single pass compares stored keys with reference keys of the same format
    Planes refs_red = refs;
    if (RL.rank) {
        if ((rc = buf_ensure(ws.A, ws.refK, planes_bytes(W, J.n, 8, RL.topb))))
            return rc;
        refs_red = planes_of(ws.refK, W, J.n, 8, RL.topb);
        HIPCHK(launch_refs_rank(sys, refs, J.n, refs_red, st));
    }
    // hash records: the references' hashes sorted, with their indices, and
    // every reference's energy and g vector (H_aa is taken from the parent)
    Planes refs_hash{};
    uint32_t hash_digits = 0;  // digit positions a hash-record sort must take (0: from histograms)
    uint64_t anc_hash[MAXW] = {0, 0, 0, 0};
    bool ref_compact = false, ref_compact4 = false;
    const uint32_t *ref_ex4 = nullptr;
    if (RL.hash) {
        if (J.n >= ((int64_t)1 << 32))
            return fail(PT2_E_INVALID, "hash records take fewer than 2^32 reference determinants");
        const int nso = 2 * c->norb;
        if ((rc = buf_ensure(ws.A, ws.refH0, planes_bytes(1, J.n, 8, 8))) ||
            (rc = buf_ensure(ws.A, ws.refH1, planes_bytes(1, J.n, 8, 8))) ||
            (rc = buf_ensure(ws.A, ws.hp, (size_t)J.n * 16)) ||
            (rc = buf_ensure(ws.A, ws.gv, (size_t)J.n * nso * 16)) ||
            (rc = buf_ensure(ws.A, ws.refX, (size_t)J.n * (c->W == 3 ? 4 : c->W) * 8)))
            return rc;
        HIPCHK(launch_refs_aos(sys, refs, J.n, (uint64_t *)ws.refX.p, st));
        HIPCHK(launch_parent_g(sys, refs, J.n, J.e0, (double *)ws.hp.p, (double *)ws.gv.p, st));
        // the compact forms of the same table: 8 bytes per reference when
        // every reference is within four excitations of the first, 4 bytes
        // within two (the single pass reads one entry per record)
        const size_t ex_bytes = ((size_t)std::max<int64_t>(J.n, 1) * 8 + 255) & ~(size_t)255;
        if ((rc = buf_ensure(ws.A, ws.refE, ex_bytes + (size_t)std::max<int64_t>(J.n, 1) * 4)))
            return rc;
        Small *d0 = ws.dsmall();
        HIPCHK(launch_zero_u32(&d0->ref_far, 1, st));
        HIPCHK(launch_refs_ex(sys, refs, J.n, (uint64_t *)ws.refE.p, (uint32_t *)((char *)ws.refE.p + ex_bytes),
                              d0->anc.bits, &d0->ref_far, st));
        HIPCHK(hipMemcpyAsync(ws.host_small->anc.bits, d0->anc.bits, sizeof(d0->anc.bits), hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(&ws.host_small->ref_far, &d0->ref_far, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int w = 0; w < MAXW; w++)
            anc_hash[w] = ws.host_small->anc.bits[w];
        ref_compact = ws.host_small->ref_far <= 8 && c->opt.compact_refs != 0;
        ref_compact4 = ws.host_small->ref_far <= 4 && c->opt.compact_refs != 0;
        ref_ex4 = (const uint32_t *)((const char *)ws.refE.p + ex_bytes);
    }
    // the anchor of the diagonals of bitstring and rank-key records: the first
    // sorted reference, its energy and g vector, and its hot pair rows (their
    // count sizes the single pass's LDS); hash records take each diagonal
    // relative to the record's parent instead
    int anc_nh = 0;
    if (!RL.hash) {
        Small *d0 = ws.dsmall();
        HIPCHK(launch_anchor(sys, refs, J.n, J.e0, &d0->anc, st));
        HIPCHK(hipMemcpyAsync(&ws.host_small->anc.nh, &d0->anc.nh, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        anc_nh = ws.host_small->anc.nh;
    }
    // subtraction form: sum_i c_i^2 (E0 - H_ii), removed from the total below
    double ref_terms = 0.0;
    if (subtract) {
        Small *d0 = ws.dsmall();
        HIPCHK(launch_ref_terms(sys, refs, J.n, J.e0, d0->partials, &d0->result, st));
        Partial pr;
        HIPCHK(hipMemcpyAsync(&pr, &d0->result, sizeof pr, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ref_terms = pr.e_sum + pr.e_comp;
    }
    Plan P;
    Job JJ = J;
    if (J.dump)
        JJ.forced_log2p = 0;
    if ((rc = plan_job(c, sys, L, RL, ws, refs, J.n, JJ, st, P)))
        return rc;
    uint64_t mx = 0;
    for (auto s : P.sizes)
        mx = std::max(mx, s);
    uint32_t key_bits = (uint32_t)RL.bits;
    if (RL.hash) {
        // sort on the top b bits of the hash, the fewest digit passes for
        // which the expected number of colliding pairs among the largest
        // subset's N records, N^2 / 2^(b - log2p + 1), stays at N/512 or
        // fewer (the subset fixes the top log2p bits; N bounds the number of
        // distinct determinants).  Collided runs are resolved exactly, each by
        // a revisit of its own records: at the bound, with every record a
        // distinct determinant, the revisits would cost about as much as the
        // 24-byte digit pass the bits save; with several records per
        // determinant, as generation gives, far less.  Among choices with
        // equal passes, the most bits.  A byte of the hash with no kept,
        // varying bit is a digit with one value, which the sort skips: with
        // 512 subsets of 1.9e9 records, 48 bits take 5 passes.
        int b = 64;
        if (c->opt.hash_bits == 0) {
            auto passes = [&](int bits) {
                int np = 0;
                for (int d = 0; d < 8; d++)
                    np += (8 * d + 8 > 64 - bits && 8 * d < 64 - P.log2p) ? 1 : 0;
                return np;
            };
            int best = 64;
            for (int bits = 64; bits >= 32; bits -= 8) {
                if ((double)mx * (double)mx / std::ldexp(1.0, bits - P.log2p + 1) > (double)mx / 512.0)
                    break;
                if (passes(bits) < passes(best))
                    best = bits;
            }
            // packed records take the low bits of the hash word
            b = RL.packed && best > HC_KEPT_BITS ? HC_KEPT_BITS : best;
            sys.kc.hash_mask = b >= 64 ? ~0ull : ~((1ull << (64 - b)) - 1);
        } else {
            b = c->opt.hash_bits >= 64 ? 64 : c->opt.hash_bits;
        }
        key_bits = (uint32_t)b;
        if (c->opt.hash_bits == 0) {
            // the digits that can vary: bytes holding kept bits below the
            // subset's fixed top log2p bits (the others hold one value)
            for (int d = 0; d < 8; d++)
                if (8 * d + 8 > 64 - b && 8 * d < 64 - P.log2p)
                    hash_digits |= 1u << d;
        }
        // the references' hashes (same bits), sorted, with their indices
        Planes h0 = planes_of(ws.refH0, 1, J.n, 8, 8), h1 = planes_of(ws.refH1, 1, J.n, 8, 8);
        HIPCHK(launch_refs_hash(sys, refs, J.n, h0, st));
        Timing none;
        if ((rc = radix_sort(ws, 1, 8, h0, h1, J.n, 64, st, none, nullptr, nullptr)))
            return rc;
        refs_hash = h0;
    }
    if ((rc = ensure_records(ws, W, pb, RL.topb, (int64_t)std::max<uint64_t>(std::max(mx, P.cap_hint), 1))))
        return rc;
    const double rbytes = record_bytes(W, pb, RL.topb);
    res.record_bytes = (uint32_t)rbytes;
    res.key_bits = key_bits;
    Small *ds = ws.dsmall();
    // same-spin doubles shared between references of one spin string (direct
    // generation with bitstring keys)
    int64_t nga = 0, ngb = 0;
    const bool want = c->opt.string_reuse == 2 ? L.nDaa + L.nDbb > 0 : c->opt.string_reuse == 1 && L.nDaa > 0;
    const bool reuse = !P.compact && want && !sys.kc.on && !sys.kc.hash && spin_reuse_ok(L, W);
    if (reuse && (rc = spin_groups(ws, refs, W, c->norb, J.n, c->opt.string_reuse == 2, st, nga, ngb)))
        return rc;
    res.n_alpha_groups = (uint64_t)nga;
    res.n_beta_groups = (uint64_t)ngb;
    std::vector<Partial> part_res(P.parts.size());
    for (size_t q = 0; q < P.parts.size(); q++) {
        const int64_t n = (int64_t)P.sizes[q];
        res.n_contrib += P.structural[q];
        res.n_after_cutoff += (uint64_t)n;
        Planes A = planes_of(ws.recA, W, ws.rec_cap, pb, RL.topb), B = planes_of(ws.recB, W, ws.rec_cap, pb, RL.topb);
        hipEvent_t a;
        if ((rc = timed_begin(ws, tm, st, a)))
            return rc;
        if (!P.compact) {
            const int kinds = nga > 0 ? (ngb > 0 ? 2 : 1) : 0;
            HIPCHK(launch_gen_direct(sys, L, pm, refs, J.n, P.chunk, kinds, A, st));
            if (kinds > 0) {
                const uint32_t *G = (const uint32_t *)ws.agrp.p, *I = G + 2 * ws.agrp_ngrp;
                HIPCHK(launch_gen_spin(sys, L, pm, refs, 0, G, I, nga, A, st));
                if (kinds == 2)
                    HIPCHK(launch_gen_spin(sys, L, pm, refs, 1, G + 2 * nga, I + J.n, ngb, A, st));
            }
        }
        else if (P.target)
            HIPCHK(launch_gen_target(sys, L, pm, refs, J.n, P.log2p, P.parts[q], c->opt.cutoff,
                                     (const uint64_t *)ws.off.p + (size_t)q * P.nchunks,
                                     (const uint64_t *)ws.tot.p + q, A, &ds->flags, P.bk, st));
        else
            HIPCHK(launch_gen_compact(sys, L, pm, refs, J.n, P.chunk,
                                      P.log2p, P.parts[q], c->opt.cutoff,
                                      (const uint64_t *)ws.off.p + (size_t)q * P.nchunks, P.nchunks,
                                      (uint64_t)ws.rec_cap, A, &ds->flags, st));
        if ((rc = timed_end(ws, tm, st, a, 0)))
            return rc;
        res.bytes_gen += (double)n * rbytes;
        if (J.dump == 1)
            break;  // generation order: the records are in recA
        if ((rc = radix_sort(ws, W, pb, A, B, n, RL.bits, st, tm, &res.n_sort_passes, &res.bytes_sort,
                             RL.hash ? SORT_ITEMS_WIDE : SORT_ITEMS, hash_digits)))
            return rc;
        if (J.dump == 2 || J.dump == 3) {
            // hand the sorted planes to the inspection copy below (it reads recA)
            if (ws.recA.p != (void *)A.key[0])
                std::swap(ws.recA, ws.recB);
            break;
        }
        if ((rc = timed_begin(ws, tm, st, a)))
            return rc;
        if ((rc = buf_ensure(ws.A, ws.tref, (size_t)((n + RED_TILE - 1) / RED_TILE + 1) * 16)))
            return rc;
        if (RL.hash)
            HIPCHK(launch_reduce_hash(sys, pm, A, n, refs, (const uint64_t *)ws.refX.p,
                                      ref_compact && !ref_compact4 ? (const uint64_t *)ws.refE.p : nullptr,
                                      ref_compact4 ? ref_ex4 : nullptr, anc_hash, refs_hash, J.n,
                                      (const double *)ws.hp.p, (const double *)ws.gv.p, J.e0, subtract ? 0 : 1,
                                      ds->partials, ds->coll, (int64_t *)B.key[0], &ds->flags, st));
        else
            HIPCHK(launch_reduce(sys, fp32, W, A, n, refs_red, J.n, J.e0, &ds->anc, anc_nh, (int64_t *)ws.tref.p,
                                 subtract ? 0 : 1, ds->partials, &ds->flags, st));
        HIPCHK(launch_final(ds->partials, &ds->result, st));
        if ((rc = timed_end(ws, tm, st, a, 2)))
            return rc;
        res.bytes_reduce += (double)n * rbytes;
        HIPCHK(hipMemcpyAsync(&part_res[q], &ds->result, sizeof(Partial), hipMemcpyDeviceToHost, st));
    }
    if (J.dump) {
        HIPCHK(hipStreamSynchronize(st));
        const int64_t n = (int64_t)P.sizes[0];
        if (J.n_out)
            *J.n_out = n;
        if (J.dump == 1 || J.dump == 2) {
            const int64_t m = std::min<int64_t>(n, J.cap);
            Buf kb, vb;
            if ((rc = buf_alloc(ws.A, kb, (size_t)std::max<int64_t>(m, 1) * W * 8)) ||
                (rc = buf_alloc(ws.A, vb, (size_t)std::max<int64_t>(m, 1) * 8)))
                return rc;
            Planes S = planes_of(ws.recA, W, ws.rec_cap, pb, RL.topb);
            HIPCHK(launch_planes_to_aos(W, pb, S, m, (uint64_t *)kb.p, (double *)vb.p, st));
            if (m > 0) {
                HIPCHK(hipMemcpyAsync(J.keys_out, kb.p, (size_t)m * W * 8, hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(J.vals_out, vb.p, (size_t)m * 8, hipMemcpyDeviceToHost, st));
            }
            HIPCHK(hipStreamSynchronize(st));
            buf_free(ws.A, kb), buf_free(ws.A, vb);
        } else {
            Buf kb, vb, ib;
            const int64_t m = std::max<int64_t>(J.cap, 1);
            if ((rc = buf_alloc(ws.A, kb, (size_t)m * W * 8)) || (rc = buf_alloc(ws.A, vb, (size_t)m * 8)) ||
                (rc = buf_alloc(ws.A, ib, (size_t)m)))
                return rc;
            Planes S = planes_of(ws.recA, W, ws.rec_cap, pb, RL.topb);
            HIPCHK(launch_zero_u64((uint64_t *)&ds->n_out, 1, st));
            HIPCHK(launch_numerators(W, fp32, S, n, refs, J.n, (uint64_t *)kb.p, (double *)vb.p, (uint8_t *)ib.p,
                                     &ds->n_out, J.cap, st));
            unsigned long long cnt = 0;
            HIPCHK(hipMemcpyAsync(&cnt, &ds->n_out, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int64_t mm = std::min<int64_t>((int64_t)cnt, J.cap);
            std::vector<uint64_t> keys((size_t)mm * W);
            std::vector<double> vals(mm);
            std::vector<uint8_t> inr(mm);
            if (mm > 0) {
                HIPCHK(hipMemcpy(keys.data(), kb.p, (size_t)mm * W * 8, hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(vals.data(), vb.p, (size_t)mm * 8, hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(inr.data(), ib.p, (size_t)mm, hipMemcpyDeviceToHost));
            }
            buf_free(ws.A, kb), buf_free(ws.A, vb), buf_free(ws.A, ib);
            // ascending key order (slots were taken in arbitrary order)
            std::vector<int64_t> idx(mm);
            for (int64_t i = 0; i < mm; i++)
                idx[i] = i;
            std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
                for (int w = W - 1; w >= 0; w--) {
                    uint64_t a = keys[x * W + w], b = keys[y * W + w];
                    if (a != b)
                        return a < b;
                }
                return false;
            });
            for (int64_t i = 0; i < mm; i++) {
                memcpy(J.keys_out + i * W, &keys[idx[i] * W], (size_t)W * 8);
                J.vals_out[i] = vals[idx[i]];
                J.inref_out[i] = inr[idx[i]];
            }
            *J.n_out = (int64_t)cnt;
        }
        return PT2_OK;
    }
    HIPCHK(hipMemcpyAsync(&ws.host_small->flags, &ds->flags, sizeof(Flags), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint32_t err = ws.host_small->flags.err;
    if (err & ERR_BOUNDS)
        return fail(PT2_E_DEVICE, "radix scatter destination out of range");
    if (err & ERR_OVERFLOW)
        return fail(PT2_E_DEVICE, "generation did not match the count pass");
    // combine subsets in index order
    double sum = 0.0, comp = 0.0;
    for (size_t q = 0; q < P.parts.size(); q++) {
        const Partial &p = part_res[q];
        const double e = p.e_sum + p.e_comp;
        if (J.e_parts)
            J.e_parts[q] = e;
        double t = sum + e;
        if (fabs(sum) >= fabs(e))
            comp += (sum - t) + e;
        else
            comp += (e - t) + sum;
        sum = t;
        res.n_unique += p.n_unique;
        res.n_external += p.n_external;
        res.n_in_ref_hit += p.n_hit;
        res.n_nonneg_denom += p.n_nonneg;
        res.ref_cross += p.ref_cross;
        res.key_xor ^= p.key_xor;
        res.key_sum += p.key_sum;
        res.min_abs_denom = std::min(res.min_abs_denom, p.min_abs_denom);
    }
    if (subtract) {
        const double x = -ref_terms, t = sum + x;
        if (fabs(sum) >= fabs(x))
            comp += (sum - t) + x;
        else
            comp += (x - t) + sum;
        sum = t;
    }
    res.e_pt2 = sum + comp;
    res.n_partitions = (uint32_t)P.parts.size();
    for (auto &e : tm.evs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
        if (e.kind == 0)
            res.ms_gen += ms;
        else if (e.kind == 1) {
            res.ms_sort += ms;
            res.ms_sort_scatter += ms;
            res.ms_sort_pass_max = std::max(res.ms_sort_pass_max, (double)ms);
        } else if (e.kind == 4)
            res.ms_sort += ms;
        else if (e.kind == 2)
            res.ms_reduce += ms;
        else
            res.ms_hist += ms;
    }
    res.ms_total = now_ms() - t0;
    memcpy(out, &res, sizeof res);
    if (err & ERR_SINGULAR)
        return fail(PT2_E_SINGULAR, "an external determinant has E0 - H_aa == 0");
    return PT2_OK;
}

bool result_ok(const pt2_result *out) { return out && out->struct_size == sizeof(pt2_result); }

// ---------------------------------------------------------------------------
// serving scheduler (process-wide)

struct Request {
    int64_t id;
    pt2_ctx *ctx;
    std::vector<uint64_t> dets;
    std::vector<double> c;
    int64_t n;
    double e0;
    double projected;
    double cap;          // plan budget: bytes of record buffers one subset may use
    bool alone = false;  // retried after an allocation failure: run with nothing else
    int64_t cap_records = 0;       // projected records of the largest subset
    size_t arena_off = SIZE_MAX;   // slice of the device arena, if admitted into one
    int retries = 0;
    bool done = false;
    int rc = PT2_OK;
    std::string err;
    pt2_result res;
};

// One device allocation for the record and scan buffers of served
// requests, carved into slices first-fit: no allocation, mapping or
// unmapping per request.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes; disjoint, coalesced

    bool alloc(size_t bytes, size_t &off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest)
                    free_[off + bytes] = rest;
                return true;
            }
        return false;
    }

    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Worker {
    std::thread th;
    hipStream_t stream = nullptr;
    std::unique_ptr<Workspace> ws;
};

class Scheduler {
  public:
    static Scheduler &get()
    {
        static Scheduler *s = new Scheduler();  // never destroyed; workers stopped at exit
        return *s;
    }

    int submit(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, double e0, pt2_req *out)
    {
        auto r = std::make_unique<Request>();
        r->ctx = c;
        r->dets.assign(dets, dets + (size_t)n * c->W);
        r->c.assign(coeffs, coeffs + n);
        r->n = n;
        r->e0 = e0;
        const RecLayout RL = rec_layout(c, false, n);
        const int pb = RL.pb;
        const double total = (double)n * (double)c->L.nper;
        std::unique_lock<std::mutex> lk0(mu_);
        const double dev_budget = device_budget_locked(c->opt.device);
        lk0.unlock();
        // the plan depends on the request and the device budget only, so a
        // request gives the same result alone and in a mix
        double cap = c->opt.device_budget_bytes ? (double)c->opt.device_budget_bytes : dev_budget;
        if (c->opt.max_partition_bytes)
            cap = std::min(cap, (double)c->opt.max_partition_bytes);
        r->cap = cap;
        double per = subset_bytes(RL.W, pb, RL.topb, total * 1.02 + 4096.0);
        int k = 0;
        while (k < MAX_LOG2P && per > cap) {
            k++;
            per = subset_bytes(RL.W, pb, RL.topb, total / (double)(1 << k) * 1.02 + 4096.0);
        }
        r->cap_records = (int64_t)(total / (double)(1 << k) * 1.02 + 4096.0);
        r->projected = (double)slice_bytes(RL.W, pb, RL.topb, r->cap_records);
        std::unique_lock<std::mutex> lk(mu_);
        start_workers_locked(c);
        r->id = next_id_++;
        *out = r->id;
        c->inflight++;
        queue_.push_back(r.get());
        all_[r->id] = std::move(r);
        cv_.notify_all();
        return PT2_OK;
    }

    int poll(pt2_ctx *c, pt2_req id, pt2_result *out, bool wait)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = all_.find(id);
        if (it == all_.end() || it->second->ctx != c)
            return fail(PT2_E_UNKNOWN_REQ, "unknown request id %lld", (long long)id);
        if (wait)
            done_cv_.wait(lk, [&] { return it->second->done; });
        if (!it->second->done)
            return PT2_NOT_READY;
        Request *r = it->second.get();
        int rc = r->rc;
        memcpy(out, &r->res, sizeof(pt2_result));
        if (rc != PT2_OK && rc != PT2_E_SINGULAR)
            g_err = r->err;
        c->inflight--;
        all_.erase(it);
        return rc;
    }

    double device_budget(int dev)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return device_budget_locked(dev);
    }

    // bytes the scheduler may hand to the record buffers of running requests
    // on a device: 80% of what was free when it first served the device.
    // Freed request buffers stay in the device's stream-ordered pool for the
    // next request (no unmapping and remapping of hundreds of GB).
    double device_budget_locked(int dev)
    {
        auto it = dev_budget_.find(dev);
        if (it != dev_budget_.end())
            return it->second;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev);
        size_t freeb = 0, totalb = 0;
        double b = 0.0;
        if (hipMemGetInfo(&freeb, &totalb) == hipSuccess)
            b = 0.8 * (double)freeb;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
        (void)hipSetDevice(prev);
        dev_budget_[dev] = b;
        return b;
    }

    // projected bytes of the requests running on a device
    double held(int dev)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = in_use_.find(dev);
        return it == in_use_.end() ? 0.0 : it->second;
    }

    // return the stream-ordered pool's idle memory of a device when nothing
    // runs or waits there
    void trim_if_idle(int dev)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (running_[dev] != 0)
            return;
        for (Request *q : queue_)
            if (q->ctx->opt.device == dev)
                return;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
            (void)hipMemPoolTrimTo(pool, 0);
        auto it = arena_.find(dev);
        if (it != arena_.end()) {
            if (it->second.base)
                (void)hipFree(it->second.base);
            arena_.erase(it);
        }
        (void)hipGetLastError();
    }

    int inflight(pt2_ctx *c)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return c->inflight;
    }

    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
            cv_.notify_all();
        }
        for (auto &w : workers_)
            if (w->th.joinable())
                w->th.join();
        for (auto &w : workers_) {
            w->ws.reset();
            if (w->stream)
                (void)hipStreamDestroy(w->stream);
        }
        workers_.clear();
    }

  private:
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Request *> queue_;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all_;
    std::vector<std::unique_ptr<Worker>> workers_;
    int64_t next_id_ = 1;
    std::unordered_map<int, double> in_use_;  // projected bytes of running requests, per device
    std::unordered_map<int, int> running_;    // running requests, per device
    std::unordered_map<int, double> dev_budget_;
    std::unordered_map<int, Arena> arena_;

    // the device's arena, made at its first use with the device budget
    Arena &arena_locked(int dev)
    {
        auto it = arena_.find(dev);
        if (it != arena_.end())
            return it->second;
        Arena &a = arena_[dev];
        const size_t bytes = (size_t)device_budget_locked(dev) & ~(size_t)255;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev);
        void *p = nullptr;
        if (bytes && hipMalloc(&p, bytes) == hipSuccess) {
            a.base = (char *)p;
            a.size = bytes;
            a.free_[0] = bytes;
        }
        (void)hipGetLastError();
        (void)hipSetDevice(prev);
        return a;
    }
    bool stopping_ = false;
    bool atexit_ = false;

    void start_workers_locked(pt2_ctx *c)
    {
        const int want = std::max(1, c->opt.n_streams);
        if (!atexit_) {
            atexit_ = true;
            atexit([] { Scheduler::get().stop(); });
        }
        while ((int)workers_.size() < want) {
            auto w = std::make_unique<Worker>();
            w->ws = std::make_unique<Workspace>();
            w->ws->A = c->A;
            Worker *wp = w.get();
            const int dev = c->opt.device;
            w->th = std::thread([this, wp, dev] { loop(wp, dev); });
            workers_.push_back(std::move(w));
        }
    }

    // first queued request whose record and scan buffers fit a free slice of
    // its device's arena (or that would run alone there, with buffers of its
    // own); a request bypassed too often blocks the rest
    Request *pick_locked()
    {
        for (size_t i = 0; i < queue_.size(); i++) {
            Request *r = queue_[i];
            const int dev = r->ctx->opt.device;
            bool take = false;
            r->arena_off = SIZE_MAX;
            if (!r->alone || running_[dev] == 0) {
                Arena &a = arena_locked(dev);
                size_t off = 0;
                if (r->projected <= (double)a.size && a.alloc((size_t)r->projected, off)) {
                    r->arena_off = off;
                    take = true;
                } else if (running_[dev] == 0) {
                    take = true;
                }
            }
            if (take) {
                queue_.erase(queue_.begin() + (long)i);
                return r;
            }
            if (i == 0 && bypass_ >= 16)
                return nullptr;
        }
        return nullptr;
    }
    int bypass_ = 0;

    void loop(Worker *w, int dev)
    {
        (void)hipSetDevice(dev);
        if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess)
            w->stream = nullptr;
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            Request *r = nullptr;
            cv_.wait(lk, [&] { return stopping_ || (!queue_.empty() && (r = pick_locked()) != nullptr); });
            if (stopping_ && !r)
                return;
            if (!queue_.empty() && r != queue_.front())
                bypass_++;
            else
                bypass_ = 0;
            pt2_ctx *c = r->ctx;
            in_use_[c->opt.device] += r->projected;
            running_[c->opt.device]++;
            char *abase = r->arena_off != SIZE_MAX ? arena_[c->opt.device].base : nullptr;
            lk.unlock();
            (void)hipSetDevice(c->opt.device);
            Alloc A = c->A;
            A.stream = A.fa ? nullptr : w->stream;  // stream-ordered unless a hook allocates
            if (!w->ws->A.same_source(A) || w->ws->A.stream != A.stream)
                w->ws->release();  // buffers go back to the allocator that made them
            w->ws->A = A;
            if (r->arena_off != SIZE_MAX) {
                const RecLayout RL = rec_layout(c, false, r->n);
                carve_slice(*w->ws, abase + r->arena_off, RL.W, RL.pb, RL.topb, r->cap_records);
            }
            Job J{};
            J.dets = r->dets.data();
            J.coeffs = r->c.data();
            J.n = r->n;
            J.host = true;
            J.e0 = r->e0;
            J.forced_log2p = -1;
            J.plan_budget = r->cap;
            pt2_result res;
            memset(&res, 0, sizeof res);
            res.struct_size = sizeof res;
            int rc = w->stream ? run_job(c, *w->ws, w->stream, J, &res)
                               : fail(PT2_E_DEVICE, "worker stream creation failed");
            // give the record buffers back (stream-ordered, no device-wide wait)
            // so that admission by projected bytes stays truthful
            buf_free(w->ws->A, w->ws->recA), buf_free(w->ws->A, w->ws->recB);
            buf_free(w->ws->A, w->ws->counts), buf_free(w->ws->A, w->ws->offs);
            buf_free(w->ws->A, w->ws->csum), buf_free(w->ws->A, w->ws->coff);
            w->ws->rec_cap = 0;
            w->ws->scan_tiles = 0;
            if (w->stream)
                (void)hipStreamSynchronize(w->stream);
            lk.lock();
            if (r->arena_off != SIZE_MAX) {
                arena_[c->opt.device].release(r->arena_off, (size_t)r->projected);
                r->arena_off = SIZE_MAX;
            }
            if (rc == PT2_E_NOMEM && r->retries < 2) {
                // memory held outside the projections (other requests, pool
                // fragments): run it again with nothing else on the device,
                // the second time after returning the pool's idle memory
                r->retries++;
                r->alone = true;
                in_use_[c->opt.device] -= r->projected;
                running_[c->opt.device]--;
                if (r->retries == 2 && running_[c->opt.device] == 0) {
                    hipMemPool_t pool;
                    if (hipDeviceGetDefaultMemPool(&pool, c->opt.device) == hipSuccess)
                        (void)hipMemPoolTrimTo(pool, 0);
                    (void)hipGetLastError();
                }
                queue_.push_front(r);
                cv_.notify_all();
                continue;
            }
            r->rc = rc;
            r->err = rc != PT2_OK ? g_err : std::string();
            r->res = res;
            r->done = true;
            in_use_[c->opt.device] -= r->projected;
            running_[c->opt.device]--;
            done_cv_.notify_all();
            cv_.notify_all();
        }
    }
};

// The scheduler's planning budget of a device (taken once per device).
double serving_device_budget(int dev)
{
    return Scheduler::get().device_budget(dev);
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI

PT2_API void pt2_default_options(pt2_options *o)
{
    if (!o)
        return;
    memset(o, 0, sizeof *o);
    o->struct_size = sizeof *o;
    o->precision = PT2_FP64;
    o->cutoff = 0.0;
    o->log2_partitions = -1;
    o->compress_keys = -1;
    o->exclusion = PT2_EXCLUDE_SEARCH;
    o->device = 0;
    o->n_streams = 4;
    o->string_reuse = 1;
    o->compact_refs = 1;
}

PT2_API int pt2_key_words(int norb) { return (2 * norb + 63) / 64; }

PT2_API const char *pt2_last_error(void) { return g_err.c_str(); }

// The record form of a context: compress_keys forces one where it applies;
// the automatic choice (-1) prices each form by the bytes its records move
// through the digit passes and takes a compressed form only if it saves 30%
// or more against the bitstring.  Host only.
struct KeyForm {
    int mode = 0;  // 0 bitstring, 1 rank, 2 hash
    int kw = 0, kbits = 0, bb = 0, stride = 0, ktop = 0;
    std::vector<uint64_t> binom;  // C(x, j), x <= norb, j <= max(na, nb), for rank keys
};

KeyForm key_form(int norb, int nalpha, int nbeta, const pt2_options &o)
{
    KeyForm f;
    const int pb = o.precision != PT2_FP64 ? 4 : 8;
    const int W = pt2_key_words(norb);
    const double cost_bits = 2.0 * record_bytes(W, pb, top_bytes(norb)) * ((2 * norb + 7) / 8);
    double cost_rank = 1e300, cost_hash = 1e300;
    // ranks: exact binomials C(x, j), x <= norb, j <= max(na, nb)
    const int nmax = std::max(nalpha, nbeta), stride = nmax + 1;
    std::vector<unsigned __int128> C((size_t)(norb + 1) * stride, 0);
    bool fits = true;
    for (int x = 0; x <= norb; x++)
        for (int j = 0; j < stride; j++) {
            unsigned __int128 v = j == 0 ? 1 : (x == 0 ? 0 : C[(size_t)(x - 1) * stride + j - 1] +
                                                                 C[(size_t)(x - 1) * stride + j]);
            C[(size_t)x * stride + j] = v;
            if (v > (unsigned __int128)UINT64_MAX)
                fits = false;
        }
    auto bits_for = [](unsigned __int128 count) {  // bits of values 0 .. count-1
        int b = 0;
        while (count > ((unsigned __int128)1 << b))
            b++;
        return b;
    };
    const int ba = bits_for(C[(size_t)norb * stride + nalpha]);
    const int bb = bits_for(C[(size_t)norb * stride + nbeta]);
    const int kbits = ba + bb;
    const int kw = std::max(1, (kbits + 63) / 64);
    const int tb = kbits - 64 * (kw - 1);
    const int ktop = tb <= 16 ? 2 : (tb <= 32 ? 4 : 8);
    const bool rank_ok = fits && kw <= 2;
    if (rank_ok)
        cost_rank = 2.0 * record_bytes(kw, pb, ktop) * ((kbits + 7) / 8);
    // hash records: a spin-orbital index per byte, 0xFF marks an unused flip
    const bool hash_ok = 2 * norb <= 254;
    if (hash_ok)
        cost_hash = 2.0 * record_bytes(2, pb, 8) * 8;
    // FP32 payloads with the default hash width: the packed 16-byte
    // records with at most HC_KEPT_BITS kept bits (rec_layout; assumed
    // here for a reference list of fewer than HC_MAX_REFS determinants)
    if (hash_ok && pb == 4 && o.hash_bits == 0 && norb <= HC_MAX_NORB)
        cost_hash = 2.0 * 16.0 * (HC_KEPT_BITS / 8);
    if (o.compress_keys == 1 && rank_ok)
        f.mode = 1;
    else if (o.compress_keys == 2 && hash_ok)
        f.mode = 2;
    else if (o.compress_keys == -1) {
        // only a clear saving pays: compressed digits are dense, so a
        // scatter tile writes shorter runs, and both forms cost time in
        // generation and the single pass.  Measured: (10a,10b)/40 rank
        // keys (8 passes against 10) 224 ms against 192 ms; (14a,14b)/76
        // rank keys (13 against 19) 36.1 s against 39.8 s.
        // A served FP32 request of 54 orbitals (2.1e9 contributions):
        // rank keys (78 bits, ten 14-byte passes) 366 ms, sort 187 ms
        // and single pass 145 ms of it; packed hash records (40 kept
        // bits, five 16-byte passes) 214 ms, 87 ms and 110 ms.  Equal
        // costs take hash records, whose FP32 rounding is bounded: at
        // (10a,10b)/40 with FP32 payloads (60-bit ranks, eight 12-byte
        // passes) 141.9 ms and 2e-10 Eh off against 162.2 ms and 7e-9.
        const double best = std::min(cost_rank, cost_hash);
        if (best <= 0.7 * cost_bits)
            f.mode = cost_hash <= cost_rank ? 2 : 1;
    }
    if (f.mode == 1) {
        f.kw = kw, f.kbits = kbits, f.bb = bb, f.stride = stride, f.ktop = ktop;
        f.binom.resize(C.size());
        for (size_t i = 0; i < C.size(); i++)
            f.binom[i] = (uint64_t)C[i];
    }
    return f;
}

PT2_API int pt2_key_form(int norb, int nalpha, int nbeta, const pt2_options *opt, int *form, int *key_bits)
{
    g_err.clear();
    if (!form || !key_bits)
        return fail(PT2_E_INVALID, "form or key_bits is NULL");
    if (norb < 1 || norb > MAXORB)
        return fail(PT2_E_INVALID, "norb must be in [1, %d]", MAXORB);
    if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb)
        return fail(PT2_E_INVALID, "electron counts out of range");
    pt2_options o;
    pt2_default_options(&o);
    if (opt) {
        if (opt->struct_size != sizeof(pt2_options))
            return fail(PT2_E_INVALID, "pt2_options.struct_size mismatch");
        o = *opt;
    }
    if (o.precision != PT2_FP64 && o.precision != PT2_FP32_PAYLOAD && o.precision != PT2_FP32_ARITH)
        return fail(PT2_E_INVALID, "unknown precision %d", o.precision);
    if (o.hash_bits < 0 || o.hash_bits > 64)
        return fail(PT2_E_INVALID, "hash_bits must be in [0, 64]");
    if (o.compress_keys < -1 || o.compress_keys > 2)
        return fail(PT2_E_INVALID, "compress_keys must be -1, 0, 1 or 2");
    const KeyForm kf = key_form(norb, nalpha, nbeta, o);
    *form = kf.mode;
    *key_bits = kf.mode == 1 ? kf.kbits : (kf.mode == 2 ? 64 : 2 * norb);
    return PT2_OK;
}

PT2_API int pt2_create(const double *h, const double *eri, int norb, int nalpha, int nbeta, const pt2_options *opt,
                       pt2_ctx **out)
{
    g_err.clear();
    if (!out)
        return fail(PT2_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!h || !eri)
        return fail(PT2_E_INVALID, "h or eri is NULL");
    if (norb < 1 || norb > MAXORB)
        return fail(PT2_E_INVALID, "norb must be in [1, %d]", MAXORB);
    if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb)
        return fail(PT2_E_INVALID, "electron counts out of range");
    pt2_options o;
    pt2_default_options(&o);
    if (opt) {
        if (opt->struct_size != sizeof(pt2_options))
            return fail(PT2_E_INVALID, "pt2_options.struct_size mismatch");
        o = *opt;
    }
    if (o.precision != PT2_FP64 && o.precision != PT2_FP32_PAYLOAD && o.precision != PT2_FP32_ARITH)
        return fail(PT2_E_INVALID, "unknown precision %d", o.precision);
    if (o.exclusion != PT2_EXCLUDE_SEARCH && o.exclusion != PT2_EXCLUDE_SUBTRACT)
        return fail(PT2_E_INVALID, "exclusion must be PT2_EXCLUDE_SEARCH or PT2_EXCLUDE_SUBTRACT");
    if (!(o.cutoff >= 0.0))
        return fail(PT2_E_INVALID, "cutoff must be >= 0");
    if (o.log2_partitions > MAX_LOG2P)
        return fail(PT2_E_INVALID, "log2_partitions must be <= %d", MAX_LOG2P);
    if (o.hash_bits < 0 || o.hash_bits > 64)
        return fail(PT2_E_INVALID, "hash_bits must be in [0, 64]");
    if (o.spin_flip != 0 && o.spin_flip != 1)
        return fail(PT2_E_INVALID, "spin_flip must be 0 or 1");
    if (o.spin_flip && nalpha != nbeta)
        return fail(PT2_E_INVALID, "spin_flip needs nalpha == nbeta (S_z = 0)");
    if (o.string_reuse < 0 || o.string_reuse > 2)
        return fail(PT2_E_INVALID, "string_reuse must be 0, 1 or 2");
    if (o.compress_keys < -1 || o.compress_keys > 2)
        return fail(PT2_E_INVALID, "compress_keys must be -1, 0, 1 or 2");
    if ((o.alloc == nullptr) != (o.free == nullptr))
        return fail(PT2_E_INVALID, "alloc and free hooks must be given together");
    const size_t n = (size_t)norb;
    for (size_t p = 0; p < n; p++)
        for (size_t q = 0; q < n; q++) {
            if (!std::isfinite(h[p * n + q]))
                return fail(PT2_E_INVALID, "h has a non-finite entry");
            if (std::fabs(h[p * n + q] - h[q * n + p]) > 1e-12)
                return fail(PT2_E_INVALID, "h is not symmetric");
        }
    auto E = [&](size_t p, size_t q, size_t r, size_t s) { return eri[((p * n + q) * n + r) * n + s]; };
    for (size_t p = 0; p < n; p++)
        for (size_t q = 0; q < n; q++)
            for (size_t r = 0; r < n; r++)
                for (size_t s = 0; s < n; s++) {
                    const double v = E(p, q, r, s);
                    if (!std::isfinite(v))
                        return fail(PT2_E_INVALID, "eri has a non-finite entry");
                    if (std::fabs(v - E(q, p, r, s)) > 1e-12 || std::fabs(v - E(p, q, s, r)) > 1e-12 ||
                        std::fabs(v - E(r, s, p, q)) > 1e-12)
                        return fail(PT2_E_INVALID, "eri is not 8-fold symmetric at (%zu %zu|%zu %zu)", p, q, r, s);
                }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(PT2_E_DEVICE, "no HIP device available");
    }
    if (o.device < 0 || o.device >= ndev)
        return fail(PT2_E_INVALID, "device %d out of range", o.device);
    HIPCHK(hipSetDevice(o.device));

    auto c = std::make_unique<pt2_ctx>();
    c->opt = o;
    c->norb = norb, c->na = nalpha, c->nb = nbeta, c->W = pt2_key_words(norb);
    c->topb = top_bytes(norb);
    c->A.fa = o.alloc, c->A.ff = o.free, c->A.user = o.alloc_user, c->A.device = o.device;
    c->ws.A = c->A;
    c->L = make_layout(norb, nalpha, nbeta);
    if (c->L.nper >= ((int64_t)1 << 26))
        return fail(PT2_E_INVALID, "excitation space per determinant too large");
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    size_t freeb = 0, totalb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totalb));
    // memory the scheduler's running requests hold now is theirs only until
    // they finish: count it as available, admission keeps the sum in bounds
    c->budget = o.device_budget_bytes ? o.device_budget_bytes
                                      : (uint64_t)(0.8 * ((double)freeb + Scheduler::get().held(o.device)));

    // resident Hamiltonian
    const size_t n2 = n * n, n4 = n2 * n2, nso = 2 * n, ntri = nso * (nso + 1) / 2;
    // packed upper triangle over spin-orbitals b1 <= b2 (row b1 starts at
    // b1*nso - b1*(b1-1)/2, entry b2 - b1 within it)
    // Each entry is kept exactly as the pair (rounded difference, its exact
    // rounding error): the denominators E0 - H_aa are formed in double-double
    // arithmetic and must not inherit the rounding of (pp|qq) - (pq|qp).
    std::vector<double> T(ntri, 0.0), Tlo(ntri, 0.0);
    for (size_t b1 = 0, o = 0; b1 < nso; b1++) {
        const size_t p = b1 < n ? b1 : b1 - n;
        T[o++] = h[p * n + p];
        for (size_t b2 = b1 + 1; b2 < nso; b2++, o++) {
            const size_t q = b2 < n ? b2 : b2 - n;
            const bool same = (b1 < n) == (b2 < n);
            const double a = E(p, p, q, q), b = same ? -E(p, q, q, p) : 0.0;
            // two-sum: T + Tlo == a + b exactly
            const double sum = a + b;
            const double bb = sum - a;
            T[o] = sum;
            Tlo[o] = (a - (sum - bb)) + (b - bb);
        }
    }
    std::vector<uint64_t> R(nso);
    uint64_t st = 0x5054325F5A4F4252ull;
    for (size_t b = 0; b < nso; b++)
        R[b] = splitmix_next(st);
    int rc;
    if ((rc = buf_alloc(c->A, c->h, n2 * 8)) || (rc = buf_alloc(c->A, c->V, n4 * 8)) ||
        (rc = buf_alloc(c->A, c->T, ntri * 8)) || (rc = buf_alloc(c->A, c->Tlo, ntri * 8)) ||
        (rc = buf_alloc(c->A, c->R, nso * 8)))
        return rc;
    HIPCHK(hipMemcpy(c->h.p, h, n2 * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->V.p, eri, n4 * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->T.p, T.data(), ntri * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->Tlo.p, Tlo.data(), ntri * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->R.p, R.data(), nso * 8, hipMemcpyHostToDevice));
    // same-spin doubles' integral differences (ra|qb) - (rb|qa), r < q and
    // a < b, formed once (the FP64 subtraction the terms would make), when
    // the table is small beside the integrals' own footprint
    const size_t npair = (size_t)norb * (norb - 1) / 2;
    if (o.precision != PT2_FP32_ARITH && npair > 0 && npair * npair * 8 <= ((size_t)1 << 30)) {
        if ((rc = buf_alloc(c->A, c->A2, npair * npair * 8)))
            return rc;
        HIPCHK(launch_build_a2((const double *)c->V.p, norb, (double *)c->A2.p, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    if (o.precision == PT2_FP32_ARITH) {
        std::vector<float> h32(n2), V32(n4);
        for (size_t i = 0; i < n2; i++)
            h32[i] = (float)h[i];
        for (size_t i = 0; i < n4; i++)
            V32[i] = (float)eri[i];
        if ((rc = buf_alloc(c->A, c->h32, n2 * 4)) || (rc = buf_alloc(c->A, c->V32, n4 * 4)))
            return rc;
        HIPCHK(hipMemcpy(c->h32.p, h32.data(), n2 * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->V32.p, V32.data(), n4 * 4, hipMemcpyHostToDevice));
    }
    c->sys.norb = norb, c->sys.na = nalpha, c->sys.nb = nbeta, c->sys.W = c->W;
    c->sys.h = (const double *)c->h.p;
    c->sys.V = (const double *)c->V.p;
    c->sys.h32 = (const float *)c->h32.p;
    c->sys.V32 = (const float *)c->V32.p;
    c->sys.T = (const double *)c->T.p;
    c->sys.Tlo = (const double *)c->Tlo.p;
    c->sys.A2 = (const double *)c->A2.p;
    c->sys.R = (const uint64_t *)c->R.p;
    c->sys.z2 = o.spin_flip;

    // record keys: the bitstring, the combinatorial rank, or the Zobrist hash
    // (with the parent and the flips)
    memset(&c->sys.kc, 0, sizeof c->sys.kc);
    {
        const KeyForm kf = key_form(norb, nalpha, nbeta, o);
        if (kf.mode == 1) {
            if ((rc = buf_alloc(c->A, c->binom, kf.binom.size() * 8)))
                return rc;
            HIPCHK(hipMemcpy(c->binom.p, kf.binom.data(), kf.binom.size() * 8, hipMemcpyHostToDevice));
            KeyCodec &k = c->sys.kc;
            k.on = 1, k.kw = kf.kw, k.kbits = kf.kbits, k.bb = kf.bb, k.stride = kf.stride, k.ktop = kf.ktop;
            k.binom = (const uint64_t *)c->binom.p;
            c->L.rank = 1;
        } else if (kf.mode == 2) {
            c->sys.kc.hash = 1;
            c->sys.kc.hash_mask = o.hash_bits == 0 || o.hash_bits >= 64 ? ~0ull : ((1ull << o.hash_bits) - 1);
        }
    }
    *out = c.release();
    return PT2_OK;
}

namespace {
int check_eval_args(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, pt2_result *out)
{
    g_err.clear();
    if (!c)
        return fail(PT2_E_INVALID, "context is NULL");
    if (!result_ok(out))
        return fail(PT2_E_INVALID, "pt2_result is NULL or struct_size mismatch");
    if (n < 0)
        return fail(PT2_E_INVALID, "ndets < 0");
    if (n > 0 && (!dets || !coeffs))
        return fail(PT2_E_INVALID, "dets or coeffs is NULL");
    if (n >= ((int64_t)1 << 31))
        return fail(PT2_E_INVALID, "too many reference determinants");
    return PT2_OK;
}

int eval_common(pt2_ctx *c, Job &J, pt2_result *out)
{
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->opt.device) != hipSuccess)
        return fail(PT2_E_DEVICE, "hipSetDevice failed");
    return run_job(c, c->ws, c->stream, J, out);
}
}  // namespace

PT2_API int pt2_evaluate(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, double e0,
                         pt2_result *out)
{
    int rc = check_eval_args(c, dets, coeffs, n, out);
    if (rc)
        return rc;
    Job J{};
    J.dets = dets, J.coeffs = coeffs, J.n = n, J.host = true, J.e0 = e0, J.forced_log2p = -1;
    J.live_budget = true;
    return eval_common(c, J, out);
}

PT2_API int pt2_evaluate_device(pt2_ctx *c, const uint64_t *d_dets, const double *d_coeffs, int64_t n, double e0,
                                pt2_result *out)
{
    int rc = check_eval_args(c, d_dets, d_coeffs, n, out);
    if (rc)
        return rc;
    Job J{};
    J.dets = d_dets, J.coeffs = d_coeffs, J.n = n, J.host = false, J.e0 = e0, J.forced_log2p = -1;
    J.live_budget = true;
    return eval_common(c, J, out);
}

// ---------------------------------------------------------------------------
// Allocation-free evaluation: every device buffer of the call is carved from
// one file-scope device array.  In host code `scratch` names a host-side
// stand-in, not device memory: the array's device address is taken once per
// device with hipGetSymbolAddress (that device current) and only that
// address is used.  Calls on one device share the array and overlap-race.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
char *g_scratch_ptr[64];  // device address of `scratch` per device (null until taken)
Small g_scratch_host[64]; // host mirror of the control block per device

int scratch_base(int dev, char **out)
{
    if (dev < 0 || dev >= 64)
        return fail(PT2_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(PT2_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PT2_OK;
}
}  // namespace

PT2_API int pt2_evaluate_device_noalloc(pt2_ctx *c, const uint64_t *d_dets, const double *d_coeffs, int64_t n,
                                        double e0, pt2_result *out)
{
    int rc = check_eval_args(c, d_dets, d_coeffs, n, out);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    const int dev = c->opt.device;
    if (hipSetDevice(dev) != hipSuccess)
        return fail(PT2_E_DEVICE, "hipSetDevice failed");
    char *base = nullptr;
    if ((rc = scratch_base(dev, &base)))
        return rc;
    BumpArena ar;
    ar.base = base, ar.cap = NOALLOC_SCRATCH_BYTES, ar.used = 0;
    Workspace ws;
    ws.A.device = dev;
    ws.A.arena = &ar;
    ws.zero_stream = c->stream;
    ws.host_small = &g_scratch_host[dev];
    ws.own_host_small = false;
    Job J{};
    J.dets = d_dets, J.coeffs = d_coeffs, J.n = n, J.host = false, J.e0 = e0, J.forced_log2p = -1;
    // the record buffers of a subset take at most 60% of the scratch; the
    // rest holds the reference planes, counts and control data
    J.plan_budget = 0.6 * (double)NOALLOC_SCRATCH_BYTES;
    rc = run_job(c, ws, c->stream, J, out);
    if (rc == PT2_OK)
        HIPCHK(hipStreamSynchronize(c->stream));
    return rc;
}

static int eval_parts(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, double e0, int log2p,
                      const uint32_t *parts, int nparts, double *e_parts, pt2_result *out, bool host)
{
    int rc = check_eval_args(c, dets, coeffs, n, out);
    if (rc)
        return rc;
    if (log2p < 0 || log2p > MAX_LOG2P)
        return fail(PT2_E_INVALID, "log2p must be in [0, %d]", MAX_LOG2P);
    if (nparts < 0 || (nparts > 0 && (!parts || !e_parts)))
        return fail(PT2_E_INVALID, "parts / e_parts invalid");
    for (int i = 0; i < nparts; i++)
        if (parts[i] >= (1u << log2p))
            return fail(PT2_E_INVALID, "subset index out of range");
    Job J{};
    J.dets = dets, J.coeffs = coeffs, J.n = n, J.host = host, J.e0 = e0, J.forced_log2p = log2p;
    J.parts = parts, J.nparts = nparts, J.e_parts = e_parts;
    if (nparts == 0) {
        memset(out, 0, sizeof *out);
        out->struct_size = sizeof *out;
        return PT2_OK;
    }
    return eval_common(c, J, out);
}

PT2_API int pt2_evaluate_parts(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, double e0,
                               int log2p, const uint32_t *parts, int nparts, double *e_parts, pt2_result *out)
{
    return eval_parts(c, dets, coeffs, n, e0, log2p, parts, nparts, e_parts, out, true);
}

PT2_API int pt2_evaluate_parts_device(pt2_ctx *c, const uint64_t *d_dets, const double *d_coeffs, int64_t n,
                                      double e0, int log2p, const uint32_t *parts, int nparts, double *e_parts,
                                      pt2_result *out)
{
    return eval_parts(c, d_dets, d_coeffs, n, e0, log2p, parts, nparts, e_parts, out, false);
}

PT2_API int pt2_dump_records(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, int sorted,
                             uint64_t *keys_out, double *payload_out, int64_t cap, int64_t *n_out)
{
    pt2_result tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.struct_size = sizeof tmp;
    int rc = check_eval_args(c, dets, coeffs, n, &tmp);
    if (rc)
        return rc;
    if (!n_out || cap < 0 || (cap > 0 && (!keys_out || !payload_out)))
        return fail(PT2_E_INVALID, "output buffers invalid");
    Job J{};
    J.dets = dets, J.coeffs = coeffs, J.n = n, J.host = true, J.e0 = 0.0, J.forced_log2p = 0;
    J.dump = sorted ? 2 : 1, J.keys_out = keys_out, J.vals_out = payload_out, J.cap = cap, J.n_out = n_out;
    return eval_common(c, J, &tmp);
}

PT2_API int pt2_dump_numerators(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, uint64_t *keys_out,
                                double *num_out, uint8_t *in_ref_out, int64_t cap, int64_t *n_out)
{
    pt2_result tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.struct_size = sizeof tmp;
    int rc = check_eval_args(c, dets, coeffs, n, &tmp);
    if (rc)
        return rc;
    if (!n_out || cap < 0 || (cap > 0 && (!keys_out || !num_out || !in_ref_out)))
        return fail(PT2_E_INVALID, "output buffers invalid");
    Job J{};
    J.dets = dets, J.coeffs = coeffs, J.n = n, J.host = true, J.e0 = 0.0, J.forced_log2p = 0;
    J.dump = 3, J.keys_out = keys_out, J.vals_out = num_out, J.inref_out = in_ref_out, J.cap = cap, J.n_out = n_out;
    return eval_common(c, J, &tmp);
}

PT2_API int pt2_submit(pt2_ctx *c, const uint64_t *dets, const double *coeffs, int64_t n, double e0, pt2_req *out)
{
    pt2_result tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.struct_size = sizeof tmp;
    int rc = check_eval_args(c, dets, coeffs, n, &tmp);
    if (rc)
        return rc;
    if (!out)
        return fail(PT2_E_INVALID, "request id pointer is NULL");
    return Scheduler::get().submit(c, dets, coeffs, n, e0, out);
}

PT2_API int pt2_poll(pt2_ctx *c, pt2_req req, pt2_result *out)
{
    g_err.clear();
    if (!c || !result_ok(out))
        return fail(PT2_E_INVALID, "invalid arguments");
    return Scheduler::get().poll(c, req, out, false);
}

PT2_API int pt2_wait(pt2_ctx *c, pt2_req req, pt2_result *out)
{
    g_err.clear();
    if (!c || !result_ok(out))
        return fail(PT2_E_INVALID, "invalid arguments");
    return Scheduler::get().poll(c, req, out, true);
}

PT2_API int pt2_destroy(pt2_ctx *c)
{
    g_err.clear();
    if (!c)
        return PT2_OK;
    if (Scheduler::get().inflight(c) > 0)
        return fail(PT2_E_BUSY, "requests in flight");
    Scheduler::get().trim_if_idle(c->opt.device);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        (void)hipSetDevice(c->opt.device);
        if (c->stream)
            (void)hipStreamSynchronize(c->stream);
        c->ws.release();
        buf_free(c->A, c->h), buf_free(c->A, c->V), buf_free(c->A, c->h32), buf_free(c->A, c->V32);
        buf_free(c->A, c->A2);
        buf_free(c->A, c->T), buf_free(c->A, c->Tlo), buf_free(c->A, c->R), buf_free(c->A, c->binom);
        if (c->own_stream && c->stream)
            (void)hipStreamDestroy(c->stream);
    }
    delete c;
    return PT2_OK;
}

PT2_API int pt2_sort_records(int device, int W, int key_bits, uint64_t *keys, void *payload, int payload_bytes,
                             int64_t n)
{
    g_err.clear();
    if (W < 1 || W > MAXW || key_bits < 0 || key_bits > 64 * W || (payload_bytes != 4 && payload_bytes != 8) ||
        n < 0 || (n > 0 && (!keys || !payload)))
        return fail(PT2_E_INVALID, "invalid arguments");
    if (n <= 1)
        return PT2_OK;
    HIPCHK(hipSetDevice(device));
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    Workspace ws;
    int rc;
    const size_t pbytes = planes_bytes(W, n, payload_bytes, 8);
    if ((rc = ensure_small(ws)) || (rc = buf_alloc(ws.A, ws.recA, pbytes)) || (rc = buf_alloc(ws.A, ws.recB, pbytes))) {
        (void)hipStreamDestroy(st);
        return rc;
    }
    std::vector<uint64_t> planes((size_t)n * W);
    for (int64_t i = 0; i < n; i++)
        for (int w = 0; w < W; w++)
            planes[(size_t)w * n + i] = keys[i * W + w];
    Planes A = planes_of(ws.recA, W, n, payload_bytes, 8), B = planes_of(ws.recB, W, n, payload_bytes, 8);
    Timing none;
    rc = PT2_OK;
    bool up_ok = true;
    for (int w = 0; w < W; w++)
        up_ok = up_ok && hipMemcpy(A.key[w], planes.data() + (size_t)w * n, (size_t)n * 8, hipMemcpyHostToDevice) ==
                             hipSuccess;
    if (!up_ok ||
        hipMemcpy(A.pay, payload, (size_t)n * payload_bytes, hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(PT2_E_DEVICE, "upload failed");
    if (!rc)
        rc = radix_sort(ws, W, payload_bytes, A, B, n, key_bits, st, none, nullptr, nullptr);
    if (!rc) {
        Flags f;
        if (hipStreamSynchronize(st) != hipSuccess ||
            hipMemcpy(&f, &ws.dsmall()->flags, sizeof f, hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(PT2_E_DEVICE, "sort failed");
        else if (f.err & ERR_BOUNDS)
            rc = fail(PT2_E_DEVICE, "radix scatter destination out of range");
    }
    if (!rc) {
        for (int w = 0; w < W; w++)
            if (hipMemcpy(planes.data() + (size_t)w * n, A.key[w], (size_t)n * 8, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(PT2_E_DEVICE, "download failed");
        if (!rc && hipMemcpy(payload, A.pay, (size_t)n * payload_bytes, hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(PT2_E_DEVICE, "download failed");
        if (!rc)
            for (int64_t i = 0; i < n; i++)
                for (int w = 0; w < W; w++)
                    keys[i * W + w] = planes[(size_t)w * n + i];
    }
    ws.release();
    (void)hipStreamDestroy(st);
    return rc;
}
