/*
 * pt2.h -- C-ABI of the MI355X (gfx950) Epstein-Nesbet PT2 engine.
 *
 * The engine evaluates, for a selected-CI reference psi = sum_i c_i |D_i>,
 *
 *     E_PT2 = sum_{a not in psi} N_a^2 / (E0 - H_aa),   N_a = sum_i H_ai c_i
 *
 * (Tubman et al., arXiv:1808.02049, Section II, the Epstein-Nesbet equation),
 * by the sort-based method of Section III: generate every single and double
 * excitation of every reference determinant together with its numerator term
 * H_ai c_i (Algorithm 1, generation step), sort the terms by determinant
 * bitstring (Algorithm 1, sort step), and make one pass over the sorted terms
 * to form N_a, drop determinants that are in the reference, and accumulate the
 * energy (Algorithm 1, single pass).  When the terms do not fit in device
 * memory the external space is split into non-overlapping, complete subsets
 * that are processed one after another (Algorithm 2, constraint PT2); here the
 * subset of a determinant is the top k bits of a Zobrist hash of its
 * bitstring, so the split has 2^k subsets.
 *
 * Conventions (the paper fixes only that alpha orbitals are the most
 * significant digits of the bitstring, Section III, triplet constraints):
 *   - determinant bitstring: 2*norb bits in W = pt2_key_words(norb) uint64
 *     words, word 0 least significant; beta orbital p is bit p, alpha orbital
 *     p is bit norb + p; bits at or above 2*norb are zero;
 *   - |D> = product of creators of the occupied spin-orbitals in ascending bit
 *     order acting on the vacuum; coefficients c_i refer to this ordering;
 *   - integrals are real, chemists' notation (pq|rs), no constant term:
 *     H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q.
 *
 * Memory ownership: the caller owns every pointer it passes.  Host inputs are
 * copied before the call returns.  The library owns the device memory it
 * allocates (through the optional allocator hook, else hipMalloc) and frees
 * it in pt2_destroy.
 *
 * Errors: every entry point returns a PT2_* code; no exception crosses the
 * boundary.  pt2_last_error() gives a message for the calling thread.
 *
 * Threading: pt2_submit and pt2_poll may be called from any thread.  The
 * pt2_evaluate* entry points serialise per context.
 */
#ifndef PT2_H
#define PT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt2_ctx pt2_ctx;
typedef int64_t pt2_req;

enum {
    PT2_OK = 0,
    PT2_NOT_READY = 1,      /* pt2_poll: request still running                   */
    PT2_E_INVALID = -1,     /* bad argument or input (see pt2_last_error)        */
    PT2_E_NOMEM = -2,       /* device or host allocation failed / budget too low */
    PT2_E_DEVICE = -3,      /* HIP runtime error or a device-side bound tripped  */
    PT2_E_BUSY = -4,        /* pt2_destroy with requests in flight               */
    PT2_E_SINGULAR = -5,    /* an external E0 - H_aa is exactly zero             */
    PT2_E_UNKNOWN_REQ = -6  /* pt2_poll: no such request                         */
};

enum {
    PT2_EXCLUDE_SEARCH = 0,
    PT2_EXCLUDE_SUBTRACT = 1
};

enum {
    PT2_FP64 = 0,          /* FP64 integrals and numerator terms                 */
    PT2_FP32_PAYLOAD = 1,  /* H_ai c_i computed in FP64 and stored rounded to
                              FP32 (4 bytes less per record and sort pass);
                              N_a, H_aa, denominators and sums stay FP64         */
    PT2_FP32_ARITH = 2     /* as PT2_FP32_PAYLOAD, but the integrals are rounded
                              to FP32 and H_ai c_i is computed in FP32; the
                              rounding of the integrals is shared by every term,
                              so the error in E_PT2 grows with the system (about
                              1e-8 relative at 1e11 terms)                       */
};

typedef struct {
    uint32_t struct_size;          /* sizeof(pt2_options)                            */
    int precision;                 /* PT2_FP64, PT2_FP32_PAYLOAD or PT2_FP32_ARITH   */
    double cutoff;                 /* drop a term when |H_ai c_i| < cutoff (strict;
                                      Section IV uses 1e-8); 0 keeps every term      */
    uint64_t device_budget_bytes;  /* device memory the engine may hold for
                                      record buffers; 0 = 80% of free memory: for
                                      pt2_evaluate* free memory at the call plus
                                      the buffers the context already holds, for
                                      pt2_submit free memory at pt2_create.  The
                                      budget sets the hash split, and the split
                                      sets the summation grouping: for results
                                      that are bit-identical across calls, fix
                                      this or log2_partitions                      */
    uint64_t max_partition_bytes;  /* cap on the record buffers of one subset;
                                      0 = the budget                                 */
    int log2_partitions;           /* -1: the planner picks the split; 0 <= k <= 12
                                      forces 2^k subsets                             */
    int device;                    /* HIP device ordinal                             */
    int n_streams;                 /* requests that may run at once (pt2_submit)     */
    void *(*alloc)(size_t bytes, void *user);        /* optional device allocator   */
    void (*free)(void *ptr, size_t bytes, void *user);
    void *alloc_user;
    void *stream;                  /* hipStream_t for pt2_evaluate*; NULL = own      */
    int timing;                    /* nonzero: time phases with HIP events            */
    int compress_keys;             /* -1 (default): stored terms carry the
                                      combinatorial rank of their determinant
                                      (per spin, sum_i C(o_i, i) over the ascending
                                      occupied orbitals o_i; alpha rank above beta
                                      rank) when both ranks fit 64 bits and this
                                      saves at least 30% of the sort digits;
                                      it orders terms exactly as the bitstrings,
                                      so results are unchanged.  0: always the
                                      bitstring; 1: the rank whenever it fits; 2:
                                      hash records whenever 2 norb <= 254: the
                                      64-bit Zobrist hash of the determinant (8
                                      digit passes whatever norb is) with the parent
                                      index and the flipped spin-orbitals, from
                                      which the single pass rebuilds the bitstring
                                      and separates determinants whose hashes
                                      collide.  The automatic choice takes the form
                                      that moves the fewest bytes through the digit
                                      passes if it saves 30% or more (hash records
                                      priced as 16-byte records of six passes with
                                      FP32 payloads and hash_bits 0; a tie takes
                                      hash records)                                */
    int exclusion;                 /* PT2_EXCLUDE_SEARCH (default): drop reference
                                      determinants by a search of the sorted
                                      reference (Section V, direct check);
                                      PT2_EXCLUDE_SUBTRACT: keep them and subtract
                                      sum_i c_i^2 (E0 - H_ii), exact only when the
                                      coefficients are an eigenvector of H in the
                                      reference space with eigenvalue E0 (Section V,
                                      removal of duplicate contributions).  With
                                      subtraction the counts and checksums cover
                                      every distinct determinant                      */
    int hash_bits;                 /* hash records: bits of the hash kept as the sort
                                      key.  0 (default): per evaluation, the top 32,
                                      40, 48, 56 or 64 bits, the choice with the
                                      fewest digit passes (then the most bits) for
                                      which the expected number of colliding pairs
                                      among the largest subset's N records,
                                      N^2 / 2^(bits - log2p + 1) with 2^log2p
                                      subsets, is N/512 or fewer (collided runs are
                                      resolved exactly).  1-64: exactly that many
                                      low bits (few bits make collisions common, to
                                      test their handling)                          */
    int spin_flip;                 /* 1: use the alpha/beta swap symmetry of an S_z = 0
                                      reference (Section V, spin symmetry): only
                                      determinants whose alpha string is not below
                                      their beta string are generated, and the term
                                      of each with alpha != beta counts twice.  Needs
                                      nalpha == nbeta (else PT2_E_INVALID at create)
                                      and a reference closed under the swap with
                                      c(swap(D)) = c(D) for all D, or = -c(D) for all
                                      D (else PT2_E_INVALID at evaluation).  Counts
                                      and checksums then cover the generated half;
                                      n_contrib stays the structural count of all
                                      terms.  Default 0                              */
    int string_reuse;              /* when every term of every reference is
                                      generated (one subset, no cutoff, no spin
                                      flip) with bitstring keys, same-spin doubles
                                      and their matrix elements are computed once
                                      per group of up to 32 references sharing the
                                      spin string they excite and written for each
                                      of them (Section V, data reuse for unique
                                      alpha and beta strings); the records, and so
                                      every result, are identical.  1 (default):
                                      alpha-alpha doubles, grouped by alpha string;
                                      2: also beta-beta doubles, grouped by beta
                                      string; 0: each reference computes its own   */
    int compact_refs;              /* hash records: 1 (default): when every
                                      reference is within four excitations of the
                                      first sorted one, the single pass rebuilds
                                      parents from that one and up to eight flipped
                                      spin-orbitals per reference (8 B each; 4 B
                                      with up to four flips when every reference
                                      is within two excitations) instead of a full
                                      bitstring per reference; results are
                                      identical.  0: always the full bitstrings    */
} pt2_options;

typedef struct {
    uint32_t struct_size;     /* sizeof(pt2_result), set by the caller               */
    double e_pt2;             /* the energy (FP64)                                   */
    uint64_t n_contrib;       /* structural single+double terms, duplicates and
                                 reference hits included, before the cutoff          */
    uint64_t n_after_cutoff;  /* terms stored and sorted                             */
    uint64_t n_unique;        /* distinct bitstrings among stored terms              */
    uint64_t n_external;      /* distinct bitstrings outside the reference           */
    uint64_t n_in_ref_hit;    /* distinct bitstrings found in the reference          */
    uint32_t n_partitions;    /* subsets evaluated                                   */
    uint32_t n_sort_passes;   /* 8-bit digit passes run, all subsets                 */
    uint32_t record_bytes;    /* bytes of one stored term: key planes + payload     */
    double min_abs_denom;     /* min |E0 - H_aa| over external bitstrings            */
    uint64_t n_nonneg_denom;  /* external bitstrings with E0 - H_aa >= 0             */
    double ref_cross;         /* sum over reference hits of c_i * N_i                */
    uint64_t key_xor;         /* XOR of a 64-bit mix of every external bitstring     */
    uint64_t key_sum;         /* sum (mod 2^64) of the same mix                      */
    double ms_total;          /* wall time of the call (host clock)                  */
    double ms_gen;            /* device time (timing != 0): generation kernels       */
    double ms_sort;           /*   radix digit passes (count, scan, scatter)         */
    double ms_sort_scatter;   /*   of which the rank-and-scatter kernels             */
    double ms_reduce;         /*   single pass and final sum                         */
    double ms_hist;           /*   digit histograms, count pass, reference sort      */
    double ms_sort_pass_max;  /*   slowest single scatter kernel                     */
    double bytes_gen, bytes_sort, bytes_reduce; /* algorithmic bytes per phase (a
                                 digit pass: every record read and written once by
                                 the scatter, the digit's key plane read once by
                                 the count)                                          */
    uint32_t key_bits;        /* bits of the sort key of a stored term (2 norb for
                                 bitstrings, fewer for rank keys, the hash bits
                                 kept for hash records)                              */
    uint64_t n_alpha_groups;  /* groups of references sharing an alpha string whose
                                 alpha-alpha doubles were generated once for the
                                 group (string_reuse); 0 when not used             */
    uint64_t n_beta_groups;   /* the same for beta strings and beta-beta doubles    */
} pt2_result;

/* Fills *opt with defaults (FP64, cutoff 0, planner-chosen split, device 0). */
void pt2_default_options(pt2_options *opt);

/* W = ceil(2*norb/64), the number of uint64 words of a determinant bitstring. */
int pt2_key_words(int norb);

/*
 * The record form pt2_create takes for these sizes and options (opt may be
 * NULL: the defaults).  Host only; no device is touched.  *form = 0 bitstring
 * keys, 1 combinatorial rank keys, 2 hash records (Section V, compression
 * with hash functions), the values compress_keys forces; *key_bits = the bits
 * of that key: 2*norb, the two spin ranks' bits, or 64 for hash records, of
 * which an evaluation keeps 32-64 (hash_bits).  PT2_E_INVALID for a NULL
 * output, sizes out of range, or an option pt2_create rejects for its value.
 */
int pt2_key_form(int norb, int nalpha, int nbeta, const pt2_options *opt, int *form, int *key_bits);

/*
 * Create a context for one Hamiltonian; integrals stay resident on the device.
 *   h    host, norb*norb FP64, row-major, symmetric
 *   eri  host, norb^4 FP64, row-major (pq|rs) at ((p*norb+q)*norb+r)*norb+s,
 *        8-fold symmetric to 1e-12
 *   1 <= norb <= 128, 0 <= nalpha, nbeta <= norb
 *   opt  may be NULL (defaults)
 * Errors: PT2_E_INVALID (sizes, symmetry), PT2_E_NOMEM, PT2_E_DEVICE.
 */
int pt2_create(const double *h, const double *eri, int norb, int nalpha, int nbeta,
               const pt2_options *opt, pt2_ctx **out);

/*
 * Synchronous evaluation from host arrays (Algorithm 2 over the planner's
 * split, Algorithm 1 within each subset).
 *   dets    host, ndets x W uint64 (row i = determinant i)
 *   coeffs  host, ndets FP64 (used as given; the library never normalises)
 *   e0      the variational energy E_ASCI of the Epstein-Nesbet equation
 *   out     result; out->struct_size must be sizeof(pt2_result)
 * Every determinant must have nalpha alpha and nbeta beta electrons, no bits
 * at or above 2*norb, and no determinant may repeat (PT2_E_INVALID).
 * Returns PT2_E_SINGULAR if an external E0 - H_aa is exactly zero.
 */
int pt2_evaluate(pt2_ctx *ctx, const uint64_t *dets, const double *coeffs, int64_t ndets,
                 double e0, pt2_result *out);

/*
 * As pt2_evaluate, but dets and coeffs are device pointers already resident
 * in HBM (same layout).  Work is queued on opt->stream (or the context's
 * stream); the call returns after the result has been copied to the host.
 * Input checks run on the device; a violation returns PT2_E_INVALID.
 */
int pt2_evaluate_device(pt2_ctx *ctx, const uint64_t *d_dets, const double *d_coeffs,
                        int64_t ndets, double e0, pt2_result *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * pt2_evaluate_device, but the call allocates nothing.  Every device buffer
 * of the evaluation (reference planes, record and sort buffers, counts,
 * partial sums, control data) is carved from one static device array of
 * 256 MiB that the library holds on each device it runs on until the
 * process ends; no hipMalloc, hipFree, pinned host allocation, stream or
 * event is created, and per-kernel timings are not recorded.  The record
 * buffers of one subset are planned to fit 60% of it (the planner splits
 * the work into more subsets as needed); an evaluation that does not fit
 * returns PT2_E_NOMEM with a message naming the scratch size.  The call
 * clears what must start at zero and returns after its work is done.  All
 * calls on one device share the array: calls that overlap on one device
 * (different contexts or threads) race.  Inputs, errors and results as
 * pt2_evaluate_device.
 */
int pt2_evaluate_device_noalloc(pt2_ctx *ctx, const uint64_t *d_dets, const double *d_coeffs,
                                int64_t ndets, double e0, pt2_result *out);

/*
 * Evaluate only the listed subsets of a 2^log2p split (0 <= log2p <= 12) of the external space
 * (Algorithm 2; each subset on its own), from host arrays.
 *   parts   host, nparts distinct subset indices in [0, 2^log2p) (an index
 *           out of range or listed twice: PT2_E_INVALID)
 *   e_parts host, nparts FP64 outputs, the energy of each listed subset
 * out holds the totals over the listed subsets.  Used to check sampled
 * subsets of large workloads, and to shard a workload over devices.
 */
int pt2_evaluate_parts(pt2_ctx *ctx, const uint64_t *dets, const double *coeffs, int64_t ndets,
                       double e0, int log2p, const uint32_t *parts, int nparts, double *e_parts,
                       pt2_result *out);

/*
 * As pt2_evaluate_parts, but d_dets and d_coeffs are device pointers already
 * resident in HBM (layout as pt2_evaluate); parts and e_parts stay host
 * arrays.  Evaluating the 2^log2p subsets in several calls of contiguous
 * groups, and summing e_parts in subset order, gives the full energy with
 * each call's work bounded (Algorithm 2: the subsets are independent).
 */
int pt2_evaluate_parts_device(pt2_ctx *ctx, const uint64_t *d_dets, const double *d_coeffs,
                              int64_t ndets, double e0, int log2p, const uint32_t *parts, int nparts,
                              double *e_parts, pt2_result *out);

/*
 * Serving form.  pt2_submit copies dets and coeffs (host arrays) and queues
 * the request; it returns at once with a request id.  Requests of every
 * context share one device scheduler: a request starts when a stream is free
 * and its projected record-buffer bytes fit in the device budget, and runs
 * concurrently with the others.  pt2_poll returns PT2_NOT_READY until the
 * request is done, then fills *out once and forgets the id (a second poll
 * returns PT2_E_UNKNOWN_REQ).  A request that fails reports its error code
 * from pt2_poll.  pt2_wait blocks until the request is done.
 */
int pt2_submit(pt2_ctx *ctx, const uint64_t *dets, const double *coeffs, int64_t ndets,
               double e0, pt2_req *out);
int pt2_poll(pt2_ctx *ctx, pt2_req req, pt2_result *out);
int pt2_wait(pt2_ctx *ctx, pt2_req req, pt2_result *out);

/* Free the context; PT2_E_BUSY (and nothing freed) while requests are in flight. */
int pt2_destroy(pt2_ctx *ctx);

/* Message describing the last error on the calling thread ("" if none). */
const char *pt2_last_error(void);

/*
 * Inspection entry points (small inputs; single subset, 2^0 split).
 *
 * pt2_dump_records: the generated terms in generation order (sorted == 0) or
 * after the radix sort (sorted != 0).  keys_out: cap x W uint64 (row-major);
 * payload_out: cap FP64 (FP32 terms are widened).  *n_out = number of terms
 * (only the first cap are written).
 *
 * pt2_dump_numerators: every distinct bitstring with its numerator N_a,
 * ascending, and in_ref_out[k] = 1 if it is in the reference.
 */
int pt2_dump_records(pt2_ctx *ctx, const uint64_t *dets, const double *coeffs, int64_t ndets,
                     int sorted, uint64_t *keys_out, double *payload_out, int64_t cap,
                     int64_t *n_out);
int pt2_dump_numerators(pt2_ctx *ctx, const uint64_t *dets, const double *coeffs, int64_t ndets,
                        uint64_t *keys_out, double *num_out, uint8_t *in_ref_out, int64_t cap,
                        int64_t *n_out);

/*
 * The engine's stable LSD radix sort on its own (Algorithm 1, sort step):
 * sorts n records by the low key_bits bits of their W-word keys, ascending,
 * equal keys keeping their input order.  keys: host, n x W uint64 row-major
 * (sorted in place); payload: host, n elements of payload_bytes (4 or 8),
 * permuted alongside.  device selects the GPU.
 */
int pt2_sort_records(int device, int W, int key_bits, uint64_t *keys, void *payload,
                     int payload_bytes, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* PT2_H */
