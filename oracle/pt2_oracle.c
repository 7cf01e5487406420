/*
 * FP64 CPU oracle for the Epstein-Nesbet PT2 energy of a selected-CI
 * reference.  TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and
 * the benchmark's CPU-baseline leg load this file.  It shares no code with
 * the HIP engine.
 *
 * What it computes (Tubman et al., arXiv:1808.02049):
 *   E_PT2 = sum over determinants a outside the reference set R of
 *           N_a^2 / (E0 - H_aa),   N_a = sum_{i in R} H_ai c_i
 * (Section II, the Epstein-Nesbet equation; the sum is restricted to
 * determinants not in the reference, as Algorithm 1 and the duplicate-removal
 * subsection of Section V state; Algorithm 1 prints the per-determinant term
 * without the square, which is read as the square of the summed numerator so
 * that it agrees with the Epstein-Nesbet equation).
 *
 * How (Algorithm 1, fundamental algorithm; Algorithm 2 for the constraint
 * loop): every reference determinant is expanded into all its single and
 * double excitations; each emits the pair (bitstring, H_ai * c_i); the pairs
 * are grouped by bitstring with the C library's qsort (a library primitive);
 * a single pass over the groups forms N_a, skips bitstrings present in the
 * reference (found by bsearch), forms the denominator E0 - H_aa from scratch
 * as one compensated sum (orc_denominator: exact to a few units in the last
 * place of the difference, which near-singular denominators need) and
 * accumulates the energy with Neumaier compensated summation.
 *
 * Constraints: the external space is split into 2^k non-overlapping, complete
 * subsets by the top k bits of a Zobrist hash of the bitstring (XOR of one
 * random word per set bit; the words come from the SplitMix64 generator of
 * Steele, Lea and Flood (2014) seeded with 0x5054325F5A4F4252).  This replaces
 * the paper's triplet constraint (Section III) by a hash constraint, which has
 * the same two properties the method needs: every bitstring belongs to exactly
 * one subset, and the subset is a function of the bitstring alone.
 *
 * Conventions (the paper is silent on them): real orbitals, chemists'
 * notation (pq|rs), no constant energy term; determinant
 * |D> = prod over occupied spin-orbitals in ascending bit order of creators;
 * beta orbital p is bit p, alpha orbital p is bit norb+p (alpha most
 * significant, as the triplet-constraint subsection fixes).
 *
 * Fermionic phases are counted with explicit loops over the orbitals lying
 * strictly between the two indices, never with popcount.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXW 4
#define ORC_MAXORB 128
#define ORC_MAXTHREADS 256

typedef struct {
    int norb, nalpha, nbeta;
    const double *h;   /* norb*norb, symmetric                  */
    const double *eri; /* norb^4, (pq|rs) at ((p*n+q)*n+r)*n+s   */
} orc_system;

typedef struct {
    double e_pt2;
    uint64_t n_contrib;      /* structural candidates in the evaluated subsets */
    uint64_t n_kept;         /* after the numerator cutoff                    */
    uint64_t n_unique;       /* distinct bitstrings among kept records        */
    uint64_t n_external;     /* distinct bitstrings not in the reference      */
    uint64_t n_in_ref_hit;   /* distinct bitstrings found in the reference    */
    double min_abs_denom;
    uint64_t n_nonneg_denom;
    double ref_cross;        /* sum over hits of c_i * N_i                    */
    uint64_t key_xor;        /* XOR of mix(key) over external bitstrings      */
    uint64_t key_sum;        /* sum of mix(key) over external bitstrings      */
} orc_result;

/* ------------------------------------------------------------------------ */
/* bit helpers                                                               */

int orc_key_words(int norb) { return (2 * norb + 63) / 64; }

static int get_bit(const uint64_t *k, int b) { return (int)((k[b >> 6] >> (b & 63)) & 1u); }
static void flip_bit(uint64_t *k, int b) { k[b >> 6] ^= (uint64_t)1 << (b & 63); }

/* spin 0 = alpha, spin 1 = beta */
static int spin_bit(const orc_system *s, int spin, int p) { return spin == 0 ? s->norb + p : p; }

static double ERI(const orc_system *s, int p, int q, int r, int t)
{
    size_t n = (size_t)s->norb;
    return s->eri[((p * n + q) * n + r) * n + t];
}

static double H1(const orc_system *s, int p, int q) { return s->h[(size_t)p * s->norb + q]; }

/* (-1)^(number of occupied orbitals of this spin strictly between from and to) */
static int phase_move(const orc_system *s, const uint64_t *key, int spin, int from, int to)
{
    int lo = from < to ? from : to, hi = from < to ? to : from, cnt = 0;
    for (int p = lo + 1; p < hi; p++)
        cnt += get_bit(key, spin_bit(s, spin, p));
    return (cnt & 1) ? -1 : 1;
}

/* ------------------------------------------------------------------------ */
/* Zobrist hash and the partition (constraint) function                      */

static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_zobrist_table(int norb, uint64_t *R)
{
    uint64_t st = 0x5054325F5A4F4252ull;
    for (int b = 0; b < 2 * norb; b++)
        R[b] = splitmix64_next(&st);
}

static uint64_t zobrist(const uint64_t *R, const uint64_t *key, int nbits)
{
    uint64_t z = 0;
    for (int b = 0; b < nbits; b++)
        if (get_bit(key, b))
            z ^= R[b];
    return z;
}

static uint32_t part_of(uint64_t z, int log2p) { return log2p == 0 ? 0u : (uint32_t)(z >> (64 - log2p)); }

/* A 64-bit mix of a bitstring, for order-independent checksums of key sets. */
static uint64_t key_mix(const uint64_t *key, int W)
{
    uint64_t acc = 0x243F6A8885A308D3ull;
    for (int w = 0; w < W; w++) {
        uint64_t st = key[w] ^ acc;
        acc = splitmix64_next(&st);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Matrix elements                                                          */

/* Neumaier's compensated summation: sum + comp carries the running total,
 * comp the exact rounding errors of the additions (each recovered by the
 * two-sum error-free transformation). */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/* <D|H|D> from scratch:  sum_p h_pp + sum_{p<q} [(pp|qq) - delta_spin (pq|qp)] */
double orc_diag(const orc_system *s, const uint64_t *key)
{
    int orb[2 * ORC_MAXORB], spn[2 * ORC_MAXORB], n = 0;
    for (int spin = 0; spin < 2; spin++)
        for (int p = 0; p < s->norb; p++)
            if (get_bit(key, spin_bit(s, spin, p))) {
                orb[n] = p;
                spn[n] = spin;
                n++;
            }
    double e = 0.0;
    for (int i = 0; i < n; i++) {
        e += H1(s, orb[i], orb[i]);
        for (int j = i + 1; j < n; j++) {
            e += ERI(s, orb[i], orb[i], orb[j], orb[j]);
            if (spn[i] == spn[j])
                e -= ERI(s, orb[i], orb[j], orb[j], orb[i]);
        }
    }
    return e;
}

/* The Epstein-Nesbet denominator E0 - <D|H|D> (Section II), as ONE
 * compensated sum of E0 and the negated diagonal summands.
 *
 * E0 and <D|H|D> are each of order 10^2 Eh while their difference can be
 * 10^-6 Eh or less for some external determinants, and such a determinant's
 * term N^2 / (E0 - H_DD) moves by its own size for every relative change of
 * the difference.  Rounding <D|H|D> to FP64 first (orc_diag) leaves an error
 * of about 1e-13 Eh in the difference, which is amplified there by
 * (N / (E0 - H_DD))^2, up to 1e6 on the synthetic systems.  Every summand here
 * (E0, -h_pp, -(pp|qq), +(pq|qp)) is an exact FP64 number, and the
 * compensated sum returns their exact total to within a few units in the last
 * place of the total itself, whatever its size. */
double orc_denominator(const orc_system *s, const uint64_t *key, double e0)
{
    int orb[2 * ORC_MAXORB], spn[2 * ORC_MAXORB], n = 0;
    for (int spin = 0; spin < 2; spin++)
        for (int p = 0; p < s->norb; p++)
            if (get_bit(key, spin_bit(s, spin, p))) {
                orb[n] = p;
                spn[n] = spin;
                n++;
            }
    double sum = e0, comp = 0.0;
    for (int i = 0; i < n; i++) {
        neumaier_add(&sum, &comp, -H1(s, orb[i], orb[i]));
        for (int j = i + 1; j < n; j++) {
            neumaier_add(&sum, &comp, -ERI(s, orb[i], orb[i], orb[j], orb[j]));
            if (spn[i] == spn[j])
                neumaier_add(&sum, &comp, ERI(s, orb[i], orb[j], orb[j], orb[i]));
        }
    }
    return sum + comp;
}

/* <D'|H|D> for D' = D with r -> a in one spin (phase excluded):
 * h_ra + sum_{j occ, any spin} (ra|jj) - sum_{j occ, same spin} (rj|ja)      */
static double single_value(const orc_system *s, const uint64_t *key, int spin, int r, int a)
{
    double v = H1(s, r, a);
    for (int t = 0; t < 2; t++)
        for (int j = 0; j < s->norb; j++) {
            if (!get_bit(key, spin_bit(s, t, j)))
                continue;
            v += ERI(s, r, a, j, j);
            if (t == spin)
                v -= ERI(s, r, j, j, a);
        }
    return v;
}

/* Same-spin double r<s -> a<b applied as r->a then s->b. */
static double double_same(const orc_system *sy, const uint64_t *key, int spin, int r, int s, int a, int b)
{
    uint64_t mid[ORC_MAXW];
    int W = orc_key_words(sy->norb);
    memcpy(mid, key, sizeof(uint64_t) * W);
    int ph1 = phase_move(sy, key, spin, r, a);
    flip_bit(mid, spin_bit(sy, spin, r));
    flip_bit(mid, spin_bit(sy, spin, a));
    int ph2 = phase_move(sy, mid, spin, s, b);
    return (double)(ph1 * ph2) * (ERI(sy, r, a, s, b) - ERI(sy, r, b, s, a));
}

/* Opposite-spin double: alpha r->a, beta s->b. */
static double double_opp(const orc_system *sy, const uint64_t *key, int r, int a, int s, int b)
{
    int ph = phase_move(sy, key, 0, r, a) * phase_move(sy, key, 1, s, b);
    return (double)ph * ERI(sy, r, a, s, b);
}

/* General <Di|H|Dj> (Slater-Condon rules; zero beyond double excitations). */
double orc_hij(const orc_system *s, const uint64_t *ki, const uint64_t *kj)
{
    int rem[2][2], add[2][2], nrem[2] = {0, 0}, nadd[2] = {0, 0}, total = 0;
    for (int spin = 0; spin < 2; spin++)
        for (int p = 0; p < s->norb; p++) {
            int b = spin_bit(s, spin, p);
            int in_i = get_bit(ki, b), in_j = get_bit(kj, b);
            if (in_j && !in_i) {
                if (nrem[spin] >= 2 || total >= 2)
                    return 0.0;
                rem[spin][nrem[spin]++] = p;
                total++;
            } else if (in_i && !in_j) {
                if (nadd[spin] >= 2)
                    return 0.0;
                add[spin][nadd[spin]++] = p;
            }
        }
    if (nrem[0] != nadd[0] || nrem[1] != nadd[1])
        return 0.0; /* different particle numbers per spin */
    if (total == 0)
        return orc_diag(s, ki);
    if (total == 1) {
        int spin = nrem[0] ? 0 : 1;
        int r = rem[spin][0], a = add[spin][0];
        return phase_move(s, kj, spin, r, a) * single_value(s, kj, spin, r, a);
    }
    if (nrem[0] == 2 || nrem[1] == 2) {
        int spin = nrem[0] == 2 ? 0 : 1;
        return double_same(s, kj, spin, rem[spin][0], rem[spin][1], add[spin][0], add[spin][1]);
    }
    return double_opp(s, kj, rem[0][0], add[0][0], rem[1][0], add[1][0]);
}

/* ------------------------------------------------------------------------ */
/* Excitation enumeration                                                    */

typedef struct {
    uint64_t key[ORC_MAXW];
    double v;
    uint64_t seq; /* emission order: (reference index, local index) flattened */
} orc_rec;

typedef struct {
    orc_rec *r;
    size_t n, cap;
} orc_vec;

static int vec_push(orc_vec *v, const uint64_t *key, int W, double val, uint64_t seq)
{
    if (v->n == v->cap) {
        size_t nc = v->cap ? 2 * v->cap : 4096;
        orc_rec *nr = (orc_rec *)realloc(v->r, nc * sizeof(orc_rec));
        if (!nr)
            return -1;
        v->r = nr;
        v->cap = nc;
    }
    orc_rec *o = &v->r[v->n++];
    memset(o->key, 0, sizeof(o->key));
    memcpy(o->key, key, sizeof(uint64_t) * W);
    o->v = val;
    o->seq = seq;
    return 0;
}

typedef struct {
    const orc_system *s;
    const uint64_t *R; /* Zobrist table */
    int W, log2p;
    double cutoff;
    /* slot[part]: where records of that subset go (index into outs), or -1
     * for a subset not evaluated; with log2p == 0 everything goes to slot 0 */
    const int32_t *slot;
    uint64_t *n_candidates; /* per slot: candidates whose subset is kept */
    orc_vec *outs;          /* per slot: emitted records */
} orc_emit_ctx;

/* Slot of a candidate with Zobrist hash z (-1: its subset is not evaluated).
 * Tested before the matrix element is evaluated.  z is the parent's hash XOR
 * the words of the flipped bits (XOR hashing is incremental by construction). */
static int kept(const orc_emit_ctx *E, uint64_t z) { return E->log2p == 0 ? 0 : E->slot[part_of(z, E->log2p)]; }

/* Emit one candidate of a kept subset if it passes the cutoff. */
static int emit(orc_emit_ctx *E, int slot, const uint64_t *key, double hval, double ci, uint64_t seq)
{
    E->n_candidates[slot]++;
    double v = hval * ci;
    if (E->cutoff > 0.0 && fabs(v) < E->cutoff)
        return 0;
    return vec_push(&E->outs[slot], key, E->W, v, seq);
}

/* All singles and doubles of one reference determinant, in a fixed order:
 * alpha singles, beta singles, alpha-alpha doubles, beta-beta doubles,
 * alpha-beta doubles. */
static int expand_det(orc_emit_ctx *E, const uint64_t *key, double ci, uint64_t seq0)
{
    const orc_system *s = E->s;
    int n = s->norb, W = E->W;
    uint64_t k1[ORC_MAXW], k2[ORC_MAXW];
    uint64_t seq = seq0;
    const uint64_t zp = zobrist(E->R, key, 2 * n);
    const uint64_t *R = E->R;

    for (int spin = 0; spin < 2; spin++)
        for (int r = 0; r < n; r++) {
            if (!get_bit(key, spin_bit(s, spin, r)))
                continue;
            for (int a = 0; a < n; a++) {
                if (get_bit(key, spin_bit(s, spin, a)))
                    continue;
                memcpy(k1, key, sizeof(uint64_t) * W);
                flip_bit(k1, spin_bit(s, spin, r));
                flip_bit(k1, spin_bit(s, spin, a));
                uint64_t z = zp ^ R[spin_bit(s, spin, r)] ^ R[spin_bit(s, spin, a)];
                const int sl = kept(E, z);
                if (sl < 0) {
                    seq++;
                    continue;
                }
                double hv = phase_move(s, key, spin, r, a) * single_value(s, key, spin, r, a);
                if (emit(E, sl, k1, hv, ci, seq++))
                    return -1;
            }
        }

    for (int spin = 0; spin < 2; spin++)
        for (int r = 0; r < n; r++) {
            if (!get_bit(key, spin_bit(s, spin, r)))
                continue;
            for (int t = r + 1; t < n; t++) {
                if (!get_bit(key, spin_bit(s, spin, t)))
                    continue;
                for (int a = 0; a < n; a++) {
                    if (get_bit(key, spin_bit(s, spin, a)))
                        continue;
                    for (int b = a + 1; b < n; b++) {
                        if (get_bit(key, spin_bit(s, spin, b)))
                            continue;
                        memcpy(k2, key, sizeof(uint64_t) * W);
                        flip_bit(k2, spin_bit(s, spin, r));
                        flip_bit(k2, spin_bit(s, spin, t));
                        flip_bit(k2, spin_bit(s, spin, a));
                        flip_bit(k2, spin_bit(s, spin, b));
                        uint64_t z = zp ^ R[spin_bit(s, spin, r)] ^ R[spin_bit(s, spin, t)] ^
                                     R[spin_bit(s, spin, a)] ^ R[spin_bit(s, spin, b)];
                        const int sl = kept(E, z);
                        if (sl < 0) {
                            seq++;
                            continue;
                        }
                        double hv = double_same(s, key, spin, r, t, a, b);
                        if (emit(E, sl, k2, hv, ci, seq++))
                            return -1;
                    }
                }
            }
        }

    for (int r = 0; r < n; r++) {
        if (!get_bit(key, spin_bit(s, 0, r)))
            continue;
        for (int a = 0; a < n; a++) {
            if (get_bit(key, spin_bit(s, 0, a)))
                continue;
            for (int t = 0; t < n; t++) {
                if (!get_bit(key, spin_bit(s, 1, t)))
                    continue;
                for (int b = 0; b < n; b++) {
                    if (get_bit(key, spin_bit(s, 1, b)))
                        continue;
                    uint64_t z = zp ^ R[spin_bit(s, 0, r)] ^ R[spin_bit(s, 0, a)] ^ R[spin_bit(s, 1, t)] ^
                                 R[spin_bit(s, 1, b)];
                    const int sl = kept(E, z);
                    if (sl < 0) {
                        seq++;
                        continue;
                    }
                    memcpy(k2, key, sizeof(uint64_t) * W);
                    flip_bit(k2, spin_bit(s, 0, r));
                    flip_bit(k2, spin_bit(s, 0, a));
                    flip_bit(k2, spin_bit(s, 1, t));
                    flip_bit(k2, spin_bit(s, 1, b));
                    double hv = double_opp(s, key, r, a, t, b);
                    if (emit(E, sl, k2, hv, ci, seq++))
                        return -1;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Grouping and the single pass                                              */

static int cmp_key(const uint64_t *a, const uint64_t *b, int W)
{
    for (int w = W - 1; w >= 0; w--) {
        if (a[w] < b[w])
            return -1;
        if (a[w] > b[w])
            return 1;
    }
    return 0;
}

static int cmp_rec(const void *pa, const void *pb)
{
    const orc_rec *a = (const orc_rec *)pa, *b = (const orc_rec *)pb;
    int c = cmp_key(a->key, b->key, ORC_MAXW); /* unused words are zero */
    if (c)
        return c;
    return a->seq < b->seq ? -1 : (a->seq > b->seq ? 1 : 0);
}

typedef struct {
    const uint64_t *keys; /* sorted reference keys, n x W */
    const double *c;      /* coefficients in the same order */
    int64_t n;
    int W;
} orc_refset;

static int64_t ref_find(const orc_refset *R, const uint64_t *key)
{
    int64_t lo = 0, hi = R->n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_key(R->keys + mid * R->W, key, R->W);
        if (c == 0)
            return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* Walk records sorted by (key, seq). Returns the subset energy (compensated). */
static double single_pass(const orc_system *s, const orc_refset *R, double e0, orc_rec *rec, size_t n,
                          orc_result *res)
{
    int W = R->W;
    double sum = 0.0, comp = 0.0;
    size_t i = 0;
    while (i < n) {
        size_t j = i;
        double num = 0.0;
        while (j < n && cmp_key(rec[j].key, rec[i].key, W) == 0) {
            num += rec[j].v;
            j++;
        }
        res->n_unique++;
        int64_t hit = ref_find(R, rec[i].key);
        if (hit >= 0) {
            res->n_in_ref_hit++;
            res->ref_cross += R->c[hit] * num;
        } else {
            double denom = orc_denominator(s, rec[i].key, e0);
            res->n_external++;
            if (fabs(denom) < res->min_abs_denom)
                res->min_abs_denom = fabs(denom);
            if (denom >= 0.0)
                res->n_nonneg_denom++;
            neumaier_add(&sum, &comp, num * num / denom);
            uint64_t m = key_mix(rec[i].key, W);
            res->key_xor ^= m;
            res->key_sum += m;
        }
        i = j;
    }
    return sum + comp;
}

/* ------------------------------------------------------------------------ */
/* Driver                                                                    */

static void result_init(orc_result *r)
{
    memset(r, 0, sizeof(*r));
    r->min_abs_denom = INFINITY;
}

/* Expansion of a contiguous slice of the reference determinants into the
 * slots of the subsets being evaluated (one job per thread). */
typedef struct {
    const uint64_t *dets;
    const double *c;
    int64_t lo, hi;
    orc_emit_ctx E;
    int err;
} gen_job;

static void *gen_worker(void *arg)
{
    gen_job *J = (gen_job *)arg;
    for (int64_t i = J->lo; i < J->hi; i++)
        if (expand_det(&J->E, J->dets + i * J->E.W, J->c[i], (uint64_t)i << 32)) {
            J->err = -1;
            return NULL;
        }
    return NULL;
}

/* Grouping and single pass of the slots first, first+stride, ... */
typedef struct {
    const orc_system *s;
    const orc_refset *refs;
    double e0;
    gen_job *gen;
    int ngen, nslot, stride, first;
    double *e_slot;
    orc_result *res_slot;
    int err;
} pass_job;

static void *pass_worker(void *arg)
{
    pass_job *J = (pass_job *)arg;
    for (int k = J->first; k < J->nslot; k += J->stride) {
        orc_result *res = &J->res_slot[k];
        result_init(res);
        size_t tot = 0;
        for (int t = 0; t < J->ngen; t++) {
            tot += J->gen[t].E.outs[k].n;
            res->n_contrib += J->gen[t].E.n_candidates[k];
        }
        orc_rec *all = (orc_rec *)malloc(sizeof(orc_rec) * (tot ? tot : 1));
        if (!all) {
            J->err = -1;
            return NULL;
        }
        size_t o = 0;
        for (int t = 0; t < J->ngen; t++) {
            orc_vec *v = &J->gen[t].E.outs[k];
            if (v->n)
                memcpy(all + o, v->r, sizeof(orc_rec) * v->n);
            o += v->n;
            free(v->r);
            v->r = NULL, v->n = v->cap = 0;
        }
        res->n_kept = tot;
        /* the sequence number makes the order total: emission order within a key */
        qsort(all, tot, sizeof(orc_rec), cmp_rec);
        J->e_slot[k] = single_pass(J->s, J->refs, J->e0, all, tot, res);
        res->e_pt2 = J->e_slot[k];
        free(all);
    }
    return NULL;
}

static void run_threads(void *(*fn)(void *), void *jobs, size_t size, int nt)
{
    pthread_t th[ORC_MAXTHREADS];
    if (nt == 1) {
        fn(jobs);
        return;
    }
    for (int t = 0; t < nt; t++)
        pthread_create(&th[t], NULL, fn, (char *)jobs + (size_t)t * size);
    for (int t = 0; t < nt; t++)
        pthread_join(th[t], NULL);
}

/* Expand every reference determinant once for the subsets parts[0..nslot)
 * (threads over slices of the reference), then group and pass each subset
 * (threads over subsets).  The records of a subset are the same set, and
 * after sorting by (bitstring, emission order) in the same order, whatever
 * the thread count. */
static int run_batch(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, double e0,
                     double cutoff, int log2p, const uint64_t *R, const orc_refset *refs, int32_t *slot,
                     const uint32_t *parts, int nslot, int nthreads, double *e_slot, orc_result *res_slot)
{
    const int W = orc_key_words(s->norb);
    int ng = nthreads;
    if (ng > n)
        ng = n > 0 ? (int)n : 1;
    if (log2p > 0)
        for (int k = 0; k < nslot; k++)
            slot[parts[k]] = k;
    gen_job *gen = (gen_job *)calloc((size_t)ng, sizeof(gen_job));
    int err = gen ? 0 : -1;
    for (int t = 0; t < ng && !err; t++) {
        gen_job *g = &gen[t];
        g->dets = dets, g->c = c;
        g->lo = n * t / ng, g->hi = n * (t + 1) / ng;
        g->E.s = s, g->E.R = R, g->E.W = W, g->E.log2p = log2p, g->E.cutoff = cutoff, g->E.slot = slot;
        g->E.n_candidates = (uint64_t *)calloc((size_t)nslot, sizeof(uint64_t));
        g->E.outs = (orc_vec *)calloc((size_t)nslot, sizeof(orc_vec));
        if (!g->E.n_candidates || !g->E.outs)
            err = -1;
    }
    if (!err) {
        run_threads(gen_worker, gen, sizeof(gen_job), ng);
        for (int t = 0; t < ng; t++)
            if (gen[t].err)
                err = -1;
    }
    if (!err) {
        int np = nthreads < nslot ? nthreads : nslot;
        pass_job *pj = (pass_job *)calloc((size_t)np, sizeof(pass_job));
        if (!pj)
            err = -1;
        for (int t = 0; t < np && !err; t++) {
            pass_job j = {s, refs, e0, gen, ng, nslot, np, t, e_slot, res_slot, 0};
            pj[t] = j;
        }
        if (!err) {
            run_threads(pass_worker, pj, sizeof(pass_job), np);
            for (int t = 0; t < np; t++)
                if (pj[t].err)
                    err = -1;
        }
        free(pj);
    }
    if (log2p > 0)
        for (int k = 0; k < nslot; k++)
            slot[parts[k]] = -1;
    for (int t = 0; gen && t < ng; t++) {
        for (int k = 0; gen[t].E.outs && k < nslot; k++)
            free(gen[t].E.outs[k].r);
        free(gen[t].E.outs), free(gen[t].E.n_candidates);
    }
    free(gen);
    return err;
}

static int cmp_idx_W;
static const uint64_t *cmp_idx_keys;
static int cmp_idx(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return cmp_key(cmp_idx_keys + a * cmp_idx_W, cmp_idx_keys + b * cmp_idx_W, cmp_idx_W);
}

/*
 * Evaluate the PT2 energy restricted to the listed subsets of a 2^log2p
 * split of the external space (parts == NULL: all subsets).  Subsets are
 * taken nthreads at a time; per-subset results are combined in list order,
 * so the result does not depend on the thread count.
 *
 * Returns 0 on success, -1 on allocation failure, -2 on invalid input
 * (duplicate reference determinants).
 */
int orc_pt2(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, double e0, double cutoff,
            int log2p, const uint32_t *parts, int nparts, int nthreads, orc_result *total, double *e_part)
{
    int W = orc_key_words(s->norb);
    uint64_t R[2 * ORC_MAXORB];
    orc_zobrist_table(s->norb, R);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > ORC_MAXTHREADS)
        nthreads = ORC_MAXTHREADS;

    /* sorted reference set (input order kept for emission) */
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    uint64_t *rk = (uint64_t *)malloc(sizeof(uint64_t) * W * (n > 0 ? n : 1));
    double *rc = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!idx || !rk || !rc) {
        free(idx), free(rk), free(rc);
        return -1;
    }
    for (int64_t i = 0; i < n; i++)
        idx[i] = i;
    cmp_idx_W = W;
    cmp_idx_keys = dets;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_idx);
    for (int64_t i = 0; i < n; i++) {
        memcpy(rk + i * W, dets + idx[i] * W, sizeof(uint64_t) * W);
        rc[i] = c[idx[i]];
        if (i > 0 && cmp_key(rk + i * W, rk + (i - 1) * W, W) == 0) {
            free(idx), free(rk), free(rc);
            return -2;
        }
    }
    orc_refset refs = {rk, rc, n, W};

    uint32_t *all = NULL;
    if (!parts) {
        nparts = 1 << log2p;
        all = (uint32_t *)malloc(sizeof(uint32_t) * nparts);
        for (int p = 0; p < nparts; p++)
            all[p] = (uint32_t)p;
        parts = all;
    }
    orc_result *rp = (orc_result *)calloc((size_t)(nparts > 0 ? nparts : 1), sizeof(orc_result));
    double *ep = (double *)calloc((size_t)(nparts > 0 ? nparts : 1), sizeof(double));
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * ((size_t)1 << log2p));
    int err = (rp && ep && slot) ? 0 : -1;
    for (size_t p = 0; slot && p < ((size_t)1 << log2p); p++)
        slot[p] = -1;
    for (int k0 = 0; k0 < nparts && !err; k0 += nthreads) {
        int nb = nparts - k0 < nthreads ? nparts - k0 : nthreads;
        err = run_batch(s, dets, c, n, e0, cutoff, log2p, R, &refs, slot, parts + k0, nb, nthreads, ep + k0,
                        rp + k0);
    }

    result_init(total);
    double sum = 0.0, comp = 0.0;
    for (int k = 0; k < nparts && !err; k++) {
        neumaier_add(&sum, &comp, ep[k]);
        if (e_part)
            e_part[k] = ep[k];
        total->n_contrib += rp[k].n_contrib;
        total->n_kept += rp[k].n_kept;
        total->n_unique += rp[k].n_unique;
        total->n_external += rp[k].n_external;
        total->n_in_ref_hit += rp[k].n_in_ref_hit;
        if (rp[k].min_abs_denom < total->min_abs_denom)
            total->min_abs_denom = rp[k].min_abs_denom;
        total->n_nonneg_denom += rp[k].n_nonneg_denom;
        total->ref_cross += rp[k].ref_cross;
        total->key_xor ^= rp[k].key_xor;
        total->key_sum += rp[k].key_sum;
    }
    total->e_pt2 = sum + comp;
    free(all), free(rp), free(ep), free(slot), free(idx), free(rk), free(rc);
    return err;
}

/* Records of one subset in emission order (single thread). */
static int emit_one(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, double cutoff,
                    int log2p, uint32_t part, orc_vec *v, uint64_t *ncand)
{
    int W = orc_key_words(s->norb);
    uint64_t R[2 * ORC_MAXORB];
    orc_zobrist_table(s->norb, R);
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * ((size_t)1 << log2p));
    if (!slot)
        return -1;
    for (size_t p = 0; p < ((size_t)1 << log2p); p++)
        slot[p] = -1;
    slot[part] = 0;
    orc_emit_ctx E = {s, R, W, log2p, cutoff, slot, ncand, v};
    int err = 0;
    for (int64_t i = 0; i < n && !err; i++)
        err = expand_det(&E, dets + i * W, c[i], (uint64_t)i << 32);
    free(slot);
    return err;
}

/*
 * Emit the raw (bitstring, H_ai c_i) records of one subset, in emission order,
 * without grouping.  Returns the number of records (which may exceed cap; only
 * the first cap are written), or -1 on allocation failure.
 */
int64_t orc_emit(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, double cutoff, int log2p,
                 uint32_t part, uint64_t *keys_out, double *vals_out, int64_t cap)
{
    int W = orc_key_words(s->norb);
    orc_vec v = {NULL, 0, 0};
    uint64_t ncand = 0;
    if (emit_one(s, dets, c, n, cutoff, log2p, part, &v, &ncand)) {
        free(v.r);
        return -1;
    }
    for (size_t i = 0; i < v.n && (int64_t)i < cap; i++) {
        memcpy(keys_out + i * W, v.r[i].key, sizeof(uint64_t) * W);
        vals_out[i] = v.r[i].v;
    }
    int64_t cnt = (int64_t)v.n;
    free(v.r);
    return cnt;
}

/*
 * The distinct bitstrings of one subset with their numerators N_a, sorted
 * ascending.  Returns the count (only the first cap are written) or -1 on
 * allocation failure.
 */
int64_t orc_numerators(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, int log2p,
                       uint32_t part, uint64_t *keys_out, double *num_out, int64_t cap)
{
    int W = orc_key_words(s->norb);
    orc_vec v = {NULL, 0, 0};
    uint64_t ncand = 0;
    if (emit_one(s, dets, c, n, 0.0, log2p, part, &v, &ncand)) {
        free(v.r);
        return -1;
    }
    qsort(v.r, v.n, sizeof(orc_rec), cmp_rec);
    int64_t cnt = 0;
    size_t i = 0;
    while (i < v.n) {
        size_t j = i;
        double num = 0.0;
        while (j < v.n && cmp_key(v.r[j].key, v.r[i].key, W) == 0)
            num += v.r[j++].v;
        if (cnt < cap) {
            memcpy(keys_out + cnt * W, v.r[i].key, sizeof(uint64_t) * W);
            num_out[cnt] = num;
        }
        cnt++;
        i = j;
    }
    free(v.r);
    return cnt;
}

/* Diagonal energies of many determinants (threaded over slices). */
typedef struct {
    const orc_system *s;
    const uint64_t *keys;
    double *out;
    int64_t lo, hi;
    int W;
} diag_job;

static void *diag_worker(void *arg)
{
    diag_job *J = (diag_job *)arg;
    for (int64_t i = J->lo; i < J->hi; i++)
        J->out[i] = orc_diag(J->s, J->keys + i * J->W);
    return NULL;
}

/* E0 - H_aa (orc_denominator) of many determinants, one thread. */
void orc_denominator_many(const orc_system *s, const uint64_t *keys, int64_t n, double e0, double *out)
{
    int W = orc_key_words(s->norb);
    for (int64_t i = 0; i < n; i++)
        out[i] = orc_denominator(s, keys + i * W, e0);
}

void orc_diag_many(const orc_system *s, const uint64_t *keys, int64_t n, double *out, int nthreads)
{
    int W = orc_key_words(s->norb);
    if (nthreads < 1)
        nthreads = 1;
    diag_job jobs[256];
    pthread_t th[256];
    if (nthreads > 256)
        nthreads = 256;
    for (int t = 0; t < nthreads; t++) {
        jobs[t].s = s, jobs[t].keys = keys, jobs[t].out = out, jobs[t].W = W;
        jobs[t].lo = n * t / nthreads, jobs[t].hi = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, diag_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++)
        pthread_join(th[t], NULL);
}

/* Dense H_RR (n x n, row-major) by pairwise Slater-Condon rules. */
void orc_hrr(const orc_system *s, const uint64_t *dets, int64_t n, double *H)
{
    int W = orc_key_words(s->norb);
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < n; j++)
            H[i * n + j] = orc_hij(s, dets + i * W, dets + j * W);
}

/* <c|H|c> = sum_ij c_i H_ij c_j by pairwise Slater-Condon rules (threaded). */
typedef struct {
    const orc_system *s;
    const uint64_t *dets;
    const double *c;
    int64_t n, lo, hi;
    double sum, comp;
} exp_job;

static void *exp_worker(void *arg)
{
    exp_job *J = (exp_job *)arg;
    int W = orc_key_words(J->s->norb);
    for (int64_t i = J->lo; i < J->hi; i++) {
        double row = 0.0, rc = 0.0;
        for (int64_t j = 0; j < J->n; j++) {
            /* H_ij vanishes beyond double excitations (more than four differing
             * spin-orbitals); orc_hij returns 0 there too, this only skips the call */
            int ndiff = 0;
            for (int w = 0; w < W; w++)
                ndiff += __builtin_popcountll(J->dets[i * W + w] ^ J->dets[j * W + w]);
            if (ndiff > 4)
                continue;
            double hij = orc_hij(J->s, J->dets + i * W, J->dets + j * W);
            if (hij != 0.0)
                neumaier_add(&row, &rc, hij * J->c[j]);
        }
        neumaier_add(&J->sum, &J->comp, J->c[i] * (row + rc));
    }
    return NULL;
}

double orc_expectation(const orc_system *s, const uint64_t *dets, const double *c, int64_t n, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    exp_job jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) {
        exp_job j = {s, dets, c, n, n * t / nthreads, n * (t + 1) / nthreads, 0.0, 0.0};
        jobs[t] = j;
        pthread_create(&th[t], NULL, exp_worker, &jobs[t]);
    }
    double sum = 0.0, comp = 0.0;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        neumaier_add(&sum, &comp, jobs[t].sum + jobs[t].comp);
    }
    return sum + comp;
}

/* Zobrist subset of each key (for tests of the split's completeness). */
void orc_parts(int norb, const uint64_t *keys, int64_t n, int log2p, uint32_t *out)
{
    int W = orc_key_words(norb);
    uint64_t R[2 * ORC_MAXORB];
    orc_zobrist_table(norb, R);
    for (int64_t i = 0; i < n; i++)
        out[i] = part_of(zobrist(R, keys + i * W, 2 * norb), log2p);
}

uint64_t orc_key_mix(const uint64_t *key, int W) { return key_mix(key, W); }

/* The SplitMix64 stream from a seed (exposed so tests can pin the generator
 * to its published outputs). */
void orc_splitmix64_stream(uint64_t seed, int n, uint64_t *out)
{
    uint64_t st = seed;
    for (int i = 0; i < n; i++)
        out[i] = splitmix64_next(&st);
}
