/*
 * Brute-force full-CI checker.  TEST INFRASTRUCTURE ONLY: it pins the PT2
 * oracle and shares no code with it or with the HIP engine.
 *
 * It applies the second-quantised Hamiltonian
 *   H = sum_{pq,sigma} h_pq a+_{p sigma} a_{q sigma}
 *     + 1/2 sum_{pqrs,sigma tau} (pq|rs) a+_{p sigma} a+_{r tau} a_{s tau} a_{q sigma}
 * (real orbitals, chemists' notation, no constant) term by term to
 * determinants, using nothing but the action of single creation and
 * annihilation operators on an ordered product of creators.  No
 * Slater-Condon case analysis appears here: a term whose annihilators find
 * an empty orbital, or whose creators find an occupied one, vanishes by the
 * operator definition.
 *
 * A determinant is the ordered list of occupied spin-orbitals
 * so_1 < so_2 < ... (spin-orbital index = bit index: beta orbital p is p,
 * alpha orbital p is norb + p), standing for a+_{so_1} a+_{so_2} ... |0>.
 *   a_x   on the list: zero if x absent; else remove it, sign (-1)^(its position)
 *   a+_x  on the list: zero if x present; else insert it, sign (-1)^(its position)
 *
 * The full-CI space is indexed by (alpha string rank) * (number of beta
 * strings) + (beta string rank), with strings ranked in the combinatorial
 * number system.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FB_MAXEL 64
#define FB_MAXSO 256

typedef struct {
    int norb, nalpha, nbeta;
    const double *h;
    const double *eri;
} fb_system;

typedef struct {
    int n;
    int so[FB_MAXEL];
} fb_det;

/* ---------------------------------------------------------------- operators */

/* returns sign (+1/-1) or 0 if the result vanishes */
static int op_annihilate(fb_det *d, int x)
{
    for (int k = 0; k < d->n; k++)
        if (d->so[k] == x) {
            for (int m = k; m < d->n - 1; m++)
                d->so[m] = d->so[m + 1];
            d->n--;
            return (k & 1) ? -1 : 1;
        }
    return 0;
}

static int op_create(fb_det *d, int x)
{
    int k = 0;
    while (k < d->n && d->so[k] < x)
        k++;
    if (k < d->n && d->so[k] == x)
        return 0;
    for (int m = d->n; m > k; m--)
        d->so[m] = d->so[m - 1];
    d->so[k] = x;
    d->n++;
    return (k & 1) ? -1 : 1;
}

/* ------------------------------------------------------------ conversions */

static int W_of(int norb) { return (2 * norb + 63) / 64; }

static void det_from_key(const fb_system *s, const uint64_t *key, fb_det *d)
{
    d->n = 0;
    for (int b = 0; b < 2 * s->norb; b++)
        if ((key[b >> 6] >> (b & 63)) & 1u)
            d->so[d->n++] = b;
}

static void key_from_det(const fb_system *s, const fb_det *d, uint64_t *key)
{
    memset(key, 0, sizeof(uint64_t) * W_of(s->norb));
    for (int k = 0; k < d->n; k++)
        key[d->so[k] >> 6] |= (uint64_t)1 << (d->so[k] & 63);
}

static double binom_tab[FB_MAXSO + 1][FB_MAXEL + 1];
static pthread_once_t binom_once = PTHREAD_ONCE_INIT;

static void binom_init(void)
{
    for (int n = 0; n <= FB_MAXSO; n++)
        for (int k = 0; k <= FB_MAXEL; k++) {
            if (k == 0)
                binom_tab[n][k] = 1.0;
            else if (n == 0)
                binom_tab[n][k] = 0.0;
            else
                binom_tab[n][k] = binom_tab[n - 1][k - 1] + binom_tab[n - 1][k];
        }
}

static double binom(int n, int k)
{
    pthread_once(&binom_once, binom_init);
    if (k < 0 || n < 0 || k > n)
        return 0.0;
    return binom_tab[n][k];
}

int64_t fb_dim(int norb, int na, int nb) { return (int64_t)(binom(norb, na) * binom(norb, nb)); }

/* rank of an occupied-orbital set (ascending list) in the combinatorial number system */
static int64_t string_rank(const int *occ, int n)
{
    int64_t r = 0;
    for (int k = 0; k < n; k++)
        r += (int64_t)binom(occ[k], k + 1);
    return r;
}

static void string_unrank(int64_t r, int norb, int n, int *occ)
{
    for (int k = n - 1; k >= 0; k--) {
        int p = k;
        while (p + 1 < norb && (int64_t)binom(p + 1, k + 1) <= r)
            p++;
        occ[k] = p;
        r -= (int64_t)binom(p, k + 1);
    }
}

/* FCI index of a determinant, or -1 if its electron counts do not match */
static int64_t det_index(const fb_system *s, const fb_det *d)
{
    int oa[FB_MAXEL], ob[FB_MAXEL], na = 0, nb = 0;
    for (int k = 0; k < d->n; k++) {
        if (d->so[k] >= s->norb)
            oa[na++] = d->so[k] - s->norb;
        else
            ob[nb++] = d->so[k];
    }
    if (na != s->nalpha || nb != s->nbeta)
        return -1;
    int64_t nbs = (int64_t)binom(s->norb, s->nbeta);
    return string_rank(oa, na) * nbs + string_rank(ob, nb);
}

static void det_of_index(const fb_system *s, int64_t idx, fb_det *d)
{
    int64_t nbs = (int64_t)binom(s->norb, s->nbeta);
    int oa[FB_MAXEL], ob[FB_MAXEL];
    string_unrank(idx / nbs, s->norb, s->nalpha, oa);
    string_unrank(idx % nbs, s->norb, s->nbeta, ob);
    d->n = 0;
    for (int k = 0; k < s->nbeta; k++)
        d->so[d->n++] = ob[k];
    for (int k = 0; k < s->nalpha; k++)
        d->so[d->n++] = s->norb + oa[k];
}

int64_t fb_index_of_key(const fb_system *s, const uint64_t *key)
{
    fb_det d;
    det_from_key(s, key, &d);
    return det_index(s, &d);
}

void fb_key_of_index(const fb_system *s, int64_t idx, uint64_t *key)
{
    fb_det d;
    det_of_index(s, idx, &d);
    key_from_det(s, &d, key);
}

/* ---------------------------------------------------------- H application */

static double eri_at(const fb_system *s, int p, int q, int r, int t)
{
    size_t n = (size_t)s->norb;
    return s->eri[((p * n + q) * n + r) * n + t];
}

/* spatial orbital and spin of a spin-orbital */
static int orb_of(const fb_system *s, int so) { return so >= s->norb ? so - s->norb : so; }
static int spin_of(const fb_system *s, int so) { return so >= s->norb ? 0 : 1; }

/*
 * out[index] += weight * <index|H|D> for every determinant index reached.
 * Every term of H is visited; a term vanishes as soon as one of its
 * operators does.  With out == NULL only the component on determinant
 * `target` is accumulated, into *acc.
 */
static void deposit(double *out, int64_t idx, double x, int64_t target, double *acc)
{
    if (out)
        out[idx] += x;
    else if (idx == target)
        *acc += x;
}

static void apply_H(const fb_system *s, const fb_det *D, double weight, double *out, int64_t target,
                    double *acc)
{
    int nso = 2 * s->norb;
    /* one-body: a+_p a_q, same spin */
    for (int q = 0; q < nso; q++) {
        fb_det d1 = *D;
        int s1 = op_annihilate(&d1, q);
        if (!s1)
            continue;
        for (int p = 0; p < nso; p++) {
            if (spin_of(s, p) != spin_of(s, q))
                continue;
            fb_det d2 = d1;
            int s2 = op_create(&d2, p);
            if (!s2)
                continue;
            int64_t idx = det_index(s, &d2);
            deposit(out, idx, weight * s1 * s2 * s->h[(size_t)orb_of(s, p) * s->norb + orb_of(s, q)], target,
                    acc);
        }
    }
    /* two-body: 1/2 (pq|rs) a+_p a+_r a_s a_q with spin(p)=spin(q), spin(r)=spin(s) */
    for (int q = 0; q < nso; q++) {
        fb_det d1 = *D;
        int s1 = op_annihilate(&d1, q);
        if (!s1)
            continue;
        for (int t = 0; t < nso; t++) {
            fb_det d2 = d1;
            int s2 = op_annihilate(&d2, t);
            if (!s2)
                continue;
            for (int r = 0; r < nso; r++) {
                if (spin_of(s, r) != spin_of(s, t))
                    continue;
                fb_det d3 = d2;
                int s3 = op_create(&d3, r);
                if (!s3)
                    continue;
                for (int p = 0; p < nso; p++) {
                    if (spin_of(s, p) != spin_of(s, q))
                        continue;
                    fb_det d4 = d3;
                    int s4 = op_create(&d4, p);
                    if (!s4)
                        continue;
                    int64_t idx = det_index(s, &d4);
                    double g = eri_at(s, orb_of(s, p), orb_of(s, q), orb_of(s, r), orb_of(s, t));
                    deposit(out, idx, weight * 0.5 * s1 * s2 * s3 * s4 * g, target, acc);
                }
            }
        }
    }
}

/* v[FCI] = H * (sum_i c_i |D_i>) over the full space (v zeroed here). */
void fb_h_times(const fb_system *s, const uint64_t *dets, const double *c, int64_t n, double *v)
{
    int W = W_of(s->norb);
    memset(v, 0, sizeof(double) * fb_dim(s->norb, s->nalpha, s->nbeta));
    for (int64_t i = 0; i < n; i++) {
        fb_det d;
        det_from_key(s, dets + i * W, &d);
        apply_H(s, &d, c[i], v, -1, NULL);
    }
}

/* <D|H|D> by applying H to D and keeping the component on D itself. */
typedef struct {
    const fb_system *s;
    const int64_t *idx;
    double *out;
    int64_t lo, hi;
} diag_job;

static void *diag_worker(void *arg)
{
    diag_job *J = (diag_job *)arg;
    for (int64_t k = J->lo; k < J->hi; k++) {
        fb_det d;
        double acc = 0.0;
        det_of_index(J->s, J->idx[k], &d);
        apply_H(J->s, &d, 1.0, NULL, J->idx[k], &acc);
        J->out[k] = acc;
    }
    return NULL;
}

void fb_diag_many(const fb_system *s, const int64_t *idx, int64_t n, double *out, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 64)
        nthreads = 64;
    diag_job jobs[64];
    pthread_t th[64];
    for (int t = 0; t < nthreads; t++) {
        diag_job j = {s, idx, out, n * t / nthreads, n * (t + 1) / nthreads};
        jobs[t] = j;
        pthread_create(&th[t], NULL, diag_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++)
        pthread_join(th[t], NULL);
}

/* Dense FCI Hamiltonian (dim x dim, row-major) for tiny spaces. */
void fb_dense(const fb_system *s, double *H)
{
    int64_t dim = fb_dim(s->norb, s->nalpha, s->nbeta);
    double *col = (double *)calloc((size_t)dim, sizeof(double));
    for (int64_t j = 0; j < dim; j++) {
        fb_det d;
        det_of_index(s, j, &d);
        memset(col, 0, sizeof(double) * (size_t)dim);
        apply_H(s, &d, 1.0, col, -1, NULL);
        for (int64_t i = 0; i < dim; i++)
            H[i * dim + j] = col[i];
    }
    free(col);
}
