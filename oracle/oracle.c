/*
 * CPU oracle for the product of two sparse multivariate polynomials in
 * distributed format.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg call it; the library's product
 * path never does.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Section 2, problem statement and Fig. 1): for
 *   A = sum_i a_i x^{alpha_i},  B = sum_j b_j x^{beta_j}
 * the product is the sum of all pairwise term products
 *   P_{i,j} = a_i b_j x^{gamma_{i,j}},  gamma_{i,j} = alpha_i + beta_j,
 * with equal monomials grouped, like terms summed and zero terms removed, and
 * the result returned sorted ascending by monomial (Algorithm 1 returns its
 * containers concatenated in ascending order; Section 2 calls this the
 * canonical form).  Exponents are packed into one 64-bit word (Section 6), so
 * gamma_{i,j} is the integer sum of the two packed keys as long as no field
 * carries into its neighbour; that is checked first.
 *
 * This is the plain definition written out: a double loop over (i, j) in
 * row-major order, one hash-map accumulator per distinct monomial, then a
 * sort of the distinct monomials.  Nothing of Algorithms 1 or 2 (grid
 * sampling, intervals, FindEdge) is used: those reach the same result faster.
 *
 * Coefficient rings:
 *   ring 0  integers mod p = 2^61 - 1; residues in [0, p); products reduced
 *           with a 128-bit remainder (a plain '%', not a Mersenne fold).
 *   ring 1  IEEE double; each product rounded once, contributions to one
 *           monomial added left to right in row-major (i, j) order starting
 *           from +0.0; the sum of |fl(a_i b_j)| is also returned per monomial.
 *   ring 2  int64; exact sums in a three-word (192-bit) signed accumulator,
 *           mirroring the three-word accumulator of the paper's benchmark
 *           section; a result that does not fit int64 is reported.
 *   ring 3  integers mod q = 2^64 - 59 (a prime); residues in [0, q);
 *           products and sums reduced with a 128-bit remainder.
 *   ring 4  integers as three-word (192-bit) two's-complement values, all
 *           arithmetic modulo 2^192: operands, products and sums wrap.  The
 *           result is the exact integer product whenever every output
 *           coefficient lies in [-2^191, 2^191).  Coefficient arrays hold
 *           three words per term, least significant first.
 * Only an exact +/-0.0 (ring 1) or 0 (rings 0, 2, 3, 4) is dropped.
 *
 * Build: gcc -O2 -ffp-contract=off -shared -fPIC oracle.c -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EUNSORTED (-2)
#define OR_EOVERFLOW (-3)
#define OR_ERANGE (-4)
#define OR_ECAPACITY (-5)
#define OR_ENOMEM (-6)
#define OR_EINT64 (-9)

#define OR_MODP 0
#define OR_F64 1
#define OR_I64 2
#define OR_MODQ 3
#define OR_Z192 4

static const uint64_t P61 = (((uint64_t)1) << 61) - 1;
static const uint64_t Q64 = ~(uint64_t)0 - 58; /* 2^64 - 59 */

/* Three-word two's-complement accumulator (w[0] least significant). */
typedef struct { uint64_t w[3]; } acc192;

static void acc192_add_i128(acc192 *a, __int128 v) {
    uint64_t lo = (uint64_t)v;
    uint64_t mid = (uint64_t)(v >> 64);
    uint64_t hi = (v < 0) ? ~(uint64_t)0 : 0;
    uint64_t s0 = a->w[0] + lo;
    uint64_t c0 = s0 < lo;
    uint64_t s1 = a->w[1] + mid;
    uint64_t c1 = s1 < mid;
    uint64_t s1c = s1 + c0;
    c1 += s1c < s1;
    a->w[0] = s0;
    a->w[1] = s1c;
    a->w[2] = a->w[2] + hi + c1;
}

static int acc192_is_zero(const acc192 *a) { return (a->w[0] | a->w[1] | a->w[2]) == 0; }

/* a += b (mod 2^192). */
static void acc192_add(acc192 *a, const acc192 *b) {
    unsigned __int128 t = (unsigned __int128)a->w[0] + b->w[0];
    a->w[0] = (uint64_t)t;
    t = (t >> 64) + a->w[1] + b->w[1];
    a->w[1] = (uint64_t)t;
    a->w[2] = (uint64_t)(t >> 64) + a->w[2] + b->w[2];
}

/* a * b (mod 2^192): schoolbook over 64-bit words, dropping every partial
   product of weight 2^192 or more.  Two's-complement operands need no
   special case, since the product is taken modulo 2^192. */
static acc192 acc192_mul(const uint64_t *a, const uint64_t *b) {
    acc192 r;
    unsigned __int128 t = (unsigned __int128)a[0] * b[0];
    r.w[0] = (uint64_t)t;
    unsigned __int128 u = (t >> 64) + (unsigned __int128)a[0] * b[1];
    unsigned __int128 v = (unsigned __int128)(uint64_t)u + (unsigned __int128)a[1] * b[0];
    r.w[1] = (uint64_t)v;
    r.w[2] = (uint64_t)(u >> 64) + (uint64_t)(v >> 64) + a[0] * b[2] + a[1] * b[1] + a[2] * b[0];
    return r;
}

/* Returns 1 and stores the value when the accumulator fits int64. */
static int acc192_to_i64(const acc192 *a, int64_t *out) {
    int64_t v = (int64_t)a->w[0];
    uint64_t ext = (v < 0) ? ~(uint64_t)0 : 0;
    if (a->w[1] != ext || a->w[2] != ext) return 0;
    *out = v;
    return 1;
}

typedef struct {
    uint64_t key;
    uint64_t modp;   /* rings 0 and 3 */
    acc192 exact;    /* rings 2 and 4 */
    double sum;      /* ring 1 */
    double abssum;   /* ring 1 */
} entry;

typedef struct {
    entry *e;
    unsigned char *used;
    uint64_t cap;   /* power of two */
    uint64_t n;
} table;

static uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static int table_init(table *t, uint64_t cap) {
    t->cap = cap;
    t->n = 0;
    t->e = (entry *)malloc(cap * sizeof(entry));
    t->used = (unsigned char *)calloc(cap, 1);
    return (t->e && t->used) ? OR_OK : OR_ENOMEM;
}

static void table_free(table *t) {
    free(t->e);
    free(t->used);
    t->e = NULL;
    t->used = NULL;
}

static entry *table_slot(table *t, uint64_t key) {
    uint64_t m = t->cap - 1;
    uint64_t h = mix64(key) & m;
    while (t->used[h] && t->e[h].key != key) h = (h + 1) & m;
    if (!t->used[h]) {
        t->used[h] = 1;
        memset(&t->e[h], 0, sizeof(entry));
        t->e[h].key = key;
        t->n++;
    }
    return &t->e[h];
}

static int table_grow(table *t) {
    table nt;
    if (table_init(&nt, t->cap * 2) != OR_OK) {
        table_free(&nt);
        return OR_ENOMEM;
    }
    for (uint64_t s = 0; s < t->cap; s++) {
        if (!t->used[s]) continue;
        uint64_t m = nt.cap - 1;
        uint64_t h = mix64(t->e[s].key) & m;
        while (nt.used[h]) h = (h + 1) & m;
        nt.used[h] = 1;
        nt.e[h] = t->e[s];
        nt.n++;
    }
    table_free(t);
    *t = nt;
    return OR_OK;
}

/* Input checks.  Fields: variable v occupies bits [(nvars-1-v)*bits, +bits). */
int oracle_validate(int nvars, int bits, int ring, int64_t na, const uint64_t *fk, const void *fc,
                    int64_t nb, const uint64_t *gk, const void *gc) {
    if (nvars < 1 || bits < 1 || nvars * bits > 64) return OR_EINVAL;
    if (ring != OR_MODP && ring != OR_F64 && ring != OR_I64 && ring != OR_MODQ && ring != OR_Z192) return OR_EINVAL;
    if (na < 0 || nb < 0) return OR_EINVAL;
    if ((na > 0 && (!fk || !fc)) || (nb > 0 && (!gk || !gc))) return OR_EINVAL;
    int used = nvars * bits;
    uint64_t fieldmask = (bits == 64) ? ~(uint64_t)0 : ((((uint64_t)1) << bits) - 1);
    uint64_t maxf[64], maxg[64];
    for (int v = 0; v < nvars; v++) maxf[v] = maxg[v] = 0;
    for (int side = 0; side < 2; side++) {
        int64_t n = side ? nb : na;
        const uint64_t *k = side ? gk : fk;
        const void *c = side ? gc : fc;
        uint64_t *mx = side ? maxg : maxf;
        for (int64_t i = 0; i < n; i++) {
            if (used < 64 && (k[i] >> used) != 0) return OR_EINVAL;
            if (i > 0 && !(k[i] > k[i - 1])) return OR_EUNSORTED;
            for (int v = 0; v < nvars; v++) {
                uint64_t e = (k[i] >> ((nvars - 1 - v) * bits)) & fieldmask;
                if (e > mx[v]) mx[v] = e;
            }
            if (ring == OR_MODP && ((const uint64_t *)c)[i] >= P61) return OR_ERANGE;
            if (ring == OR_MODQ && ((const uint64_t *)c)[i] >= Q64) return OR_ERANGE;
            if (ring == OR_F64 && !isfinite(((const double *)c)[i])) return OR_ERANGE;
        }
    }
    if (na > 0 && nb > 0) {
        for (int v = 0; v < nvars; v++) {
            /* the sum of the two maxima must still fit the field */
            if (maxf[v] > fieldmask - maxg[v]) return OR_EOVERFLOW;
        }
    }
    return OR_OK;
}

static int cmp_entry_key(const void *a, const void *b) {
    uint64_t x = ((const entry *)a)->key, y = ((const entry *)b)->key;
    return (x > y) - (x < y);
}

/*
 * h = f * g.  Outputs go to caller arrays of capacity `cap`; *nh receives the
 * number of terms.  If the result has more than `cap` terms, nothing is
 * written, *nh holds the required count and OR_ECAPACITY is returned.
 * habs (ring 1 only, may be NULL) receives sum |fl(a_i b_j)| per output term.
 */
int oracle_mul(int nvars, int bits, int ring, int64_t na, const uint64_t *fk, const void *fc,
               int64_t nb, const uint64_t *gk, const void *gc, int64_t cap, uint64_t *hk, void *hc,
               double *habs, int64_t *nh) {
    int rc = oracle_validate(nvars, bits, ring, na, fk, fc, nb, gk, gc);
    if (rc != OR_OK) return rc;
    if (!nh) return OR_EINVAL;
    *nh = 0;
    if (na == 0 || nb == 0) return OR_OK;

    table t;
    if (table_init(&t, (uint64_t)1 << 16) != OR_OK) {
        table_free(&t);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < na; i++) {
        for (int64_t j = 0; j < nb; j++) {
            if (2 * (t.n + 1) > t.cap && table_grow(&t) != OR_OK) {
                table_free(&t);
                return OR_ENOMEM;
            }
            entry *e = table_slot(&t, fk[i] + gk[j]);
            if (ring == OR_MODP) {
                uint64_t a = ((const uint64_t *)fc)[i], b = ((const uint64_t *)gc)[j];
                uint64_t c = (uint64_t)(((unsigned __int128)a * b) % P61);
                e->modp = (e->modp + c) % P61;
            } else if (ring == OR_I64) {
                int64_t a = ((const int64_t *)fc)[i], b = ((const int64_t *)gc)[j];
                acc192_add_i128(&e->exact, (__int128)a * b);
            } else if (ring == OR_MODQ) {
                uint64_t a = ((const uint64_t *)fc)[i], b = ((const uint64_t *)gc)[j];
                uint64_t c = (uint64_t)(((unsigned __int128)a * b) % Q64);
                e->modp = (uint64_t)(((unsigned __int128)e->modp + c) % Q64);
            } else if (ring == OR_Z192) {
                acc192 c = acc192_mul((const uint64_t *)fc + 3 * i, (const uint64_t *)gc + 3 * j);
                acc192_add(&e->exact, &c);
            } else {
                double a = ((const double *)fc)[i], b = ((const double *)gc)[j];
                volatile double c = a * b; /* rounded once, never fused with the add */
                e->sum = e->sum + c;
                e->abssum = e->abssum + fabs(c);
            }
        }
    }
    /* gather non-zero terms */
    entry *out = (entry *)malloc((t.n ? t.n : 1) * sizeof(entry));
    if (!out) {
        table_free(&t);
        return OR_ENOMEM;
    }
    uint64_t m = 0;
    for (uint64_t s = 0; s < t.cap; s++) {
        if (!t.used[s]) continue;
        const entry *e = &t.e[s];
        int zero = (ring == OR_MODP || ring == OR_MODQ) ? (e->modp == 0)
                   : (ring == OR_I64 || ring == OR_Z192)  ? acc192_is_zero(&e->exact)
                                                          : (e->sum == 0.0);
        if (!zero) out[m++] = *e;
    }
    table_free(&t);
    qsort(out, m, sizeof(entry), cmp_entry_key);
    *nh = (int64_t)m;
    if ((int64_t)m > cap) {
        free(out);
        return OR_ECAPACITY;
    }
    for (uint64_t s = 0; s < m; s++) {
        hk[s] = out[s].key;
        if (ring == OR_MODP || ring == OR_MODQ) {
            ((uint64_t *)hc)[s] = out[s].modp;
        } else if (ring == OR_Z192) {
            for (int k = 0; k < 3; k++) ((uint64_t *)hc)[3 * s + k] = out[s].exact.w[k];
        } else if (ring == OR_I64) {
            int64_t v;
            if (!acc192_to_i64(&out[s].exact, &v)) {
                free(out);
                return OR_EINT64;
            }
            ((int64_t *)hc)[s] = v;
        } else {
            ((double *)hc)[s] = out[s].sum;
            if (habs) habs[s] = out[s].abssum;
        }
    }
    free(out);
    return OR_OK;
}

/* Upper bound on the number of output terms: min(na*nb, degree-box size). */
int oracle_bound(int nvars, int bits, int64_t na, const uint64_t *fk, int64_t nb, const uint64_t *gk,
                 int64_t *bound) {
    if (nvars < 1 || bits < 1 || nvars * bits > 64 || !bound) return OR_EINVAL;
    if (na == 0 || nb == 0) {
        *bound = 0;
        return OR_OK;
    }
    uint64_t fieldmask = (bits == 64) ? ~(uint64_t)0 : ((((uint64_t)1) << bits) - 1);
    double box = 1.0;
    for (int v = 0; v < nvars; v++) {
        uint64_t lo = ~(uint64_t)0, hi = 0, lo2 = ~(uint64_t)0, hi2 = 0;
        for (int64_t i = 0; i < na; i++) {
            uint64_t e = (fk[i] >> ((nvars - 1 - v) * bits)) & fieldmask;
            if (e < lo) lo = e;
            if (e > hi) hi = e;
        }
        for (int64_t j = 0; j < nb; j++) {
            uint64_t e = (gk[j] >> ((nvars - 1 - v) * bits)) & fieldmask;
            if (e < lo2) lo2 = e;
            if (e > hi2) hi2 = e;
        }
        box *= (double)(hi + hi2 - lo - lo2 + 1);
    }
    double prod = (double)na * (double)nb;
    double b = box < prod ? box : prod;
    *bound = (int64_t)b;
    return OR_OK;
}
