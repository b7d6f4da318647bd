/*
 * LearnedSort 2.0 oracle -- TEST INFRASTRUCTURE ONLY (see lsort_oracle.h).
 *
 * Plain single-threaded C, built with -O2 -ffp-contract=off: every floating
 * point operation below is rounded exactly as written (the only fused
 * multiply-add is the explicit fma() of the leaf model).
 *
 * Readings taken where the paper is silent or garbled (numbered as in the
 * design notes):
 *   R1/R2  Alg. 1 bucket prediction at level p under parent i is
 *          floor(F * f^(1+p)) - p*i*f, clamped to [0, f).
 *   R3     the tail flush of Alg. 1 clears the fragment it just copied.
 *   R4     loops over buckets run over [0, f).
 *   R5     the fragment log records (bucket, size) pairs.
 *   R6     partial fragments are flushed in bucket order.
 *   R7     Defragment is a stable out-of-place gather by bucket in log order.
 *   R8     homogeneous = every key bitwise equal (ord); size <= 1 counts.
 *   R9     counting-sort slot = clamp(floor((F*f^2 - (i*f+j)) * n'), 0, n'-1).
 *   R10    running totals are inclusive; placement decrements then writes,
 *          walking the sub-bucket backwards.
 *   R11/12 histogram of n' slots, reused buffers.
 *   R13    the touch-up insertion sort covers the whole array, ord order.
 *   R14    model: two-layer linear spline over the sorted sample (root linear
 *          in the totalOrder word; leaf k knotted at its most repeated
 *          sample value; a start knot at the sample minimum; the sample
 *          eCDF exact just below, at (mid-rank) and just above each knot; a
 *          key uses the segment of the largest knot not above it).
 *   R15    every copy of a key gets the same prediction: its mid-rank in the
 *          sample when it is a knot.
 *   R16    sample with replacement, m = max(1, ceil(rate*n)).
 *   R17    n <= 1: nothing; n <= small_n: insertion sort.
 *   R18    optional recursion (s_max > 0) into over-full sub-buckets with a
 *          local model; a partition that leaves more than 7/8 of the keys
 *          in one bucket is redone on the bits just below the highest
 *          differing bit (MSD fallback); past a provable depth bound the
 *          sort stops with ORC_ERR_DEPTH.
 *   R20    non-finite f64 keys: F = 0 for negative, 1 for positive.
 *   R24    u64 -> f64 conversion rounds to nearest even.
 */
#include "lsort_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ keys -- */

/* Order-preserving map of IEEE-754 double bits (totalOrder). */
static uint64_t f64_bits_to_ord(uint64_t b)
{
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

static uint64_t ord_to_f64_bits(uint64_t o)
{
    return (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
}

static uint64_t raw_to_ord(uint64_t raw, uint32_t dtype)
{
    return dtype == ORC_F64 ? f64_bits_to_ord(raw) : raw;
}

static uint64_t ord_to_raw(uint64_t o, uint32_t dtype)
{
    return dtype == ORC_F64 ? ord_to_f64_bits(o) : o;
}

/* The real value the model sees: the double itself, or the u64 rounded to
 * the nearest double (ties to even). */
static double ord_value(uint64_t o, uint32_t dtype)
{
    if (dtype == ORC_U64)
        return (double)o;
    uint64_t b = ord_to_f64_bits(o);
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

/* ---------------------------------------------------------------- sample -- */

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is the state passed through the
 * variant-13 mixing function.  Output t (0-based) of a stream seeded with s is
 * mix(s + (t+1) * gamma). */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + (t + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* Uniform index in [0, n): high 64 bits of the 128-bit product. */
uint64_t orc_sample_index(uint64_t seed, uint64_t t, uint64_t n)
{
    unsigned __int128 p = (unsigned __int128)orc_splitmix64_at(seed, t) * n;
    return (uint64_t)(p >> 64);
}

uint64_t orc_sample_size(uint64_t n, double rate, uint64_t cap)
{
    double want = ceil(rate * (double)n);
    uint64_t m = want < 1.0 ? 1u : (uint64_t)want;
    if (cap && m > cap)
        m = cap;
    return m;
}

/* ----------------------------------------------------------------- model -- */

/* Reading R14.  A two-layer model of the sample eCDF:
 *  - root: leaf = floor((r(x) - r(xmin)) * L / (r(xmax) - r(xmin))), clamped
 *    to [0, L), where r(x) is the totalOrder word of the double x read as a
 *    number (log-like spacing: every binade gets leaves, so skewed data
 *    still spreads over them);
 *  - leaf k: one spline knot X_k: the value with the most copies among the
 *    sample values falling into leaf k (ties: the smallest) when it holds at
 *    least 2 copies and at least 1/L of the sample, else the leaf's smallest
 *    value; with the exact sample eCDF just below it (y), at it (mid-rank ym)
 *    and at or below it (y1);
 *  - a start knot at the sample minimum (index L);
 *  - between a knot with B sample values below it and d copies and the next
 *    knot (B' below it), linear from ylo = (B + d - 1/2)/m' to
 *    (B' + 1/2)/m' (mid-ranks of the last copy and of the next first copy),
 *    or to (xmax, 1) after the last knot.
 * A key uses the largest knot not above it: ym at the knot, the segment
 * above it otherwise, 0 below the sample minimum. */
typedef struct {
    double xmin, xmax, rs, r0;
    uint64_t mfin;       /* m': finite sample values */
    uint32_t L;
    /* L + 1 knots (leaves, then the start knot): X, y, ym, y1, ylo, yhi, s;
     * ye: where the segment arriving at the knot ends (training only) */
    double *X, *y, *ym, *y1, *ylo, *yhi, *s, *ye;
} model_t;

static void model_free(model_t* M)
{
    free(M->X);
    M->X = M->y = M->ym = M->y1 = M->ylo = M->yhi = M->s = M->ye = NULL;
}

static int model_alloc(model_t* M, uint32_t L)
{
    memset(M, 0, sizeof *M);
    M->L = L;
    size_t K = (size_t)L + 1;
    M->X = (double*)calloc(8u * K, sizeof(double));
    if (!M->X)
        return ORC_ERR_NOMEM;
    M->y = M->X + K;
    M->ym = M->y + K;
    M->y1 = M->ym + K;
    M->ylo = M->y1 + K;
    M->yhi = M->ylo + K;
    M->s = M->yhi + K;
    M->ye = M->s + K;
    return ORC_OK;
}

/* Root coordinate: the totalOrder word of a double, read as a number. */
static double root_coord(double x)
{
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    return (double)f64_bits_to_ord(b);
}

/* Root model: which leaf a finite value belongs to. */
static uint32_t model_leaf(const model_t* M, double x)
{
    double t = (root_coord(x) - M->r0) * M->rs;
    if (!(t >= 1.0))
        return 0;
    if (t >= (double)(M->L - 1u))
        return M->L - 1u;
    return (uint32_t)t;
}

/* Largest non-empty leaf j < k, or L (the start knot) if there is none. */
static uint32_t model_prev(const model_t* M, uint32_t k)
{
    while (k-- > 0)
        if (!isinf(M->X[k]))
            return k;
    return M->L;
}

/* F_A(x): estimated fraction of keys smaller than x (Sec. 2: the model
 * returns the count of keys less than x, scaled).  Monotone non-decreasing:
 * knots increase with the leaf index, and each segment is clamped to
 * [ylo_j, yhi_j] with ylo_j >= ym_j and yhi_j <= the next knot's ym. */
static double model_F(const model_t* M, double x)
{
    if (isnan(x) || isinf(x))
        return signbit(x) ? 0.0 : 1.0;
    uint32_t k = model_leaf(M, x);
    uint32_t j = (x >= M->X[k]) ? k : model_prev(M, k);
    if (j == M->L && !(x >= M->X[j]))
        return 0.0;
    if (x == M->X[j])
        return M->ym[j];
    if (M->s[j] == 0.0)
        return M->ylo[j];
    double F = fma(x - M->X[j], M->s[j], M->ylo[j]);
    if (F < M->ylo[j])
        F = M->ylo[j];
    if (F > M->yhi[j])
        F = M->yhi[j];
    return F;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y);
}

/* The values of one knot: B sample values below it, d copies of it. */
static void set_knot(model_t* M, uint32_t k, double X, uint64_t B, uint64_t d)
{
    const double m2 = (double)(2 * M->mfin);
    M->X[k] = X;
    M->y[k] = (double)B / (double)M->mfin;
    M->ym[k] = (double)(2 * B + d) / m2;
    M->y1[k] = (double)(B + d) / (double)M->mfin;
    M->ylo[k] = (double)(2 * (B + d) - 1) / m2;
    M->ye[k] = (double)(2 * B + 1) / m2;
}

/* Train on sample values given as ord words (order-independent: the sample
 * is sorted first). */
static int model_train(model_t* M, const uint64_t* sample, uint64_t m, uint32_t L, uint32_t dtype)
{
    int rc = model_alloc(M, L);
    if (rc)
        return rc;
    uint64_t* v = (uint64_t*)malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    uint64_t* best = (uint64_t*)calloc((size_t)L, sizeof(uint64_t));   /* per leaf: longest run */
    uint64_t* bstart = (uint64_t*)calloc((size_t)L, sizeof(uint64_t));
    uint64_t* first = (uint64_t*)malloc((size_t)L * sizeof(uint64_t)); /* per leaf: first sample index */
    uint64_t* flen = (uint64_t*)calloc((size_t)L, sizeof(uint64_t));  /* and the length of its run */
    if (!v || !best || !bstart || !first || !flen) {
        free(v);
        free(best);
        free(bstart);
        free(first);
        free(flen);
        model_free(M);
        return ORC_ERR_NOMEM;
    }
    uint64_t mfin = 0;
    for (uint64_t t = 0; t < m; ++t) {
        double x = ord_value(sample[t], dtype);
        if (!isnan(x) && !isinf(x))
            v[mfin++] = sample[t];
    }
    M->mfin = mfin;
    for (uint32_t k = 0; k <= L; ++k)
        M->X[k] = INFINITY;
    if (mfin == 0) {                 /* no knot at all: every F = 0 */
        free(v);
        free(best);
        free(bstart);
        free(first);
        free(flen);
        return ORC_OK;
    }
    qsort(v, (size_t)mfin, sizeof(uint64_t), cmp_u64);
    M->xmin = ord_value(v[0], dtype);
    M->xmax = ord_value(v[mfin - 1], dtype);
    M->r0 = root_coord(M->xmin);
    double r1 = root_coord(M->xmax);
    M->rs = (r1 > M->r0) ? (double)L / (r1 - M->r0) : 0.0;
    for (uint32_t k = 0; k < L; ++k)
        first[k] = mfin;
    /* runs of equal values (as doubles; a run starts at its smallest word) */
    uint64_t run0_len = 0;
    for (uint64_t a = 0; a < mfin;) {
        double x = ord_value(v[a], dtype);
        uint64_t e = a + 1;
        while (e < mfin && ord_value(v[e], dtype) == x)
            ++e;
        uint32_t k = model_leaf(M, x);
        if (first[k] == mfin) {
            first[k] = a;
            flen[k] = e - a;
        }
        if (e - a > best[k]) {
            best[k] = e - a;
            bstart[k] = a;
        }
        if (a == 0)
            run0_len = e;
        a = e;
    }
    /* leaf knots; an empty leaf has none (X = +inf, constant at the count
     * of the sample below the leaf) */
    for (uint32_t k = 0; k < L; ++k) {
        if (best[k] >= 2 && best[k] * L >= mfin) {
            set_knot(M, k, ord_value(v[bstart[k]], dtype), bstart[k], best[k]);
        } else if (best[k]) {
            set_knot(M, k, ord_value(v[first[k]], dtype), first[k], flen[k]);
        } else {
            /* samples in earlier leaves = first sample index of the next
             * non-empty leaf, or all of them */
            uint64_t nb = mfin;
            for (uint32_t j = k + 1; j < L; ++j)
                if (first[j] != mfin) {
                    nb = first[j];
                    break;
                }
            M->X[k] = INFINITY;
            M->y[k] = M->ym[k] = M->y1[k] = M->ylo[k] = (double)nb / (double)mfin;
        }
        M->yhi[k] = M->ylo[k];
        M->s[k] = 0.0;
    }
    set_knot(M, L, M->xmin, 0, run0_len);
    M->yhi[L] = M->ylo[L];
    M->s[L] = 0.0;
    /* segment from just above each knot (leaves, then the start knot) to
     * the next knot, or to (xmax, 1) */
    for (uint32_t k = 0; k <= L; ++k) {
        if (isinf(M->X[k]))
            continue;
        double Xh = M->xmax, yh = 1.0;
        for (uint32_t j = (k == L ? 0 : k + 1); j < L; ++j) {
            if (!isinf(M->X[j])) {
                Xh = M->X[j];
                yh = M->ye[j];
                break;
            }
        }
        double sl = (yh - M->ylo[k]) / (Xh - M->X[k]);
        if (!(sl > 0.0) || isinf(sl))
            sl = 0.0;
        M->yhi[k] = yh;
        M->s[k] = sl;
    }
    free(v);
    free(best);
    free(bstart);
    free(first);
    free(flen);
    return ORC_OK;
}

static void model_export(const model_t* M, double* out)
{
    out[0] = M->xmin;
    out[1] = M->xmax;
    out[2] = M->rs;
    out[3] = (double)M->mfin;
    for (uint32_t k = 0; k <= M->L; ++k) {
        double* o = out + 4 + 7 * (size_t)k;
        o[0] = M->X[k];
        o[1] = M->y[k];
        o[2] = M->ym[k];
        o[3] = M->y1[k];
        o[4] = M->ylo[k];
        o[5] = M->yhi[k];
        o[6] = M->s[k];
    }
}

static int model_import(model_t* M, const double* in, uint32_t L)
{
    int rc = model_alloc(M, L);
    if (rc)
        return rc;
    M->xmin = in[0];
    M->xmax = in[1];
    M->rs = in[2];
    M->mfin = (uint64_t)in[3];
    M->r0 = root_coord(M->xmin);
    for (uint32_t k = 0; k <= L; ++k) {
        const double* o = in + 4 + 7 * (size_t)k;
        M->X[k] = o[0];
        M->y[k] = o[1];
        M->ym[k] = o[2];
        M->y1[k] = o[3];
        M->ylo[k] = o[4];
        M->yhi[k] = o[5];
        M->s[k] = o[6];
    }
    return ORC_OK;
}

/* Sample m keys of A[0..n) (ord) with the counter-based stream and train. */
static int model_fit_range(model_t* M, const uint64_t* A, uint64_t n, uint64_t m,
                           uint64_t seed, uint32_t L, uint32_t dtype, uint64_t* idx_out)
{
    uint64_t* smp = (uint64_t*)malloc((size_t)m * sizeof(uint64_t));
    if (!smp)
        return ORC_ERR_NOMEM;
    for (uint64_t t = 0; t < m; ++t) {
        uint64_t i = orc_sample_index(seed, t, n);
        if (idx_out)
            idx_out[t] = i;
        smp[t] = A[i];
    }
    int rc = model_train(M, smp, m, L, dtype);
    free(smp);
    return rc;
}

/* -------------------------------------------------------------- bucketer -- */

enum { BK_MODEL = 0, BK_MSD = 1 };

typedef struct {
    int kind;
    const model_t* M;
    uint32_t dtype;
    double scale;        /* f^(1+p) */
    int64_t offset;      /* p * i * f */
    uint32_t fanout;
    uint32_t shift;      /* MSD fallback digit */
    uint64_t mask;
} bucketer_t;

static uint32_t bucket_of(const bucketer_t* B, uint64_t o)
{
    if (B->kind == BK_MSD)
        return (uint32_t)((o >> B->shift) & B->mask);
    double v = model_F(B->M, ord_value(o, B->dtype)) * B->scale;
    int64_t q = (int64_t)v - B->offset;          /* v >= 0: truncation is floor */
    if (q < 0)
        return 0;
    if (q > (int64_t)B->fanout - 1)
        return B->fanout - 1;
    return (uint32_t)q;
}

/* ------------------------------------------------------------- Alg. 1 ---- */

typedef struct {
    uint64_t* pairs;     /* (bucket, size) */
    uint64_t n, cap;
} fraglog_t;

static int log_push(fraglog_t* L, uint64_t b, uint64_t s)
{
    if (L->n == L->cap) {
        uint64_t nc = L->cap ? 2 * L->cap : 64;
        uint64_t* p = (uint64_t*)realloc(L->pairs, (size_t)nc * 2 * sizeof(uint64_t));
        if (!p)
            return ORC_ERR_NOMEM;
        L->pairs = p;
        L->cap = nc;
    }
    L->pairs[2 * L->n] = b;
    L->pairs[2 * L->n + 1] = s;
    L->n++;
    return ORC_OK;
}

/* Partition A[0..n) into f buckets through fragments of capacity c that are
 * copied back to A at the write head as soon as they fill (Alg. 1). */
static int partition(uint64_t* A, uint64_t n, const bucketer_t* B, uint32_t c,
                     uint64_t* SB, fraglog_t* log, orc_stats* st)
{
    uint32_t f = B->fanout;
    uint64_t* frag = (uint64_t*)malloc((size_t)f * c * sizeof(uint64_t));
    uint32_t* fsz = (uint32_t*)calloc(f, sizeof(uint32_t));
    if (!frag || !fsz) {
        free(frag);
        free(fsz);
        return ORC_ERR_NOMEM;
    }
    memset(SB, 0, (size_t)f * sizeof(uint64_t));
    log->n = 0;
    uint64_t w = 0;
    int rc = ORC_OK;
    for (uint64_t t = 0; t < n && rc == ORC_OK; ++t) {
        uint64_t x = A[t];
        uint32_t b = bucket_of(B, x);
        frag[(size_t)b * c + fsz[b]++] = x;
        SB[b]++;
        if (fsz[b] == c) {
            if (w + c > t + 1) {           /* would overwrite unread keys */
                rc = ORC_ERR_WRITE_HEAD;
                break;
            }
            memcpy(A + w, frag + (size_t)b * c, (size_t)c * sizeof(uint64_t));
            w += c;
            rc = log_push(log, b, c);
            fsz[b] = 0;
        }
    }
    for (uint32_t i = 0; i < f && rc == ORC_OK; ++i) {
        uint32_t s = fsz[i];
        if (!s)
            continue;
        memcpy(A + w, frag + (size_t)i * c, (size_t)s * sizeof(uint64_t));
        w += s;
        rc = log_push(log, i, s);
        fsz[i] = 0;
    }
    if (rc == ORC_OK && w != n)
        rc = ORC_ERR_PARTITION;
    if (st) {
        st->partitions++;
        st->fragments += log->n;
    }
    free(frag);
    free(fsz);
    return rc;
}

/* Make each bucket's fragments contiguous: bucket b ends up at
 * [sum_{<b} S_B, sum_{<=b} S_B), fragments in log order. */
static int defragment(uint64_t* A, uint64_t n, const uint64_t* SB, uint32_t f,
                      const uint64_t* pairs, uint64_t nfrag)
{
    uint64_t* cur = (uint64_t*)malloc((size_t)f * sizeof(uint64_t));
    uint64_t* tmp = (uint64_t*)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    if (!cur || !tmp) {
        free(cur);
        free(tmp);
        return ORC_ERR_NOMEM;
    }
    uint64_t run = 0;
    for (uint32_t b = 0; b < f; ++b) {
        cur[b] = run;
        run += SB[b];
    }
    int rc = run == n ? ORC_OK : ORC_ERR_PARTITION;
    uint64_t r = 0;
    for (uint64_t k = 0; k < nfrag && rc == ORC_OK; ++k) {
        uint64_t b = pairs[2 * k], s = pairs[2 * k + 1];
        if (b >= f || r + s > n || cur[b] + s > n) {
            rc = ORC_ERR_PARTITION;
            break;
        }
        memcpy(tmp + cur[b], A + r, (size_t)s * sizeof(uint64_t));
        cur[b] += s;
        r += s;
    }
    if (rc == ORC_OK && r != n)
        rc = ORC_ERR_PARTITION;
    if (rc == ORC_OK)
        memcpy(A, tmp, (size_t)n * sizeof(uint64_t));
    free(cur);
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------- Alg. 2 ---- */

static int homogeneous(const uint64_t* A, uint64_t n)
{
    for (uint64_t k = 1; k < n; ++k)
        if (A[k] != A[0])
            return 0;
    return 1;
}

static uint64_t orc_insertion_sort_ord(uint64_t* A, uint64_t n)
{
    uint64_t moves = 0;
    for (uint64_t i = 1; i < n; ++i) {
        uint64_t x = A[i];
        uint64_t j = i;
        while (j > 0 && A[j - 1] > x) {
            A[j] = A[j - 1];
            --j;
            ++moves;
        }
        A[j] = x;
    }
    return moves;
}

/* Model-based counting sort of one sub-bucket (readings R9-R12). */
static int counting_sort(uint64_t* A, uint64_t n, const model_t* M, uint32_t dtype,
                         double scale, double offset, orc_stats* st)
{
    if (n <= 1)
        return ORC_OK;
    uint64_t* K = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
    uint64_t* T = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    uint64_t* P = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    if (!K || !T || !P) {
        free(K);
        free(T);
        free(P);
        return ORC_ERR_NOMEM;
    }
    for (uint64_t k = 0; k < n; ++k) {
        double v = (model_F(M, ord_value(A[k], dtype)) * scale - offset) * (double)n;
        uint64_t pos;
        if (!(v >= 1.0))
            pos = 0;
        else if (v >= (double)(n - 1))
            pos = n - 1;
        else
            pos = (uint64_t)v;
        P[k] = pos;
        K[pos]++;
    }
    for (uint64_t k = 1; k < n; ++k)
        K[k] += K[k - 1];
    for (uint64_t k = n; k-- > 0;)
        T[--K[P[k]]] = A[k];
    memcpy(A, T, (size_t)n * sizeof(uint64_t));
    free(K);
    free(T);
    free(P);
    if (st)
        st->counting_sorts++;
    return ORC_OK;
}

typedef struct {
    const orc_params* p;
    orc_stats* st;
    uint32_t f, c, L, dtype;
    uint64_t s_max;
    uint32_t depth_max;  /* deepest recursion level allowed (depth_bound) */
} ctx_t;

static uint64_t local_seed(uint64_t seed, uint64_t start, uint32_t depth)
{
    return orc_splitmix64_at(seed ^ start, depth);
}

static uint64_t local_sample_size(const ctx_t* C, uint64_t n)
{
    uint64_t m = orc_sample_size(n, C->p->sample_rate, 0);
    uint64_t lo = C->p->local_min_sample < n ? C->p->local_min_sample : n;
    return m > lo ? m : lo;
}

static int recurse_local(const ctx_t* C, uint64_t* A, uint64_t n, uint64_t start, uint32_t depth);
static uint32_t depth_bound(uint64_t n);

/* Base case of a range no model bucket covers (children of an MSD split):
 * train a local model on the range and counting-sort by F * n. */
static int local_base(const ctx_t* C, uint64_t* A, uint64_t n, uint64_t start, uint32_t depth)
{
    model_t M;
    int rc = model_fit_range(&M, A, n, local_sample_size(C, n), local_seed(C->p->seed, start, depth),
                             C->L, C->dtype, NULL);
    if (rc)
        return rc;
    rc = counting_sort(A, n, &M, C->dtype, 1.0, 0.0, C->st);
    model_free(&M);
    return rc;
}

/* Handle child j of a partition done with bucketer B. */
static int finish_child(const ctx_t* C, uint64_t* A, uint64_t n, uint64_t start, uint32_t depth,
                        const bucketer_t* B, uint32_t j)
{
    if (n <= 1 || homogeneous(A, n)) {
        if (n > 1)
            C->st->homogeneous++;
        return ORC_OK;
    }
    if (C->s_max && n > C->s_max)
        return recurse_local(C, A, n, start, depth + 1);
    if (B->kind == BK_MODEL)
        return counting_sort(A, n, B->M, C->dtype, B->scale, (double)(B->offset + (int64_t)j), C->st);
    return local_base(C, A, n, start, depth + 1);
}

/* Partition + Defragment of A[0..n) with bucketer B; S_B returned in SB. */
static int partition_defrag(const ctx_t* C, uint64_t* A, uint64_t n, const bucketer_t* B, uint64_t* SB)
{
    fraglog_t log = {0};
    int rc = partition(A, n, B, C->c, SB, &log, C->st);
    if (rc == ORC_OK)
        rc = defragment(A, n, SB, B->fanout, log.pairs, log.n);
    free(log.pairs);
    return rc;
}

/* Highest differing bit of a range's extreme words: the MSD fallback of
 * reading R18 partitions on the bits just below it. */
static void range_extremes(const uint64_t* A, uint64_t n, uint64_t* lo, uint64_t* hi)
{
    *lo = ~0ull;
    *hi = 0;
    for (uint64_t k = 0; k < n; ++k) {
        if (A[k] < *lo) *lo = A[k];
        if (A[k] > *hi) *hi = A[k];
    }
}

/* The MSD digit of reading R18 for a range whose extremes differ first at
 * bit d: the b' = min(floor(log2 f), d+1) bits at [d+1-b', d] of the word.
 * Keys of the range agree above bit d, so the digit is monotone in the word,
 * and lo and hi get different digits (their bit d differs). */
static void msd_bucketer(bucketer_t* B, uint64_t lo, uint64_t hi, uint32_t f)
{
    uint32_t d = 63u - (uint32_t)__builtin_clzll(lo ^ hi);
    uint32_t lf = 0;
    while ((1u << (lf + 1)) <= f)
        ++lf;                                 /* floor(log2 f) */
    uint32_t bits = lf < d + 1 ? lf : d + 1;
    if (bits == 0)
        bits = 1;
    B->kind = BK_MSD;
    B->fanout = 1u << bits;
    B->shift = d + 1 - bits;
    B->mask = (1ull << bits) - 1u;
}

/* One split of reading R18 on a non-homogeneous range A[0..n): Partition +
 * Defragment by a local model trained on the range (Sec. 2's eCDF model on
 * a sample of the range).  When the largest bucket still holds more than
 * 7/8 of the keys the model made no real progress, and the range is
 * partitioned again on its MSD digit instead (force_msd: directly).  Every
 * child of a model split then holds at most 7/8 of the range, and every
 * child of an MSD split differs first at a lower bit than the range, which
 * bounds the depth (see depth_bound).  B, SB (C->f entries) and M (model
 * storage, freed by the caller when B->kind == BK_MODEL) receive the split. */
static int split_range(const ctx_t* C, uint64_t* A, uint64_t n, uint64_t start, uint32_t depth,
                       int force_msd, model_t* M, bucketer_t* B, uint64_t* SB)
{
    int rc = ORC_OK;
    memset(M, 0, sizeof *M);
    uint64_t biggest = n;
    if (!force_msd) {
        rc = model_fit_range(M, A, n, local_sample_size(C, n), local_seed(C->p->seed, start, depth),
                             C->L, C->dtype, NULL);
        if (rc)
            return rc;
        bucketer_t BM = {BK_MODEL, M, C->dtype, (double)C->f, 0, C->f, 0, 0};
        *B = BM;
        rc = partition_defrag(C, A, n, B, SB);
        biggest = 0;
        for (uint32_t j = 0; j < C->f; ++j)
            if (SB[j] > biggest)
                biggest = SB[j];
    }
    if (rc == ORC_OK && 8 * biggest > 7 * n) {
        uint64_t lo, hi;
        range_extremes(A, n, &lo, &hi);
        msd_bucketer(B, lo, hi, C->f);
        B->M = M;
        C->st->fallbacks++;
        rc = partition_defrag(C, A, n, B, SB);
    }
    return rc;
}

/* Reading R18: recursion into an over-full, non-homogeneous range. */
static int recurse_local(const ctx_t* C, uint64_t* A, uint64_t n, uint64_t start, uint32_t depth)
{
    if (n <= 1 || homogeneous(A, n))
        return ORC_OK;
    if (depth > C->depth_max)
        return ORC_ERR_DEPTH;
    if (depth > C->st->max_depth)
        C->st->max_depth = depth;
    uint64_t* SB = (uint64_t*)malloc((size_t)C->f * sizeof(uint64_t));
    if (!SB)
        return ORC_ERR_NOMEM;
    model_t M;
    bucketer_t B;
    int rc = split_range(C, A, n, start, depth, 0, &M, &B, SB);
    uint64_t r = 0;
    for (uint32_t j = 0; j < B.fanout && rc == ORC_OK; ++j) {
        rc = finish_child(C, A + r, SB[j], start + r, depth, &B, j);
        r += SB[j];
    }
    free(SB);
    model_free(&M);
    return rc;
}

/* Deepest level a sort of n keys may reach: levels 0 and 1, then at most
 * ceil(log_{8/7} n) <= 6 ceil(log2 n) model splits (each child keeps at most
 * 7/8 of its range) and at most 64 MSD splits (each lowers the highest bit
 * in which a range's keys differ). */
static uint32_t depth_bound(uint64_t n)
{
    uint32_t lg = 0;
    while (lg < 64 && (1ull << lg) < n)
        ++lg;
    return 2u + 64u + 6u * lg;
}

void orc_default_params(orc_params* p, uint32_t dtype)
{
    memset(p, 0, sizeof *p);
    p->fanout = 1000;
    p->frag_cap = 100;
    p->leaves = 1000;
    p->small_n = 0;
    p->s_max = 0;
    p->sample_rate = 0.01;
    p->sample_cap = 0;
    p->seed = 0x2107032900000001ull;
    p->local_min_sample = 1024;
    p->dtype = dtype;
}

static int check_params(const orc_params* p)
{
    if (!p || p->fanout < 2 || p->frag_cap < 1 || p->leaves < 1)
        return ORC_ERR_ARG;
    if (p->dtype != ORC_F64 && p->dtype != ORC_U64)
        return ORC_ERR_ARG;
    if (!(p->sample_rate > 0.0))
        return ORC_ERR_ARG;
    return ORC_OK;
}

/* LearnedSort 2.0 (Alg. 2) on ord keys. */
static int learned_sort(const ctx_t* C, uint64_t* A, uint64_t n)
{
    uint32_t f = C->f;
    uint32_t small = C->p->small_n ? C->p->small_n : 2u * f;
    if (n <= 1)
        return ORC_OK;
    if (n <= small) {
        C->st->touchup_moves += orc_insertion_sort_ord(A, n);
        return ORC_OK;
    }
    model_t M;
    uint64_t m = orc_sample_size(n, C->p->sample_rate, C->p->sample_cap);
    int rc = model_fit_range(&M, A, n, m, C->p->seed, C->L, C->dtype, NULL);
    if (rc)
        return rc;
    uint64_t* SB = (uint64_t*)malloc((size_t)f * sizeof(uint64_t));
    uint64_t* SB1 = (uint64_t*)malloc((size_t)f * sizeof(uint64_t));
    if (!SB || !SB1) {
        free(SB);
        free(SB1);
        model_free(&M);
        return ORC_ERR_NOMEM;
    }
    /* Level 0: Partition + Defragment. */
    bucketer_t B0 = {BK_MODEL, &M, C->dtype, (double)f, 0, f, 0, 0};
    rc = partition_defrag(C, A, n, &B0, SB);
    /* Level 1: re-partition each non-homogeneous bucket, then sort the
     * sub-buckets. */
    uint64_t r = 0;
    for (uint32_t i = 0; i < f && rc == ORC_OK; ++i) {
        uint64_t ni = SB[i];
        uint64_t s = r;
        if (homogeneous(A + s, ni)) {
            if (ni > 1)
                C->st->homogeneous++;
            r += ni;
            continue;
        }
        if (C->st->max_depth < 1)
            C->st->max_depth = 1;
        bucketer_t B1 = {BK_MODEL, &M, C->dtype, (double)f * (double)f, (int64_t)i * (int64_t)f, f, 0, 0};
        rc = partition_defrag(C, A + s, ni, &B1, SB1);
        for (uint32_t j = 0; j < f && rc == ORC_OK; ++j) {
            uint64_t nj = SB1[j];
            rc = finish_child(C, A + r, nj, r, 1, &B1, j);
            r += nj;
        }
    }
    free(SB);
    free(SB1);
    model_free(&M);
    if (rc)
        return rc;
    /* Touch-up over the whole array. */
    C->st->touchup_moves += orc_insertion_sort_ord(A, n);
    return ORC_OK;
}

int orc_sort(uint64_t* keys, size_t n, const orc_params* p, orc_stats* st)
{
    orc_stats local;
    if (!st)
        st = &local;
    memset(st, 0, sizeof *st);
    int rc = check_params(p);
    if (rc || (n && !keys)) {
        st->status = ORC_ERR_ARG;
        return ORC_ERR_ARG;
    }
    ctx_t C = {p, st, p->fanout, p->frag_cap, p->leaves, p->dtype, p->s_max, depth_bound(n)};
    for (size_t k = 0; k < n; ++k)
        keys[k] = raw_to_ord(keys[k], p->dtype);
    rc = learned_sort(&C, keys, n);
    for (size_t k = 0; k < n; ++k)
        keys[k] = ord_to_raw(keys[k], p->dtype);
    st->status = rc;
    return rc;
}

/* ------------------------------------------------------- stage exports ---- */

static uint64_t* to_ord_copy(const uint64_t* keys, size_t n, uint32_t dtype)
{
    uint64_t* A = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    if (A)
        for (size_t k = 0; k < n; ++k)
            A[k] = raw_to_ord(keys[k], dtype);
    return A;
}

int orc_train(const uint64_t* keys, size_t n, const orc_params* p, double* model_out, uint64_t* sample_idx)
{
    if (check_params(p) || !keys || n == 0 || !model_out)
        return ORC_ERR_ARG;
    uint64_t* A = to_ord_copy(keys, n, p->dtype);
    if (!A)
        return ORC_ERR_NOMEM;
    model_t M;
    uint64_t m = orc_sample_size(n, p->sample_rate, p->sample_cap);
    int rc = model_fit_range(&M, A, n, m, p->seed, p->leaves, p->dtype, sample_idx);
    if (rc == ORC_OK) {
        model_export(&M, model_out);
        model_free(&M);
    }
    free(A);
    return rc;
}

int orc_train_sample(const uint64_t* sample, uint64_t m, uint32_t leaves, uint32_t dtype,
                     double* model_out)
{
    if (!sample || m == 0 || leaves < 1 || !model_out || (dtype != ORC_F64 && dtype != ORC_U64))
        return ORC_ERR_ARG;
    uint64_t* A = to_ord_copy(sample, m, dtype);
    if (!A)
        return ORC_ERR_NOMEM;
    model_t M;
    int rc = model_train(&M, A, m, leaves, dtype);
    if (rc == ORC_OK) {
        model_export(&M, model_out);
        model_free(&M);
    }
    free(A);
    return rc;
}

double orc_model_eval(const double* model, uint32_t leaves, uint64_t key, uint32_t dtype)
{
    model_t M;
    if (model_import(&M, model, leaves))
        return -1.0;
    double F = model_F(&M, ord_value(raw_to_ord(key, dtype), dtype));
    model_free(&M);
    return F;
}

uint32_t orc_bucket(const double* model, uint32_t leaves, uint64_t key, uint32_t dtype,
                    double scale, int64_t offset, uint32_t fanout)
{
    model_t M;
    if (model_import(&M, model, leaves))
        return ~0u;
    bucketer_t B = {BK_MODEL, &M, dtype, scale, offset, fanout, 0, 0};
    uint32_t b = bucket_of(&B, raw_to_ord(key, dtype));
    model_free(&M);
    return b;
}

int orc_partition(uint64_t* keys, size_t n, const double* model, uint32_t leaves,
                  uint32_t dtype, uint32_t fanout, uint32_t frag_cap, uint32_t level,
                  uint32_t parent, uint64_t* sb, uint64_t* frag_log, uint64_t frag_log_cap,
                  uint64_t* nfrag)
{
    if (!keys || !model || !sb || fanout < 2 || frag_cap < 1 || level > 1)
        return ORC_ERR_ARG;
    model_t M;
    int rc = model_import(&M, model, leaves);
    if (rc)
        return rc;
    for (size_t k = 0; k < n; ++k)
        keys[k] = raw_to_ord(keys[k], dtype);
    double scale = level ? (double)fanout * (double)fanout : (double)fanout;
    int64_t off = level ? (int64_t)parent * (int64_t)fanout : 0;
    bucketer_t B = {BK_MODEL, &M, dtype, scale, off, fanout, 0, 0};
    fraglog_t log = {0};
    rc = partition(keys, n, &B, frag_cap, sb, &log, NULL);
    if (nfrag)
        *nfrag = log.n;
    if (frag_log)
        for (uint64_t k = 0; k < log.n && k < frag_log_cap; ++k) {
            frag_log[2 * k] = log.pairs[2 * k];
            frag_log[2 * k + 1] = log.pairs[2 * k + 1];
        }
    for (size_t k = 0; k < n; ++k)
        keys[k] = ord_to_raw(keys[k], dtype);
    free(log.pairs);
    model_free(&M);
    return rc;
}

int orc_defragment(uint64_t* keys, size_t n, const uint64_t* sb, uint32_t fanout,
                   const uint64_t* frag_log, uint64_t nfrag)
{
    if ((n && !keys) || !sb || (nfrag && !frag_log))
        return ORC_ERR_ARG;
    return defragment(keys, n, sb, fanout, frag_log, nfrag);
}

int orc_counting_sort(uint64_t* keys, size_t n, const double* model, uint32_t leaves,
                      uint32_t dtype, double scale, double offset)
{
    if ((n && !keys) || !model)
        return ORC_ERR_ARG;
    model_t M;
    int rc = model_import(&M, model, leaves);
    if (rc)
        return rc;
    for (size_t k = 0; k < n; ++k)
        keys[k] = raw_to_ord(keys[k], dtype);
    rc = counting_sort(keys, n, &M, dtype, scale, offset, NULL);
    for (size_t k = 0; k < n; ++k)
        keys[k] = ord_to_raw(keys[k], dtype);
    model_free(&M);
    return rc;
}

uint64_t orc_insertion_sort(uint64_t* keys, size_t n, uint32_t dtype)
{
    for (size_t k = 0; k < n; ++k)
        keys[k] = raw_to_ord(keys[k], dtype);
    uint64_t moves = orc_insertion_sort_ord(keys, n);
    for (size_t k = 0; k < n; ++k)
        keys[k] = ord_to_raw(keys[k], dtype);
    return moves;
}

int orc_stage_level0(const uint64_t* keys, size_t n, const orc_params* p,
                     const double* model_in,
                     uint64_t* sb, uint64_t* minmax, uint8_t* homog, uint64_t* sb1,
                     uint64_t* out_keys, uint64_t* frag_log, uint64_t frag_log_cap,
                     uint64_t* nfrag)
{
    if (check_params(p) || !keys || n == 0)
        return ORC_ERR_ARG;
    uint32_t f = p->fanout;
    orc_stats st;
    memset(&st, 0, sizeof st);
    ctx_t C = {p, &st, f, p->frag_cap, p->leaves, p->dtype, p->s_max, depth_bound(n)};
    uint64_t* A = to_ord_copy(keys, n, p->dtype);
    uint64_t* SB = (uint64_t*)malloc((size_t)f * sizeof(uint64_t));
    uint64_t* SB1 = (uint64_t*)malloc((size_t)f * sizeof(uint64_t));
    if (!A || !SB || !SB1) {
        free(A);
        free(SB);
        free(SB1);
        return ORC_ERR_NOMEM;
    }
    model_t M;
    int rc;
    if (model_in)
        rc = model_import(&M, model_in, p->leaves);
    else
        rc = model_fit_range(&M, A, n, orc_sample_size(n, p->sample_rate, p->sample_cap), p->seed,
                             p->leaves, p->dtype, NULL);
    if (rc) {
        free(A);
        free(SB);
        free(SB1);
        return rc;
    }
    bucketer_t B0 = {BK_MODEL, &M, p->dtype, (double)f, 0, f, 0, 0};
    fraglog_t log = {0};
    rc = partition(A, n, &B0, p->frag_cap, SB, &log, &st);
    if (rc == ORC_OK) {
        if (nfrag)
            *nfrag = log.n;
        if (frag_log)
            for (uint64_t k = 0; k < log.n && k < frag_log_cap; ++k) {
                frag_log[2 * k] = log.pairs[2 * k];
                frag_log[2 * k + 1] = log.pairs[2 * k + 1];
            }
        rc = defragment(A, n, SB, f, log.pairs, log.n);
    }
    free(log.pairs);
    if (rc == ORC_OK) {
        uint64_t r = 0;
        for (uint32_t i = 0; i < f && rc == ORC_OK; ++i) {
            uint64_t ni = SB[i];
            uint64_t lo = ~0ull, hi = 0;
            for (uint64_t k = 0; k < ni; ++k) {
                if (A[r + k] < lo) lo = A[r + k];
                if (A[r + k] > hi) hi = A[r + k];
            }
            int hom = homogeneous(A + r, ni);
            if (sb) sb[i] = ni;
            if (minmax) {
                minmax[2 * i] = lo;
                minmax[2 * i + 1] = hi;
            }
            if (homog) homog[i] = (uint8_t)hom;
            if (sb1) {
                memset(sb1 + (size_t)i * f, 0, (size_t)f * sizeof(uint64_t));
                if (!hom) {
                    uint64_t* tmp = (uint64_t*)malloc((size_t)ni * sizeof(uint64_t));
                    if (!tmp) {
                        rc = ORC_ERR_NOMEM;
                        break;
                    }
                    memcpy(tmp, A + r, (size_t)ni * sizeof(uint64_t));
                    bucketer_t B1 = {BK_MODEL, &M, p->dtype, (double)f * (double)f,
                                     (int64_t)i * (int64_t)f, f, 0, 0};
                    rc = partition_defrag(&C, tmp, ni, &B1, SB1);
                    if (rc == ORC_OK)
                        memcpy(sb1 + (size_t)i * f, SB1, (size_t)f * sizeof(uint64_t));
                    free(tmp);
                }
            }
            r += ni;
        }
    }
    if (rc == ORC_OK && out_keys)
        for (size_t k = 0; k < n; ++k)
            out_keys[k] = ord_to_raw(A[k], p->dtype);
    model_free(&M);
    free(A);
    free(SB);
    free(SB1);
    return rc;
}

int orc_split_stage(const uint64_t* keys, size_t n, const orc_params* p, uint64_t start, uint32_t depth,
                    int force_msd, uint64_t* out_keys, uint64_t* sb, uint32_t sb_cap, uint32_t* fanout_out,
                    uint32_t* msd_out, uint32_t* shift_out)
{
    if (check_params(p) || !keys || n < 2 || !sb || sb_cap < p->fanout)
        return ORC_ERR_ARG;
    orc_stats st;
    memset(&st, 0, sizeof st);
    ctx_t C = {p, &st, p->fanout, p->frag_cap, p->leaves, p->dtype, p->s_max, depth_bound(n)};
    uint64_t* A = to_ord_copy(keys, n, p->dtype);
    uint64_t* SB = (uint64_t*)calloc(p->fanout, sizeof(uint64_t));
    if (!A || !SB) {
        free(A);
        free(SB);
        return ORC_ERR_NOMEM;
    }
    int rc = homogeneous(A, n) ? ORC_ERR_ARG : ORC_OK;
    model_t M;
    memset(&M, 0, sizeof M);
    bucketer_t B;
    if (rc == ORC_OK)
        rc = split_range(&C, A, n, start, depth, force_msd, &M, &B, SB);
    if (rc == ORC_OK) {
        memset(sb, 0, (size_t)sb_cap * sizeof(uint64_t));
        memcpy(sb, SB, (size_t)B.fanout * sizeof(uint64_t));
        if (fanout_out) *fanout_out = B.fanout;
        if (msd_out) *msd_out = B.kind == BK_MSD;
        if (shift_out) *shift_out = B.kind == BK_MSD ? B.shift : 0;
        if (out_keys)
            for (size_t k = 0; k < n; ++k)
                out_keys[k] = ord_to_raw(A[k], p->dtype);
    }
    model_free(&M);
    free(A);
    free(SB);
    return rc;
}
