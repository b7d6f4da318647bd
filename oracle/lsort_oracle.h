/*
 * LearnedSort 2.0 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of LearnedSort 2.0
 * (Kristo, Vaidya, Kraska: "Defeating duplicates: A re-design of the
 * LearnedSort algorithm", arXiv 2107.03290), written from the paper:
 *   - Algorithm 1 (fragment partitioning with a write head),
 *   - Algorithm 2 (two-level driver, homogeneity skip, model-based counting
 *     sort, insertion-sort touch-up),
 *   - Section 6.1 (two-layer model, 1000 leaves, 1% sample, fan-out 1000,
 *     fragment capacity 100).
 *
 * Only the tests, the package smoke check and the benchmark's CPU-baseline
 * leg may load this library.  The GPU library shares no code with it.
 *
 * Keys are handled as order-preserving unsigned 64-bit words ("ord"):
 *   u64: the key itself;
 *   f64: IEEE-754 bits b mapped to b ^ (sign ? ~0 : 1<<63), i.e. totalOrder
 *        (-NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN).
 * The sorted output is the unique non-decreasing permutation under that order.
 */
#ifndef LSORT_ORACLE_H
#define LSORT_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F64 = 1, ORC_U64 = 2 };

enum {
    ORC_OK = 0,
    ORC_ERR_ARG = -1,
    ORC_ERR_NOMEM = -2,
    ORC_ERR_WRITE_HEAD = -3,   /* write head overtook the read head (Alg. 1 invariant) */
    ORC_ERR_PARTITION = -4,    /* fragments do not account for every key */
    ORC_ERR_DEPTH = -5,        /* recursion passed its depth bound (reading R18) */
};

typedef struct {
    uint32_t fanout;           /* f: buckets per partition (Sec. 6.1: 1000) */
    uint32_t frag_cap;         /* c: fragment capacity (Sec. 6.1: 100) */
    uint32_t leaves;           /* L: leaf models of the two-layer model (Sec. 6.1: 1000) */
    uint32_t small_n;          /* n <= small_n: insertion sort only (0 -> 2*f) */
    uint64_t s_max;            /* 0: paper-literal two levels; else recurse into sub-buckets > s_max */
    double   sample_rate;      /* Sec. 6.1: 1% */
    uint64_t sample_cap;       /* 0: no cap on the global sample size */
    uint64_t seed;             /* seed of the SplitMix64 sample stream */
    uint32_t local_min_sample; /* minimum sample of a local (recursion) model */
    uint32_t dtype;            /* ORC_F64 or ORC_U64 */
} orc_params;

typedef struct {
    uint64_t touchup_moves;    /* element moves made by the final insertion sort */
    uint64_t fragments;        /* fragments copied back, over every Partition call */
    uint64_t partitions;       /* Partition calls */
    uint64_t homogeneous;      /* buckets skipped as homogeneous */
    uint64_t counting_sorts;   /* model-based counting sorts run */
    uint64_t fallbacks;        /* no-progress MSD fallbacks taken */
    uint32_t max_depth;        /* deepest partition level reached (0 = level 0) */
    int32_t  status;
} orc_stats;

/* Model export layout (doubles): [xmin, xmax, rs, m'] then, for each of the
 * L leaf knots and then the start knot (at the sample minimum), [X, y, ym,
 * y1, ylo, yhi, s]: the knot; the sample eCDF just below it, its mid-rank and
 * the eCDF at and below it; the segment above the knot (from ylo, slope s,
 * up to yhi).  A leaf without sample values has X = +inf.
 * Size 4 + 7*(L+1). */
#define ORC_MODEL_DOUBLES(L) (4u + 7u * ((uint32_t)(L) + 1u))

void orc_default_params(orc_params* p, uint32_t dtype);

/* Sort keys (raw f64 bits or u64 words) in place. */
int orc_sort(uint64_t* keys, size_t n, const orc_params* p, orc_stats* st);

/* Sample size m for n keys and the t-th sample index (Sec. 6.1, 1% sample). */
uint64_t orc_sample_size(uint64_t n, double rate, uint64_t cap);
uint64_t orc_sample_index(uint64_t seed, uint64_t t, uint64_t n);
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t t);

/* Train the global model on the sample of keys[0..n); write it in the export
 * layout.  sample_idx (m entries, may be NULL) receives the sample indices. */
int orc_train(const uint64_t* keys, size_t n, const orc_params* p,
              double* model_out, uint64_t* sample_idx);

/* Train on the given sample (raw keys) instead of drawing one. */
int orc_train_sample(const uint64_t* sample, uint64_t m, uint32_t leaves, uint32_t dtype,
                     double* model_out);

/* Model evaluation F_A(x) of an exported model for one raw key. */
double orc_model_eval(const double* model, uint32_t leaves, uint64_t key, uint32_t dtype);

/* Bucket of one raw key: clamp(floor(F*scale) - offset, 0, fanout-1). */
uint32_t orc_bucket(const double* model, uint32_t leaves, uint64_t key, uint32_t dtype,
                    double scale, int64_t offset, uint32_t fanout);

/* Level-0 stage of Alg. 2 on a copy of keys: Partition + Defragment with the
 * given exported model (NULL: train it).  Outputs (each may be NULL):
 *   sb[f]        bucket sizes S_B,
 *   minmax[2f]   per bucket (min ord, max ord); empty buckets give (~0, 0),
 *   homog[f]     1 if the bucket is homogeneous (bitwise-equal keys, or size <= 1),
 *   sb1[f*f]     level-1 sizes S'_B of every non-homogeneous bucket (row i),
 *   out_keys[n]  the array after level-0 Partition + Defragment,
 *   frag_log     (bucket, size) pairs in copy-back order (2 * nfrag entries),
 *   nfrag        number of fragments of the level-0 partition. */
int orc_stage_level0(const uint64_t* keys, size_t n, const orc_params* p,
                     const double* model_in,
                     uint64_t* sb, uint64_t* minmax, uint8_t* homog, uint64_t* sb1,
                     uint64_t* out_keys, uint64_t* frag_log, uint64_t frag_log_cap,
                     uint64_t* nfrag);

/* Alg. 1 alone on keys[0..n) in place (no defragment) with an exported model,
 * level p (0: scale f, offset 0; 1: scale f^2, offset i*f).  Writes S_B and
 * the fragment log (bucket, size) pairs.  Returns ORC_OK or an error. */
int orc_partition(uint64_t* keys, size_t n, const double* model, uint32_t leaves,
                  uint32_t dtype, uint32_t fanout, uint32_t frag_cap, uint32_t level,
                  uint32_t parent, uint64_t* sb, uint64_t* frag_log, uint64_t frag_log_cap,
                  uint64_t* nfrag);

/* Defragment (bucket contiguity) given S_B and the fragment log. */
int orc_defragment(uint64_t* keys, size_t n, const uint64_t* sb, uint32_t fanout,
                   const uint64_t* frag_log, uint64_t nfrag);

/* Model-based counting sort of one sub-bucket followed by nothing else:
 * slot = clamp(floor((F*scale - offset) * n), 0, n-1).  Returns the number of
 * keys placed. */
int orc_counting_sort(uint64_t* keys, size_t n, const double* model, uint32_t leaves,
                      uint32_t dtype, double scale, double offset);

/* One recursion split of reading R18 on a copy of keys[0..n) (n >= 2, not
 * all equal), exactly as the sort takes it for a range at `start` (relative
 * to the array) and recursion level `depth`: Partition + Defragment by a
 * local model trained on the range, or, when its largest bucket keeps more
 * than 7/8 of the keys (or with force_msd), by the MSD digit below the
 * range's highest differing bit.  Outputs: out_keys[n] (may be NULL) the
 * range after the split, sb[sb_cap >= fanout] the child sizes (zero past
 * the split's fanout), *fanout_out the children, *msd_out 1 for an MSD
 * split, *shift_out its digit's shift. */
int orc_split_stage(const uint64_t* keys, size_t n, const orc_params* p, uint64_t start, uint32_t depth,
                    int force_msd, uint64_t* out_keys, uint64_t* sb, uint32_t sb_cap, uint32_t* fanout_out,
                    uint32_t* msd_out, uint32_t* shift_out);

/* Insertion sort on ord order; returns element moves. */
uint64_t orc_insertion_sort(uint64_t* keys, size_t n, uint32_t dtype);

#ifdef __cplusplus
}
#endif
#endif
