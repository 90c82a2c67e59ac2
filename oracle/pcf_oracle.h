/*
 * pcf_oracle.h -- plain, slow CPU oracle of PCF Learned Sort.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the two meet only
 * through seeded input arrays produced by a separate generator module.
 *
 * What it computes (Sato & Matsui, "PCF Learned Sort", TMLR 2025):
 *   - optionally the Spline Learned Sort of App. A.5: the same training, and
 *     inference F(x) = (b_{i-1} + frac * (b_i - b_{i-1})) / alpha with frac
 *     the key's relative position inside its bin (b_{-1} = 0, 0-based bins);
 *   - Algorithm 1 (the Learned-Sort framework, Sec. 3.2): arrays shorter than
 *     tau go to the standard sort; otherwise a CDF model is trained, every
 *     key is appended to bucket floor(F(x) * gamma) (0-based here), buckets of
 *     size >= delta go to the standard sort, the others recurse, and the
 *     buckets are concatenated.
 *   - The PCF model (Sec. 3.3): i(x) = floor((x - x_min) beta / (x_max - x_min)),
 *     b_i = #{samples a_j : i(a_j) <= i}, F(x) = b_{i(x)} / alpha.
 *   - The parameter rule of the PCF theorems (Sec. 3.3):
 *     alpha = beta = gamma = delta = floor(n^{3/4}); tau = 100 as in Sec. 4.1.
 *
 * Readings where the paper is silent:
 *   - sampling is with replacement, index j of a node drawn from SplitMix64
 *     (counter-based: the j-th output of SplitMix64 started at the node seed),
 *     reduced to [0, n) by the high 64 bits of the 128-bit product;
 *   - the node seed is SplitMix64 chained over (seed, segment, depth, offset);
 *   - i(x) is evaluated in IEEE fp64 round-to-nearest as
 *     min(beta, floor(RN(RN(x - x_min) * RN(beta / RN(x_max - x_min))))),
 *     with both operands halved first when x_max - x_min overflows, and a node
 *     whose scale beta / (x_max - x_min) is not finite counts as a bucketing
 *     failure (standard sort); for uint64 keys RN(x - x_min) is the exact
 *     integer difference rounded to fp64;
 *   - floor(F(x) gamma) is the exact integer floor(b_i * gamma / alpha);
 *   - an array whose minimum equals its maximum is returned unchanged (the
 *     single-value early exit of Sec. 4.1), checked after the n < tau test;
 *   - keys must be finite and not -0.0 (the sorted order is then unique).
 *
 * Parity status: pinned (see tests/test_oracle_*.py); nothing here is
 * "parity unpinned".
 */
#ifndef PCF_ORACLE_H
#define PCF_ORACLE_H

#include <stdint.h>

#define PCFO_OK 0
#define PCFO_ERR_ARG 1
#define PCFO_ERR_INVALID_KEY 2
#define PCFO_ERR_NOMEM 3

#define PCFO_KEY_F64 0
#define PCFO_KEY_U64 1

/* CDF model of a bucketing: the PCF of Sec. 3.3, or the spline of App. A.5
 * (same training; inference interpolates linearly inside the key's bin). */
#define PCFO_MODEL_PCF 0
#define PCFO_MODEL_SPLINE 1

/* Counters filled by a full sort (all optional). */
typedef struct {
    uint64_t levels;          /* model-based bucketings performed */
    uint64_t max_depth;       /* deepest recursion depth that was entered (root = 0) */
    uint64_t small_sorts;     /* standard sorts of arrays with n < tau */
    uint64_t fail_sorts;      /* standard sorts of buckets with |c| >= delta */
    uint64_t fail_keys;       /* keys in those buckets */
    uint64_t single_valued;   /* early exits on x_min == x_max */
    uint64_t nonfinite_scale; /* nodes whose scale overflowed (standard sort) */
    double max_quant_lhs;     /* max over nodes of beta * eta(I) / |I| */
} pcfo_stats;

/* One model-based bucketing of one array with explicit parameters. */
typedef struct {
    /* inputs */
    uint64_t alpha, beta, gamma;
    const uint64_t *sample_idx; /* optional: alpha explicit sample positions (test hook) */
    /* outputs: caller-allocated arrays */
    uint64_t *b;          /* beta + 1 entries: inclusive prefix counts of the sample */
    uint64_t *T;          /* beta + 1 entries: bucket of each bin, floor(b_i gamma / alpha) */
    uint64_t *sizes;      /* gamma + 1 entries: bucket sizes */
    void *part_keys;      /* n keys: buckets concatenated, each in input order */
    uint32_t *part_vals;  /* n payload words or NULL */
    uint64_t *sample_pos; /* optional: alpha sample positions actually used */
    /* scalar outputs */
    uint64_t min_bits, max_bits; /* raw bits of x_min, x_max */
    double scale;                /* RN(beta / RN(x_max - x_min)) (halved form if flagged) */
    int halves;                  /* 1 when x_max - x_min overflowed and halves were used */
    int status;                  /* 0 bucketed, 1 single-valued, 2 scale not finite */
    /* input */
    int model;                   /* PCFO_MODEL_PCF or PCFO_MODEL_SPLINE */
} pcfo_level_io;

uint64_t pcfo_splitmix64(uint64_t state, uint64_t k);
uint64_t pcfo_node_seed(uint64_t seed, uint64_t segment, uint64_t depth, uint64_t offset);
uint64_t pcfo_sample_index(uint64_t node_seed, uint64_t j, uint64_t n);
uint64_t pcfo_root34(uint64_t n);
double pcfo_quant_lhs_f64(uint64_t beta, double lo, double hi);
double pcfo_eta_f64(double lo, double hi);

int pcfo_level(int key_type, const void *keys, const uint32_t *vals, uint64_t n,
               uint64_t node_seed, pcfo_level_io *io);

int pcfo_sort(int key_type, const void *keys_in, const uint32_t *vals_in, void *keys_out,
              uint32_t *vals_out, uint64_t n, uint64_t seed, uint64_t segment, uint64_t tau,
              pcfo_stats *stats);

/* The same recursion with the given CDF model (PCFO_MODEL_*). */
int pcfo_sort_model(int key_type, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                    uint32_t *vals_out, uint64_t n, uint64_t seed, uint64_t segment, uint64_t tau,
                    int model, pcfo_stats *stats);

#endif
