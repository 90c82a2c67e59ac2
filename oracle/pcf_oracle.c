/*
 * pcf_oracle.c -- plain, slow CPU oracle of PCF Learned Sort.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  Build with
 *   gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 * so that every fp64 operation is one IEEE round-to-nearest step.
 * The PCFO_PLANT_* macros compile deliberate mistakes into throw-away copies
 * of the oracle; a test checks that the pins catch each one.  They are never
 * defined in the normal build.
 * See pcf_oracle.h for what is computed and the readings taken.
 */
#include "pcf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) -------------------------
 * The generator's state advances by the odd constant 0x9E3779B97F4A7C15 and
 * each output is the state passed through the published 64-bit finalizer.
 * pcfo_splitmix64(s, k) is the k-th output (k = 0, 1, ...) of the generator
 * whose state starts at s: a counter-based form of the same sequence. */
static uint64_t sm_finalize(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t pcfo_splitmix64(uint64_t state, uint64_t k)
{
    return sm_finalize(state + (k + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Seed of the node at (segment, depth, offset): SplitMix64 chained over the
 * identifiers, so the same node gets the same samples on every run. */
uint64_t pcfo_node_seed(uint64_t seed, uint64_t segment, uint64_t depth, uint64_t offset)
{
    uint64_t s = pcfo_splitmix64(seed, segment);
    s = pcfo_splitmix64(s, depth);
    return pcfo_splitmix64(s, offset);
}

/* Position of sample j in an array of n keys: uniform with replacement
 * (Sec. 3.3 takes alpha samples; the proofs treat them as independent draws). */
uint64_t pcfo_sample_index(uint64_t node_seed, uint64_t j, uint64_t n)
{
#ifdef PCFO_PLANT_SAMPLE_PREFIX
    (void)node_seed;
    return j % n; /* planted mistake: the first alpha keys instead of random draws */
#else
    unsigned __int128 p = (unsigned __int128)pcfo_splitmix64(node_seed, j) * n;
    return (uint64_t)(p >> 64);
#endif
}

/* floor(n^{3/4}) exactly: the largest m with m^4 <= n^3 (n < 2^42). */
uint64_t pcfo_root34(uint64_t n)
{
    unsigned __int128 n3 = (unsigned __int128)n * n * n;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        unsigned __int128 m2 = (unsigned __int128)mid * mid;
        if (m2 <= n3 / m2)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* eta(I) of App. A.4 for fp64 keys: the widest rounding cell meeting I =
 * [lo, hi], i.e. the spacing of doubles in the binade of max(|lo|, |hi|). */
double pcfo_eta_f64(double lo, double hi)
{
    double m = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
    int e;
    if (m == 0.0)
        return ldexp(1.0, -1074);
    frexp(m, &e); /* m = f 2^e, f in [0.5, 1): binade [2^(e-1), 2^e) */
    if (e - 53 < -1074)
        return ldexp(1.0, -1074);
    return ldexp(1.0, e - 53);
}

/* Left side of the fine-enough-quantization condition beta eta(I) / |I|. */
double pcfo_quant_lhs_f64(uint64_t beta, double lo, double hi)
{
    long double w = (long double)hi - (long double)lo;
    return (double)((long double)beta * (long double)pcfo_eta_f64(lo, hi) / w);
}

#define KEY double
#define SUFFIX f64
#define IS_F64 1
#include "pcf_oracle_impl.h"
#undef KEY
#undef SUFFIX
#undef IS_F64

#define KEY uint64_t
#define SUFFIX u64
#define IS_F64 0
#include "pcf_oracle_impl.h"
#undef KEY
#undef SUFFIX
#undef IS_F64

int pcfo_level(int key_type, const void *keys, const uint32_t *vals, uint64_t n,
               uint64_t node_seed, pcfo_level_io *io)
{
    if (!io || !keys || n == 0 || io->alpha == 0 || io->beta == 0 || !io->b || !io->T ||
        !io->sizes || !io->part_keys)
        return PCFO_ERR_ARG;
    if (io->model != PCFO_MODEL_PCF && io->model != PCFO_MODEL_SPLINE)
        return PCFO_ERR_ARG;
    if (key_type == PCFO_KEY_F64)
        return level_entry_f64((const double *)keys, vals, n, node_seed, io);
    if (key_type == PCFO_KEY_U64)
        return level_entry_u64((const uint64_t *)keys, vals, n, node_seed, io);
    return PCFO_ERR_ARG;
}

int pcfo_sort(int key_type, const void *keys_in, const uint32_t *vals_in, void *keys_out,
              uint32_t *vals_out, uint64_t n, uint64_t seed, uint64_t segment, uint64_t tau,
              pcfo_stats *stats)
{
    return pcfo_sort_model(key_type, keys_in, vals_in, keys_out, vals_out, n, seed, segment, tau,
                           PCFO_MODEL_PCF, stats);
}

int pcfo_sort_model(int key_type, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                    uint32_t *vals_out, uint64_t n, uint64_t seed, uint64_t segment, uint64_t tau,
                    int model, pcfo_stats *stats)
{
    if (model != PCFO_MODEL_PCF && model != PCFO_MODEL_SPLINE)
        return PCFO_ERR_ARG;
    pcfo_stats local;
    pcfo_stats *st = stats ? stats : &local;
    memset(st, 0, sizeof *st);
    if (n == 0)
        return PCFO_OK;
    if (!keys_in || !keys_out)
        return PCFO_ERR_ARG;
    if (key_type == PCFO_KEY_F64)
        return sort_entry_f64((const double *)keys_in, vals_in, (double *)keys_out, vals_out, n,
                              seed, segment, tau, model, st);
    if (key_type == PCFO_KEY_U64)
        return sort_entry_u64((const uint64_t *)keys_in, vals_in, (uint64_t *)keys_out, vals_out,
                              n, seed, segment, tau, model, st);
    return PCFO_ERR_ARG;
}
