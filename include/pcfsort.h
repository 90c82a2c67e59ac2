/*
 * pcfsort.h -- C ABI of libpcfsort.so, an MI355X (gfx950) implementation of
 * PCF Learned Sort (Sato & Matsui, "PCF Learned Sort: a Learning Augmented
 * Sort Algorithm with O(n log log n) Expected Complexity", TMLR 2025).
 *
 * Problem (Algorithm 1, Sec. 3.2): given n keys, produce them in ascending
 * order.  The library runs the Learned-Sort recursion on the GPU: each level
 * samples the keys, fits the piecewise-constant CDF model (Sec. 3.3: equal-
 * width bins between the array's minimum and maximum, sample counts, prefix
 * sum), predicts every key's bucket from that model, counts, scans and
 * scatters the keys into contiguous buckets, and then sorts every bucket:
 * small ones inside one workgroup's LDS, ones of size >= delta with a
 * standard sort (radix), the rest by another level.
 *
 * Conventions for every call:
 *   - Buffers named d_* are device memory owned by the caller; the library
 *     never frees them.  They must stay valid until the work is complete.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Calls return a pcf_status.  Argument errors are reported synchronously
 *     and nothing is enqueued.  The sort calls enqueue their kernels on
 *     `stream`.  Given a device status word (d_status != NULL), a call
 *     enqueues a fixed chain of recursion levels (enough for any input of n
 *     keys: the delta rule's levels plus 9 radix levels; empty levels exit at
 *     once), the LDS finish and a kernel that writes the status word, and
 *     returns without waiting: with a caller workspace such a call can be
 *     captured into a hipGraph.  Without a status word a call waits for
 *     `stream`: it reads back a few bytes of level counts after the planned
 *     levels (runs only the extra levels an input needs) and at the end, and
 *     returns the data status.  The output is complete once `stream` is
 *     synchronized.
 *   - Keys are totally ordered by value.  fp64 keys must be finite and must
 *     not be -0.0 (then the ascending order is unique bit for bit); a key that
 *     breaks this makes the call return PCF_ERR_INVALID_KEY (detected on the
 *     device; also written to *d_status when d_status is not NULL) and leaves
 *     the output unspecified.
 *   - Sorts are stable: payload words of equal keys keep their input order,
 *     so argsort breaks ties by position.
 *   - keys_in == keys_out (in place) is allowed.  Other buffers must not
 *     overlap.
 *   - Scratch memory: pass a device workspace of at least
 *     pcf_workspace_bytes(...) bytes, or d_ws = NULL to let the library
 *     allocate stream-ordered memory for the call.
 *   - n and segment lengths with a uint32 payload must be < 2^32.
 *
 * Debugging switches (environment, read once per process):
 *   - PCF_SYNC=1: every sort call waits for its work and returns its data
 *     status, also when given a status word (not while `stream` is being
 *     captured into a graph).
 *   - PCF_TRACE=1: as PCF_SYNC, and one line per call on stderr: keys,
 *     segments, payload, nodes/units/keys of every level that ran, LDS items
 *     per class, status and overflow flags.
 *   - PCF_NO_GRAPH=1: segmented calls launch eagerly instead of replaying a
 *     captured graph.
 *   - PCF_DEBUG=1: the call site of a failed HIP call is printed to stderr.
 */
#ifndef PCFSORT_H
#define PCFSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCF_OK = 0,
    PCF_ERR_INVALID_ARGUMENT = 1, /* null pointer with n > 0, bad enum, size limits */
    PCF_ERR_INVALID_KEY = 2,      /* NaN, +-inf or -0.0 among fp64 keys */
    PCF_ERR_OUT_OF_MEMORY = 3,    /* workspace too small, allocation failed, over budget */
    PCF_ERR_HIP = 4,              /* a HIP runtime call failed: see pcf_last_hip_error() */
    PCF_ERR_UNSUPPORTED = 5,      /* no gfx950 device or feature not built */
    PCF_PENDING = 6,              /* serving: request not finished yet */
    PCF_ERR_UNKNOWN_TICKET = 7,   /* serving: ticket never issued or already released */
    PCF_ERR_SHUTDOWN = 8          /* serving: server is shutting down */
} pcf_status;

typedef enum {
    PCF_KEY_F64 = 0, /* IEEE binary64, ascending numeric order */
    PCF_KEY_U64 = 1  /* unsigned 64-bit integers */
} pcf_key_type;

/* Human-readable name of a status code (static string). */
const char *pcf_status_string(int status);
/* The last hipError_t seen by a call that returned PCF_ERR_HIP on this thread. */
int pcf_last_hip_error(void);
/* Library version string. */
const char *pcf_version(void);

/*
 * Workspace size for a sort of n keys in num_segments segments
 * (num_segments = 1 for the plain calls), with or without a uint32 payload.
 * An upper bound that holds for every input of that size.
 */
size_t pcf_workspace_bytes(int key_type, size_t n, int with_payload, uint32_t num_segments);

/*
 * Sort n fp64 keys ascending (Algorithm 1).  d_in and d_out hold n doubles
 * each; d_in may equal d_out.  d_status: optional device int32 that receives
 * the data status (PCF_OK or PCF_ERR_INVALID_KEY).
 */
int pcf_sort_f64(const double *d_in, double *d_out, size_t n, void *d_ws, size_t ws_bytes,
                 int32_t *d_status, void *stream);

/* Same for uint64 keys. */
int pcf_sort_u64(const uint64_t *d_in, uint64_t *d_out, size_t n, void *d_ws, size_t ws_bytes,
                 int32_t *d_status, void *stream);

/*
 * For callers that cannot allocate (code under hipGraph capture, tight
 * serving loops, hosts that forbid allocation): pcf_sort_f64 with no
 * workspace argument and no allocation of any kind.  The workspace is a
 * static device array of PCF_STATIC_SCRATCH_BYTES that the library holds on
 * every device it runs on, until the process ends.  n is limited to what that
 * array holds (about 10 million keys; pcf_workspace_bytes(PCF_KEY_F64, n, 0, 1)
 * must not exceed it): larger n returns PCF_ERR_OUT_OF_MEMORY and enqueues
 * nothing.  d_status is required (PCF_ERR_INVALID_ARGUMENT if NULL): the call
 * enqueues the fixed chain and returns; data errors reach *d_status.  Calls
 * on one device share the one array, so calls that overlap on a device (on
 * different streams, or on one stream reordered by the caller) race; calls in
 * order on one stream do not.  Profile events are not recorded for it.
 */
#define PCF_STATIC_SCRATCH_BYTES (128ull << 20)
int pcf_sort_f64_static(const double *d_in, double *d_out, size_t n, int32_t *d_status,
                        void *stream);

/*
 * In-place variant (the in-place forms of sample sort that Sec. 5 points to):
 * sorts the n keys of d_keys within that array.  A node larger than a fixed
 * staging capacity (2^24 keys) is bucketed in place (the model's 256 buckets,
 * eight rounds of a two-way in-place partition on the bits of the bucket id);
 * buckets are then sorted through a staging buffer of at most that many keys
 * by the segmented sort, and larger ones are bucketed in place again (with the
 * standard sort's radix digits once a bucket has failed, |c_j| >= delta).
 * Keys only: the swaps are not stable.  Workspace: pcf_inplace_workspace_bytes
 * (the staging buffer and its sort workspace, plus 1/64 of the key bytes for
 * marks and block counts), or d_ws = NULL to allocate it stream-ordered.
 * Waits for `stream` and returns the outcome (PCF_ERR_INVALID_KEY for an
 * invalid fp64 key).  n < 2^32.
 */
size_t pcf_inplace_workspace_bytes(int key_type, size_t n);
int pcf_sort_inplace(int key_type, void *d_keys, size_t n, void *d_ws, size_t ws_bytes,
                     void *stream);

/*
 * Argsort (Algorithm 1 with each key carrying its input position).
 * d_idx_out[k] receives the input position of the k-th smallest key; ties
 * are broken by ascending position.  d_keys_out (nullable) receives the
 * sorted keys; when NULL the keys are sorted in workspace memory.
 * n < 2^32.
 */
int pcf_argsort(int key_type, const void *d_keys_in, void *d_keys_out, uint32_t *d_idx_out,
                size_t n, void *d_ws, size_t ws_bytes, int32_t *d_status, void *stream);

/*
 * Segmented sort: segment s is keys [d_offsets[s], d_offsets[s+1]) and is
 * sorted on its own (Algorithm 1 per array), stably, carrying the optional
 * uint32 payload d_vals_in -> d_vals_out (both NULL for keys only; with a
 * payload every segment must be shorter than 2^32).  d_offsets: device array
 * of num_segments + 1 non-decreasing uint64 CSR offsets, d_offsets[0] = 0;
 * empty segments are allowed.  total_keys = d_offsets[num_segments] < 2^32.
 * Offsets that break these rules are found on the device: the call's data
 * status is then PCF_ERR_INVALID_ARGUMENT (status word or return value) and
 * the output is unspecified; no kernel accesses memory outside the buffers.
 * With a caller workspace (d_ws != NULL) the batch runs as one fixed launch
 * chain (enough levels for any input of total_keys keys, empty levels exit at
 * once) that is captured into a hipGraph on the first call with a given
 * argument set (device, key type, buffer pointers, sizes, d_status, policy)
 * and replayed by later calls with the same set; up to 16 executable graphs
 * are cached (least recently used evicted).  The graph reads the buffers'
 * contents at replay time, so a caller may refill them between calls.  With
 * d_ws == NULL, with profiling on, or with PCF_NO_GRAPH set in the
 * environment, the launches are made one by one.  Stream-ordered: returns
 * after enqueue when d_status is given, else waits and returns the outcome.
 */
int pcf_sort_segmented(int key_type, const void *d_keys_in, void *d_keys_out,
                       const uint32_t *d_vals_in, uint32_t *d_vals_out,
                       const uint64_t *d_offsets, uint32_t num_segments, size_t total_keys,
                       void *d_ws, size_t ws_bytes, int32_t *d_status, void *stream);

/* Graph cache counters of pcf_sort_segmented (captures, replays, entries held). */
int pcf_graph_stats(uint64_t *captures, uint64_t *replays, uint64_t *cached);
/* Waits for and destroys every cached graph (e.g. before freeing its buffers). */
int pcf_graph_clear(void);

/*
 * Diagnostic: run exactly one model-based bucketing level (Sec. 3.3 with the
 * given alpha, beta, gamma) on the whole array as one node named by
 * node_seed, and report the model.  The stable partition (buckets
 * concatenated, each in input order) goes to d_part_keys / d_part_vals
 * (d_vals_in NULL = no payload).  Host arrays (may be NULL): h_b and h_T
 * receive beta + 1 uint64 values (prefix counts b_i and the bucket of each
 * bin), h_sizes receives gamma + 1 bucket sizes, h_scalars receives
 * {min bits, max bits, scale bits, halves, status} as 5 uint64.
 * Synchronizes `stream`.  Limits: beta <= 16383, gamma <= 2047 (and alpha <=
 * 65535 with the spline model).  The level uses the current policy's model;
 * with the spline model h_T receives the prefix counts b_i the model
 * interpolates between.
 */
int pcf_level_trace(int key_type, const void *d_keys_in, const uint32_t *d_vals_in, size_t n,
                    uint64_t node_seed, uint32_t alpha, uint32_t beta, uint32_t gamma,
                    void *d_part_keys, uint32_t *d_part_vals, uint64_t *h_b, uint64_t *h_T,
                    uint64_t *h_sizes, uint64_t *h_scalars, void *stream);

/*
 * The bucketing-failure experiment of Sec. 4.2 (Fig. 3): for every cell c
 * (h_cells[4c .. 4c+3] = alpha, beta, gamma, delta) and every one of `reps`
 * fp64 arrays of n keys (device, array r at d_keys + r * n), one PCF bucketing
 * of the whole array (Sec. 3.3: alpha samples with replacement, beta + 1
 * equal-width bins, gamma + 1 buckets) with node seed chained over
 * (seed, c, r, 0); h_failures[c] receives the number of arrays for which some
 * bucket holds more than delta keys.  Parameters may exceed a sort level's
 * (beta, gamma < 2^30).  Allocates and frees its scratch stream-ordered and
 * synchronizes `stream`.
 */
int pcf_lfail_grid(const double *d_keys, size_t n, uint32_t reps, const uint32_t *h_cells,
                   uint32_t ncells, uint64_t seed, uint32_t *h_failures, void *stream);

/* ---- per-kernel profile -------------------------------------------------
 * When enabled, every later sort call records hipEvents around each of its
 * kernel launches on its stream and adds the elapsed times and the number of
 * keys each launch processed to process-wide counters.  A call without a
 * device status word waits for its stream and adds its figures at once; a
 * call with one returns after enqueueing, and its figures are added at the
 * calling thread's next call without a status word or its next
 * pcf_profile_read (which waits for those calls' streams).  Used by the
 * benchmark to price each kernel against the HBM roofline.
 */
typedef enum {
    PCF_K_SETUP = 0,    /* control block + roots */
    PCF_K_RANGE = 1,    /* minimum / maximum of the top-level arrays */
    PCF_K_FIT = 2,      /* samples, histogram, prefix, bin -> bucket table */
    PCF_K_COUNT = 3,    /* bucket counts per chunk */
    PCF_K_COLSCAN = 4,  /* scan of the counts over chunks */
    PCF_K_CLASSIFY = 5, /* bucket starts, recurse / standard-sort decision */
    PCF_K_SCATTER = 6,  /* stable scatter into contiguous buckets */
    PCF_K_LDS_SMALL = 7,/* in-LDS finish, arrays of up to 2048 keys */
    PCF_K_LDS_BIG = 8,  /* in-LDS finish, arrays of up to 8192 keys */
    /* key counts only (launches and ms stay 0), summed over levels: */
    PCF_K_RADIX_KEYS = 9,   /* keys bucketed by radix levels (standard sort of failed buckets) */
    PCF_K_BITONIC_KEYS = 10,/* keys bitonic-sorted in LDS (failed buckets and bins, equal keys) */
    PCF_K_SINGLE_KEYS = 11, /* keys in arrays found single-valued (early exit) */
    PCF_K_COUNT_KINDS = 12
} pcf_kernel_kind;

typedef struct {
    uint64_t launches;
    double ms;    /* summed hipEvent elapsed time */
    double keys;  /* summed keys processed by the launches */
    /* part of ms spent on the standard sort of failed buckets (|c_j| >= delta,
     * Algorithm 1), apportioned by key share: on a global level, ms times the
     * level's keys in radix nodes over its keys; in the LDS finish, ms times
     * the bitonic-sorted keys over the keys of the LDS items */
    double fallback_ms;
} pcf_kernel_stat;

int pcf_profile_enable(int on);
/* Restricts the events to the launch kinds whose bit (1 << kind) is set in
 * kind_mask, kinds PCF_K_SETUP .. PCF_K_LDS_BIG; the others run without events
 * and add nothing to their counters.  Fewer events leave fewer gaps between
 * launches, so a benchmark can time the whole call while it prices one kernel.
 * Default: all of them.  A bit at PCF_K_RADIX_KEYS or above:
 * PCF_ERR_INVALID_ARGUMENT (the key-count kinds are always summed). */
int pcf_profile_select(uint32_t kind_mask);
/* Copies PCF_K_COUNT_KINDS entries into out; reset != 0 clears the counters. */
int pcf_profile_read(pcf_kernel_stat *out, int reset);
const char *pcf_kernel_name(int kind);

/* ---- policy (parameters of the GPU recursion) ---------------------------- */

/*
 * Parameters of the GPU recursion.  The global levels pick gamma + 1 =
 * clamp(next power of two of len / target_child, 2, max_buckets) buckets,
 * beta = min(max_bins, bins_per_bucket * (gamma + 1)) bins and
 * alpha = min(max_samples, samples_per_bucket * (gamma + 1)) samples;
 * delta = floor(len^{3/4}) as in the paper's theorems.  Arrays of at most
 * lds_cap keys are finished inside one workgroup's LDS with the paper's own
 * parameters (alpha = beta = gamma = delta = floor(len^{3/4}), tau = 100).
 * Dynamic tuning of alpha, beta, gamma is suggested in Sec. 5.
 */
typedef struct {
    uint32_t max_buckets;        /* power of two, 2..2048 */
    uint32_t target_child;       /* keys per bucket aimed at */
    uint32_t bins_per_bucket;    /* beta / (gamma + 1) */
    uint32_t max_bins;           /* <= 16383 */
    uint32_t samples_per_bucket; /* alpha / (gamma + 1) */
    uint32_t max_samples;        /* <= 1 << 20 */
    uint32_t chunk_keys;         /* keys per count/scatter work unit (minimum) */
    uint32_t lds_cap;            /* largest array finished in LDS, <= 8192 */
    uint32_t tau;                /* small-array threshold inside LDS (paper: 100) */
    uint32_t seed;               /* sampling seed */
    uint32_t model;              /* CDF model of the global levels: 0 PCF (Sec. 3.3),
                                    1 spline (Spline Learned Sort, App. A.5); the
                                    in-LDS finish uses the PCF at one bin per key */
    uint32_t scatter_tile;       /* keys per scatter tile: 0 = default (8192 keys
                                    alone, 2048 with a payload); 4096 or 8192 for
                                    keys alone, 1024 or 2048 with a payload (other
                                    values take the default) */
} pcf_policy;

/* Current process-wide policy (defaults, or what pcf_set_policy / tuning set). */
int pcf_get_policy(pcf_policy *out);
int pcf_set_policy(const pcf_policy *p);

/* The policy a call of n keys uses: the loaded tuning table's entry for
 * (key_type, with_payload, n) if there is one, else the process-wide policy.
 * With a table loaded, the recursion also picks the parameters of every global
 * node (max_buckets, target_child, bins_per_bucket, max_bins,
 * samples_per_bucket, max_samples, chunk_keys) from the entry whose size class
 * holds the node's length, so the segments of a batch and the nodes of deeper
 * levels each use the entry tuned for their own size; the call's entry gives
 * the rest (lds_cap, tau, seed, model, scatter_tile). */
int pcf_policy_for(int key_type, size_t n, int with_payload, pcf_policy *out);

/*
 * Autotuner: on the current device, for four size classes ([0, 2^18),
 * [2^18, 2^22), [2^22, 2^25), [2^25, 2^32) keys; the first two timed on a
 * segmented batch of 2^25 keys in segments of floor(2^U[10, 18]) and
 * floor(2^U[18, 22]) keys, the others on one array of 2^23 and 2^26 keys),
 * times candidate policies (max_buckets, samples_per_bucket,
 * bins_per_bucket, chunk_keys, target_child, scatter_tile; coordinate descent from the
 * process-wide policy, hipEvent-timed, median of repeats, summed over uniform,
 * normal and lognormal synthetic arrays) and writes the winners as JSON to
 * out_json (format "pcfsort-tuning-1"; an entry's rep_n is the number of keys
 * it was timed on, for the two small classes the batch's total, which lies
 * outside the class's own [min_n, max_n)).  Takes a few seconds and about
 * 4.5 GB of device memory; does not change the active policy.
 * pcf_load_tuning reads such a file, validates every entry (policy limits as
 * pcf_set_policy, no overlapping classes of one kind) and installs it as the
 * table, replacing any previous one; json_path NULL clears the table.
 * A workspace sized before a table is loaded may be too small afterwards
 * (the call then returns PCF_ERR_OUT_OF_MEMORY).
 */
int pcf_autotune(int key_type, int with_payload, const char *out_json);
int pcf_load_tuning(const char *json_path);

/* ---- serving --------------------------------------------------------------
 * A request loop with continuous batching under an HBM budget.  Submitted
 * sorts wait in an admission queue; whenever a stream slot and enough budget
 * are free, the scheduler admits every queued request that fits, gathers them
 * into one segmented batch and launches it, so requests that arrive while
 * others run join the next batch and batches on different streams overlap on
 * the device.  Results stay device-resident in server-owned memory until
 * released.
 */
typedef struct pcf_server pcf_server;

typedef struct {
    uint64_t hbm_budget_bytes; /* device memory the server may hold (results + work) */
    uint32_t max_streams;      /* concurrent batches (1..8) */
    uint32_t max_batch_requests; /* requests per batch (>= 1) */
    uint64_t max_batch_keys;   /* keys per batch (>= 1) */
    int32_t device;            /* HIP device ordinal */
    uint32_t flags;            /* reserved, 0 */
} pcf_serve_config;

typedef struct {
    void *d_keys_sorted;  /* server-owned device buffer: n sorted keys */
    uint32_t *d_idx;      /* server-owned: argsort positions, or NULL */
    uint64_t n;
    uint64_t latency_ns;  /* submit -> completion observed by the server */
    uint64_t queue_ns;    /* submit -> admission */
    int32_t status;       /* PCF_OK or the request's error */
    uint32_t batch_requests; /* requests in the batch that ran it */
} pcf_result;

typedef struct {
    uint64_t submitted, completed, released, batches;
    uint64_t budget_bytes, budget_in_use, budget_high_water;
    uint64_t queued;
} pcf_serve_stats;

int pcf_serve_create(const pcf_serve_config *cfg, pcf_server **out);
/* Never blocks.  d_keys (n keys of key_type) must already hold their final
 * contents (any device work that writes them has completed), and must stay
 * valid and unchanged until the request is done: the server's own streams
 * read them, in no order with the caller's streams.  Keys written by work
 * still in flight on a stream: use pcf_serve_submit_after.  A request that
 * alone exceeds the budget returns PCF_ERR_OUT_OF_MEMORY. */
int pcf_serve_submit(pcf_server *s, int key_type, const void *d_keys, size_t n, int want_argsort,
                     uint64_t *ticket);
/* As pcf_serve_submit, for keys that work still in flight writes: the batch
 * that sorts the request first makes its stream wait for ready_event (a
 * hipEvent_t, passed as void*, recorded by the caller after that work; NULL =
 * ready now).  The event must not be destroyed until the request is done;
 * recording it again in the meantime can only delay the batch. */
int pcf_serve_submit_after(pcf_server *s, int key_type, const void *d_keys, size_t n,
                           int want_argsort, void *ready_event, uint64_t *ticket);
/* Non-blocking: PCF_OK and *out filled when done, PCF_PENDING otherwise. */
int pcf_serve_poll(pcf_server *s, uint64_t ticket, pcf_result *out);
/* Blocks until the request is done (or timeout_ms passes: PCF_PENDING). */
int pcf_serve_wait(pcf_server *s, uint64_t ticket, uint32_t timeout_ms, pcf_result *out);
/* Returns the result memory to the budget; the ticket becomes unknown. */
int pcf_serve_release(pcf_server *s, uint64_t ticket);
int pcf_serve_get_stats(pcf_server *s, pcf_serve_stats *out);
/* Stops admission, waits for running batches, frees everything. */
int pcf_serve_destroy(pcf_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PCFSORT_H */
