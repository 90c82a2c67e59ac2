// pcf_driver.h -- host-side driver of the PCF Learned Sort library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/pcfsort.h"
#include "pcf_device.h"

namespace pcf {

// Records a failed HIP call for pcf_last_hip_error() and returns PCF_ERR_HIP
// (PCF_DEBUG=1 in the environment prints the call site to stderr).
int hip_fail(hipError_t e, const char* what = nullptr, int line = 0);

#define PCF_HIP(call)                                              \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return hip_fail(e_, #call, __LINE__);    \
  } while (0)

struct Layout {
  size_t ctl, tmp_keys, tmp_vals, int_keys, trace_b, mmr, sbuf0;
  size_t nodes[2], units[2], table[2], cm[2], mm[2], bstart[2], cmap[2], task_node[2], items[3];
  size_t total;
  uint32_t cap_nodes, cap_units, cap_aux;
  uint64_t cap_table, cap_cm;
  uint32_t cap_items[3];
  uint32_t nbmax;
};

Layout make_layout(size_t n, int has_pay, uint32_t nseg, const pcf_policy& pol, int int_keys,
                   uint32_t trace_nb, uint32_t trace_beta);

// One sort call: plain (offsets == NULL, nseg = 1) or segmented.
struct SortArgs {
  int key_type;
  const void* keys_in;
  void* keys_out;          // NULL for argsort without keys: workspace keys are used
  const uint32_t* vals_in; // NULL: none, or iota when `iota`
  uint32_t* vals_out;      // NULL: keys only
  int iota;
  const uint64_t* offsets; // device CSR offsets or NULL
  const uint64_t* seg_src; // device array of per-segment key addresses (keys_in unused), or NULL
  int no_graph;            // segmented: always launch eagerly
  const pcf_policy* pol_override;  // NULL: the tuned / default policy for n
  uint32_t nseg;
  size_t n;
  void* ws;
  size_t ws_bytes;
  int32_t* d_status;
  hipStream_t stream;
  // diagnostics (pcf_level_trace)
  int trace;
  uint64_t trace_seed;
  uint32_t trace_alpha, trace_beta, trace_nb;
  uint64_t* h_b;
  uint64_t* h_T;
  uint64_t* h_sizes;
  uint64_t* h_scalars;
  // filled on return when not NULL
  uint32_t* levels_run;
  int no_prof;             // record no profile events (they would be created on demand)
};

int run_sort(const SortArgs& a);
// Exact workspace of one call (int_keys: argsort without a key output).
size_t workspace_for(int key_type, size_t n, int has_pay, uint32_t nseg, int int_keys);
int graph_stats(uint64_t* captures, uint64_t* replays, uint64_t* cached);
int graph_clear();

pcf_policy current_policy();

// One size class of a tuning table: arrays of min_n <= n < max_n keys of the
// given type (with or without a payload) use `pol`.
struct TuneEntry {
  int key_type, with_payload;
  uint64_t min_n, max_n;
  pcf_policy pol;
  double ms;  // measured time of the representative size
};
pcf_policy policy_for(int key_type, size_t n, int has_pay);
void install_table(const std::vector<TuneEntry>& t);
int check_policy(const pcf_policy& p);
int device_cus();

}  // namespace pcf
