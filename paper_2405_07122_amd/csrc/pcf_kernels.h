// pcf_kernels.h -- declarations of the gfx950 kernels (defined and explicitly
// instantiated in pcf_kernels.hip) and the types their launches share with
// the host driver.
#pragma once

#include "pcf_device.h"

namespace pcf {

// Creates the roots: one node (or one LDS item) per non-empty segment.
// offsets == NULL means one segment [0, n).
struct RootArgs {
  const void* keys;
  const uint64_t* seg_src;  // per-segment key addresses (device), or NULL: keys + offset
  const uint32_t* vals;
  const uint64_t* offsets;
  uint64_t n;
  uint32_t nseg;
  uint32_t iota;
  uint32_t fixed_alpha, fixed_beta, fixed_nb;  // trace: explicit parameters
  uint32_t force_global;                        // trace: never an LDS item
  uint64_t fixed_seed;
  uint32_t has_fixed_seed;
};

__global__ void k_roots(Plan p, RootArgs a);
__global__ void k_init(Plan p);
// Publishes a call's outcome to the caller's device status word (when given)
// and to Ctl::status: the data error, else PCF_ERR_OUT_OF_MEMORY for a
// capacity overflow or nodes left at `check_level` (the end of a fixed chain;
// -1: no check), else PCF_ERR_HIP for a failed internal range check.
__global__ void k_finish(Plan p, int32_t* d_status, int check_level);
// Writes v to *d (the status word of a call with nothing to sort).
__global__ void k_set_status(int32_t* d, int32_t v);

struct LevelIO {
  void* dst_keys;       // where this level's scatter writes (absolute positions)
  uint32_t* dst_vals;
};

// LDS layout of the scatter (bytes), for NW waves and TS keys per tile.  The
// stable variant (with a payload) keeps per-wave bucket counters; the
// keys-only variant ranks with LDS atomics and needs none.
struct ScatterLds {
  uint32_t tab, wcnt, runoff, tstart, tcnt, mmlo, mmhi, cmapf, sk, sv, sb, total;
};
__host__ __device__ inline ScatterLds scatter_lds(uint32_t max_bins, uint32_t nbmax, int nw,
                                                  int ts, int pay, int wide_tab = 0) {
  ScatterLds l;
  uint32_t o = 0;
  auto take = [&](uint32_t bytes) {
    uint32_t r = o;
    o += (bytes + 15u) & ~15u;
    return r;
  };
  // bucket ids as bytes when they fit; spline tables hold 16-bit prefix counts
  l.tab = take((nbmax <= 256 && !wide_tab ? 1u : 2u) * (max_bins + 1));
  l.wcnt = take(pay ? 2u * nw * nbmax : 0u);
  l.runoff = take(4u * nbmax);
  l.tstart = take(4u * (nbmax + 1));
  l.tcnt = take(4u * nbmax);
  l.mmlo = take(8u * nbmax);
  l.mmhi = take(8u * nbmax);
  l.cmapf = take(1u * nbmax);
  l.sk = take(8u * ts);
  l.sv = take(pay ? 4u * ts : 0u);
  l.sb = take(2u * ts);
  l.total = o;
  return l;
}

// LDS layout of the keys-only scatter: a tile needs three barriers because
// the write-out reads per-bucket bases (wbase) that the next tile's offset
// update cannot touch before the next tile's first barrier.
struct ScatterKeysLds {
  uint32_t tab, runoff, tstart, wbase, tcnt, mmlo, mmhi, cmapf, sk, sb, total;
};
__host__ __device__ inline ScatterKeysLds scatter_keys_lds(uint32_t max_bins, uint32_t nbmax,
                                                           int ts, int wide_tab = 0) {
  ScatterKeysLds l;
  uint32_t o = 0;
  auto take = [&](uint32_t bytes) {
    uint32_t r = o;
    o += (bytes + 15u) & ~15u;
    return r;
  };
  // bucket ids as bytes when they fit; spline tables hold 16-bit prefix counts
  l.tab = take((nbmax <= 256 && !wide_tab ? 1u : 2u) * (max_bins + 1));
  l.runoff = take(4u * nbmax);
  l.tstart = take(4u * nbmax);
  l.wbase = take(4u * nbmax);
  l.tcnt = take(4u * nbmax);
  l.mmlo = take(8u * nbmax);
  l.mmhi = take(8u * nbmax);
  l.cmapf = take(1u * nbmax);
  l.sk = take(8u * ts);
  l.sb = take(2u * ts);
  l.total = o;
  return l;
}

// In-LDS finish: arrays of up to CAP keys, one bin per key at every level.
template <int CAP>
struct K5Cfg {
  static constexpr uint32_t SMAX = CAP / 16 + 8;  // ranges of >= tau (>= 16) keys
};

// Occupancy of the in-LDS finish: every class keeps 8 keys per thread (2048
// keys: 256 threads, 4096: 512, 8192: 1024), which fits 4 waves per SIMD (3 for
// uint64 keys with a payload), so a CU holds 4, 2 and 1 workgroups of the three
// classes (what their LDS allows) with 16 waves each time.  The launch uses
// exactly the resident number of workgroups: items are assigned statically, so
// a second round of workgroups would double the time of the last ones.

template <int KT, int CAP, int PAY, int NT>
struct K5Occ {
  // waves per SIMD: classes of 8 keys per thread fit 4 (uint64 with a payload:
  // 3); 16 keys per thread need twice the registers
  static constexpr int v = (CAP / NT <= 8) ? ((PAY && KT == 1) ? 3 : 4) : 2;
  static constexpr int by_waves() { return v * 4 / (NT / 64) > 0 ? v * 4 / (NT / 64) : 1; }
};

template <int KT, int CAP, int NT, int PAY>
struct K5Smem {
  uint64_t key[CAP];      // key images
  uint32_t seg[CAP];      // final segment: start | end << 16
  uint32_t cnt[CAP + 4];  // bin counts, then bin starts; cnt[CAP] = keys
  uint16_t pos[PAY ? CAP : 2];  // position inside the item (ties, payload)
  uint32_t stk[K5Cfg<CAP>::SMAX][3];  // start, end, depth | fail << 31
  uint64_t red64[2 * NT / 64];
  uint32_t red[NT / 64 + 1];
  uint32_t nstk;
  uint32_t flag;
  uint32_t sh[4];
};

// Resident workgroups per CU of an in-LDS finish class: what the waves allow,
// capped by what the 160 KiB of LDS holds.
template <int KT, int CAP, int PAY, int NT>
constexpr int k5_wg_per_cu() {
  const int by_lds = (int)((160 * 1024) / sizeof(K5Smem<KT, CAP, NT, PAY>));
  const int w = K5Occ<KT, CAP, PAY, NT>::by_waves();
  return w < by_lds ? w : (by_lds > 0 ? by_lds : 1);
}

template <int KT, int NT>
__global__ void k_range(Plan p);
template <int KT, int NT>
__global__ void k_fit(Plan p, int L, int trace);
template <int KT, int NT>
__global__ void k_count(Plan p, int L);
template <int NT>
__global__ void k_colscan(Plan p, int L);
template <int NT>
__global__ void k_classify(Plan p, int L, LevelIO io);
template <int KT, int NT, int TS, int PAY>
__global__ void k_scatter(Plan p, int L, LevelIO io, uint32_t max_bins, uint32_t nbmax);
template <int KT, int NT, int TS>
__global__ void k_scatter_keys(Plan p, int L, LevelIO io, uint32_t max_bins, uint32_t nbmax);
template <int KT, int CAP, int NT, int PAY>
__global__ void k_lds_sort(Plan p, int cls);

}  // namespace pcf
