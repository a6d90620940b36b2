// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/gx.h"
#include "gx_device.hpp"

// Device buffers of the exploration driver, owned by a table and reused by
// every exploration into it (grow-only).
struct gx_explore_buffers {
  uint32_t* img = nullptr;  // network image (in the control block, see ctr)
  uint64_t img_cap = 0;     // words
  uint32_t* img_global = nullptr;  // an image too large for LDS (own allocation)
  uint64_t img_global_cap = 0;     // words
  uint32_t* f[2] = {nullptr, nullptr};
  uint64_t f_cap[2] = {0, 0};  // states
  uint32_t* dead = nullptr;
  uint64_t dead_cap = 0;  // states
  uint32_t* succ = nullptr;  // successors of a level slice, before the table probe
  uint64_t succ_cap = 0;     // states
  // control block (device) and its pinned host mirror: the level counters
  // (one cache line each) and what a small-level launch reports, then the
  // initial state's slot and the network image; one copy up per exploration,
  // the counters' part read back after every level
  uint64_t* ctr = nullptr;
  uint64_t* ctr_host = nullptr;
  uint8_t* status = nullptr;
  uint32_t* key = nullptr;  // the initial state, 4 words (in the control block)
  // safety monitor: bad-state bitmask, violating states, their running count
  uint32_t* mon = nullptr;
  uint64_t mon_cap = 0;      // words
  uint32_t* viol = nullptr;
  uint64_t viol_cap = 0;     // states
  uint64_t* viol_ctr = nullptr;
};

struct gx_table {
  int device = 0;
  uint32_t w = 0;  // words per state
  uint32_t S = 0;  // slot words
  uint32_t B = 0;  // bucket words
  uint32_t G = 0;  // subgroup width
  uint32_t U = 1;  // keys in flight per subgroup
  uint32_t H = 8;  // hash functions
  uint64_t seed = 0;
  uint64_t n_buckets = 0;
  uint32_t* words = nullptr;     // n_buckets * B
  uint64_t* hc = nullptr;        // 2*H hash constants
  uint64_t* counters = nullptr;  // ctr_slots sets of gx::kNumCounters
  uint32_t ctr_slots = 1;
  uint64_t a0 = 0, c0 = 0;
  // something was inserted since creation or the last clear: gx_explore, whose
  // first levels place states assuming an empty table, refuses the table
  bool holds_states = false;
  gx_explore_buffers eb;

  gx::TableDev dev() const {
    gx::TableDev t;
    t.words = words;
    t.n_buckets = n_buckets;
    t.hc = hc;
    t.seed = seed;
    t.a0 = a0;
    t.c0 = c0;
    t.H = H;
    t.counters = counters;
    t.ctr_slots = ctr_slots;
    return t;
  }
};

namespace gx {

inline uint32_t slot_words(uint32_t w) { return w == 3 ? 4u : w; }

// A 4-lane subgroup holds at most 8 words of a bucket per lane, so it pairs
// with buckets of up to 32 words.  An autotuned value gives way to an
// explicit one: an explicit 4-lane subgroup caps an autotuned bucket at 32
// words, an explicit 64-word bucket turns an autotuned 4-lane subgroup into 8.
inline void fit_subgroup(uint32_t* B, uint32_t* G, bool B_given) {
  if (*G == 4 && *B > 32) {
    if (B_given) *G = 8;
    else *B = 32;
  }
}

struct FopArgs {
  TableDev t;
  const uint32_t* keys;
  uint32_t w;
  uint64_t n;
  uint8_t* status;
  uint64_t* n_new;
  uint32_t cus;  // compute units of the device
  hipStream_t stream;
};

// Find-or-put dispatch over (B, G, U) for slot width S (one translation unit
// per S).
template <int S>
hipError_t dispatch_b(uint32_t B, uint32_t G, uint32_t U, const FopArgs& a);
extern template hipError_t dispatch_b<1>(uint32_t, uint32_t, uint32_t, const FopArgs&);
extern template hipError_t dispatch_b<2>(uint32_t, uint32_t, uint32_t, const FopArgs&);
extern template hipError_t dispatch_b<4>(uint32_t, uint32_t, uint32_t, const FopArgs&);

// Launch the find-or-put kernel specialised for the table's (S, B, G, U).
hipError_t launch_find_or_put(const gx_table* t, const uint32_t* keys, uint64_t n,
                              uint8_t* status, uint64_t* n_new, hipStream_t stream);

// Fill n_words (a multiple of 4, 16-byte aligned) with value, stream-ordered
// (a kernel, never a memset node, so it may be captured in a graph).
hipError_t fill_words(uint32_t* p, uint64_t n_words, uint32_t value, int device,
                      hipStream_t stream);

// The keys stored in total_words words of bucket storage (slots of S words,
// keys of w words) on the device, sorted lexicographically, w words each.
// Waits for all device work.  *n_out receives the number of keys.
gx_status sorted_keys(const uint32_t* dev_words, uint64_t total_words, uint32_t S, uint32_t w,
                      std::vector<uint32_t>* out, uint64_t* n_out);
// The same into a malloc'd array (for gx_explore_result.states).
gx_status sorted_keys_malloc(const uint32_t* dev_words, uint64_t total_words, uint32_t S,
                             uint32_t w, uint32_t** out);

// LDS bytes one workgroup may use on the device (queried once per device).
size_t lds_per_workgroup(int device);

// Number of workgroups that keep every CU busy for a grid-stride kernel.
uint32_t resident_grid(int device, uint32_t per_cu);

}  // namespace gx
