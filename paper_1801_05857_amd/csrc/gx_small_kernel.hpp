// Small BFS levels expanded on one workgroup, level after level, with no host
// round trip between them: the device-side level loop of gx_explore for the
// levels too small to fill the device (Sec. 5.2 traces the low rate on small
// instances to small search layers and per-layer overhead).
#pragma once

#include <algorithm>
#include <cstdint>

#include "gx_explore_kernel.hpp"

namespace gx {

constexpr uint32_t kSmallThreads = 512;  // one workgroup of 8 wavefronts
constexpr uint32_t kSmallWaves = kSmallThreads / 64;
constexpr uint32_t kSmallLevels = 64;     // levels one launch may complete
constexpr uint64_t kSmallMaxLevel = 4096; // largest level the workgroup expands
constexpr uint64_t kSmallSuccBudget = 4096;  // and at most this many successors (worst case)

// What a launch leaves for the host (read back with the level counters).
struct SmallOut {
  uint64_t n_levels;     // levels completed by this launch; their sizes follow
  uint64_t n_in;         // size of the current level (0: the exploration is over)
  uint64_t cur;          // the frontier buffer holding it
  uint64_t init_status;  // find-or-put status of the initial state (when inserted)
  uint64_t log_n;        // LDS-resident launch: states it logged (they go into the table)
  uint64_t pad[3];
  uint64_t levels[kSmallLevels];
};

struct SmallArgs {
  TableDev t;
  const uint32_t* img;  // network image (global; copied to LDS)
  uint32_t img_words;
  uint32_t img_stride;
  uint32_t* f[2];       // the two frontier buffers
  uint64_t f_cap;       // states each holds
  uint32_t cur;         // buffer holding the current level
  uint64_t n_in;        // its size
  uint32_t* succ;       // a level's successors, S words each
  uint64_t succ_cap;
  uint32_t* dead;
  uint64_t dead_cap;
  uint64_t* ctr;        // the exploration's counters (see ctr_at)
  SmallOut* out;
  uint64_t limit;       // largest level this launch expands (limit * max_succ fits)
  const uint32_t* init_key;  // non-null: find-or-put it first (the level-0 state)
  // LDS-resident levels (lds_levels_kernel) only:
  uint32_t set_mask;    // entries of the LDS visited set, minus one (a power of two)
  uint32_t max_succ;    // successors a state can have at most
};

// A table that held states the launch did not put there (reported as
// GX_EINVAL: gx_explore needs an empty table).
constexpr uint32_t kFlagNotEmpty = 16;

// Every level: (1) the workgroup numbers the level's successors state by
// state (block prefix sum of the per-state counts) and writes them to the
// successor buffer with the coalesced lockstep walk of emit_window; (2) all
// eight wavefronts find-or-put those successors and append the NEW ones to
// the next frontier, one atomic add per wavefront and round; (3) thread 0 reads the level's size and decides: next level,
// done, or back to the host (a level above the limit, a full table, the
// deadlock buffer short of a level, or kSmallLevels levels done).  Probes use
// the table's bucket size with (G, U) of this kernel: the claim protocol does
// not depend on how many lanes read a bucket, and a workgroup on its own
// needs every lane's key in flight to hide the probe latency.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(kSmallThreads) void small_levels_kernel(SmallArgs a) {
  extern __shared__ uint32_t smem[];
  __shared__ uint32_t wave_tot[kSmallWaves];
  __shared__ uint64_t sh_n_in;
  __shared__ uint32_t sh_cur, sh_go, sh_levels;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid >> 6;
  const int lane = __lane_id();
  uint32_t* img = smem;
  for (uint32_t k = tid; k < a.img_words; k += kSmallThreads) img[k] = a.img[k];
  if (tid == 0) {
    const uint64_t dead = __hip_atomic_load(ctr_at(a.ctr, kCtrDead), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    sh_n_in = a.n_in;
    sh_cur = a.cur;
    sh_go = a.n_in > 0 && a.n_in <= a.limit && a.n_in <= a.dead_cap - min(dead, a.dead_cap)
                ? 1u
                : 0u;
    sh_levels = 0;
    // a level completed by the host path leaves its size in the tail
    __hip_atomic_store(ctr_at(a.ctr, kCtrTail), 0ull, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  LaneStats st;
  if (a.init_key != nullptr && wave == 0) {
    uint32_t key[S];
#pragma unroll
    for (int x = 0; x < S; ++x) key[x] = lane == 0 ? a.init_key[x] : 0u;
    const uint8_t r = find_or_put_lanes<S, B, G, U>(a.t, key, lane == 0, st);
    if (lane == 0) {
      a.out->init_status = r;
      if (r != kNew) sh_go = 0;
    }
  }
  while (true) {
    __syncthreads();
    if (!sh_go) break;
    const uint64_t n_in = sh_n_in;
    const uint32_t cur = sh_cur;
    const uint32_t* fin = a.f[cur];
    uint32_t* fout = a.f[cur ^ 1u];

    // (1) successors of the level, numbered state by state
    uint64_t n_succ = 0;
    for (uint64_t r0 = 0; r0 < n_in; r0 += kSmallThreads) {
      const uint64_t i = r0 + tid;
      const bool has = i < n_in;
      uint32_t sw[S];
#pragma unroll
      for (int x = 0; x < S; ++x) sw[x] = 0;
      if (has) load_slot<S>(fin + i * S, sw);
      const uint32_t c = has ? count_successors<S>(img, sw) : 0u;
      if (has && c == 0) {
        const uint64_t d = atomicAdd(ctr_at(a.ctr, kCtrDead), 1ull);
        if (d < a.dead_cap) store_slot<S>(a.dead + d * S, sw);
      }
      uint32_t wt = 0;
      (void)wave_exclusive_scan(c, &wt);
      if (lane == 0) wave_tot[wave] = wt;
      __syncthreads();
      uint64_t wb = n_succ, round = 0;
      for (uint32_t w = 0; w < kSmallWaves; ++w) {
        wb += w < wave ? wave_tot[w] : 0u;
        round += wave_tot[w];
      }
      // limit * max_succ <= succ_cap (host bound); refuse rather than overrun
      if (n_succ + round <= a.succ_cap) {
        if (wt) emit_window<S, false>(img, sw, has, a.succ + wb * S, 0, wt);
      } else if (tid == 0) {
        atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagFrontierOverflow);
      }
      n_succ += round;
      __syncthreads();  // wave_tot is rewritten by the next round
    }
    if (n_succ > a.succ_cap) n_succ = 0;
    if (tid == 0 && n_succ) atomicAdd(ctr_at(a.ctr, kCtrTrans), static_cast<unsigned long long>(n_succ));
    __syncthreads();  // the successors are visible to every wavefront

    // (2) find-or-put of the successors; the NEW ones of a round go to the
    // next frontier with one atomic add per wavefront (levels are small, so
    // rounds are few)
    bool full = false, over = false;
    for (uint64_t k0 = static_cast<uint64_t>(wave) * 64; k0 < n_succ; k0 += kSmallThreads) {
      const uint64_t idx = k0 + lane;
      const bool act = idx < n_succ;
      uint32_t key[S];
#pragma unroll
      for (int x = 0; x < S; ++x) key[x] = 0;
      if (act) load_slot<S>(a.succ + idx * S, key);
      const uint8_t r = find_or_put_lanes<S, B, G, U>(a.t, key, act, st);
      const bool is_new = act && r == kNew;
      full |= act && r == kFull;
      const uint64_t m = __ballot(is_new);
      if (m) {
        unsigned long long base = 0;
        if (lane == 0)
          base = atomicAdd(ctr_at(a.ctr, kCtrTail), static_cast<unsigned long long>(__popcll(m)));
        base = __shfl(base, 0, 64);
        const uint64_t pos = base + __popcll(m & ((1ull << lane) - 1ull));
        if (is_new && pos < a.f_cap) store_slot<S>(fout + pos * S, key);
        over |= is_new && pos >= a.f_cap;
      }
    }
    if (__ballot(full) && lane == 0) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagTableFull);
    if (__ballot(over) && lane == 0) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagFrontierOverflow);
    __syncthreads();  // every append of the level is done

    // (3) the level's size and what comes next
    if (tid == 0) {
      auto* tail = ctr_at(a.ctr, kCtrTail);
      const uint64_t n_next =
          __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t flags = __hip_atomic_load(ctr_at(a.ctr, kCtrFlags), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t dead = __hip_atomic_load(ctr_at(a.ctr, kCtrDead), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(tail, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (n_next) a.out->levels[sh_levels++] = n_next;
      sh_n_in = n_next;
      sh_cur = cur ^ 1u;
      sh_go = flags == 0 && n_next > 0 && n_next <= a.limit && sh_levels < kSmallLevels &&
                      n_next <= a.dead_cap - min(dead, a.dead_cap)
                  ? 1u
                  : 0u;
    }
  }
  if (tid == 0) {
    a.out->n_levels = sh_levels;
    a.out->n_in = sh_n_in;
    a.out->cur = sh_cur;
  }
  flush_stats(a.t, st, nullptr);
}


// ------------------------------------------------ LDS-resident first levels
template <int S>
constexpr uint32_t lds_chunk() {  // staged successors per wavefront chunk (2 KiB)
  return 512u / S;
}
constexpr uint32_t kLocked = 0xFFFFFFFEu;  // an LDS set entry being written (packed
                                           // states never hold it: bit 31 is 0)

// Insert-if-absent of key into the workgroup's LDS set (open addressing,
// linear probing, set_mask + 1 entries of S words); true where this lane put
// it there.  A multi-word entry is claimed by a compare-and-swap of its first
// word to kLocked and published by writing the first word last; a lane that
// meets a locked entry looks at it again in the next step (its owner
// publishes within the step that claimed it).  Must be reached by the whole
// wavefront; act false: no key.
template <int S>
__device__ inline bool lds_set_insert(uint32_t* set, uint32_t mask, const uint32_t (&key)[S],
                                      bool act) {
  bool done = !act, fresh = false;
  uint32_t h = dedup_hash<S>(key) & mask;
  while (__ballot(!done)) {
    if (!done) {
      uint32_t* e = set + h * S;
      const uint32_t w0 = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (w0 == kEmpty) {
        uint32_t expect = kEmpty;
        if (__hip_atomic_compare_exchange_strong(e, &expect, S == 1 ? key[0] : kLocked,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP)) {
          if constexpr (S > 1) {
#pragma unroll
            for (int x = 1; x < S; ++x)
              __hip_atomic_store(e + x, key[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(e, key[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
          fresh = true;
          done = true;
        }
      } else if (w0 != kLocked) {
        bool same = w0 == key[0];
        if constexpr (S > 1) {
          if (same) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
            for (int x = 1; x < S; ++x)
              same &= __hip_atomic_load(e + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ==
                      key[x];
          }
        }
        if (same)
          done = true;
        else
          h = (h + 1) & mask;
      }
    }
  }
  return fresh;
}

// The logged states into the table, by the workgroup that logged them, with
// no device-scope claim: the table held none of them and nothing else (the
// premise of an LDS-resident launch) and they are distinct (the visited set
// decided that), so each takes the next slot of the first bucket of its hash
// sequence that still has one, counted in LDS (fill, one word per bucket),
// and is written with a plain store.  That is the layout find-or-put builds:
// a bucket fills from its lowest slot, and a state lies in its j-th bucket
// only when buckets 1..j-1 of its sequence are full.  (Claimed one by one,
// the states of a small fresh table queue at a few memory channels: 29 us
// for 4096 of them.)  No slot left in any of the H buckets: FULL.  Log entry
// 0 is the initial state; its outcome goes to out->init_status.  Must be
// reached by the whole workgroup.
template <int S, int B>
__device__ inline void place_log(const SmallArgs& a, uint32_t* fill, const uint32_t* log,
                                 uint32_t log_n) {
  constexpr uint32_t kSlots = B / S;
  const uint32_t tid = threadIdx.x;
  const uint32_t nb = static_cast<uint32_t>(a.t.n_buckets);
  for (uint32_t k = tid; k < nb; k += kSmallThreads) fill[k] = 0;
  __syncthreads();
  LaneStats st;
  uint32_t stored = 0, lookups = 0, full = 0;
  for (uint32_t i = tid; i < log_n; i += kSmallThreads) {
    uint32_t key[S];
    load_slot<S>(log + static_cast<uint64_t>(i) * S, key);
    const uint64_t mix = key_mix<S>(key, a.t.seed);
    bool done = false;
    uint32_t j = 0;
    for (; j < a.t.H && !done; ++j) {
      const uint64_t ca = j == 0 ? a.t.a0 : a.t.hc[2 * j];
      const uint64_t cc = j == 0 ? a.t.c0 : a.t.hc[2 * j + 1];
      const uint64_t b = bucket_of(mix, ca, cc, a.t.n_buckets);
      const uint32_t slot = atomicAdd(&fill[b], 1u);
      ++st.probes;
      if (slot < kSlots) {
        store_slot<S>(a.t.words + b * B + slot * S, key);
        done = true;
        if (j > st.max_j) st.max_j = j;
      }
    }
    ++lookups;
    if (done) ++stored;
    else ++full;
    if (i == 0) a.out->init_status = done ? kNew : kFull;
  }
  st.stored = wave_sum(stored);
  st.lookups = wave_sum(lookups);
  st.full = wave_sum(full);
  if (st.full && __lane_id() == 0) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagTableFull);
  flush_stats(a.t, st, nullptr);
}

// The first levels of an exploration, while the table holds nothing but what
// this launch puts there: an LDS set of every state reached so far decides
// NEW or SEEN exactly, with no table probe.  New states are appended to a log
// in global memory (the successor buffer), level after level, so a level is
// a contiguous range of the log.  A level is expanded only while the set
// stays at most three quarters full even if every successor were new.  When
// the levels end (the exploration is complete, a level would not fit, or
// kSmallLevels levels are done) the current level is copied to frontier
// buffer 0 for the host, and every logged state goes into the table: placed
// by this workgroup when the table's per-bucket fill counts fit in the LDS
// the visited set used (see place_log), else by log_insert_kernel, launched
// after it.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(kSmallThreads) void lds_levels_kernel(SmallArgs a) {
  extern __shared__ uint32_t smem[];
  constexpr uint32_t kChunk = lds_chunk<S>();
  __shared__ uint32_t sh_go, sh_levels, sh_log_n, sh_ls, sh_le, sh_dead;
  __shared__ unsigned long long sh_trans, sh_dead0;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid >> 6;
  const int lane = __lane_id();
  uint32_t* img = smem;
  uint32_t* set = smem + a.img_stride;
  const uint32_t n_set = a.set_mask + 1;
  uint32_t* stage = set + n_set * S + wave * kChunk * S;
  uint32_t* log = a.succ;
  const uint64_t set_cap = static_cast<uint64_t>(n_set) / 4 * 3;
  // a wavefront's 64 states have at most 64 * max_succ successors
  const bool one_chunk = static_cast<uint64_t>(a.max_succ) * 64 <= kChunk;
  for (uint32_t k = tid; k < a.img_words; k += kSmallThreads) img[k] = a.img[k];
  for (uint32_t k = tid; k < n_set * S; k += kSmallThreads) set[k] = kEmpty;
  __syncthreads();
  if (wave == 0) {
    uint32_t key[S];
#pragma unroll
    for (int x = 0; x < S; ++x) key[x] = a.init_key[x];
    (void)lds_set_insert<S>(set, a.set_mask, key, lane == 0);
    if (lane == 0) {
      store_slot<S>(log, key);
      sh_log_n = 1;
      sh_ls = 0;
      sh_le = 1;
      sh_levels = 0;
      sh_trans = 0;
      sh_dead = 0;
      sh_dead0 = __hip_atomic_load(ctr_at(a.ctr, kCtrDead), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
      sh_go = a.limit >= 1 && 1 + static_cast<uint64_t>(a.max_succ) <= min(set_cap, a.succ_cap)
                  ? 1u
                  : 0u;
    }
  }
  while (true) {
    __syncthreads();
    if (!sh_go) break;
    const uint32_t ls = sh_ls, n_in = sh_le - sh_ls;
    for (uint32_t g0 = wave * 64; g0 < n_in; g0 += kSmallThreads) {
      const uint32_t i = g0 + lane;
      const bool has = i < n_in;
      uint32_t sw[S];
#pragma unroll
      for (int x = 0; x < S; ++x) sw[x] = 0;
      if (has) load_slot<S>(log + static_cast<uint64_t>(ls + i) * S, sw);
      uint32_t total = 0;
      bool staged = false;  // the wavefront's successors are in its stage already
      if (one_chunk) {
        // every state's successors fit one chunk: emitted at once, counted
        // on the way (this lane's for the deadlock test)
        uint32_t c = 0;
        emit_window<S, false, 1>(img, sw, has, stage, 0, kChunk, &total, &c);
        if (has && c == 0) {
          const uint64_t d = atomicAdd(ctr_at(a.ctr, kCtrDead), 1ull);
          if (d < a.dead_cap) store_slot<S>(a.dead + d * S, sw);
          atomicAdd(&sh_dead, 1u);
        }
        staged = true;
      } else {
        const uint32_t c = has ? count_successors<S>(img, sw) : 0u;
        if (has && c == 0) {
          const uint64_t d = atomicAdd(ctr_at(a.ctr, kCtrDead), 1ull);
          if (d < a.dead_cap) store_slot<S>(a.dead + d * S, sw);
          atomicAdd(&sh_dead, 1u);
        }
        (void)wave_exclusive_scan(c, &total);
      }
      if (lane == 0 && total) atomicAdd(&sh_trans, static_cast<unsigned long long>(total));
      for (uint32_t lo = 0; lo < total; lo += kChunk) {
        const uint32_t hi = min(total, lo + kChunk);
        // (a wavefront whose successors fit one chunk walks them without the
        // window's per-run wavefront sums)
        if (!staged) {
          if (lo == 0 && hi == total)
            emit_window<S, false>(img, sw, has, stage, 0, total);
          else
            emit_window<S, true>(img, sw, has, stage, lo, hi);
        }
        wave_lds_sync();
        // NEW states of the chunk are compacted in place at the front of the
        // stage (each round reads its keys before any is rewritten), then
        // logged with one reservation
        uint32_t n_new = 0;
        for (uint32_t r0 = 0; r0 < hi - lo; r0 += 64) {
          const uint32_t idx = r0 + lane;
          const bool act = idx < hi - lo;
          uint32_t key[S];
#pragma unroll
          for (int x = 0; x < S; ++x) key[x] = act ? stage[idx * S + x] : 0u;
          const bool fresh = lds_set_insert<S>(set, a.set_mask, key, act);
          const uint64_t m = __ballot(fresh);
          wave_lds_sync();  // every lane's key of this round is read before any write
          if (fresh) {
            const uint32_t pos = n_new + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
#pragma unroll
            for (int x = 0; x < S; ++x) stage[pos * S + x] = key[x];
          }
          n_new += static_cast<uint32_t>(__popcll(m));
        }
        wave_lds_sync();
        if (n_new) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&sh_log_n, n_new);
          base = __shfl(base, 0, 64);
          for (uint32_t k = lane; k < n_new * S; k += 64)
            log[static_cast<uint64_t>(base) * S + k] = stage[k];
        }
        wave_lds_sync();  // the stage is rewritten by the next chunk
      }
    }
    __syncthreads();  // the level's new states are logged
    if (tid == 0) {
      const uint32_t le = sh_le, log_n = sh_log_n, n_next = log_n - le;
      const uint64_t dead = sh_dead0 + sh_dead;
      if (n_next) a.out->levels[sh_levels++] = n_next;
      sh_ls = le;
      sh_le = log_n;
      const uint64_t worst = log_n + static_cast<uint64_t>(n_next) * a.max_succ;
      // (n_next <= limit: the level after it fits the frontier buffer, which
      // receives the current level when the launch ends)
      sh_go = n_next > 0 && n_next <= a.limit && sh_levels < kSmallLevels &&
                      worst <= min(set_cap, a.succ_cap) &&
                      n_next <= a.dead_cap - min(dead, a.dead_cap)
                  ? 1u
                  : 0u;
    }
  }
  __syncthreads();
  // the current level becomes frontier buffer 0 (when the levels go on)
  const uint32_t ls = sh_ls, n_cur = sh_le - sh_ls, log_n = sh_log_n;
  for (uint32_t k = tid; k < n_cur * S; k += kSmallThreads)
    a.f[0][k] = log[static_cast<uint64_t>(ls) * S + k];
  // the visited set is done with: its LDS holds the bucket fill counts
  const bool placed = a.t.n_buckets <= static_cast<uint64_t>(n_set) * S;
  if (placed) place_log<S, B>(a, set, log, log_n);
  if (tid == 0) {
    a.out->n_levels = sh_levels;
    a.out->n_in = n_cur;  // 0: the last level expanded found nothing new
    a.out->cur = 0;
    a.out->log_n = placed ? 0 : log_n;  // states left for log_insert_kernel
    if (sh_trans) atomicAdd(ctr_at(a.ctr, kCtrTrans), sh_trans);
  }
}

// The states an LDS-resident launch logged go into the table, spread over
// the device (launched right after it on the same stream).  They are
// distinct and the table held none of them (it was empty when the
// exploration started), so each must come back NEW: FULL raises the
// table-full flag, anything else kFlagNotEmpty.  The initial state (log
// entry 0) reports its status in out->init_status.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void log_insert_kernel(TableDev t, const uint32_t* log,
                                                         SmallOut* out, uint64_t* ctr) {
  const uint64_t n = out->log_n;
  const int lane = __lane_id();
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  LaneStats st;
  bool full = false, seen = false;
  for (uint64_t base = wave * 64; base < n; base += n_waves * 64) {
    const uint64_t idx = base + lane;
    const bool act = idx < n;
    uint32_t key[S];
#pragma unroll
    for (int x = 0; x < S; ++x) key[x] = 0;
    if (act) load_slot<S>(log + idx * S, key);
    const uint8_t r = find_or_put_lanes<S, B, G, U>(t, key, act, st);
    full |= act && r == kFull;
    seen |= act && r != kNew && r != kFull;
    if (idx == 0) out->init_status = r;
  }
  if (__ballot(full) && lane == 0) atomicOr(ctr_at(ctr, kCtrFlags), kFlagTableFull);
  if (__ballot(seen) && lane == 0) atomicOr(ctr_at(ctr, kCtrFlags), kFlagNotEmpty);
  flush_stats(t, st, nullptr);
}

template <int S, int B>
hipError_t launch_small_b(const SmallArgs& a, size_t lds, hipStream_t s) {
  constexpr int G = B <= 32 ? 4 : 8;
  constexpr int U = 4;
  const void* k = reinterpret_cast<const void*>(&small_levels_kernel<S, B, G, U>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((small_levels_kernel<S, B, G, U>), dim3(1), dim3(kSmallThreads), lds, s, a);
  return hipGetLastError();
}

// LDS bytes of an LDS-resident launch with 2^set_bits set entries.
template <int S>
size_t lds_levels_bytes(uint32_t img_stride, uint32_t set_bits) {
  return (static_cast<size_t>(img_stride) + (size_t(S) << set_bits) +
          kSmallWaves * lds_chunk<S>() * S) * sizeof(uint32_t);
}

template <int S, int B>
hipError_t launch_lds_b(const SmallArgs& a, size_t lds, hipStream_t s) {
  constexpr int G = B <= 32 ? 4 : 8;
  constexpr int U = 4;
  const void* k = reinterpret_cast<const void*>(&lds_levels_kernel<S, B, G, U>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((lds_levels_kernel<S, B, G, U>), dim3(1), dim3(kSmallThreads), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the launch places its log itself when the table's fill counts fit the
  // set's LDS (the test place_log's caller makes)
  if (a.t.n_buckets <= (static_cast<uint64_t>(a.set_mask) + 1) * S) return hipSuccess;
  // else the logged states (at most three quarters of the set) into the table
  const uint32_t grid = static_cast<uint32_t>(
      std::min<uint64_t>(256, (static_cast<uint64_t>(a.set_mask) + 1) / 256 + 1));
  hipLaunchKernelGGL((log_insert_kernel<S, B, G, U>), dim3(grid), dim3(256), 0, s, a.t, a.succ,
                     a.out, a.ctr);
  return hipGetLastError();
}

// Launch the LDS-resident first levels with the largest visited set that fits
// lds_limit bytes of LDS, then the insertion of the states they logged;
// returns hipErrorInvalidValue (nothing launched) when not even 2^10 entries
// fit.
template <int S>
hipError_t launch_lds_levels(uint32_t B, SmallArgs a, size_t lds_limit, hipStream_t s) {
  uint32_t bits = 20;
  while (bits >= 10 && lds_levels_bytes<S>(a.img_stride, bits) > lds_limit) --bits;
  if (bits < 10) return hipErrorInvalidValue;
  a.set_mask = (1u << bits) - 1u;
  const size_t lds = lds_levels_bytes<S>(a.img_stride, bits);
  switch (B) {
    case 4: return launch_lds_b<S, 4>(a, lds, s);
    case 8: return launch_lds_b<S, 8>(a, lds, s);
    case 16: return launch_lds_b<S, 16>(a, lds, s);
    case 32: return launch_lds_b<S, 32>(a, lds, s);
    case 64: return launch_lds_b<S, 64>(a, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int S>
hipError_t launch_small(uint32_t B, const SmallArgs& a, hipStream_t s) {
  const size_t lds = static_cast<size_t>(a.img_stride) * sizeof(uint32_t);  // the image
  switch (B) {
    case 4: return launch_small_b<S, 4>(a, lds, s);
    case 8: return launch_small_b<S, 8>(a, lds, s);
    case 16: return launch_small_b<S, 16>(a, lds, s);
    case 32: return launch_small_b<S, 32>(a, lds, s);
    case 64: return launch_small_b<S, 64>(a, lds, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gx
