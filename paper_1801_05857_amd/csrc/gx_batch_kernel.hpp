// Batched exploration: many explorations (instances) in one persistent
// kernel.  Each instance has its own table partition, network image and pair
// of frontier buffers; every instance advances level by level (Sec. 3), but
// instances are not synchronised with each other.
//
// Work queue: an append-only array of level entries {instance, tiles}.  A
// workgroup claims one tile (256 frontier states) of the oldest entry that
// still has unclaimed tiles, expands it (the same per-wavefront routine as
// the single-exploration level kernel) and counts it finished; the workgroup
// that finishes the last tile of a level publishes the instance's next level
// as a new entry (or marks the instance done).  Frontier data written by many
// workgroups is published with agent-scope release fences before the finish
// count and read after agent-scope acquire fences.
//
// Every workgroup leaves the loop when all instances are done, or when its
// own wait for new work exceeds a bounded number of polls (then it raises the
// abort flag, which every other workgroup also obeys), so the kernel always
// drains.
#pragma once

#include <cstdint>

#include "gx_explore_kernel.hpp"

namespace gx {

struct BatchInst {  // per instance, written by the host
  TableDev t;
  uint32_t img_off, img_words;  // network image within the shared image array
  uint32_t* f[2];               // frontier buffers
  uint64_t cap;                 // frontier capacity (states)
  uint64_t* levels;             // level counts (max_levels entries)
  uint32_t max_levels;
  uint32_t pad;
};

struct BatchState {  // per instance, device-updated
  uint64_t ctr[kCtrCount * kCtrSpread];  // counters, one cache line each (ctr_at)
  uint64_t n_in;     // states in the current level
  uint32_t level;    // index of the current level
  uint32_t cur;      // which frontier buffer holds it
  uint32_t done;
  uint32_t pad[27];  // the next instance's counters start on a fresh line
};

static_assert(sizeof(BatchState) % 128 == 0, "instance counters on their own cache lines");

struct BatchEntry {
  uint32_t inst;
  uint32_t tiles;
  uint32_t claimed;
  uint32_t finished;
  uint32_t ready;
  uint32_t pad[3];
};

static_assert(sizeof(BatchEntry) == 32, "queue slots are cleared as 8 words each");

struct BatchGlobal {
  uint32_t head;      // oldest entry that may still have unclaimed tiles
  uint32_t tail;      // entries published or being published
  uint32_t done;      // instances finished
  uint32_t abort;     // set when a wait exceeded its bound or the queue overflowed
  uint64_t dead_used; // deadlock records used
};

struct BatchArgs {
  const BatchInst* inst;
  BatchState* state;
  BatchEntry* queue;
  uint32_t queue_cap;
  BatchGlobal* g;
  uint32_t n;          // instances of this class
  const uint32_t* img; // all network images
  uint32_t img_stride; // LDS words reserved for an image
  uint32_t* dead;      // deadlock records: S words each
  uint32_t* dead_tag;  // instance of each record
  uint64_t dead_cap;
  uint64_t spin_limit; // polls a workgroup may wait for new work
  const uint32_t* init_states;  // n x S initial states
};

enum : uint32_t { kFlagLevelsOverflow = 4, kFlagQueueOverflow = 8 };

__device__ inline uint32_t ld_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Put every instance's initial state into its frontier buffer 0 and insert it
// into its table: one wavefront per instance, lane 0 holds the key.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(64) void batch_init_kernel(BatchArgs a) {
  const uint32_t i = blockIdx.x;
  if (i >= a.n) return;
  const BatchInst& in = a.inst[i];
  uint32_t key[S];
#pragma unroll
  for (int x = 0; x < S; ++x) key[x] = a.init_states[static_cast<uint64_t>(i) * S + x];
  if (__lane_id() == 0) {
#pragma unroll
    for (int x = 0; x < S; ++x) in.f[0][x] = key[x];
  }
  LaneStats st;
  const uint8_t r = find_or_put_lanes<S, B, G, U>(in.t, key, __lane_id() == 0, st);
  if (__lane_id() == 0 && r != kNew) {
    // table not empty of it, or full: the instance fails before its first level
    atomicOr(ctr_at(a.state[i].ctr, kCtrFlags),
             static_cast<unsigned long long>(r == kFull ? kFlagTableFull : kFlagFrontierOverflow));
  }
}

template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void batch_explore_kernel(BatchArgs a) {
  extern __shared__ uint32_t smem[];
  __shared__ uint32_t sh_inst, sh_tile, sh_entry, sh_stop;
  uint32_t* img = smem;
  uint32_t* stage = smem + a.img_stride + (threadIdx.x >> 6) * (kStageWords / 4);
  uint32_t cached = 0xFFFFFFFFu;
  LaneStats st;

  while (true) {
    if (threadIdx.x == 0) {
      uint32_t stop = 0;
      uint64_t polls = 0;
      // Flags and indices are polled with relaxed agent-scope loads; the one
      // acquire is the load of the entry's ready flag, which orders this
      // workgroup after the publisher of the level (and, through its own
      // acquire, after every workgroup that wrote the level's frontier).  An
      // agent-scope acquire costs an L2 invalidate, a release an L2
      // write-back.
      while (true) {
        if (ld_rlx(&a.g->abort)) {
          stop = 1;
          break;
        }
        if (ld_rlx(&a.g->done) >= a.n) {
          stop = 1;
          break;
        }
        const uint32_t h = ld_rlx(&a.g->head);
        const uint32_t tl = ld_rlx(&a.g->tail);
        bool got = false;
        if (h < tl && h < a.queue_cap) {
          BatchEntry* e = &a.queue[h];
          if (ld_acq(&e->ready)) {
            if (e->inst >= a.n || e->tiles == 0) {
              // a published entry is never like this: refuse to index with it
              __hip_atomic_store(&a.g->abort, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
              stop = 1;
              break;
            }
            const uint32_t tile = atomicAdd(&e->claimed, 1u);
            if (tile < e->tiles) {
              sh_inst = e->inst;
              sh_tile = tile;
              sh_entry = h;
              got = true;
            } else {
              atomicCAS(&a.g->head, h, h + 1);  // exhausted: move on
              continue;
            }
          }
        }
        if (got) break;
        if (++polls > a.spin_limit) {
          __hip_atomic_store(&a.g->abort, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          stop = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      sh_stop = stop;
    }
    // the barrier orders every wavefront after thread 0's acquire: the
    // level's frontier and instance state are visible without a fence of
    // their own
    __syncthreads();
    if (sh_stop) break;
    const uint32_t iid = uniform32(sh_inst);
    const uint32_t tile = uniform32(sh_tile);
    const BatchInst& in = a.inst[iid];
    BatchState& bs = a.state[iid];
    if (iid != cached) {
      for (uint32_t k = threadIdx.x; k < in.img_words; k += 256) img[k] = a.img[in.img_off + k];
      cached = iid;
    }
    __syncthreads();
    WaveJob j;
    j.t = uniform_table(in.t);
    j.img = img;
    const uint32_t cur = uniform32(bs.cur);
    j.frontier_in = uniform_ptr(static_cast<const uint32_t*>(in.f[cur]));
    j.first = static_cast<uint64_t>(tile) * 256 + (threadIdx.x & ~63u);
    j.n_in = uniform64(bs.n_in);
    j.frontier_out = uniform_ptr(in.f[cur ^ 1]);
    j.cap_out = uniform64(in.cap);
    j.dead = a.dead;
    j.dead_tag = a.dead_tag;
    j.tag = iid;
    j.dead_cap = a.dead_cap;
    j.dead_ctr = &a.g->dead_used;
    j.ctr = bs.ctr;
    j.dtab = nullptr;
    if (j.first < j.n_in) expand_wave<S, B, G, U>(j, stage, st);
    __syncthreads();
    if (threadIdx.x == 0) {
      // release this tile's frontier writes (an L2 write-back; no
      // invalidate unless this is the level's last tile)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      BatchEntry* e = &a.queue[sh_entry];
      const uint32_t fin = atomicAdd(&e->finished, 1u) + 1u;
      if (fin == e->tiles) {
        // last tile of the level: publish the next level or finish
        __threadfence();
        const uint64_t n_next = __hip_atomic_load(&bs.ctr[kCtrTail * kCtrSpread], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        uint64_t flags = __hip_atomic_load(&bs.ctr[kCtrFlags * kCtrSpread], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        bool finished = flags != 0 || n_next == 0;
        if (!finished) {
          if (bs.level + 1 >= in.max_levels) {
            atomicOr(ctr_at(bs.ctr, kCtrFlags), kFlagLevelsOverflow);
            finished = true;
          } else {
            in.levels[bs.level + 1] = n_next;
            const uint32_t slot = atomicAdd(&a.g->tail, 1u);
            if (slot >= a.queue_cap) {
              atomicOr(ctr_at(bs.ctr, kCtrFlags), kFlagQueueOverflow);
              finished = true;
            } else {
              bs.level += 1;
              bs.cur ^= 1u;
              bs.n_in = n_next;
              bs.ctr[kCtrTail * kCtrSpread] = 0;
              BatchEntry* ne = &a.queue[slot];
              ne->inst = iid;
              ne->tiles = static_cast<uint32_t>((n_next + 255) / 256);
              ne->claimed = 0;
              ne->finished = 0;
              __threadfence();
              __hip_atomic_store(&ne->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
        if (finished) {
          bs.done = 1;
          __threadfence();
          atomicAdd(&a.g->done, 1u);
        }
      }
    }
  }
  // no table statistics: they would keep six counters per lane live across
  // the whole persistent loop (12 more VGPRs, two fewer waves per SIMD)
  (void)st;
}

template <int S, int B, int G, int U>
struct BatchKernels {  // init + persistent launch of one (S, B, G, U) class
  static hipError_t launch(const BatchArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((batch_init_kernel<S, B, G, U>), dim3(a.n), dim3(64), 0, s, a);
    hipLaunchKernelGGL((batch_explore_kernel<S, B, G, U>), dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
  }
  static hipError_t init(const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((batch_init_kernel<S, B, G, U>), dim3(a.n), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  static int resident_per_cu(size_t lds) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_explore_kernel<S, B, G, U>, 256,
                                                     lds) != hipSuccess)
      return 1;
    return b > 0 ? b : 1;
  }
};

}  // namespace gx

namespace gx {

template <int S>
hipError_t batch_launch(uint32_t B, uint32_t G, uint32_t U, const BatchArgs& a, uint32_t grid,
                        size_t lds, hipStream_t s) {
#define GX_BATCH_CASE(BB, GG, UU) \
  if (B == BB && G == GG && U == UU) return BatchKernels<S, BB, GG, UU>::launch(a, grid, lds, s);
#define GX_BATCH_B(BB) GX_BATCH_CASE(BB, 8, 1) GX_BATCH_CASE(BB, 8, 2) GX_BATCH_CASE(BB, 16, 1) GX_BATCH_CASE(BB, 16, 2)
#define GX_BATCH_B4(BB) GX_BATCH_B(BB) GX_BATCH_CASE(BB, 4, 1) GX_BATCH_CASE(BB, 4, 2)
  GX_BATCH_B4(8) GX_BATCH_B4(16) GX_BATCH_B4(32) GX_BATCH_B(64)
#undef GX_BATCH_B4
#undef GX_BATCH_B
#undef GX_BATCH_CASE
  return hipErrorInvalidValue;
}

// The initial states alone (the stepped schedule expands the levels with
// the multi-job step kernel).
template <int S>
hipError_t batch_init(uint32_t B, uint32_t G, uint32_t U, const BatchArgs& a, hipStream_t s) {
#define GX_BATCH_CASE(BB, GG, UU) \
  if (B == BB && G == GG && U == UU) return BatchKernels<S, BB, GG, UU>::init(a, s);
#define GX_BATCH_B(BB) GX_BATCH_CASE(BB, 8, 1) GX_BATCH_CASE(BB, 8, 2) GX_BATCH_CASE(BB, 16, 1) GX_BATCH_CASE(BB, 16, 2)
#define GX_BATCH_B4(BB) GX_BATCH_B(BB) GX_BATCH_CASE(BB, 4, 1) GX_BATCH_CASE(BB, 4, 2)
  GX_BATCH_B4(8) GX_BATCH_B4(16) GX_BATCH_B4(32) GX_BATCH_B(64)
#undef GX_BATCH_B4
#undef GX_BATCH_B
#undef GX_BATCH_CASE
  return hipErrorInvalidValue;
}

template <int S>
int batch_resident(uint32_t B, uint32_t G, uint32_t U, size_t lds) {
#define GX_BATCH_CASE(BB, GG, UU) \
  if (B == BB && G == GG && U == UU) return BatchKernels<S, BB, GG, UU>::resident_per_cu(lds);
#define GX_BATCH_B(BB) GX_BATCH_CASE(BB, 8, 1) GX_BATCH_CASE(BB, 8, 2) GX_BATCH_CASE(BB, 16, 1) GX_BATCH_CASE(BB, 16, 2)
#define GX_BATCH_B4(BB) GX_BATCH_B(BB) GX_BATCH_CASE(BB, 4, 1) GX_BATCH_CASE(BB, 4, 2)
  GX_BATCH_B4(8) GX_BATCH_B4(16) GX_BATCH_B4(32) GX_BATCH_B(64)
#undef GX_BATCH_B4
#undef GX_BATCH_B
#undef GX_BATCH_CASE
  return 1;
}

}  // namespace gx
