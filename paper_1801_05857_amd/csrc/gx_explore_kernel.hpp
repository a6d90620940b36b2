// Exploration level kernel and its (B, G, U) dispatch for one slot width S;
// each slot width is instantiated in a translation unit of its own.
#pragma once

#include <cstdint>

#include "gx_internal.hpp"

namespace gx {

constexpr uint32_t kImgMaxWords = 11776;  // 46 KiB of LDS for the network image
constexpr uint32_t kStageWords = 4096;    // 16 KiB of LDS for staged successors

// ------------------------------------------------------------------ kernel
struct ExploreArgs {
  TableDev t;
  const uint32_t* img;
  uint32_t img_words;
  uint32_t img_stride;  // img_words rounded up to 4
  const uint32_t* frontier_in;
  uint64_t n_in;
  uint32_t* frontier_out;
  uint64_t cap_out;
  uint32_t* dead;
  uint64_t dead_cap;
  uint64_t* ctr;  // [0] next-frontier tail [1] deadlocks [2] transitions [3] flags [4] local duplicates
  uint32_t dedup; // nonzero: drop duplicates within each staged chunk before probing
};

enum : uint32_t { kFlagFrontierOverflow = 1, kFlagTableFull = 2 };

// Per-wavefront LDS hash set of the local duplicate filter: twice as many
// entries as a chunk holds successors, so it is never more than half full.
template <int S>
__host__ __device__ constexpr uint32_t dedup_entries() {
  return 2u * (kStageWords / 4u / S);
}

// Field access with mask arithmetic only: a select chain over the words is
// folded by the compiler into an indexed load from a private array, which
// would live in scratch memory.
template <int S>
__device__ __forceinline__ uint32_t get_field(const uint32_t (&sw)[S], uint32_t f) {
  const uint32_t word = f & 0xFF, shift = (f >> 8) & 0xFF, width = f >> 16;
  uint32_t x = 0;
#pragma unroll
  for (int t = 0; t < S; ++t) x |= sw[t] & (0u - static_cast<uint32_t>(word == static_cast<uint32_t>(t)));
  return (x >> shift) & ((1u << width) - 1u);
}

template <int S>
__device__ __forceinline__ void set_field(uint32_t (&sw)[S], uint32_t f, uint32_t v) {
  const uint32_t word = f & 0xFF, shift = (f >> 8) & 0xFF, width = f >> 16;
  const uint32_t m = ((1u << width) - 1u) << shift;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const uint32_t sel = 0u - static_cast<uint32_t>(word == static_cast<uint32_t>(t));
    sw[t] = (sw[t] & ~(m & sel)) | ((v << shift) & sel);
  }
}

template <int S>
__device__ __forceinline__ uint32_t count_successors(const uint32_t* img, const uint32_t (&sw)[S]) {
  const uint32_t P = img[0], R = img[1];
  uint32_t c = 0;
  for (uint32_t p = 0; p < P; ++p) {
    const uint32_t l = get_field<S>(sw, img[4 + p]);
    const uint32_t ob = img[4 + P + p];
    c += img[ob + l + 1] - img[ob + l];
  }
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t rb = img[4 + 2 * P + r];
    const uint32_t np = img[rb];
    uint32_t prod = 1;
    for (uint32_t i = 0; i < np && prod; ++i) {
      const uint32_t q = img[rb + 1 + 2 * i], ob = img[rb + 2 + 2 * i];
      const uint32_t l = get_field<S>(sw, img[4 + q]);
      prod *= img[ob + l + 1] - img[ob + l];
    }
    c += prod;
  }
  return c;
}

// Write successors with ordinals in [lo, hi) of this state to stage[(k-lo)*S].
template <int S>
__device__ __forceinline__ void emit_successors(const uint32_t* img, const uint32_t (&sw)[S], int lo,
                                       int hi, uint32_t* stage) {
  const uint32_t P = img[0], R = img[1];
  int k = 0;
  for (uint32_t p = 0; p < P; ++p) {
    const uint32_t f = img[4 + p];
    const uint32_t l = get_field<S>(sw, f);
    const uint32_t ob = img[4 + P + p];
    const uint32_t s0 = img[ob + l], s1 = img[ob + l + 1];
    const int n = static_cast<int>(s1 - s0);
    if (k + n <= lo) {
      k += n;
      continue;
    }
    for (uint32_t t = s0; t < s1; ++t, ++k) {
      if (k >= hi) return;
      if (k >= lo) {
        uint32_t succ[S];
#pragma unroll
        for (int x = 0; x < S; ++x) succ[x] = sw[x];
        set_field<S>(succ, f, img[t]);
#pragma unroll
        for (int x = 0; x < S; ++x) stage[(k - lo) * S + x] = succ[x];
      }
    }
  }
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t rb = img[4 + 2 * P + r];
    const uint32_t np = img[rb];
    uint32_t prod = 1;
    for (uint32_t i = 0; i < np && prod; ++i) {
      const uint32_t q = img[rb + 1 + 2 * i], ob = img[rb + 2 + 2 * i];
      const uint32_t l = get_field<S>(sw, img[4 + q]);
      prod *= img[ob + l + 1] - img[ob + l];
    }
    const int n = static_cast<int>(prod);
    if (k + n <= lo) {
      k += n;
      continue;
    }
    for (uint32_t c = 0; c < prod; ++c, ++k) {
      if (k >= hi) return;
      if (k >= lo) {
        uint32_t succ[S];
#pragma unroll
        for (int x = 0; x < S; ++x) succ[x] = sw[x];
        uint32_t rem = c;
        for (uint32_t i = 0; i < np; ++i) {
          const uint32_t q = img[rb + 1 + 2 * i], ob = img[rb + 2 + 2 * i];
          const uint32_t fq = img[4 + q];
          const uint32_t l = get_field<S>(sw, fq);
          const uint32_t b0 = img[ob + l], cnt = img[ob + l + 1] - b0;
          set_field<S>(succ, fq, img[b0 + rem % cnt]);
          rem /= cnt;
        }
#pragma unroll
        for (int x = 0; x < S; ++x) stage[(k - lo) * S + x] = succ[x];
      }
    }
  }
}

// Exclusive prefix sum over the 64 lanes of a wavefront; *total receives the
// wavefront's sum.
__device__ inline uint32_t wave_exclusive_scan(uint32_t v, uint32_t* total) {
  const int lane = __lane_id();
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// Orders the LDS accesses of one wavefront (its lanes exchange staged
// successors through LDS; no other wavefront touches that region).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront's share of a BFS level: frontier states [first, first + 64)
// (those below n_in) of one exploration.  Counters of that exploration:
// ctr[0] next-frontier tail, ctr[1] deadlocks, ctr[2] transitions, ctr[3] flags.
struct WaveJob {
  TableDev t;
  const uint32_t* img;  // network image, in LDS
  const uint32_t* frontier_in;
  uint64_t first, n_in;
  uint32_t* frontier_out;
  uint64_t cap_out;
  uint32_t* dead;       // deadlock states (S words each)
  uint32_t* dead_tag;   // nullable: per deadlock record, the exploration's tag
  uint32_t tag;
  uint64_t dead_cap;
  uint64_t* dead_ctr;   // deadlock records used (may be shared by explorations)
  uint64_t* ctr;
  uint32_t* dtab;       // nullable: this wavefront's LDS duplicate filter
};

// Hash of a staged successor for the duplicate filter (any mix will do: it
// only spreads the chunk over the filter's entries).
template <int S>
__device__ __forceinline__ uint32_t dedup_hash(const uint32_t (&k)[S]) {
  uint32_t h = 0x9E3779B9u;
#pragma unroll
  for (int x = 0; x < S; ++x) h = (h ^ k[x]) * 0x85EBCA6Bu;
  return h ^ (h >> 15);
}

// A wavefront owns 64 frontier states and its own slice of the LDS staging
// buffer, and runs generate -> find-or-put -> append on its own; no barrier
// couples it to the other wavefronts of its workgroup, so successor
// generation (ALU) of one wavefront overlaps the table probes (memory) of the
// others.  Must be reached by the whole wavefront.
template <int S, int B, int G, int U>
__device__ inline void expand_wave(const WaveJob& j, uint32_t* stage, LaneStats& st) {
  constexpr uint32_t kWaveWords = kStageWords / 4;
  constexpr uint32_t CAP = kWaveWords / S;  // staged successors per chunk
  const int lane = __lane_id();
  const uint64_t i = j.first + lane;
  const bool has = i < j.n_in;
  uint32_t sw[S];
#pragma unroll
  for (int x = 0; x < S; ++x) sw[x] = has ? j.frontier_in[i * S + x] : 0u;
  const uint32_t c = has ? count_successors<S>(j.img, sw) : 0u;
  if (has && c == 0) {
    const uint64_t d = atomicAdd(reinterpret_cast<unsigned long long*>(j.dead_ctr), 1ull);
    if (j.dead_ctr != &j.ctr[1]) atomicAdd(reinterpret_cast<unsigned long long*>(&j.ctr[1]), 1ull);
    if (d < j.dead_cap) {
#pragma unroll
      for (int x = 0; x < S; ++x) j.dead[d * S + x] = sw[x];
      if (j.dead_tag) j.dead_tag[d] = j.tag;
    }
  }
  uint32_t total = 0;
  const uint32_t off = wave_exclusive_scan(c, &total);
  if (lane == 0 && total)
    atomicAdd(reinterpret_cast<unsigned long long*>(&j.ctr[2]), static_cast<unsigned long long>(total));

  for (uint32_t lo = 0; lo < total; lo += CAP) {
    const uint32_t hi = min(total, lo + CAP);
    if (c && off < hi && off + c > lo)
      emit_successors<S>(j.img, sw, static_cast<int>(lo) - static_cast<int>(off),
                         static_cast<int>(hi) - static_cast<int>(off), stage);
    wave_lds_sync();
    const uint32_t n_st = hi - lo;
    // Local duplicate filter (the block-local state cache of the tool): the
    // first occurrence of a successor in this chunk claims an entry of the
    // wavefront's LDS set; later occurrences find it and skip the table
    // probe (their result would be SEEN).  dupmask bit r: this lane's key of
    // round r is such a later occurrence.
    uint32_t dupmask = 0;
    if (j.dtab) {
      constexpr uint32_t D = dedup_entries<S>();
      for (uint32_t e = lane; e < D; e += 64) j.dtab[e] = kEmpty;
      wave_lds_sync();
      uint32_t dups = 0;
      for (uint32_t r0 = 0, r = 0; r0 < n_st; r0 += 64, ++r) {
        const uint32_t idx = r0 + lane;
        if (idx < n_st) {
          uint32_t key[S];
#pragma unroll
          for (int x = 0; x < S; ++x) key[x] = stage[idx * S + x];
          uint32_t h = dedup_hash<S>(key) & (D - 1);
          while (true) {
            uint32_t prev = kEmpty;
            if (__hip_atomic_compare_exchange_strong(&j.dtab[h], &prev, idx, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WAVEFRONT))
              break;  // first occurrence
            bool same = true;
#pragma unroll
            for (int x = 0; x < S; ++x) same &= stage[prev * S + x] == key[x];
            if (same) {
              dupmask |= 1u << r;
              ++dups;
              break;
            }
            h = (h + 1) & (D - 1);
          }
        }
      }
      const uint32_t wd = wave_sum(dups);
      if (lane == 0 && wd) atomicAdd(reinterpret_cast<unsigned long long*>(&j.ctr[4]), wd);
      wave_lds_sync();
    }
    for (uint32_t r0 = 0, r = 0; r0 < n_st; r0 += 64, ++r) {
      const uint32_t idx = r0 + lane;
      const bool act = idx < n_st && !((dupmask >> r) & 1u);
      uint32_t key[S];
#pragma unroll
      for (int x = 0; x < S; ++x) key[x] = act ? stage[idx * S + x] : 0u;
      const uint8_t res = find_or_put_lanes<S, B, G, U>(j.t, key, act, st);
      const bool is_new = act && res == kNew;
      const uint64_t m = __ballot(is_new);
      if (m) {
        unsigned long long base = 0;
        if (lane == 0)
          base = atomicAdd(reinterpret_cast<unsigned long long*>(&j.ctr[0]),
                           static_cast<unsigned long long>(__popcll(m)));
        base = __shfl(base, 0, 64);
        if (is_new) {
          const uint64_t pos = base + __popcll(m & ((1ull << lane) - 1ull));
          if (pos < j.cap_out) {
#pragma unroll
            for (int x = 0; x < S; ++x) j.frontier_out[pos * S + x] = key[x];
          } else {
            atomicOr(reinterpret_cast<unsigned long long*>(&j.ctr[3]), kFlagFrontierOverflow);
          }
        }
      }
      if (act && res == kFull)
        atomicOr(reinterpret_cast<unsigned long long*>(&j.ctr[3]), kFlagTableFull);
    }
    wave_lds_sync();
  }
}

// One BFS level of one exploration: 256 frontier states per workgroup.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void explore_level_kernel(ExploreArgs a) {
  extern __shared__ uint32_t smem[];
  uint32_t* img = smem;
  uint32_t* stage = smem + a.img_stride + (threadIdx.x >> 6) * (kStageWords / 4);
  for (uint32_t i = threadIdx.x; i < a.img_words; i += 256) img[i] = a.img[i];
  __syncthreads();
  WaveJob j;
  j.t = a.t;
  j.img = img;
  j.frontier_in = a.frontier_in;
  j.first = static_cast<uint64_t>(blockIdx.x) * 256 + (threadIdx.x & ~63u);
  j.n_in = a.n_in;
  j.frontier_out = a.frontier_out;
  j.cap_out = a.cap_out;
  j.dead = a.dead;
  j.dead_tag = nullptr;
  j.tag = 0;
  j.dead_cap = a.dead_cap;
  j.dead_ctr = &a.ctr[1];
  j.ctr = a.ctr;
  j.dtab = a.dedup ? smem + a.img_stride + kStageWords + (threadIdx.x >> 6) * dedup_entries<S>()
                   : nullptr;
  LaneStats st;
  if (j.first < j.n_in) expand_wave<S, B, G, U>(j, stage, st);
  flush_stats(a.t, st, nullptr);
}

template <int S, int B, int G, int U>
hipError_t launch_level(const ExploreArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  if (lds > 65536) {  // more than the default per-workgroup LDS: ask for it
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&explore_level_kernel<S, B, G, U>),
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((explore_level_kernel<S, B, G, U>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int S, int B, int G>
hipError_t level_u(uint32_t U, const ExploreArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  switch (U) {
    case 1: return launch_level<S, B, G, 1>(a, grid, lds, s);
    case 2: return launch_level<S, B, G, 2>(a, grid, lds, s);
    case 4: return launch_level<S, B, G, 4>(a, grid, lds, s);
    case 8: return launch_level<S, B, G, 8>(a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int S, int B>
hipError_t level_g(uint32_t G, uint32_t U, const ExploreArgs& a, uint32_t grid, size_t lds,
                   hipStream_t s) {
  switch (G) {
    case 8: return level_u<S, B, 8>(U, a, grid, lds, s);
    case 16: return level_u<S, B, 16>(U, a, grid, lds, s);
    case 32: return level_u<S, B, 32>(U, a, grid, lds, s);
    case 64: return level_u<S, B, 64>(U, a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int S>
hipError_t level_b(uint32_t B, uint32_t G, uint32_t U, const ExploreArgs& a, uint32_t grid,
                   size_t lds, hipStream_t s) {
  switch (B) {
    case 4: return level_g<S, 4>(G, U, a, grid, lds, s);
    case 8: return level_g<S, 8>(G, U, a, grid, lds, s);
    case 16: return level_g<S, 16>(G, U, a, grid, lds, s);
    case 32: return level_g<S, 32>(G, U, a, grid, lds, s);
    case 64: return level_g<S, 64>(G, U, a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gx
