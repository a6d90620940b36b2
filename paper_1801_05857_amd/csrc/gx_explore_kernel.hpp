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
  uint64_t* ctr;  // [0] next-frontier tail [1] deadlocks [2] transitions [3] flags
};

enum : uint32_t { kFlagFrontierOverflow = 1, kFlagTableFull = 2 };

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

// Exclusive prefix sum over the 256 threads; *total receives the sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
  const int lane = __lane_id();
  const int wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) scratch[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < 4; ++w) {
      const uint32_t t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[4] = run;
  }
  __syncthreads();
  const uint32_t ex = scratch[wid] + x - v;
  *total = scratch[4];
  return ex;
}

template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void explore_level_kernel(ExploreArgs a) {
  extern __shared__ uint32_t smem[];
  constexpr int CAP = kStageWords / S;  // staged successors per chunk
  uint32_t* img = smem;
  uint32_t* stage = smem + a.img_stride;
  uint32_t* scratch = stage + kStageWords;

  for (uint32_t i = threadIdx.x; i < a.img_words; i += 256) img[i] = a.img[i];
  __syncthreads();

  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
  const bool has = i < a.n_in;
  uint32_t sw[S];
#pragma unroll
  for (int x = 0; x < S; ++x) sw[x] = has ? a.frontier_in[i * S + x] : 0u;
  const uint32_t c = has ? count_successors<S>(img, sw) : 0u;
  if (has && c == 0) {
    const uint64_t d = atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctr[1]), 1ull);
    if (d < a.dead_cap) {
#pragma unroll
      for (int x = 0; x < S; ++x) a.dead[d * S + x] = sw[x];
    }
  }
  uint32_t total = 0;
  const uint32_t off = block_exclusive_scan(c, scratch, &total);
  if (threadIdx.x == 0 && total)
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctr[2]), static_cast<unsigned long long>(total));

  const int lane = __lane_id();
  LaneStats st;
  for (uint32_t lo = 0; lo < total; lo += CAP) {
    const uint32_t hi = min(total, lo + static_cast<uint32_t>(CAP));
    if (c && off < hi && off + c > lo)
      emit_successors<S>(img, sw, static_cast<int>(lo) - static_cast<int>(off),
                         static_cast<int>(hi) - static_cast<int>(off), stage);
    __syncthreads();
    const uint32_t n_st = hi - lo;
    for (uint32_t r0 = 0; r0 < n_st; r0 += 256) {
      const uint32_t idx = r0 + threadIdx.x;
      const bool act = idx < n_st;
      uint32_t key[S];
#pragma unroll
      for (int x = 0; x < S; ++x) key[x] = act ? stage[idx * S + x] : 0u;
      const uint8_t res = find_or_put_lanes<S, B, G, U>(a.t, key, act, st);
      const bool is_new = act && res == kNew;
      const uint64_t m = __ballot(is_new);
      if (m) {
        unsigned long long base = 0;
        if (lane == 0)
          base = atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctr[0]),
                           static_cast<unsigned long long>(__popcll(m)));
        base = __shfl(base, 0, 64);
        if (is_new) {
          const uint64_t pos = base + __popcll(m & ((1ull << lane) - 1ull));
          if (pos < a.cap_out) {
#pragma unroll
            for (int x = 0; x < S; ++x) a.frontier_out[pos * S + x] = key[x];
          } else {
            atomicOr(reinterpret_cast<unsigned long long*>(&a.ctr[3]), kFlagFrontierOverflow);
          }
        }
      }
      if (act && res == kFull)
        atomicOr(reinterpret_cast<unsigned long long*>(&a.ctr[3]), kFlagTableFull);
    }
    __syncthreads();
  }
  flush_stats(a.t, st, nullptr);
}

template <int S, int B, int G, int U>
hipError_t launch_level(const ExploreArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
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
    case 8: return level_g<S, 8>(G, U, a, grid, lds, s);
    case 16: return level_g<S, 16>(G, U, a, grid, lds, s);
    case 32: return level_g<S, 32>(G, U, a, grid, lds, s);
    case 64: return level_g<S, 64>(G, U, a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gx
