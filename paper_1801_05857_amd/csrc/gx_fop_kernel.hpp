// Find-or-put kernel and its (B, G, U) dispatch for one slot width S; each
// slot width is instantiated in a translation unit of its own so the
// specialisations compile in parallel.
#pragma once

#include <algorithm>

#include "gx_internal.hpp"

namespace gx {

template <int S>
__device__ inline void load_key(const uint32_t* keys, uint32_t w, uint64_t idx,
                                uint32_t (&k)[S]) {
  if constexpr (S == 1) {
    k[0] = keys[idx];
  } else if constexpr (S == 2) {
    uint2 t = reinterpret_cast<const uint2*>(keys)[idx];
    k[0] = t.x;
    k[1] = t.y;
  } else {
    if (w == 4) {
      uint4 t = reinterpret_cast<const uint4*>(keys)[idx];
      k[0] = t.x;
      k[1] = t.y;
      k[2] = t.z;
      k[3] = t.w;
    } else {
      const uint32_t* p = keys + idx * 3;
      k[0] = p[0];
      k[1] = p[1];
      k[2] = p[2];
      k[3] = 0;
    }
  }
}

// One key per lane: a wavefront handles 64 consecutive keys per round (one
// coalesced read of the keys, one coalesced write of the statuses), its
// subgroups probing them U at a time.  Grid-stride over rounds.
template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void fop_kernel(TableDev t, const uint32_t* keys, uint32_t w,
                                                  uint64_t n, uint8_t* status, uint64_t* n_new) {
  const int lane = __lane_id();
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  LaneStats st;
  for (uint64_t base = wave * 64; base < n; base += n_waves * 64) {
    const uint64_t idx = base + lane;
    const bool act = idx < n;
    uint32_t key[S];
#pragma unroll
    for (int x = 0; x < S; ++x) key[x] = 0;
    if (act) load_key<S>(keys, w, idx, key);
    const uint8_t r = find_or_put_lanes<S, B, G, U>(t, key, act, st);
    if (act) status[idx] = r;
  }
  flush_stats(t, st, n_new);
}


template <int S, int B, int G, int U>
hipError_t launch_fop(const FopArgs& a) {
  // as many workgroups as can be resident at once (grid-stride over rounds)
  static int per_cu = 0;
  if (per_cu == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fop_kernel<S, B, G, U>, 256, 0) !=
            hipSuccess ||
        b <= 0)
      b = 2;
    per_cu = b;
  }
  const uint64_t want = (a.n + 255) / 256;  // one key per thread per round
  uint32_t grid = static_cast<uint32_t>(
      std::min<uint64_t>(want, static_cast<uint64_t>(a.cus) * static_cast<uint32_t>(per_cu)));
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL((fop_kernel<S, B, G, U>), dim3(grid), dim3(256), 0, a.stream, a.t, a.keys,
                     a.w, a.n, a.status, a.n_new);
  return hipGetLastError();
}

template <int S, int B, int G>
hipError_t dispatch_u(uint32_t U, const FopArgs& a) {
  switch (U) {
    case 1: return launch_fop<S, B, G, 1>(a);
    case 2: return launch_fop<S, B, G, 2>(a);
    case 4: return launch_fop<S, B, G, 4>(a);
    case 8:
      if constexpr (G >= 8) return launch_fop<S, B, G, 8>(a);
      break;
  }
  return hipErrorInvalidValue;
}

template <int S, int B>
hipError_t dispatch_g(uint32_t G, uint32_t U, const FopArgs& a) {
  switch (G) {
    case 4:
      if constexpr (B <= 32) return dispatch_u<S, B, 4>(U, a);
      break;
    case 8: return dispatch_u<S, B, 8>(U, a);
    case 16: return dispatch_u<S, B, 16>(U, a);
    case 32: return dispatch_u<S, B, 32>(U, a);
    case 64: return dispatch_u<S, B, 64>(U, a);
  }
  return hipErrorInvalidValue;
}

template <int S>
hipError_t dispatch_b(uint32_t B, uint32_t G, uint32_t U, const FopArgs& a) {
  switch (B) {
    case 4: return dispatch_g<S, 4>(G, U, a);
    case 8: return dispatch_g<S, 8>(G, U, a);
    case 16: return dispatch_g<S, 16>(G, U, a);
    case 32: return dispatch_g<S, 32>(G, U, a);
    case 64: return dispatch_g<S, 64>(G, U, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace gx
