// Step kernel of the exploration server and of the stepped batch schedule:
// one launch expands the current BFS level of every active job (jobs of one
// kernel class).  Workgroup b takes tile b of the concatenation of all jobs'
// levels (256 states per tile), finds its job by binary search over the jobs'
// first tiles, loads that job's network image into LDS and expands the tile
// with the same per-wavefront routine as the single-exploration kernel.  Jobs
// join and leave between launches.
#pragma once

#include <cstdint>

#include "gx_explore_kernel.hpp"

namespace gx {

struct ServeJob {
  TableDev t;
  uint32_t img_off, img_words;
  const uint32_t* frontier_in;
  uint64_t n_in;
  uint32_t* frontier_out;
  uint64_t cap_out;
  uint32_t* dead;
  uint64_t dead_cap;
  uint64_t* ctr;        // the job's counters (ctr_at)
  uint64_t tile_begin;  // first tile of this job in the step
  // a deadlock buffer shared by several jobs: records used (null: the job's
  // own kCtrDead counter) and, per record, the job's tag (nullable)
  uint64_t* dead_ctr;
  uint32_t* dead_tag;
  uint32_t tag;
  uint32_t pad;
};

struct ServeArgs {
  const ServeJob* jobs;
  uint32_t n_jobs;
  const uint32_t* img;  // all jobs' network images
  uint32_t img_stride;  // LDS words reserved for one image
};

template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void serve_step_kernel(ServeArgs a) {
  extern __shared__ uint32_t smem[];
  uint32_t* img = smem;
  uint32_t* stage = smem + a.img_stride + (threadIdx.x >> 6) * (kStageWords / 4);
  const uint64_t tile = blockIdx.x;
  // last job whose first tile is <= this tile
  uint32_t lo = 0, hi = a.n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (a.jobs[mid].tile_begin <= tile) lo = mid;
    else hi = mid;
  }
  const ServeJob& jb = a.jobs[lo];
  for (uint32_t k = threadIdx.x; k < jb.img_words; k += 256) img[k] = a.img[jb.img_off + k];
  __syncthreads();
  WaveJob j;
  j.t = jb.t;
  j.img = img;
  j.frontier_in = jb.frontier_in;
  j.first = (tile - jb.tile_begin) * 256 + (threadIdx.x & ~63u);
  j.n_in = jb.n_in;
  j.frontier_out = jb.frontier_out;
  j.cap_out = jb.cap_out;
  j.dead = jb.dead;
  j.dead_tag = jb.dead_tag;
  j.tag = jb.tag;
  j.dead_cap = jb.dead_cap;
  j.dead_ctr = jb.dead_ctr ? jb.dead_ctr : reinterpret_cast<uint64_t*>(ctr_at(jb.ctr, kCtrDead));
  j.ctr = jb.ctr;
  j.dtab = nullptr;
  LaneStats st;
  if (j.first < j.n_in) expand_wave<S, B, G, U>(j, stage, st);
}

template <int S>
hipError_t serve_launch(uint32_t B, uint32_t G, uint32_t U, const ServeArgs& a, uint32_t grid,
                        size_t lds, hipStream_t s) {
#define GX_SERVE_CASE(BB, GG, UU)                                                              \
  if (B == BB && G == GG && U == UU) {                                                         \
    hipLaunchKernelGGL((serve_step_kernel<S, BB, GG, UU>), dim3(grid), dim3(256), lds, s, a); \
    return hipGetLastError();                                                                  \
  }
#define GX_SERVE_B(BB) GX_SERVE_CASE(BB, 8, 1) GX_SERVE_CASE(BB, 8, 2) GX_SERVE_CASE(BB, 16, 1) GX_SERVE_CASE(BB, 16, 2)
#define GX_SERVE_B4(BB) GX_SERVE_B(BB) GX_SERVE_CASE(BB, 4, 1) GX_SERVE_CASE(BB, 4, 2)
  GX_SERVE_B4(8) GX_SERVE_B4(16) GX_SERVE_B4(32) GX_SERVE_B(64)
#undef GX_SERVE_B4
#undef GX_SERVE_B
#undef GX_SERVE_CASE
  return hipErrorInvalidValue;
}

}  // namespace gx
