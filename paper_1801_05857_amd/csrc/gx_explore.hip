// Level-synchronous breadth-first exploration of the synchronous product of a
// network of LTSs (Sec. 3 of the paper), built on the bucketed find-or-put.
//
// Per BFS level one kernel launch expands the current frontier:
//   1. a workgroup of 256 threads takes 256 frontier states, one per thread,
//      and counts each state's product successors from the LDS-resident
//      network image; a state with none is a deadlock;
//   2. a block-wide prefix sum of the counts gives every successor a slot;
//      successors are generated into an LDS staging buffer, in chunks when
//      the tile has more successors than the buffer holds;
//   3. subgroups of G lanes find-or-put the staged successors; those reported
//      NEW are appended to the next frontier with one atomic add per
//      wavefront (ballot + popcount ranks).
// The paper's tool scans the hash table for states still to explore and keeps
// a per-block cache of new states (Sec. 3); here the next level is an explicit
// compacted frontier, so no scan of the table is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gx_internal.hpp"

namespace gx {

// ------------------------------------------------------------ network image
// Layout (32-bit words, indices absolute within the image):
//   [0] P  [1] R  [2] S  [3] words per state
//   [4 + p]         field of process p: word | shift << 8 | width << 16
//   [4 + P + p]     index of the start of p's free-transition offsets
//   [4 + 2P + r]    index of rule r's record
//   rule record:    n_parts, then per participant (process q, index of the
//                   start of its offsets for this rule)
//   offsets arrays: n_q + 1 entries each; entry l is the index of the first
//                   target of local state l, entry l+1 one past its last
//   target arrays:  target local states
constexpr uint32_t kImgMaxWords = 11776;  // 46 KiB of LDS
constexpr uint32_t kStageWords = 4096;    // 16 KiB of LDS for staged successors
constexpr uint32_t kMaxSuccPerState = 1u << 20;

struct NetImage {
  std::vector<uint32_t> img;
  uint32_t words = 0;
  std::vector<uint32_t> field;  // per process
  std::vector<uint32_t> initial;
  uint64_t max_succ = 0;
};

namespace {

uint32_t field_bits(uint32_t n) {
  uint32_t b = 1;
  while (b < 32 && (uint64_t(1) << b) < n) ++b;
  return b;
}

gx_status compile_network(const gx_network* net, NetImage* out) {
  if (!net || net->n_procs == 0 || !net->procs) return GX_EINVAL;
  if (net->n_rules && !net->rules) return GX_EINVAL;
  const uint32_t P = net->n_procs, R = net->n_rules, NL = net->n_labels;
  // packing plan
  std::vector<uint32_t> field(P);
  uint32_t word = 0, used = 0;
  for (uint32_t p = 0; p < P; ++p) {
    const gx_lts& l = net->procs[p];
    if (l.n_states == 0 || l.initial >= l.n_states) return GX_EINVAL;
    if (l.n_trans && (!l.src || !l.label || !l.dst)) return GX_EINVAL;
    const uint32_t b = field_bits(l.n_states);
    if (b > 31) return GX_EINVAL;
    if (used + b > 31) {
      ++word;
      used = 0;
    }
    field[p] = word | (used << 8) | (b << 16);
    used += b;
  }
  const uint32_t words = word + 1;
  if (words > 4) return GX_EINVAL;
  // which labels of each process are named by a rule at its position
  std::vector<std::vector<uint8_t>> governed(P, std::vector<uint8_t>(NL, 0));
  std::vector<std::vector<uint32_t>> parts(R);
  for (uint32_t r = 0; r < R; ++r) {
    for (uint32_t p = 0; p < P; ++p) {
      const int32_t a = net->rules[size_t(r) * P + p];
      if (a < -1 || a >= int32_t(NL)) return GX_EINVAL;
      if (a >= 0) {
        governed[p][a] = 1;
        parts[r].push_back(p);
      }
    }
    if (parts[r].empty()) return GX_EINVAL;
  }
  for (uint32_t p = 0; p < P; ++p) {
    const gx_lts& l = net->procs[p];
    for (uint32_t t = 0; t < l.n_trans; ++t)
      if (l.src[t] >= l.n_states || l.dst[t] >= l.n_states || l.label[t] >= NL) return GX_EINVAL;
  }

  std::vector<uint32_t> img(4 + 2 * P + R, 0);
  img[0] = P;
  img[1] = R;
  img[2] = slot_words(words);
  img[3] = words;
  for (uint32_t p = 0; p < P; ++p) img[4 + p] = field[p];
  // rule records
  for (uint32_t r = 0; r < R; ++r) {
    img[4 + 2 * P + r] = static_cast<uint32_t>(img.size());
    img.push_back(static_cast<uint32_t>(parts[r].size()));
    for (uint32_t q : parts[r]) {
      img.push_back(q);
      img.push_back(0);  // patched below
    }
  }
  auto too_big = [&]() { return img.size() > kImgMaxWords; };
  // CSR of targets selected by `keep` for process p: offsets then targets
  auto emit_csr = [&](uint32_t p, auto keep, uint64_t* max_deg) -> uint32_t {
    const gx_lts& l = net->procs[p];
    std::vector<std::vector<uint32_t>> by_src(l.n_states);
    for (uint32_t t = 0; t < l.n_trans; ++t)
      if (keep(l.label[t])) by_src[l.src[t]].push_back(l.dst[t]);
    const uint32_t off_at = static_cast<uint32_t>(img.size());
    img.resize(img.size() + l.n_states + 1);
    uint64_t md = 0;
    for (uint32_t s = 0; s < l.n_states; ++s) {
      img[off_at + s] = static_cast<uint32_t>(img.size());
      for (uint32_t d : by_src[s]) img.push_back(d);
      md = std::max<uint64_t>(md, by_src[s].size());
      if (too_big()) return 0;
    }
    img[off_at + l.n_states] = static_cast<uint32_t>(img.size());
    *max_deg = md;
    return off_at;
  };
  uint64_t max_succ = 0;
  for (uint32_t p = 0; p < P && !too_big(); ++p) {
    uint64_t md = 0;
    const uint32_t at = emit_csr(p, [&](uint32_t a) { return !governed[p][a]; }, &md);
    img[4 + P + p] = at;
    max_succ += md;
  }
  for (uint32_t r = 0; r < R && !too_big(); ++r) {
    const uint32_t rec = img[4 + 2 * P + r];
    uint64_t prod = 1;
    for (size_t i = 0; i < parts[r].size() && !too_big(); ++i) {
      const uint32_t q = parts[r][i];
      const uint32_t want = static_cast<uint32_t>(net->rules[size_t(r) * P + q]);
      uint64_t md = 0;
      const uint32_t at = emit_csr(q, [&](uint32_t a) { return a == want; }, &md);
      img[rec + 2 + 2 * i] = at;
      prod = std::min<uint64_t>(prod * md, uint64_t(1) << 40);
    }
    max_succ += prod;
  }
  if (too_big()) return GX_EINVAL;
  if (max_succ > kMaxSuccPerState) return GX_EINVAL;
  out->img = std::move(img);
  out->words = words;
  out->field = std::move(field);
  out->initial.resize(P);
  for (uint32_t p = 0; p < P; ++p) out->initial[p] = net->procs[p].initial;
  out->max_succ = max_succ;
  return GX_OK;
}

void pack_host(const NetImage& ni, const uint32_t* local, uint32_t* out) {
  for (uint32_t k = 0; k < ni.words; ++k) out[k] = 0;
  for (size_t p = 0; p < ni.field.size(); ++p) {
    const uint32_t f = ni.field[p];
    out[f & 0xFF] |= local[p] << ((f >> 8) & 0xFF);
  }
}

}  // namespace

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

template <int S, int B, int G>
__global__ __launch_bounds__(256) void explore_level_kernel(ExploreArgs a) {
  extern __shared__ uint32_t smem[];
  constexpr int CAP = kStageWords / S;  // staged successors per chunk
  constexpr int NSUB = 256 / G;
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
  const int li = lane % G;
  const int sub = threadIdx.x / G;
  LaneStats st;
  for (uint32_t lo = 0; lo < total; lo += CAP) {
    const uint32_t hi = min(total, lo + static_cast<uint32_t>(CAP));
    if (c && off < hi && off + c > lo)
      emit_successors<S>(img, sw, static_cast<int>(lo) - static_cast<int>(off),
                         static_cast<int>(hi) - static_cast<int>(off), stage);
    __syncthreads();
    const uint32_t n_st = hi - lo;
    for (uint32_t r0 = 0; r0 < n_st; r0 += NSUB) {
      const uint32_t idx = r0 + sub;
      uint32_t key[1][S];
      bool act[1] = {idx < n_st};
      uint8_t res[1];
#pragma unroll
      for (int x = 0; x < S; ++x) key[0][x] = act[0] ? stage[idx * S + x] : 0u;
      find_or_put<S, B, G, 1>(a.t, key, act, res, st);
      const bool is_new = act[0] && res[0] == kNew && li == 0;
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
            for (int x = 0; x < S; ++x) a.frontier_out[pos * S + x] = key[0][x];
          } else {
            atomicOr(reinterpret_cast<unsigned long long*>(&a.ctr[3]), kFlagFrontierOverflow);
          }
        }
      }
      if (act[0] && res[0] == kFull && li == 0)
        atomicOr(reinterpret_cast<unsigned long long*>(&a.ctr[3]), kFlagTableFull);
    }
    __syncthreads();
  }
  flush_stats(a.t, st, nullptr);
}

namespace {

template <int S, int B, int G>
hipError_t launch_level(const ExploreArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((explore_level_kernel<S, B, G>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int S, int B>
hipError_t level_g(uint32_t G, const ExploreArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  switch (G) {
    case 8: return launch_level<S, B, 8>(a, grid, lds, s);
    case 16: return launch_level<S, B, 16>(a, grid, lds, s);
    case 32: return launch_level<S, B, 32>(a, grid, lds, s);
    case 64: return launch_level<S, B, 64>(a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int S>
hipError_t level_b(uint32_t B, uint32_t G, const ExploreArgs& a, uint32_t grid, size_t lds,
                   hipStream_t s) {
  switch (B) {
    case 8: return level_g<S, 8>(G, a, grid, lds, s);
    case 16: return level_g<S, 16>(G, a, grid, lds, s);
    case 32: return level_g<S, 32>(G, a, grid, lds, s);
    case 64: return level_g<S, 64>(G, a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_level_any(const gx_table* t, const ExploreArgs& a, uint32_t grid, size_t lds,
                            hipStream_t s) {
  switch (t->S) {
    case 1: return level_b<1>(t->B, t->G, a, grid, lds, s);
    case 2: return level_b<2>(t->B, t->G, a, grid, lds, s);
    case 4: return level_b<4>(t->B, t->G, a, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

struct DeviceBuffers {
  uint32_t* img = nullptr;
  uint32_t* f[2] = {nullptr, nullptr};
  uint32_t* dead = nullptr;
  uint64_t* ctr = nullptr;
  uint8_t* status = nullptr;
  ~DeviceBuffers() {
    if (img) (void)hipFree(img);
    if (f[0]) (void)hipFree(f[0]);
    if (f[1]) (void)hipFree(f[1]);
    if (dead) (void)hipFree(dead);
    if (ctr) (void)hipFree(ctr);
    if (status) (void)hipFree(status);
  }
};

}  // namespace
}  // namespace gx

// ====================================================================== ABI
extern "C" {

gx_status gx_network_words(const gx_network* net, uint32_t* words) {
  if (!words) return GX_EINVAL;
  gx::NetImage ni;
  const gx_status s = gx::compile_network(net, &ni);
  if (s != GX_OK) return s;
  *words = ni.words;
  return GX_OK;
}

gx_status gx_network_pack(const gx_network* net, const uint32_t* local, uint64_t n,
                          uint32_t* out) {
  if ((n && (!local || !out))) return GX_EINVAL;
  gx::NetImage ni;
  const gx_status s = gx::compile_network(net, &ni);
  if (s != GX_OK) return s;
  const uint32_t P = net->n_procs;
  for (uint64_t i = 0; i < n; ++i) {
    for (uint32_t p = 0; p < P; ++p)
      if (local[i * P + p] >= net->procs[p].n_states) return GX_EINVAL;
  }
  for (uint64_t i = 0; i < n; ++i) gx::pack_host(ni, local + i * P, out + i * ni.words);
  return GX_OK;
}

void gx_explore_result_free(gx_explore_result* r) {
  if (!r) return;
  std::free(r->level_counts);
  std::free(r->deadlocks);
  r->level_counts = nullptr;
  r->deadlocks = nullptr;
}

gx_status gx_explore(const gx_network* net, gx_table* t, const gx_explore_opts* opts,
                     gx_explore_result* out) {
  if (!t || !out) return GX_EINVAL;
  gx::NetImage ni;
  gx_status s = gx::compile_network(net, &ni);
  if (s != GX_OK) return s;
  if (ni.words != t->w) return GX_EINVAL;
  const uint32_t S = t->S;
  const uint64_t n_slots = t->n_buckets * (t->B / S);
  const uint64_t cap = opts && opts->frontier_capacity ? opts->frontier_capacity : n_slots;
  const uint64_t dead_cap = opts && opts->deadlock_capacity ? opts->deadlock_capacity : (1u << 20);
  hipStream_t stream = opts ? static_cast<hipStream_t>(opts->hip_stream) : nullptr;

  gx::DeviceBuffers d;
  const uint32_t img_words = static_cast<uint32_t>(ni.img.size());
  const uint32_t img_stride = (img_words + 3) & ~3u;
  if (hipMalloc(&d.img, img_stride * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&d.f[0], cap * S * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&d.f[1], cap * S * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&d.dead, dead_cap * S * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&d.ctr, 8 * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc(&d.status, 8) != hipSuccess) {
    (void)hipGetLastError();
    return GX_ENOMEM;
  }
  uint32_t init[4] = {0, 0, 0, 0};
  gx::pack_host(ni, ni.initial.data(), init);
  uint64_t ctr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hipMemcpyAsync(d.img, ni.img.data(), img_words * sizeof(uint32_t), hipMemcpyHostToDevice,
                     stream) != hipSuccess ||
      hipMemcpyAsync(d.f[0], init, S * sizeof(uint32_t), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemsetAsync(d.ctr, 0, 8 * sizeof(uint64_t), stream) != hipSuccess)
    return GX_EDEVICE;
  // the initial state: must be new, i.e. the table was empty of it
  std::vector<uint32_t> init_key(init, init + t->w);
  uint32_t* d_key = d.dead;  // borrow: the deadlock buffer is unused yet
  if (hipMemcpyAsync(d_key, init_key.data(), t->w * sizeof(uint32_t), hipMemcpyHostToDevice,
                     stream) != hipSuccess ||
      gx::launch_find_or_put(t, d_key, 1, d.status, nullptr, stream) != hipSuccess)
    return GX_EDEVICE;
  uint8_t st0 = 0;
  if (hipMemcpyAsync(&st0, d.status, 1, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return GX_EDEVICE;
  if (st0 == gx::kFull) return GX_ETABLEFULL;
  if (st0 != gx::kNew) return GX_EINVAL;

  gx::ExploreArgs a;
  a.t = t->dev();
  a.img = d.img;
  a.img_words = img_words;
  a.img_stride = img_stride;
  a.dead = d.dead;
  a.dead_cap = dead_cap;
  a.ctr = d.ctr;
  a.cap_out = cap;
  const size_t lds = (img_stride + gx::kStageWords + 8) * sizeof(uint32_t);

  std::vector<uint64_t> levels{1};
  uint64_t n_in = 1;
  int cur = 0;
  while (n_in > 0) {
    a.frontier_in = d.f[cur];
    a.n_in = n_in;
    a.frontier_out = d.f[cur ^ 1];
    if (hipMemsetAsync(d.ctr, 0, sizeof(uint64_t), stream) != hipSuccess) return GX_EDEVICE;
    const uint64_t grid = (n_in + 255) / 256;
    if (grid > 0xFFFFFFFFull) return GX_ENOMEM;
    if (gx::launch_level_any(t, a, static_cast<uint32_t>(grid), lds, stream) != hipSuccess)
      return GX_EDEVICE;
    if (hipMemcpyAsync(ctr, d.ctr, sizeof(ctr), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GX_EDEVICE;
    if (ctr[3] & gx::kFlagTableFull) return GX_ETABLEFULL;
    if (ctr[3] & gx::kFlagFrontierOverflow) return GX_ENOMEM;
    n_in = ctr[0];
    if (n_in) levels.push_back(n_in);
    cur ^= 1;
  }
  const uint64_t n_dead = ctr[1];
  if (n_dead > dead_cap) return GX_ENOMEM;
  std::vector<uint32_t> raw(n_dead * S);
  if (n_dead && hipMemcpy(raw.data(), d.dead, raw.size() * sizeof(uint32_t),
                          hipMemcpyDeviceToHost) != hipSuccess)
    return GX_EDEVICE;
  std::vector<std::array<uint32_t, 4>> dl(n_dead);
  for (uint64_t i = 0; i < n_dead; ++i) {
    dl[i] = {0, 0, 0, 0};
    for (uint32_t k = 0; k < t->w; ++k) dl[i][k] = raw[i * S + k];
  }
  std::sort(dl.begin(), dl.end());

  uint64_t* lv = static_cast<uint64_t*>(std::malloc(sizeof(uint64_t) * levels.size()));
  uint32_t* dd = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (n_dead * t->w + 1)));
  if (!lv || !dd) {
    std::free(lv);
    std::free(dd);
    return GX_ENOMEM;
  }
  uint64_t n_states = 0;
  for (size_t k = 0; k < levels.size(); ++k) {
    lv[k] = levels[k];
    n_states += levels[k];
  }
  for (uint64_t i = 0; i < n_dead; ++i)
    for (uint32_t k = 0; k < t->w; ++k) dd[i * t->w + k] = dl[i][k];
  out->n_states = n_states;
  out->n_transitions = ctr[2];
  out->words_per_state = t->w;
  out->n_levels = static_cast<uint32_t>(levels.size());
  out->level_counts = lv;
  out->n_deadlocks = n_dead;
  out->deadlocks = dd;
  return GX_OK;
}

}  // extern "C"
