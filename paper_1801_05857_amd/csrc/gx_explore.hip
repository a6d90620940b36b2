// Level-synchronous breadth-first exploration of the synchronous product of a
// network of LTSs (Sec. 3 of the paper), built on the bucketed find-or-put.
//
// A level is expanded in slices; each slice is two kernels on the caller's
// stream:
//   1. gen_level_kernel: 256 frontier states per workgroup, one per lane;
//      every lane counts its state's product successors from the
//      LDS-resident network image (none: a deadlock, recorded at once), one
//      atomic add per workgroup reserves their room in the successor buffer,
//      and the wavefront writes them with coalesced stores;
//   2. append_kernel: find-or-put of the successor buffer by subgroups of G
//      lanes; NEW states are gathered per wavefront in LDS and moved to the
//      next frontier with one atomic add and coalesced stores.
// The paper's tool scans the hash table for states still to explore and keeps
// a per-block cache of new states (Sec. 3); here the next level is an explicit
// compacted frontier, so no scan of the table is needed.  With a safety
// monitor, every completed level is scanned once for states whose monitor
// process is in a bad state.
//
// Levels of at most kSmallMaxLevel states (the first levels of every
// exploration, the last ones of most, all of a small one) are instead
// expanded on one workgroup, up to kSmallLevels of them per launch with no
// host round trip in between: the first levels by lds_levels_kernel, which
// decides NEW or SEEN from an LDS set of the states reached so far (the
// table holds nothing else yet) and puts them into the table at the end;
// later small levels by small_levels_kernel, which probes the table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "gx_small_kernel.hpp"

namespace gx {
// instantiated in gx_explore_s1.hip, gx_explore_s2.hip and gx_explore_s4.hip
extern template hipError_t launch_gen<1>(const GenArgs&, uint32_t, size_t, hipStream_t);
extern template hipError_t launch_gen<2>(const GenArgs&, uint32_t, size_t, hipStream_t);
extern template hipError_t launch_gen<4>(const GenArgs&, uint32_t, size_t, hipStream_t);
extern template hipError_t append_b<1>(uint32_t, uint32_t, uint32_t, const AppendArgs&, uint32_t,
                                       hipStream_t);
extern template hipError_t append_b<2>(uint32_t, uint32_t, uint32_t, const AppendArgs&, uint32_t,
                                       hipStream_t);
extern template hipError_t append_b<4>(uint32_t, uint32_t, uint32_t, const AppendArgs&, uint32_t,
                                       hipStream_t);
extern template hipError_t launch_small<1>(uint32_t, const SmallArgs&, hipStream_t);
extern template hipError_t launch_small<2>(uint32_t, const SmallArgs&, hipStream_t);
extern template hipError_t launch_small<4>(uint32_t, const SmallArgs&, hipStream_t);
extern template hipError_t launch_lds_levels<1>(uint32_t, SmallArgs, size_t, hipStream_t);
extern template hipError_t launch_lds_levels<2>(uint32_t, SmallArgs, size_t, hipStream_t);
extern template hipError_t launch_lds_levels<4>(uint32_t, SmallArgs, size_t, hipStream_t);
}  // namespace gx

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
constexpr uint32_t kMaxSuccPerState = 1u << 20;
// Largest image of any kernel: one that exceeds kImgMaxWords (the LDS budget)
// is read from global memory by the exploration's generation kernel.
constexpr uint32_t kImgGlobalMaxWords = 1u << 26;

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

gx_status compile_network(const gx_network* net, NetImage* out,
                          uint32_t max_words = kImgGlobalMaxWords) {
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
  auto too_big = [&]() { return img.size() > max_words; };
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

void pack_host(const NetImage& ni, const uint32_t* local, uint32_t* out);

}  // namespace

gx_status compile_network_image(const gx_network* net, std::vector<uint32_t>* img,
                                uint32_t* words, std::vector<uint32_t>* packed_initial,
                                uint64_t* max_succ) {
  NetImage ni;
  // batches and the server keep every image in LDS
  const gx_status s = compile_network(net, &ni, kImgMaxWords);
  if (s != GX_OK) return s;
  packed_initial->assign(4, 0);
  pack_host(ni, ni.initial.data(), packed_initial->data());
  *img = std::move(ni.img);
  *words = ni.words;
  *max_succ = ni.max_succ;
  return GX_OK;
}

namespace {

void pack_host(const NetImage& ni, const uint32_t* local, uint32_t* out) {
  for (uint32_t k = 0; k < ni.words; ++k) out[k] = 0;
  for (size_t p = 0; p < ni.field.size(); ++p) {
    const uint32_t f = ni.field[p];
    out[f & 0xFF] |= local[p] << ((f >> 8) & 0xFF);
  }
}

}  // namespace

namespace {

// Safety monitor: the states among states[0, n) whose monitor field f (word
// | shift << 8 | width << 16) holds a local state marked in the bitmask
// `bad` are counted in *ctr and, below cap, copied to out (S words each).
// One atomic add per wavefront that finds any.
template <int S>
__global__ __launch_bounds__(256) void monitor_scan_kernel(const uint32_t* states, uint64_t n,
                                                           uint32_t f, const uint32_t* bad,
                                                           uint32_t* out, uint64_t cap,
                                                           unsigned long long* ctr) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * 256 + (threadIdx.x & ~63u);
  const int lane = __lane_id();
  for (uint64_t base = first; base < n; base += stride) {  // wavefront-uniform
    const uint64_t i = base + lane;
    uint32_t sw[S] = {};
    bool hit = false;
    if (i < n) {
      load_slot<S>(states + i * S, sw);
      const uint32_t l = get_field<S>(sw, f);
      hit = (bad[l >> 5] >> (l & 31)) & 1u;
    }
    const uint64_t m = __ballot(hit);
    if (m == 0) continue;
    unsigned long long k = 0;
    if (lane == 0) k = atomicAdd(ctr, static_cast<unsigned long long>(__popcll(m)));
    k = __shfl(k, 0, 64) + __popcll(m & ((1ull << lane) - 1ull));
    if (hit && k < cap) store_slot<S>(out + k * S, sw);
  }
}

hipError_t launch_monitor_scan(uint32_t S, const uint32_t* states, uint64_t n, uint32_t f,
                               const uint32_t* bad, uint32_t* out, uint64_t cap, uint64_t* ctr,
                               uint32_t cus, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid =
      static_cast<uint32_t>(std::min<uint64_t>((n + 255) / 256, static_cast<uint64_t>(cus) * 8));
  auto* c = reinterpret_cast<unsigned long long*>(ctr);
  switch (S) {
    case 1:
      hipLaunchKernelGGL((monitor_scan_kernel<1>), dim3(grid), dim3(256), 0, s, states, n, f, bad,
                         out, cap, c);
      break;
    case 2:
      hipLaunchKernelGGL((monitor_scan_kernel<2>), dim3(grid), dim3(256), 0, s, states, n, f, bad,
                         out, cap, c);
      break;
    default:
      hipLaunchKernelGGL((monitor_scan_kernel<4>), dim3(grid), dim3(256), 0, s, states, n, f, bad,
                         out, cap, c);
      break;
  }
  return hipGetLastError();
}

// One slice of a level: successor generation, then find-or-put-and-append.
hipError_t launch_slice(const gx_table* t, const GenArgs& g, uint32_t grid, size_t lds,
                        const AppendArgs& ap, uint32_t cus, hipStream_t s) {
  hipError_t e = hipSuccess;
  switch (t->S) {
    case 1:
      if ((e = launch_gen<1>(g, grid, lds, s)) != hipSuccess) return e;
      return append_b<1>(t->B, t->G, t->U, ap, cus, s);
    case 2:
      if ((e = launch_gen<2>(g, grid, lds, s)) != hipSuccess) return e;
      return append_b<2>(t->B, t->G, t->U, ap, cus, s);
    case 4:
      if ((e = launch_gen<4>(g, grid, lds, s)) != hipSuccess) return e;
      return append_b<4>(t->B, t->G, t->U, ap, cus, s);
  }
  return hipErrorInvalidValue;
}

// Grow a device buffer of `cap` elements of `elem` bytes to at least `need`
// elements, keeping its first `keep` elements.  Waits for the stream first.
hipError_t grow(void** p, uint64_t* cap, uint64_t need, size_t elem, uint64_t keep,
                hipStream_t stream, uint64_t limit) {
  if (*cap >= need && *p) return hipSuccess;
  // at least half again the old size (amortised growth), never above limit
  const uint64_t nc = std::max<uint64_t>(need, std::min<uint64_t>(limit, *cap + *cap / 2));
  void* q = nullptr;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  e = hipMalloc(&q, nc * elem);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  if (keep && *p) {
    e = hipMemcpy(q, *p, keep * elem, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      (void)hipFree(q);
      return e;
    }
  }
  if (*p) (void)hipFree(*p);
  *p = q;
  *cap = nc;
  return hipSuccess;
}


}  // namespace
}  // namespace gx

namespace gx {

// The control block of an exploration's buffers: the level counters (one
// cache line each), what a small-level launch reports, the initial state's
// slot and the network image.
constexpr size_t kCtrWords = kCtrCount * kCtrSpread;
constexpr size_t kBlockWords = kCtrWords + sizeof(SmallOut) / sizeof(uint64_t);
constexpr size_t kControlBytes =
    kBlockWords * sizeof(uint64_t) + 4 * sizeof(uint32_t) + kImgMaxWords * sizeof(uint32_t);

// Where gx_explore_noalloc puts its results.
struct FixedOut {
  uint64_t* level_counts;
  uint32_t max_levels;
  uint32_t* deadlocks;
  uint64_t max_deadlocks;
  gx_explore_summary* summary;
};

// Level counts: a growing host vector, or (fixed) the caller's array, which
// records an overflow instead of growing.
class LevelList {
 public:
  explicit LevelList(FixedOut* f) : f_(f) {}
  void push(uint64_t x) {
    if (f_) {
      if (n_ < f_->max_levels) f_->level_counts[n_] = x;
      else overflow_ = true;
    } else {
      vec_.push_back(x);
    }
    ++n_;
  }
  uint64_t size() const { return n_; }
  uint64_t at(uint64_t k) const { return f_ ? f_->level_counts[k] : vec_[k]; }
  bool overflow() const { return overflow_; }

 private:
  FixedOut* f_;
  std::vector<uint64_t> vec_;
  uint64_t n_ = 0;
  bool overflow_ = false;
};

template <int W>
int cmp_records(const void* a, const void* b) {
  const uint32_t* x = static_cast<const uint32_t*>(a);
  const uint32_t* y = static_cast<const uint32_t*>(b);
  for (int k = 0; k < W; ++k)
    if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
  return 0;
}

// Results of a fixed (no-alloc) exploration into the caller's arrays: the
// deadlock records (S words each on the device) are copied into the caller's
// array in chunks through a small host buffer, cut to w words and sorted.
gx_status finish_fixed(FixedOut& f, const LevelList& levels, uint64_t n_dead,
                       uint64_t transitions, const uint32_t* dead, uint32_t S, uint32_t w) {
  if (levels.overflow() || n_dead > f.max_deadlocks) return GX_ENOMEM;
  constexpr uint64_t kChunk = 1024;
  static thread_local uint32_t chunk[kChunk * 4];
  for (uint64_t i0 = 0; i0 < n_dead; i0 += kChunk) {
    const uint64_t n = std::min<uint64_t>(kChunk, n_dead - i0);
    if (hipMemcpy(chunk, dead + i0 * S, n * S * sizeof(uint32_t), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return GX_EDEVICE;
    for (uint64_t i = 0; i < n; ++i)
      for (uint32_t k = 0; k < w; ++k) f.deadlocks[(i0 + i) * w + k] = chunk[i * S + k];
  }
  static int (*const cmp[5])(const void*, const void*) = {nullptr, cmp_records<1>,
                                                          cmp_records<2>, cmp_records<3>,
                                                          cmp_records<4>};
  if (n_dead) std::qsort(f.deadlocks, n_dead, w * sizeof(uint32_t), cmp[w]);
  uint64_t n_states = 0;
  for (uint64_t k = 0; k < levels.size(); ++k) n_states += levels.at(k);
  f.summary->n_states = n_states;
  f.summary->n_transitions = transitions;
  f.summary->n_levels = static_cast<uint32_t>(levels.size());
  f.summary->words_per_state = w;
  f.summary->n_deadlocks = n_dead;
  return GX_OK;
}

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
  std::free(r->violations);
  std::free(r->states);
  r->level_counts = nullptr;
  r->deadlocks = nullptr;
  r->violations = nullptr;
  r->states = nullptr;
}

// The exploration of gx_explore into table t, with its device buffers in eb.
// fixed == nullptr: eb is the table's resident set, grown on demand, and the
// result arrays are malloc'd into out.  fixed != nullptr (gx_explore_noalloc):
// eb views preallocated memory that never grows (a buffer that would have to
// is GX_ENOMEM), the control block's host side is plain memory, and the
// level counts and deadlocks go to the caller's arrays in fixed.
static gx_status explore_impl(const gx_network* net, gx_table* t, const gx_explore_opts* opts,
                              gx_explore_buffers& eb, gx::FixedOut* fixed,
                              gx_explore_result* out) {
  gx::NetImage ni;
  // (with preallocated buffers the image must fit the control block)
  gx_status s = gx::compile_network(net, &ni, fixed ? gx::kImgMaxWords : gx::kImgGlobalMaxWords);
  if (s != GX_OK) return s;
  if (ni.words != t->w) return GX_EINVAL;
  const bool monitor = opts && opts->monitor_bad;
  if (monitor && (fixed || opts->monitor_proc >= ni.field.size())) return GX_EINVAL;
  // the table must be empty: its first levels are placed assuming so
  if (t->holds_states) return GX_EINVAL;
  const uint32_t S = t->S;
  const size_t state_bytes = S * sizeof(uint32_t);
  // 0: limited only by device memory
  const uint64_t max_cap = opts && opts->frontier_capacity ? opts->frontier_capacity : ~0ull;
  const uint64_t max_dead = opts && opts->deadlock_capacity ? opts->deadlock_capacity : ~0ull;
  hipStream_t stream = opts ? static_cast<hipStream_t>(opts->hip_stream) : nullptr;
  const uint64_t max_succ = std::max<uint64_t>(1, ni.max_succ);

  auto grow_buf = [&](uint32_t** p, uint64_t* cap, uint64_t need, uint64_t keep,
                      uint64_t limit) -> gx_status {
    if (*cap >= need && *p) return GX_OK;
    if (need > limit || fixed) return GX_ENOMEM;
    const uint64_t want = std::min<uint64_t>(limit, std::max<uint64_t>(need, 1u << 16));
    const hipError_t e = gx::grow(reinterpret_cast<void**>(p), cap, want, state_bytes, keep,
                                  stream, limit);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GX_ENOMEM;
    return e == hipSuccess ? GX_OK : GX_EDEVICE;
  };

  // resident buffers of the table (allocated on first use, grow-only)
  const uint32_t img_words = static_cast<uint32_t>(ni.img.size());
  // an image beyond the LDS budget stays in global memory (a buffer of its
  // own), read there by the generation kernel; such networks take no
  // small-level path (its kernels keep the image in LDS)
  const bool global_img = img_words > gx::kImgMaxWords;
  const uint32_t img_stride = global_img ? 0u : (img_words + 3) & ~3u;
  // the control block: the level's counters, what a small-level launch
  // reports (read back together), the initial state's slot, the image
  constexpr size_t kCtrWords = gx::kCtrWords;
  constexpr size_t kBlockWords = gx::kBlockWords;
  constexpr size_t kControlBytes = gx::kControlBytes;
  if (global_img) {
    if (fixed) return GX_EINVAL;
    if (eb.img_global_cap < img_words) {
      if (eb.img_global) (void)hipFree(eb.img_global);
      eb.img_global = nullptr;
      eb.img_global_cap = 0;
      if (hipMalloc(&eb.img_global, img_words * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return GX_ENOMEM;
      }
      eb.img_global_cap = img_words;
    }
    if (hipMemcpyAsync(eb.img_global, ni.img.data(), img_words * sizeof(uint32_t),
                       hipMemcpyHostToDevice, stream) != hipSuccess)
      return GX_EDEVICE;
  }
  if (!eb.ctr && (hipMalloc(&eb.ctr, kControlBytes) != hipSuccess ||
                  hipHostMalloc(&eb.ctr_host, kControlBytes) != hipSuccess ||
                  hipMalloc(&eb.status, 8) != hipSuccess)) {
    (void)hipGetLastError();
    return GX_ENOMEM;
  }
  eb.key = reinterpret_cast<uint32_t*>(eb.ctr + kBlockWords);
  eb.img = eb.key + 4;
  eb.img_cap = gx::kImgMaxWords;
  for (int k = 0; k < 2; ++k)
    if ((s = grow_buf(&eb.f[k], &eb.f_cap[k], 1, 0, max_cap)) != GX_OK) return s;
  if ((s = grow_buf(&eb.dead, &eb.dead_cap, 1, 0, max_dead)) != GX_OK) return s;
  // Small levels run on one workgroup (small_levels_kernel) when a level of
  // `small_limit` states has room for all its successors in the frontier and
  // successor buffers as they are; not with a safety monitor or the local
  // duplicate filter, whose per-level work stays on the host path.
  const bool dedup = opts && opts->local_dedup;
  uint64_t small_limit = 0;
  if (!monitor && !dedup && !global_img) {
    if ((s = grow_buf(&eb.succ, &eb.succ_cap, 1, 0, ~0ull)) != GX_OK) return s;
    const uint64_t room = std::min<uint64_t>(
        std::min<uint64_t>(eb.f_cap[0], eb.f_cap[1]),
        std::min<uint64_t>(eb.succ_cap, max_cap));
    small_limit = std::min<uint64_t>(
        gx::kSmallMaxLevel, std::min<uint64_t>(room, gx::kSmallSuccBudget) / max_succ);
  }

  uint32_t init[4] = {0, 0, 0, 0};
  gx::pack_host(ni, ni.initial.data(), init);
  // the level's counters, spread over cache lines on the device, read back
  // into pinned host memory
  uint64_t* ctr_raw = eb.ctr_host;
  const gx::SmallOut* small_out = reinterpret_cast<const gx::SmallOut*>(ctr_raw + kCtrWords);
  auto ctr = [&](uint32_t k) { return ctr_raw[k * gx::kCtrSpread]; };
  t->holds_states = true;  // from here on the exploration writes the table
  {
    // zeroed counters, the initial state's whole slot (a 3-word state's
    // fourth word is 0) and the image, up in one copy from pinned memory
    std::memset(ctr_raw, 0, kBlockWords * sizeof(uint64_t));
    uint32_t* hkey = reinterpret_cast<uint32_t*>(ctr_raw + kBlockWords);
    std::memcpy(hkey, init, 4 * sizeof(uint32_t));
    const uint32_t lds_img = global_img ? 0u : img_words;
    std::memcpy(hkey + 4, ni.img.data(), lds_img * sizeof(uint32_t));
    const size_t up = kBlockWords * sizeof(uint64_t) + (4 + lds_img) * sizeof(uint32_t);
    if (hipMemcpyAsync(eb.ctr, ctr_raw, up, hipMemcpyHostToDevice, stream) != hipSuccess)
      return GX_EDEVICE;
  }
  // the first level for the table-probing kernels (the small-level kernels
  // take the initial state from eb.key)
  if (small_limit == 0 &&
      hipMemcpyAsync(eb.f[0], eb.key, state_bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return GX_EDEVICE;
  // the initial state must be new, i.e. the table must not hold it yet (with
  // small levels, the first small launch inserts it)
  if (small_limit == 0) {
    if (gx::launch_find_or_put(t, eb.key, 1, eb.status, nullptr, stream) != hipSuccess)
      return GX_EDEVICE;
    uint8_t st0 = 0;
    if (hipMemcpyAsync(&st0, eb.status, 1, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GX_EDEVICE;
    if (st0 == gx::kFull) return GX_ETABLEFULL;
    if (st0 != gx::kNew) return GX_EINVAL;
  }

  // Safety monitor: a bitmask of the bad local states of the monitor
  // process; every completed level is scanned for states holding one.  The
  // initial state (level 0) is checked here.
  uint32_t mon_field = 0;
  std::vector<uint32_t> mon_mask;
  bool init_violates = false;
  uint32_t viol_level = 0xFFFFFFFFu;
  uint64_t viol_total = 0;  // violating states the device has recorded
  bool stop = false;
  if (monitor) {
    const uint32_t mp = opts->monitor_proc;
    const uint32_t n_local = net->procs[mp].n_states;
    mon_mask.assign((n_local + 31) / 32, 0u);
    for (uint32_t l = 0; l < n_local; ++l)
      if (opts->monitor_bad[l]) mon_mask[l >> 5] |= 1u << (l & 31);
    if (eb.mon_cap < mon_mask.size()) {
      if (eb.mon) (void)hipFree(eb.mon);
      eb.mon = nullptr;
      eb.mon_cap = 0;
      if (hipMalloc(&eb.mon, mon_mask.size() * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return GX_ENOMEM;
      }
      eb.mon_cap = mon_mask.size();
    }
    if (!eb.viol_ctr && hipMalloc(&eb.viol_ctr, sizeof(uint64_t)) != hipSuccess) {
      (void)hipGetLastError();
      return GX_ENOMEM;
    }
    if (hipMemcpy(eb.mon, mon_mask.data(), mon_mask.size() * sizeof(uint32_t),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(eb.viol_ctr, 0, sizeof(uint64_t), stream) != hipSuccess)
      return GX_EDEVICE;
    mon_field = ni.field[mp];
    if (opts->monitor_bad[ni.initial[mp]]) {
      init_violates = true;
      viol_level = 0;
      stop = opts->stop_on_violation != 0;
    }
  }

  gx::GenArgs g;
  g.img = global_img ? eb.img_global : eb.img;
  g.img_words = img_words;
  g.img_stride = img_stride;  // LDS words of the image (0: read from global memory)
  g.global_img = global_img ? 1u : 0u;
  g.ctr = eb.ctr;
  g.dedup = opts && opts->local_dedup ? 1u : 0u;
  gx::AppendArgs ap;
  ap.t = t->dev();
  ap.keys = nullptr;
  ap.n_keys = nullptr;  // per slice: the successor counter its generation uses
  ap.ctr = eb.ctr;
  ap.count_trans = g.dedup ? 0u : 1u;  // the filtered generation counts its own
  // a three-word state's successors go through the successor buffer as three
  // words, not as their four-word slots (a quarter less written and read;
  // the filtered generation stages whole slots)
  g.succ_words = S == 4 && t->w == 3 && !g.dedup ? 3u : S;
  g.pad = 0;
  ap.key_words = g.succ_words;
  const uint32_t dedup_words =
      g.dedup ? 4u * (S == 1 ? gx::dedup_entries<1>() : S == 2 ? gx::dedup_entries<2>()
                                                               : gx::dedup_entries<4>())
              : 0u;
  const size_t lds =
      (img_stride + (g.dedup ? gx::kStageWords + dedup_words : 0u) + 8) * sizeof(uint32_t);
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, t->device);
  auto read_ctr = [&]() -> gx_status {
    if (hipMemcpyAsync(ctr_raw, eb.ctr, kBlockWords * sizeof(uint64_t), hipMemcpyDeviceToHost,
                       stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GX_EDEVICE;
    if (ctr(gx::kCtrFlags) & gx::kFlagTableFull) return GX_ETABLEFULL;
    if (ctr(gx::kCtrFlags) & gx::kFlagFrontierOverflow) return GX_ENOMEM;
    if (ctr(gx::kCtrFlags) & gx::kFlagNotEmpty) return GX_EINVAL;
    return GX_OK;
  };

  // Levels are expanded in slices small enough that even if every successor
  // were new the next frontier could not overflow: slice * max_succ <= free
  // frontier room (and slice <= free deadlock room, one record per state at
  // most).  The room is tracked from these worst-case bounds; only when it is
  // short of a full slice is the exact fill read back (one synchronisation),
  // and the buffers grow, keeping their contents, to hold a full slice.
  gx::LevelList levels(fixed);
  levels.push(1);
  uint64_t n_in = 1;
  int cur = 0;
  uint64_t dead_known = 0;
  // 16384 workgroups per launch unless the caller asks for less
  const uint64_t kTargetSlice = opts && opts->slice_states ? opts->slice_states : 1u << 22;
  constexpr uint64_t kMaxRoom = 1ull << 28;    // states of frontier room one slice may claim
  uint64_t slice_no = 0;  // successor counters alternate from slice to slice
  bool init_inserted = small_limit == 0;
  while (n_in > 0 && !stop) {
    bool small = n_in <= small_limit;
    if (small && std::min<uint64_t>(eb.dead_cap, max_dead) - dead_known < n_in) {
      // every state of a small level may be a deadlock: room for a level
      s = grow_buf(&eb.dead, &eb.dead_cap, std::min<uint64_t>(dead_known + n_in, max_dead),
                   dead_known, max_dead);
      if (s != GX_OK && s != GX_ENOMEM) return s;
      small = std::min<uint64_t>(eb.dead_cap, max_dead) - dead_known >= n_in;
    }
    if (small) {
      // small levels on one workgroup, as many as stay small (up to
      // kSmallLevels per launch), then one read-back
      gx::SmallArgs sa;
      sa.t = t->dev();
      sa.img = eb.img;
      sa.img_words = img_words;
      sa.img_stride = img_stride;
      sa.f[0] = eb.f[0];
      sa.f[1] = eb.f[1];
      sa.f_cap = std::min<uint64_t>(std::min<uint64_t>(eb.f_cap[0], eb.f_cap[1]), max_cap);
      sa.cur = static_cast<uint32_t>(cur);
      sa.n_in = n_in;
      sa.succ = eb.succ;
      sa.succ_cap = eb.succ_cap;
      sa.dead = eb.dead;
      sa.dead_cap = std::min<uint64_t>(eb.dead_cap, max_dead);
      sa.ctr = eb.ctr;
      sa.out = reinterpret_cast<gx::SmallOut*>(eb.ctr + kCtrWords);
      sa.limit = small_limit;
      sa.init_key = init_inserted ? nullptr : eb.key;
      sa.set_mask = 0;
      sa.max_succ = static_cast<uint32_t>(max_succ);
      hipError_t e = hipErrorInvalidValue;
      bool lds_mode = false;
      if (!init_inserted) {
        // the first levels: LDS-resident while the table holds nothing else
        const size_t lds_limit = gx::lds_per_workgroup(t->device);
        switch (S) {
          case 1: e = gx::launch_lds_levels<1>(t->B, sa, lds_limit, stream); break;
          case 2: e = gx::launch_lds_levels<2>(t->B, sa, lds_limit, stream); break;
          case 4: e = gx::launch_lds_levels<4>(t->B, sa, lds_limit, stream); break;
        }
        lds_mode = e == hipSuccess;
        if (!lds_mode) (void)hipGetLastError();
      }
      if (!lds_mode) {
        switch (S) {
          case 1: e = gx::launch_small<1>(t->B, sa, stream); break;
          case 2: e = gx::launch_small<2>(t->B, sa, stream); break;
          case 4: e = gx::launch_small<4>(t->B, sa, stream); break;
        }
      }
      if (e != hipSuccess) return GX_EDEVICE;
      if ((s = read_ctr()) != GX_OK) return s;
      if (!init_inserted) {
        init_inserted = true;
        if (small_out->init_status == gx::kFull) return GX_ETABLEFULL;
        if (small_out->init_status != gx::kNew) return GX_EINVAL;
      }
      for (uint64_t k = 0; k < small_out->n_levels; ++k) levels.push(small_out->levels[k]);
      dead_known = ctr(gx::kCtrDead);
      if (dead_known > std::min<uint64_t>(eb.dead_cap, max_dead)) return GX_ENOMEM;
      n_in = small_out->n_in;
      cur = static_cast<int>(small_out->cur);
      // (an LDS-resident launch may hand its first level straight to the
      // table-probing kernels)
      if (!lds_mode && small_out->n_levels == 0 && n_in > 0) return GX_EDEVICE;  // no progress
      continue;
    }
    const int nxt = cur ^ 1;
    uint64_t tail_known = 0, bound = 0, dead_bound = dead_known, pos = 0;
    while (pos < n_in) {
      // full slices, but never more than kMaxRoom states of frontier room
      const uint64_t want = std::min<uint64_t>(
          n_in - pos, std::min<uint64_t>(kTargetSlice, std::max<uint64_t>(1, kMaxRoom / max_succ)));
      // usable capacities: a buffer left larger by an earlier call still
      // honours this call's limits
      auto f_cap = [&]() { return std::min<uint64_t>(eb.f_cap[nxt], max_cap); };
      auto d_cap = [&]() { return std::min<uint64_t>(eb.dead_cap, max_dead); };
      auto f_room = [&]() { return (f_cap() - bound) / max_succ; };
      // a deadlock buffer at its limit no longer bounds the slice: records
      // past it are counted, not stored, and the call ends with GX_ENOMEM
      auto d_room = [&]() { return d_cap() >= max_dead ? ~0ull : d_cap() - dead_bound; };
      if (std::min<uint64_t>(f_room(), d_room()) < want) {
        if (bound != tail_known || dead_bound != dead_known) {
          if ((s = read_ctr()) != GX_OK) return s;
          tail_known = bound = ctr(gx::kCtrTail);
          dead_known = dead_bound = ctr(gx::kCtrDead);
        }
        if (f_room() < want) {
          s = grow_buf(&eb.f[nxt], &eb.f_cap[nxt], bound + want * max_succ, tail_known, max_cap);
          if (s == GX_ENOMEM)  // no room for a full slice: settle for one state
            s = grow_buf(&eb.f[nxt], &eb.f_cap[nxt], bound + max_succ, tail_known,
                         std::min<uint64_t>(max_cap, bound + max_succ));
          if (s != GX_OK) return s;
        }
        if (d_room() < want) {
          s = grow_buf(&eb.dead, &eb.dead_cap, std::min<uint64_t>(dead_bound + want, max_dead),
                       std::min<uint64_t>(dead_known, eb.dead_cap), max_dead);
          if (s != GX_OK) return s;
        }
      }
      const uint64_t slice = std::min<uint64_t>(want, std::min<uint64_t>(f_room(), d_room()));
      if (slice == 0) return GX_ENOMEM;
      // the slice's successors (all of them, in the worst case) fit the
      // successor buffer
      const uint64_t slice_keys = slice * max_succ;
      if (eb.succ_cap < slice_keys) {
        s = grow_buf(&eb.succ, &eb.succ_cap, slice_keys, 0, ~0ull);
        if (s == GX_ENOMEM)  // settle for what fits, at least one state
          s = grow_buf(&eb.succ, &eb.succ_cap, max_succ, 0, ~0ull);
        if (s != GX_OK) return s;
      }
      const uint64_t run = std::min<uint64_t>(slice, eb.succ_cap / max_succ);
      g.frontier_in = eb.f[cur] + pos * S;
      g.n_in = run;
      g.succ = eb.succ;
      g.succ_cap = eb.succ_cap;
      g.dead = eb.dead;
      g.dead_cap = d_cap();
      ap.keys = eb.succ;
      ap.keys_cap = eb.succ_cap;
      ap.frontier_out = eb.f[nxt];
      ap.cap_out = f_cap();
      // the first slice's generation clears the next-frontier tail; each
      // slice's clears the other successor counter for the next slice
      g.reset_tail = pos == 0 ? 1u : 0u;
      g.succ_ctr = (slice_no++ & 1) ? gx::kCtrSuccAlt : gx::kCtrSucc;
      ap.n_keys = eb.ctr + g.succ_ctr * gx::kCtrSpread;
      const uint64_t grid = (run + 255) / 256;
      if (gx::launch_slice(t, g, static_cast<uint32_t>(grid), lds, ap, static_cast<uint32_t>(cus),
                           stream) != hipSuccess)
        return GX_EDEVICE;
      pos += run;
      bound += run * max_succ;
      dead_bound += run;
    }
    if ((s = read_ctr()) != GX_OK) return s;
    dead_known = ctr(gx::kCtrDead);
    n_in = ctr(gx::kCtrTail);
    if (n_in) levels.push(n_in);
    if (monitor && n_in) {
      // scan the level just completed; if the record buffer was short, grow
      // it (keeping earlier levels' records) and scan the level again
      const uint64_t prev = viol_total;
      for (int pass = 0; pass < 2; ++pass) {
        if (gx::launch_monitor_scan(S, eb.f[nxt], n_in, mon_field, eb.mon, eb.viol, eb.viol_cap,
                                    eb.viol_ctr, static_cast<uint32_t>(cus), stream) !=
            hipSuccess)
          return GX_EDEVICE;
        uint64_t got = 0;
        if (hipMemcpyAsync(&got, eb.viol_ctr, sizeof(got), hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
          return GX_EDEVICE;
        viol_total = got;
        if (got <= eb.viol_cap) break;
        if ((s = grow_buf(&eb.viol, &eb.viol_cap, got, prev, ~0ull)) != GX_OK) return s;
        if (hipMemcpy(eb.viol_ctr, &prev, sizeof(prev), hipMemcpyHostToDevice) != hipSuccess)
          return GX_EDEVICE;
      }
      if (viol_total > prev) {
        if (viol_level == 0xFFFFFFFFu) viol_level = static_cast<uint32_t>(levels.size() - 1);
        if (opts->stop_on_violation) stop = true;
      }
    }
    cur = nxt;
  }
  const uint64_t n_dead = ctr(gx::kCtrDead);
  if (n_dead > std::min<uint64_t>(eb.dead_cap, max_dead)) return GX_ENOMEM;
  if (fixed) return gx::finish_fixed(*fixed, levels, n_dead, ctr(gx::kCtrTrans), eb.dead, S, t->w);
  std::vector<uint32_t> raw(n_dead * S);
  if (n_dead && hipMemcpy(raw.data(), eb.dead, raw.size() * sizeof(uint32_t),
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
  for (uint64_t k = 0; k < levels.size(); ++k) {
    lv[k] = levels.at(k);
    n_states += levels.at(k);
  }
  for (uint64_t i = 0; i < n_dead; ++i)
    for (uint32_t k = 0; k < t->w; ++k) dd[i * t->w + k] = dl[i][k];
  out->n_states = n_states;
  out->n_transitions = ctr(gx::kCtrTrans);
  out->words_per_state = t->w;
  out->n_levels = static_cast<uint32_t>(levels.size());
  out->level_counts = lv;
  out->n_deadlocks = n_dead;
  out->deadlocks = dd;
  out->local_duplicates = ctr(gx::kCtrDups);
  out->n_violations = 0;
  out->violations = nullptr;
  out->violation_level = viol_level;
  out->reserved = 0;
  out->states = nullptr;
  if (monitor) {
    std::vector<uint32_t> vraw(viol_total * S);
    if (viol_total && hipMemcpy(vraw.data(), eb.viol, vraw.size() * sizeof(uint32_t),
                                hipMemcpyDeviceToHost) != hipSuccess) {
      gx_explore_result_free(out);
      return GX_EDEVICE;
    }
    std::vector<std::array<uint32_t, 4>> vl(viol_total);
    for (uint64_t i = 0; i < viol_total; ++i) {
      vl[i] = {0, 0, 0, 0};
      for (uint32_t k = 0; k < t->w; ++k) vl[i][k] = vraw[i * S + k];
    }
    if (init_violates) vl.push_back({init[0], init[1], init[2], init[3]});
    std::sort(vl.begin(), vl.end());
    uint32_t* vv = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (vl.size() * t->w + 1)));
    if (!vv) {
      gx_explore_result_free(out);
      return GX_ENOMEM;
    }
    for (size_t i = 0; i < vl.size(); ++i)
      for (uint32_t k = 0; k < t->w; ++k) vv[i * t->w + k] = vl[i][k];
    out->n_violations = vl.size();
    out->violations = vv;
  }
  return GX_OK;
}

gx_status gx_explore(const gx_network* net, gx_table* t, const gx_explore_opts* opts,
                     gx_explore_result* out) {
  if (!t || !out) return GX_EINVAL;
  return explore_impl(net, t, opts, t->eb, nullptr, out);
}

}  // extern "C"

// ---------------------------------------------------- no-alloc exploration
// Every device buffer gx_explore_noalloc needs beyond the table: one array
// per GPU the library runs on, held until the process ends.  In host code
// the name `scratch` is only a stand-in; its device address comes from
// hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) uint8_t scratch[GX_NOALLOC_SCRATCH_BYTES];

namespace gx {
namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};

// The device address of this GPU's scratch array, looked up once per device
// (with that device current) and kept.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_dev[device] = p;
  }
  return scratch_dev[device];
}

}  // namespace
}  // namespace gx

extern "C" {

gx_status gx_explore_noalloc(const gx_network* net, gx_table* t, const gx_explore_opts* opts,
                             uint64_t* level_counts, uint32_t max_levels, uint32_t* deadlocks,
                             uint64_t max_deadlocks, gx_explore_summary* out) {
  if (!t || !out || !level_counts || max_levels == 0 || (max_deadlocks && !deadlocks))
    return GX_EINVAL;
  if (opts && opts->monitor_bad) return GX_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  if (dev != t->device) return GX_EINVAL;
  char* base = static_cast<char*>(gx::scratch_address(dev));
  if (!base) return GX_EDEVICE;
  // control block | status | frontier 0 | frontier 1 | successors | deadlocks
  constexpr uint64_t kCtl = (gx::kControlBytes + 65535) / 65536 * 65536;
  constexpr uint64_t kRegion = (GX_NOALLOC_SCRATCH_BYTES - kCtl - 256) / 4 / 256 * 256;
  static_assert(kCtl + 256 + 4 * kRegion <= GX_NOALLOC_SCRATCH_BYTES, "scratch layout");
  const uint64_t cap = kRegion / (t->S * sizeof(uint32_t));
  static thread_local uint64_t host_block[(gx::kControlBytes + 7) / 8];
  gx_explore_buffers eb;  // views of the scratch array; never grown
  eb.ctr = reinterpret_cast<uint64_t*>(base);
  eb.ctr_host = host_block;
  eb.status = reinterpret_cast<uint8_t*>(base + kCtl);
  char* r = base + kCtl + 256;
  eb.f[0] = reinterpret_cast<uint32_t*>(r);
  eb.f[1] = reinterpret_cast<uint32_t*>(r + kRegion);
  eb.succ = reinterpret_cast<uint32_t*>(r + 2 * kRegion);
  eb.dead = reinterpret_cast<uint32_t*>(r + 3 * kRegion);
  eb.f_cap[0] = eb.f_cap[1] = eb.succ_cap = eb.dead_cap = cap;
  gx::FixedOut f{level_counts, max_levels, deadlocks, max_deadlocks, out};
  gx_explore_result unused{};
  return explore_impl(net, t, opts, eb, &f, &unused);
}

}  // extern "C"
