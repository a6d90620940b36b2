// Batched exploration (many networks explored together, each in its own table
// partition) and the find-or-put autotuner.
//
// Two schedules.  Stepped (the default): every unfinished instance advances
// one BFS level per step; a step is one multi-instance launch per kernel
// class (the server's step kernel over the concatenated tiles of the class's
// current levels), a summary kernel per class that copies each instance's
// next-level size and flags into a compact array and clears its tail, and
// one read-back of those arrays; gx_batch_run returns when every instance has
// finished.  Persistent (with use_graph or persistent): one persistent launch
// per class pulls (instance, level, tile) work from a device queue with no
// host involvement, so a whole run can be captured in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "gx_batch_kernel.hpp"
#include "gx_serve_kernel.hpp"

namespace gx {

// implemented in gx_explore.hip
gx_status compile_network_image(const gx_network* net, std::vector<uint32_t>* img,
                                uint32_t* words, std::vector<uint32_t>* packed_initial,
                                uint64_t* max_succ);

// instantiated in gx_batch_s1.hip, gx_batch_s2.hip, gx_batch_s4.hip
template <int S>
hipError_t batch_launch(uint32_t B, uint32_t G, uint32_t U, const BatchArgs& a, uint32_t grid,
                        size_t lds, hipStream_t s);
template <int S>
int batch_resident(uint32_t B, uint32_t G, uint32_t U, size_t lds);
extern template hipError_t batch_launch<1>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t batch_launch<2>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t batch_launch<4>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template int batch_resident<1>(uint32_t, uint32_t, uint32_t, size_t);
extern template int batch_resident<2>(uint32_t, uint32_t, uint32_t, size_t);
extern template int batch_resident<4>(uint32_t, uint32_t, uint32_t, size_t);
template <int S>
hipError_t batch_init(uint32_t B, uint32_t G, uint32_t U, const BatchArgs& a, hipStream_t s);
extern template hipError_t batch_init<1>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                         hipStream_t);
extern template hipError_t batch_init<2>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                         hipStream_t);
extern template hipError_t batch_init<4>(uint32_t, uint32_t, uint32_t, const BatchArgs&,
                                         hipStream_t);
// instantiated in gx_serve_s1.hip, gx_serve_s2.hip, gx_serve_s4.hip
extern template hipError_t serve_launch<1>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t serve_launch<2>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t serve_launch<4>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);

namespace {

constexpr uint32_t kDefaultMaxLevels = 4096;
constexpr uint64_t kSpinLimit = 1ull << 23;  // polls of one to two microseconds each

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- autotuner
// Tables are tuned per size class: a table's size decides where most of its
// buckets live (an XCD's L2, the last-level cache or HBM), and with it the
// cost of a probe.  Classes: up to 2^16, 2^20, 2^24 slots, and larger.
constexpr uint32_t kSizeClasses = 4;

uint32_t size_class(uint64_t capacity) {
  if (capacity <= (uint64_t(1) << 16)) return 0;
  if (capacity <= (uint64_t(1) << 20)) return 1;
  if (capacity <= (uint64_t(1) << 24)) return 2;
  return 3;
}

struct TuneKey {
  uint32_t S;
  uint32_t load_pct;
  uint32_t size_class;
  bool operator<(const TuneKey& o) const {
    return std::tie(S, load_pct, size_class) < std::tie(o.S, o.load_pct, o.size_class);
  }
};
std::map<TuneKey, gx_tune_info> g_tuned;
std::mutex g_tune_mutex;
constexpr uint32_t kDefaultB = 16, kDefaultG = 4;  // kept unless beaten by > 3%

__global__ void tune_keys_kernel(uint32_t* keys, uint32_t S, uint64_t n, uint64_t n_distinct,
                                 uint64_t seed) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // position i holds distinct key (i * odd) mod n_distinct: each key about
  // n / n_distinct times, far apart in the stream
  const uint64_t d = (i * 0x9E3779B97F4A7C15ull >> 11) % n_distinct;
  const uint64_t x = fmix64(d ^ seed);
  for (uint32_t k = 0; k < S; ++k)
    keys[i * S + k] = static_cast<uint32_t>((k & 1) ? (x >> 33) : (x & 0x7FFFFFFFu)) ^ k;
}

// After a step of the stepped schedule: instance k's next-level size and
// flags to sum[2k], sum[2k + 1]; its next-level tail cleared for the step
// after.
__global__ void batch_step_summary_kernel(BatchState* state, uint32_t n, uint64_t* sum) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint64_t* c = state[k].ctr;
  sum[2 * k] = c[kCtrTail * kCtrSpread];
  sum[2 * k + 1] = c[kCtrFlags * kCtrSpread];
  c[kCtrTail * kCtrSpread] = 0;
}

}  // namespace
}  // namespace gx

struct gx_batch {
  struct Class {
    uint32_t S = 0, B = 0, G = 0, U = 0;
    std::vector<uint32_t> members;  // instance ids
    // device
    gx::BatchInst* inst = nullptr;
    std::vector<gx::BatchInst> h_inst;  // host copy of inst
    gx::BatchState* state = nullptr;
    gx::BatchState* state_init = nullptr;
    gx::BatchEntry* queue = nullptr;
    gx::BatchEntry* queue_init = nullptr;
    uint32_t queue_cap = 0;
    gx::BatchGlobal* g = nullptr;
    gx::BatchGlobal* g_init = nullptr;
    uint32_t* img = nullptr;
    uint32_t img_stride = 0;
    uint32_t* init_states = nullptr;  // n_c x S
    uint32_t* tables = nullptr;
    uint64_t table_words = 0;
    uint32_t* frontiers = nullptr;
    uint64_t* levels = nullptr;
    uint32_t* dead = nullptr;
    uint32_t* dead_tag = nullptr;
    uint64_t dead_cap = 0;
    uint64_t* stats = nullptr;  // table counters the descriptors point at (not updated)
    uint32_t grid = 0;
    size_t lds = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_done = nullptr;
    // stepped schedule: job descriptors (device, pinned staging) and the
    // per-step summary (device, pinned read-back), nc entries each
    gx::ServeJob* d_jobs = nullptr;
    gx::ServeJob* h_jobs = nullptr;
    uint64_t* d_sum = nullptr;
    uint64_t* h_sum = nullptr;
  };
  int device = 0;
  uint32_t n = 0;
  uint32_t max_levels = 0;
  uint64_t* hc = nullptr;  // hash constants shared by every table
  uint64_t seed = 0;
  uint32_t H = 8;
  std::vector<uint32_t> w, cls;  // per instance: words, class index
  std::vector<uint32_t> Bi, Gi, Ui;
  std::vector<uint64_t> tab_off, tab_words;  // per instance: its table partition in its class
  bool keep_states = false;
  std::vector<Class> classes;
  hipEvent_t ev_fork = nullptr;
  bool use_graph = false;
  bool stepped = false;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture_stream = nullptr;
  bool ran = false;
  // the last stepped run: per instance, its level counts and status
  std::vector<std::vector<uint64_t>> step_levels;
  std::vector<gx_status> step_status;
};

namespace gx {
namespace {

void free_batch(gx_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (auto& c : b->classes) {
    for (void* p : {static_cast<void*>(c.inst), static_cast<void*>(c.state),
                    static_cast<void*>(c.state_init), static_cast<void*>(c.queue),
                    static_cast<void*>(c.queue_init), static_cast<void*>(c.g),
                    static_cast<void*>(c.g_init), static_cast<void*>(c.img),
                    static_cast<void*>(c.init_states), static_cast<void*>(c.tables),
                    static_cast<void*>(c.frontiers), static_cast<void*>(c.levels),
                    static_cast<void*>(c.dead), static_cast<void*>(c.dead_tag),
                    static_cast<void*>(c.stats)})
      if (p) (void)hipFree(p);
    if (c.side) (void)hipStreamDestroy(c.side);
    if (c.ev_done) (void)hipEventDestroy(c.ev_done);
    if (c.d_jobs) (void)hipFree(c.d_jobs);
    if (c.d_sum) (void)hipFree(c.d_sum);
    if (c.h_jobs) (void)hipHostFree(c.h_jobs);
    if (c.h_sum) (void)hipHostFree(c.h_sum);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->hc) (void)hipFree(b->hc);
  delete b;
}

template <typename T>
hipError_t dmalloc(T** p, uint64_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<uint64_t>(1, count) * sizeof(T));
}

BatchArgs class_args(const gx_batch::Class& c) {
  BatchArgs a;
  a.inst = c.inst;
  a.state = c.state;
  a.queue = c.queue;
  a.queue_cap = c.queue_cap;
  a.g = c.g;
  a.n = static_cast<uint32_t>(c.members.size());
  a.img = c.img;
  a.img_stride = c.img_stride;
  a.dead = c.dead;
  a.dead_tag = c.dead_tag;
  a.dead_cap = c.dead_cap;
  a.spin_limit = kSpinLimit;
  a.init_states = c.init_states;
  return a;
}

// Enqueue one full run of the batch on `stream`: reset every class, then the
// persistent launch of each class on its own stream, joined back.
hipError_t enqueue_run(gx_batch* b, hipStream_t stream) {
  hipError_t e = hipEventRecord(b->ev_fork, stream);
  if (e != hipSuccess) return e;
  for (auto& c : b->classes) {
    const uint32_t nc = static_cast<uint32_t>(c.members.size());
    if ((e = hipStreamWaitEvent(c.side, b->ev_fork, 0)) != hipSuccess) return e;
    if ((e = fill_words(c.tables, c.table_words, kEmpty, b->device, c.side)) != hipSuccess) return e;
    // every queue slot must read "not ready" until a finisher publishes it:
    // zero the whole queue, then put the initial levels in front
    if ((e = fill_words(reinterpret_cast<uint32_t*>(c.queue),
                        static_cast<uint64_t>(c.queue_cap) * (sizeof(BatchEntry) / 4), 0,
                        b->device, c.side)) != hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(c.state, c.state_init, nc * sizeof(BatchState),
                            hipMemcpyDeviceToDevice, c.side)) != hipSuccess ||
        (e = hipMemcpyAsync(c.queue, c.queue_init, nc * sizeof(BatchEntry),
                            hipMemcpyDeviceToDevice, c.side)) != hipSuccess ||
        (e = hipMemcpyAsync(c.g, c.g_init, sizeof(BatchGlobal), hipMemcpyDeviceToDevice,
                            c.side)) != hipSuccess)
      return e;
    const BatchArgs a = class_args(c);
    switch (c.S) {
      case 1: e = batch_launch<1>(c.B, c.G, c.U, a, c.grid, c.lds, c.side); break;
      case 2: e = batch_launch<2>(c.B, c.G, c.U, a, c.grid, c.lds, c.side); break;
      default: e = batch_launch<4>(c.B, c.G, c.U, a, c.grid, c.lds, c.side); break;
    }
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(c.ev_done, c.side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(stream, c.ev_done, 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// One whole run under the stepped schedule on `stream` (see the top of this
// file); synchronous.  The per-instance outcome goes to b->step_levels and
// b->step_status.
gx_status run_stepped(gx_batch* b, hipStream_t stream) {
  const size_t nk = b->classes.size();
  std::vector<std::vector<uint64_t>> n_in(nk);
  std::vector<std::vector<uint8_t>> cur(nk), live(nk);
  b->step_levels.assign(b->n, std::vector<uint64_t>(1, 1));
  b->step_status.assign(b->n, GX_OK);
  for (size_t ci = 0; ci < nk; ++ci) {
    gx_batch::Class& c = b->classes[ci];
    const uint32_t nc = static_cast<uint32_t>(c.members.size());
    n_in[ci].assign(nc, 1);
    cur[ci].assign(nc, 0);
    live[ci].assign(nc, 1);
    // clear the tables, reset the counters and the shared deadlock count,
    // put and insert every initial state
    if (fill_words(c.tables, c.table_words, kEmpty, b->device, stream) != hipSuccess ||
        hipMemcpyAsync(c.state, c.state_init, nc * sizeof(BatchState), hipMemcpyDeviceToDevice,
                       stream) != hipSuccess ||
        hipMemcpyAsync(c.g, c.g_init, sizeof(BatchGlobal), hipMemcpyDeviceToDevice, stream) !=
            hipSuccess)
      return GX_EDEVICE;
    const BatchArgs a = class_args(c);
    hipError_t e;
    switch (c.S) {
      case 1: e = batch_init<1>(c.B, c.G, c.U, a, stream); break;
      case 2: e = batch_init<2>(c.B, c.G, c.U, a, stream); break;
      default: e = batch_init<4>(c.B, c.G, c.U, a, stream); break;
    }
    if (e != hipSuccess) return GX_EDEVICE;
  }
  while (true) {
    bool any = false;
    // the classes' launches of a step run side by side, each on its own
    // stream, forked from and joined to `stream`
    if (hipEventRecord(b->ev_fork, stream) != hipSuccess) return GX_EDEVICE;
    for (size_t ci = 0; ci < nk; ++ci) {
      gx_batch::Class& c = b->classes[ci];
      const uint32_t nc = static_cast<uint32_t>(c.members.size());
      uint32_t n_jobs = 0;
      uint64_t tiles = 0;
      for (uint32_t k = 0; k < nc; ++k) {
        if (!live[ci][k]) continue;
        // the descriptor from the instance's static part (BatchInst, mirrored
        // on the host at creation) and its current level
        ServeJob& x = c.h_jobs[n_jobs++];
        const BatchInst& in = c.h_inst[k];
        x.t = in.t;
        x.img_off = in.img_off;
        x.img_words = in.img_words;
        x.frontier_in = in.f[cur[ci][k]];
        x.n_in = n_in[ci][k];
        x.frontier_out = in.f[cur[ci][k] ^ 1];
        x.cap_out = in.cap;
        x.dead = c.dead;
        x.dead_cap = c.dead_cap;
        x.ctr = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(c.state) +
                                            k * sizeof(BatchState) + offsetof(BatchState, ctr));
        x.tile_begin = tiles;
        x.dead_ctr = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(c.g) +
                                                 offsetof(BatchGlobal, dead_used));
        x.dead_tag = c.dead_tag;
        x.tag = k;
        x.pad = 0;
        tiles += (n_in[ci][k] + 255) / 256;
      }
      if (n_jobs == 0) continue;
      any = true;
      if (tiles > 0x7FFFFFFFull) return GX_EINVAL;
      ServeArgs sa;
      sa.jobs = c.d_jobs;
      sa.n_jobs = n_jobs;
      sa.img = c.img;
      sa.img_stride = c.img_stride;
      const hipStream_t cs = c.side;
      hipError_t e = hipStreamWaitEvent(cs, b->ev_fork, 0);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c.d_jobs, c.h_jobs, n_jobs * sizeof(ServeJob), hipMemcpyHostToDevice,
                           cs);
      if (e == hipSuccess) {
        const uint32_t grid = static_cast<uint32_t>(tiles);
        switch (c.S) {
          case 1: e = serve_launch<1>(c.B, c.G, c.U, sa, grid, c.lds, cs); break;
          case 2: e = serve_launch<2>(c.B, c.G, c.U, sa, grid, c.lds, cs); break;
          default: e = serve_launch<4>(c.B, c.G, c.U, sa, grid, c.lds, cs); break;
        }
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_step_summary_kernel, dim3((nc + 255) / 256), dim3(256), 0, cs,
                           c.state, nc, c.d_sum);
        e = hipGetLastError();
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(c.h_sum, c.d_sum, 2ull * nc * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           cs);
      if (e == hipSuccess) e = hipEventRecord(c.ev_done, cs);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, c.ev_done, 0);
      if (e != hipSuccess) return GX_EDEVICE;
    }
    if (!any) break;
    // one synchronisation per step (every class joined `stream`): the staged
    // descriptors of this step are reused only after it
    if (hipStreamSynchronize(stream) != hipSuccess) return GX_EDEVICE;
    for (size_t ci = 0; ci < nk; ++ci) {
      gx_batch::Class& c = b->classes[ci];
      const uint32_t nc = static_cast<uint32_t>(c.members.size());
      for (uint32_t k = 0; k < nc; ++k) {
        if (!live[ci][k]) continue;
        const uint32_t i = c.members[k];
        const uint64_t n_next = c.h_sum[2 * k], flags = c.h_sum[2 * k + 1];
        std::vector<uint64_t>& L = b->step_levels[i];
        gx_status st = GX_OK;
        bool done = true;
        if (flags & kFlagTableFull) st = GX_ETABLEFULL;
        else if (flags) st = GX_ENOMEM;
        else if (n_next == 0) st = GX_OK;
        else if (L.size() >= b->max_levels) st = GX_ENOMEM;  // deeper than max_levels
        else done = false;
        if (done) {
          live[ci][k] = 0;
          b->step_status[i] = st;
        } else {
          L.push_back(n_next);
          n_in[ci][k] = n_next;
          cur[ci][k] ^= 1;
        }
      }
    }
  }
  return GX_OK;
}

bool valid_pow2(uint32_t x, uint32_t lo, uint32_t hi) {
  return x >= lo && x <= hi && (x & (x - 1)) == 0;
}

// Times every candidate (B in 8..64 words, subgroup 4 (B <= 32), 8 or 16; one
// key in flight per subgroup, as the exploration kernels keep) on a stream
// shaped like an exploration's successor lookups: every distinct key about
// dup times, shuffled, into a table of the class's size filled to `load` by
// the end.  One measurement runs the stream r times back to back (clearing
// the table before each run; the clears are timed alone and subtracted), at
// least 2^25 keys in all; a candidate's time is the median of three
// measurements.  The pick is the fastest candidate, unless the default
// (B = 16, subgroup 4) is within 3% of it: near-ties keep the default, so
// that run-to-run noise does not flip the choice.
gx_status tune_class(uint32_t S, double load, uint32_t sc, gx_tune_info* out) {
  // capacity (states) of the timed table: the top of the class (2^25 for the
  // open-ended last class)
  const uint64_t cap_states = sc == 0 ? (uint64_t(1) << 16)
                              : sc == 1 ? (uint64_t(1) << 20)
                              : sc == 2 ? (uint64_t(1) << 24)
                                        : (uint64_t(1) << 25);
  const uint64_t n_distinct =
      std::max<uint64_t>(1024, static_cast<uint64_t>(static_cast<double>(cap_states) * load));
  const uint64_t dup = std::max<uint64_t>(2, std::min<uint64_t>(8, (uint64_t(1) << 26) / n_distinct));
  const uint64_t n = n_distinct * dup;
  const uint64_t reps = std::max<uint64_t>(1, (uint64_t(1) << 25) / n);
  const uint64_t slots = static_cast<uint64_t>(static_cast<double>(n_distinct) / load) + 1;
  uint32_t* keys = nullptr;
  uint8_t* status = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (keys) (void)hipFree(keys);
    if (status) (void)hipFree(status);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&keys, n * S * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&status, n) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return GX_ENOMEM;
  }
  hipLaunchKernelGGL(tune_keys_kernel, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0,
                     nullptr, keys, S, n, n_distinct, 0x5EEDull);
  // wall time on the device of `reps` runs of (clear, and find-or-put of the
  // stream unless clear_only)
  auto time_runs = [&](gx_table* t, bool clear_only, float* ms) -> bool {
    if (hipEventRecord(e0, nullptr) != hipSuccess) return false;
    for (uint64_t r = 0; r < reps; ++r) {
      if (gx_table_clear(t, nullptr) != GX_OK) return false;
      if (!clear_only && gx_find_or_put(t, keys, n, status, nullptr, nullptr) != GX_OK) return false;
    }
    return hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(ms, e0, e1) == hipSuccess;
  };
  struct Cand {
    uint32_t B, G;
    double ns;
  };
  std::vector<Cand> cands;
  gx_status st = GX_OK;
  for (uint32_t B : {8u, 16u, 32u, 64u}) {
    if (B < S * 2) continue;
    for (uint32_t G : {4u, 8u, 16u}) {
      if (G == 4 && B > 32) continue;
      gx_table_opts o{0, 64, G, 1, 0};
      gx_table* t = nullptr;
      if (gx_table_create(S, B, slots, &o, &t) != GX_OK) {
        st = GX_ENOMEM;
        continue;
      }
      float clear_ms = 0, ms[3] = {0, 0, 0};
      bool ok = time_runs(t, false, &ms[0]);  // warm-up
      ok = ok && time_runs(t, true, &clear_ms);
      for (int m = 0; m < 3 && ok; ++m) ok = time_runs(t, false, &ms[m]);
      gx_table_destroy(t);
      if (!ok) {
        st = GX_EDEVICE;
        continue;
      }
      std::sort(ms, ms + 3);
      const double work = std::max(1e-6, static_cast<double>(ms[1] - clear_ms));
      cands.push_back({B, G, work * 1e6 / static_cast<double>(reps * n)});
    }
  }
  cleanup();
  if (cands.empty()) return st == GX_OK ? GX_EDEVICE : st;
  size_t best = 0, def = cands.size();
  for (size_t k = 0; k < cands.size(); ++k) {
    if (cands[k].ns < cands[best].ns) best = k;
    if (cands[k].B == kDefaultB && cands[k].G == kDefaultG) def = k;
  }
  size_t pick = best;
  if (def < cands.size() && cands[def].ns <= cands[best].ns * 1.03) pick = def;
  double runner = 0;
  for (size_t k = 0; k < cands.size(); ++k)
    if (k != pick && (runner == 0 || cands[k].ns < runner)) runner = cands[k].ns;
  out->bucket_words = cands[pick].B;
  out->subgroup = cands[pick].G;
  out->keys_per_subgroup = 1;
  out->candidates = static_cast<uint32_t>(cands.size());
  out->ns_per_key = cands[pick].ns;
  out->ns_per_key_default = def < cands.size() ? cands[def].ns : 0.0;
  out->ns_per_key_runner_up = runner;
  out->table_slots = slots;
  out->size_class = sc;
  out->pad = 0;
  return GX_OK;
}

}  // namespace
}  // namespace gx

// ====================================================================== ABI
extern "C" {

gx_status gx_autotune_capacity(uint32_t w, double load, uint64_t capacity, gx_tune_info* info) {
  if (w < 1 || w > 4 || !(load > 0.0) || load > 0.95 || capacity == 0 || !info)
    return GX_EINVAL;
  const uint32_t S = gx::slot_words(w);
  const gx::TuneKey key{S, static_cast<uint32_t>(load * 100.0 + 0.5), gx::size_class(capacity)};
  std::lock_guard<std::mutex> lock(gx::g_tune_mutex);
  auto it = gx::g_tuned.find(key);
  if (it == gx::g_tuned.end()) {
    gx_tune_info t{};
    const gx_status st = gx::tune_class(S, load, key.size_class, &t);
    if (st != GX_OK) return st;
    it = gx::g_tuned.emplace(key, t).first;
  }
  *info = it->second;
  return GX_OK;
}

gx_status gx_autotune(uint32_t w, double load, uint32_t* B_out, uint32_t* G_out,
                      uint32_t* U_out) {
  if (w < 1 || w > 4 || !(load > 0.0) || load > 0.95 || !B_out || !G_out || !U_out)
    return GX_EINVAL;
  // the size class of a table for 2^23 states at this load
  gx_tune_info t{};
  const gx_status st = gx_autotune_capacity(
      w, load, static_cast<uint64_t>(static_cast<double>(uint64_t(1) << 23) / load) + 1, &t);
  if (st != GX_OK) return st;
  *B_out = t.bucket_words;
  *G_out = t.subgroup;
  *U_out = t.keys_per_subgroup;
  return GX_OK;
}

gx_status gx_batch_create(const gx_network* nets, uint32_t n, const gx_batch_opts* opts,
                          gx_batch** out) {
  if (!nets || n == 0 || !opts || !opts->capacity || !out) return GX_EINVAL;
  if (opts->bucket_words && !gx::valid_pow2(opts->bucket_words, 8, 64)) return GX_EINVAL;
  if (opts->subgroup && !(opts->subgroup == 4 || opts->subgroup == 8 || opts->subgroup == 16))
    return GX_EINVAL;
  if (opts->subgroup == 4 && opts->bucket_words > 32) return GX_EINVAL;
  if (opts->keys_per_subgroup && !(opts->keys_per_subgroup == 1 || opts->keys_per_subgroup == 2))
    return GX_EINVAL;
  // compile every network on the host first: argument errors before device work
  std::vector<std::vector<uint32_t>> imgs(n), inits(n);
  std::vector<uint32_t> words(n);
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t ms = 0;
    const gx_status s = gx::compile_network_image(&nets[i], &imgs[i], &words[i], &inits[i], &ms);
    if (s != GX_OK) return s;
    if (opts->capacity[i] == 0) return GX_EINVAL;
  }
  gx_batch* b = new (std::nothrow) gx_batch;
  if (!b) return GX_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return GX_EDEVICE;
  }
  b->n = n;
  b->max_levels = opts->max_levels ? opts->max_levels : gx::kDefaultMaxLevels;
  b->use_graph = opts->use_graph != 0;
  b->stepped = !b->use_graph && !opts->persistent;
  if (!b->stepped && static_cast<uint64_t>(n) * b->max_levels >= (uint64_t(1) << 31)) {
    delete b;
    return GX_EINVAL;
  }
  b->seed = opts->hash_seed ? opts->hash_seed : 0x1801058570ull;
  b->H = opts->max_hashes ? opts->max_hashes : 8;
  b->w = words;
  b->cls.resize(n);
  b->Bi.resize(n);
  b->Gi.resize(n);
  b->Ui.resize(n);
  b->tab_off.resize(n);
  b->tab_words.resize(n);
  b->keep_states = opts->keep_states != 0;
  // per-instance kernel configuration: explicit, else the autotuner's pick
  // for the instance's slot width and the combined capacity of the batch's
  // instances of that width: they run side by side, so their tables share
  // the caches, and the footprint that decides a probe's cost is theirs
  // together (tuned for its own size alone, a small instance's pick assumes
  // a table resident in an XCD's L2)
  uint64_t footprint[5] = {0, 0, 0, 0, 0};
  for (uint32_t i = 0; i < n; ++i) footprint[gx::slot_words(words[i])] += opts->capacity[i];
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t B = opts->bucket_words, G = opts->subgroup, U = opts->keys_per_subgroup;
    if (!B || !G || !U) {
      gx_tune_info ti{};
      const gx_status s =
          gx_autotune_capacity(words[i], 0.5, footprint[gx::slot_words(words[i])], &ti);
      if (s != GX_OK) {
        gx::free_batch(b);
        return s;
      }
      B = B ? B : ti.bucket_words;
      G = G ? G : ti.subgroup;
      // one key in flight per subgroup unless asked: more keys in flight cost
      // the exploration kernels a wave per SIMD of occupancy
      U = U ? U : 1;
      gx::fit_subgroup(&B, &G, opts->bucket_words != 0);
    }
    const uint32_t S = gx::slot_words(words[i]);
    if (B < 2 * S) B = 2 * S;
    b->Bi[i] = B;
    b->Gi[i] = G;
    b->Ui[i] = U;
    uint32_t k = 0;
    for (; k < b->classes.size(); ++k) {
      const auto& c = b->classes[k];
      if (c.S == S && c.B == B && c.G == G && c.U == U) break;
    }
    if (k == b->classes.size()) {
      b->classes.emplace_back();
      auto& c = b->classes.back();
      c.S = S;
      c.B = B;
      c.G = G;
      c.U = U;
    }
    b->classes[k].members.push_back(i);
    b->cls[i] = k;
  }
  // Largest declared capacity first: the initial queue holds the instances
  // in member order, so the explorations with the longest chain of levels
  // start first and the small ones fill the device around them.
  for (auto& c : b->classes)
    std::stable_sort(c.members.begin(), c.members.end(), [&](uint32_t x, uint32_t y) {
      return opts->capacity[x] > opts->capacity[y];
    });
  // shared hash constants
  std::vector<uint64_t> hc(2 * b->H);
  for (uint32_t j = 0; j < b->H; ++j) gx::hash_constants(b->seed, j, &hc[2 * j], &hc[2 * j + 1]);
  if (gx::dmalloc(&b->hc, hc.size()) != hipSuccess ||
      hipMemcpy(b->hc, hc.data(), hc.size() * sizeof(uint64_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
    gx::free_batch(b);
    return GX_ENOMEM;
  }
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  for (auto& c : b->classes) {
    const uint32_t nc = static_cast<uint32_t>(c.members.size());
    const uint32_t S = c.S;
    // layout of the class's tables and frontiers (256-byte aligned pieces)
    std::vector<uint64_t> tab_off(nc), nb(nc), fr_off(nc);
    uint64_t tw = 0, fw = 0, imgw = 0, max_img = 0;
    std::vector<uint64_t> img_off(nc);
    for (uint32_t k = 0; k < nc; ++k) {
      const uint32_t i = c.members[k];
      const uint64_t cap = opts->capacity[i];
      nb[k] = (cap + c.B / S - 1) / (c.B / S);
      tab_off[k] = tw;
      b->tab_off[i] = tw;
      b->tab_words[i] = nb[k] * c.B;
      tw += gx::align_up(nb[k] * c.B, 64);
      fr_off[k] = fw;
      fw += 2 * gx::align_up(cap * S, 64);
      img_off[k] = imgw;
      imgw += imgs[i].size();
      max_img = std::max<uint64_t>(max_img, imgs[i].size());
    }
    c.table_words = tw;
    c.img_stride = static_cast<uint32_t>(gx::align_up(max_img, 4));
    // every instance publishes at most one entry per level, so the queue
    // never overflows (checked against 2^31 entries when the batch is made);
    // the stepped schedule has no queue
    c.queue_cap = b->stepped ? 0 : nc * b->max_levels;
    uint64_t sum_cap = 0;
    for (uint32_t i : c.members) sum_cap += opts->capacity[i];
    c.dead_cap = opts->deadlock_capacity ? opts->deadlock_capacity
                                         : std::min<uint64_t>(sum_cap, uint64_t(1) << 26);
    if (gx::dmalloc(&c.tables, tw) != hipSuccess || gx::dmalloc(&c.frontiers, fw) != hipSuccess ||
        gx::dmalloc(&c.inst, nc) != hipSuccess || gx::dmalloc(&c.state, nc) != hipSuccess ||
        gx::dmalloc(&c.state_init, nc) != hipSuccess ||
        (!b->stepped && (gx::dmalloc(&c.queue, c.queue_cap) != hipSuccess ||
                         gx::dmalloc(&c.queue_init, nc) != hipSuccess)) ||
        (b->stepped && (gx::dmalloc(&c.d_jobs, nc) != hipSuccess ||
                        gx::dmalloc(&c.d_sum, 2ull * nc) != hipSuccess ||
                        hipHostMalloc(&c.h_jobs, nc * sizeof(gx::ServeJob)) != hipSuccess ||
                        hipHostMalloc(&c.h_sum, 2ull * nc * sizeof(uint64_t)) != hipSuccess)) ||
        gx::dmalloc(&c.g, 1) != hipSuccess ||
        gx::dmalloc(&c.g_init, 1) != hipSuccess || gx::dmalloc(&c.img, imgw) != hipSuccess ||
        gx::dmalloc(&c.init_states, static_cast<uint64_t>(nc) * S) != hipSuccess ||
        (!b->stepped &&
         gx::dmalloc(&c.levels, static_cast<uint64_t>(nc) * b->max_levels) != hipSuccess) ||
        gx::dmalloc(&c.dead, c.dead_cap * S) != hipSuccess ||
        gx::dmalloc(&c.dead_tag, c.dead_cap) != hipSuccess ||
        gx::dmalloc(&c.stats, 2 * gx::kNumCounters) != hipSuccess ||
        hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c.ev_done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      gx::free_batch(b);
      return GX_ENOMEM;
    }
    std::vector<gx::BatchInst> hi(nc);
    std::vector<gx::BatchState> hs(nc);
    std::vector<gx::BatchEntry> he(nc);
    std::vector<uint32_t> himg(imgw), hinit(static_cast<size_t>(nc) * S, 0);
    for (uint32_t k = 0; k < nc; ++k) {
      const uint32_t i = c.members[k];
      gx::BatchInst& in = hi[k];
      std::memset(&in, 0, sizeof(in));
      in.t.words = c.tables + tab_off[k];
      in.t.n_buckets = nb[k];
      in.t.hc = b->hc;
      in.t.seed = b->seed;
      in.t.a0 = hc[0];
      in.t.c0 = hc[1];
      in.t.H = b->H;
      in.t.counters = c.stats;
      in.t.ctr_slots = 1;  // the batch kernels keep no statistics
      in.img_off = static_cast<uint32_t>(img_off[k]);
      in.img_words = static_cast<uint32_t>(imgs[i].size());
      const uint64_t fcap = gx::align_up(opts->capacity[i] * S, 64);
      in.f[0] = c.frontiers + fr_off[k];
      in.f[1] = c.frontiers + fr_off[k] + fcap;
      in.cap = opts->capacity[i];
      in.levels = c.levels ? c.levels + static_cast<uint64_t>(k) * b->max_levels : nullptr;
      in.max_levels = b->max_levels;
      std::copy(imgs[i].begin(), imgs[i].end(), himg.begin() + img_off[k]);
      for (uint32_t x = 0; x < words[i]; ++x) hinit[static_cast<size_t>(k) * S + x] = inits[i][x];
      std::memset(&hs[k], 0, sizeof(gx::BatchState));
      hs[k].n_in = 1;
      std::memset(&he[k], 0, sizeof(gx::BatchEntry));
      he[k].inst = k;
      he[k].tiles = 1;
      he[k].ready = 1;
    }
    gx::BatchGlobal hg;
    std::memset(&hg, 0, sizeof(hg));
    hg.tail = nc;
    if (hipMemcpy(c.inst, hi.data(), nc * sizeof(gx::BatchInst), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.state_init, hs.data(), nc * sizeof(gx::BatchState), hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!b->stepped && hipMemcpy(c.queue_init, he.data(), nc * sizeof(gx::BatchEntry),
                                  hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(c.g_init, &hg, sizeof(hg), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.img, himg.data(), himg.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c.init_states, hinit.data(), hinit.size() * sizeof(uint32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      gx::free_batch(b);
      return GX_EDEVICE;
    }
    c.h_inst = std::move(hi);
    c.lds = (c.img_stride + gx::kStageWords) * sizeof(uint32_t);
    int per_cu = 1;
    switch (S) {
      case 1: per_cu = gx::batch_resident<1>(c.B, c.G, c.U, c.lds); break;
      case 2: per_cu = gx::batch_resident<2>(c.B, c.G, c.U, c.lds); break;
      default: per_cu = gx::batch_resident<4>(c.B, c.G, c.U, c.lds); break;
    }
    c.grid = static_cast<uint32_t>(per_cu) * static_cast<uint32_t>(cus);
  }
  // Classes run concurrently on their own streams.  A persistent grid sized
  // to the whole device would keep every other class's workgroups out until
  // it drains, so each class gets the share of the device its instances'
  // declared capacities claim of the total (at least one workgroup per CU).
  if (b->classes.size() > 1) {
    double total = 0;
    std::vector<double> work(b->classes.size(), 0.0);
    for (size_t k = 0; k < b->classes.size(); ++k) {
      for (uint32_t i : b->classes[k].members) work[k] += static_cast<double>(opts->capacity[i]);
      total += work[k];
    }
    for (size_t k = 0; k < b->classes.size(); ++k) {
      auto& c = b->classes[k];
      const double share = total > 0 ? work[k] / total : 1.0;
      c.grid = std::max<uint32_t>(static_cast<uint32_t>(cus),
                                  static_cast<uint32_t>(c.grid * share + 0.5));
    }
  }
  if (b->use_graph) {
    hipGraph_t graph = nullptr;
    if (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      gx::free_batch(b);
      return GX_EDEVICE;
    }
    const hipError_t e = gx::enqueue_run(b, b->capture_stream);
    const hipError_t e2 = hipStreamEndCapture(b->capture_stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess ||
        hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      gx::free_batch(b);
      return GX_EDEVICE;
    }
    (void)hipGraphDestroy(graph);
  }
  *out = b;
  return GX_OK;
}

gx_status gx_batch_destroy(gx_batch* b) {
  gx::free_batch(b);
  return GX_OK;
}

gx_status gx_batch_instance_config(const gx_batch* b, uint32_t i, uint32_t* bucket_words,
                                   uint32_t* subgroup, uint32_t* keys_per_subgroup) {
  if (!b || i >= b->n || !bucket_words || !subgroup || !keys_per_subgroup) return GX_EINVAL;
  *bucket_words = b->Bi[i];
  *subgroup = b->Gi[i];
  *keys_per_subgroup = b->Ui[i];
  return GX_OK;
}

gx_status gx_batch_run(gx_batch* b, void* hip_stream) {
  if (!b) return GX_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (b->stepped) {
    const gx_status st = gx::run_stepped(b, s);
    if (st != GX_OK) return st;
    b->ran = true;
    return GX_OK;
  }
  hipError_t e;
  if (b->use_graph) {
    e = hipGraphLaunch(b->exec, s);
  } else {
    e = gx::enqueue_run(b, s);
  }
  if (e != hipSuccess) return GX_EDEVICE;
  b->ran = true;
  return GX_OK;
}

gx_status gx_batch_results(gx_batch* b, gx_explore_result* outs, gx_status* inst_status) {
  if (!b || !outs || !inst_status || !b->ran) return GX_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return GX_EDEVICE;
  for (uint32_t i = 0; i < b->n; ++i) {
    std::memset(&outs[i], 0, sizeof(gx_explore_result));
    inst_status[i] = GX_EDEVICE;
  }
  for (auto& c : b->classes) {
    const uint32_t nc = static_cast<uint32_t>(c.members.size());
    const uint32_t S = c.S;
    std::vector<gx::BatchState> hs(nc);
    std::vector<uint64_t> lv(b->stepped ? 0 : static_cast<size_t>(nc) * b->max_levels);
    gx::BatchGlobal hg;
    if (hipMemcpy(hs.data(), c.state, nc * sizeof(gx::BatchState), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        (!b->stepped && hipMemcpy(lv.data(), c.levels, lv.size() * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost) != hipSuccess) ||
        hipMemcpy(&hg, c.g, sizeof(hg), hipMemcpyDeviceToHost) != hipSuccess)
      return GX_EDEVICE;
    const uint64_t n_rec = std::min<uint64_t>(hg.dead_used, c.dead_cap);
    std::vector<uint32_t> dead(n_rec * S), tag(n_rec);
    if (n_rec && (hipMemcpy(dead.data(), c.dead, dead.size() * sizeof(uint32_t),
                            hipMemcpyDeviceToHost) != hipSuccess ||
                  hipMemcpy(tag.data(), c.dead_tag, tag.size() * sizeof(uint32_t),
                            hipMemcpyDeviceToHost) != hipSuccess))
      return GX_EDEVICE;
    std::vector<std::vector<std::array<uint32_t, 4>>> per(nc);
    for (uint64_t r = 0; r < n_rec; ++r) {
      std::array<uint32_t, 4> v{0, 0, 0, 0};
      for (uint32_t x = 0; x < S; ++x) v[x] = dead[r * S + x];
      if (tag[r] < nc) per[tag[r]].push_back(v);
    }
    for (uint32_t k = 0; k < nc; ++k) {
      const uint32_t i = c.members[k];
      const uint32_t w = b->w[i];
      const gx::BatchState& st = hs[k];
      const uint64_t flags = st.ctr[gx::kCtrFlags * gx::kCtrSpread];
      outs[i] = gx_explore_result{};  // no safety monitor in batches
      outs[i].violation_level = 0xFFFFFFFFu;
      gx_status s = GX_OK;
      if (b->stepped)
        s = b->step_status[i];
      else if (!st.done || hg.abort)
        s = GX_EDEVICE;
      else if (flags & gx::kFlagTableFull)
        s = GX_ETABLEFULL;
      else if (flags)
        s = GX_ENOMEM;
      if (s == GX_OK && per[k].size() != st.ctr[gx::kCtrDead * gx::kCtrSpread])
        s = GX_ENOMEM;  // deadlock records overflowed
      inst_status[i] = s;
      if (s != GX_OK) continue;
      const uint32_t n_levels =
          b->stepped ? static_cast<uint32_t>(b->step_levels[i].size()) : st.level + 1;
      uint64_t* L = static_cast<uint64_t*>(std::malloc(sizeof(uint64_t) * n_levels));
      auto& dl = per[k];
      std::sort(dl.begin(), dl.end());
      uint32_t* D = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (dl.size() * w + 1)));
      if (!L || !D) {
        std::free(L);
        std::free(D);
        inst_status[i] = GX_ENOMEM;
        continue;
      }
      uint64_t total = 0;
      for (uint32_t l = 0; l < n_levels; ++l) {
        L[l] = l == 0         ? 1
               : b->stepped ? b->step_levels[i][l]
                            : lv[static_cast<size_t>(k) * b->max_levels + l];
        total += L[l];
      }
      for (size_t r = 0; r < dl.size(); ++r)
        for (uint32_t x = 0; x < w; ++x) D[r * w + x] = dl[r][x];
      outs[i].n_states = total;
      outs[i].n_transitions = st.ctr[gx::kCtrTrans * gx::kCtrSpread];
      outs[i].words_per_state = w;
      outs[i].n_levels = n_levels;
      outs[i].level_counts = L;
      outs[i].n_deadlocks = dl.size();
      outs[i].deadlocks = D;
      if (b->keep_states) {
        const gx_status ks = gx::sorted_keys_malloc(c.tables + b->tab_off[i], b->tab_words[i], S,
                                                    w, &outs[i].states);
        if (ks != GX_OK) {
          gx_explore_result_free(&outs[i]);
          inst_status[i] = ks;
        }
      }
    }
  }
  return GX_OK;
}

gx_status gx_explore_batch(const gx_network* nets, uint32_t n, const gx_batch_opts* opts,
                           gx_explore_result* outs, gx_status* inst_status) {
  if (!outs || !inst_status) return GX_EINVAL;
  gx_batch* b = nullptr;
  gx_status s = gx_batch_create(nets, n, opts, &b);
  if (s != GX_OK) return s;
  s = gx_batch_run(b, opts->hip_stream);
  if (s == GX_OK) s = gx_batch_results(b, outs, inst_status);
  gx_batch_destroy(b);
  return s;
}

}  // extern "C"
