// Exploration server: requests (networks with a declared size bound) are
// admitted when their HBM reservation fits the budget, get their table,
// frontiers and deadlock buffer as one block of a device arena allocated
// once with the server (a buddy allocator: reservations are powers of two,
// so admitting a request allocates nothing), and are advanced one BFS level
// per step by a multi-job launch over every active request (continuous
// batching: requests join and leave between steps).  A request whose table
// fills up is retried with four times its bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "gx_buddy.hpp"
#include "gx_serve_kernel.hpp"

namespace gx {

gx_status compile_network_image(const gx_network* net, std::vector<uint32_t>* img,
                                uint32_t* words, std::vector<uint32_t>* packed_initial,
                                uint64_t* max_succ);

// instantiated in gx_serve_s1.hip, gx_serve_s2.hip and gx_serve_s4.hip
extern template hipError_t serve_launch<1>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t serve_launch<2>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);
extern template hipError_t serve_launch<4>(uint32_t, uint32_t, uint32_t, const ServeArgs&,
                                           uint32_t, size_t, hipStream_t);

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint32_t kMaxAttempts = 12;
// a job's counters: kCtrCount counters kCtrSpread words apart (one cache line each)
constexpr uint64_t kSlotCtrWords = uint64_t(kCtrCount) * kCtrSpread;

struct Request {
  uint64_t id = 0;
  std::vector<uint32_t> img, init;
  uint32_t w = 0;
  uint64_t declared = 0;
  uint32_t attempts = 0;
  Clock::time_point arrival;
  bool done = false;
  gx_status status = GX_OK;
  gx_explore_result result{};
  uint64_t latency_ns = 0;
};

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}


// Device words a job's small state takes: table counters, the initial key
// and its status byte.
constexpr uint64_t kSlotSmallBytes = 128;

}  // namespace
}  // namespace gx

struct gx_server {
  struct Job {
    gx::Request* r = nullptr;
    gx_table* t = nullptr;   // a view of its arena block
    uint64_t reserved = 0;   // bytes of that block
    uint64_t block = 0;      // its offset in the arena
    uint64_t n_in = 0;
    int cur = 0;
    uint32_t slot = 0;
    std::vector<uint64_t> levels;
  };
  // configuration
  uint64_t budget = 0;
  uint32_t max_active = 0;
  bool keep_states = false;
  double load = 0.5;
  uint64_t seed = 0;
  uint32_t H = 8;
  uint32_t cfg[5][3] = {};  // per slot width: bucket words, subgroup, keys per subgroup
  int device = 0;
  hipStream_t stream = nullptr;
  // state, guarded by mu
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_id = 1;
  std::map<uint64_t, std::unique_ptr<gx::Request>> reqs;
  std::deque<gx::Request*> waiting;
  uint64_t reserved = 0;        // bytes reserved by active jobs
  // device arena of budget bytes, shared hash constants, per-slot small state
  char* arena = nullptr;
  uint64_t arena_bytes = 0;
  gx::Buddy buddy;
  uint64_t a0 = 0, c0 = 0;  // first hash constant pair (host copy)
  uint64_t* d_hc = nullptr;
  char* d_small = nullptr;
  gx_server_stats stats{};
  // owned by the step thread
  std::vector<Job> active;
  std::vector<uint32_t> free_slots;
  gx::ServeJob* d_jobs = nullptr;
  uint32_t* d_img = nullptr;
  uint64_t* d_ctr = nullptr;
  uint64_t* h_ctr = nullptr;   // pinned host copy of d_ctr (per-step read-back)
  gx::ServeJob* h_jobs = nullptr;  // pinned staging of the step's job descriptors
  std::thread th;
};

namespace gx {
namespace {

uint64_t table_bytes_for(uint32_t w, uint64_t slots) {
  // table + two frontiers + deadlock buffer, each slots x S words
  return 4ull * slots * slot_words(w) * sizeof(uint32_t);
}

void complete(gx_server* s, Request* r, gx_status st) {
  r->status = st;
  r->latency_ns = static_cast<uint64_t>(
      std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - r->arrival).count());
  r->done = true;
  r->img.clear();
  r->img.shrink_to_fit();
  if (st == GX_OK) ++s->stats.completed;
  else ++s->stats.failed;
}

// A table over the arena block at `off` for w words and `slots` slots (a
// power of two): the table, then the two frontiers and the deadlock buffer,
// slots states each; counters, initial key and status in the job slot's
// small state; the server's shared hash constants.  Nothing is allocated on
// the device.  mu held.
gx_table* job_table(gx_server* s, uint32_t w, uint64_t slots, uint64_t off, uint32_t slot) {
  const uint32_t S = slot_words(w);
  const uint32_t* c = s->cfg[S];
  gx_table* t = new (std::nothrow) gx_table;
  if (!t) return nullptr;
  t->device = s->device;
  t->w = w;
  t->S = S;
  t->B = c[0];
  t->G = c[1];
  t->U = c[2];
  t->H = s->H;
  t->seed = s->seed;
  t->n_buckets = slots * S / c[0];
  t->a0 = s->a0;
  t->c0 = s->c0;
  const uint64_t T = slots * S * sizeof(uint32_t);
  char* base = s->arena + off;
  char* small = s->d_small + static_cast<uint64_t>(slot) * kSlotSmallBytes;
  t->words = reinterpret_cast<uint32_t*>(base);
  t->hc = s->d_hc;
  t->counters = nullptr;  // job tables keep no statistics
  t->ctr_slots = 1;
  t->eb.key = reinterpret_cast<uint32_t*>(small + 64);
  t->eb.status = reinterpret_cast<uint8_t*>(small + 96);
  for (int k = 0; k < 2; ++k) {
    t->eb.f[k] = reinterpret_cast<uint32_t*>(base + (k + 1) * T);
    t->eb.f_cap[k] = slots;
  }
  t->eb.dead = reinterpret_cast<uint32_t*>(base + 3 * T);
  t->eb.dead_cap = slots;
  return t;
}

// Admit waiting requests while their reservations fit.  mu held.
void admit(gx_server* s) {
  while (!s->waiting.empty() && !s->free_slots.empty()) {
    Request* r = s->waiting.front();
    const uint64_t slots = pow2_at_least(
        std::max<uint64_t>(64, static_cast<uint64_t>(static_cast<double>(r->declared) / s->load) + 1));
    const uint64_t need = table_bytes_for(r->w, slots);
    if (need > s->buddy.largest()) {  // can never fit
      s->waiting.pop_front();
      complete(s, r, GX_ENOMEM);
      s->cv_done.notify_all();
      continue;
    }
    const uint64_t off = s->buddy.alloc(need);
    if (off == ~0ull) break;  // wait for running jobs to finish
    const uint32_t slot = s->free_slots.back();
    gx_table* t = job_table(s, r->w, slots, off, slot);
    if (!t) {
      s->buddy.release(off, need);
      break;
    }
    s->waiting.pop_front();
    gx_server::Job j;
    j.r = r;
    j.t = t;
    j.reserved = need;
    j.block = off;
    j.slot = slot;
    s->free_slots.pop_back();
    s->reserved += need;
    s->stats.reserved_peak = std::max(s->stats.reserved_peak, s->reserved);
    // reset the table, place the initial state, insert it
    uint32_t init[4] = {0, 0, 0, 0};
    for (uint32_t x = 0; x < r->w; ++x) init[x] = r->init[x];
    bool ok = gx_table_clear(t, s->stream) == GX_OK &&
              hipMemcpyAsync(t->eb.f[0], init, t->S * sizeof(uint32_t), hipMemcpyHostToDevice,
                             s->stream) == hipSuccess &&
              hipMemcpyAsync(t->eb.key, init, r->w * sizeof(uint32_t), hipMemcpyHostToDevice,
                             s->stream) == hipSuccess &&
              hipMemsetAsync(s->d_ctr + kSlotCtrWords * j.slot, 0, kSlotCtrWords * sizeof(uint64_t),
                             s->stream) ==
                  hipSuccess &&
              launch_find_or_put(t, t->eb.key, 1, t->eb.status, nullptr, s->stream) == hipSuccess &&
              hipMemcpyAsync(s->d_img + static_cast<uint64_t>(j.slot) * kImgMaxWords,
                             r->img.data(), r->img.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, s->stream) == hipSuccess &&
              hipStreamSynchronize(s->stream) == hipSuccess;
    if (!ok) {
      s->reserved -= need;
      s->free_slots.push_back(j.slot);
      s->buddy.release(off, need);
      delete t;
      complete(s, r, GX_EDEVICE);
      s->cv_done.notify_all();
      continue;
    }
    j.n_in = 1;
    j.cur = 0;
    j.levels.assign(1, 1);
    s->active.push_back(std::move(j));
    s->stats.active_peak = std::max<uint64_t>(s->stats.active_peak, s->active.size());
  }
}

// Finish job k of s->active (mu held): store its result or retry it.
void finish_job(gx_server* s, size_t k, gx_status st, uint64_t transitions, uint64_t n_dead) {
  gx_server::Job& j = s->active[k];
  Request* r = j.r;
  if (st == GX_ETABLEFULL && r->attempts + 1 < kMaxAttempts) {
    ++r->attempts;
    // four times the bound, and at least twice the states already found
    uint64_t found = 0;
    for (uint64_t c : j.levels) found += c;
    r->declared = std::max<uint64_t>(r->declared * 4, 2 * found);
    ++s->stats.retried;
    s->waiting.push_front(r);
  } else if (st != GX_OK) {
    complete(s, r, st);
  } else {
    const uint32_t w = r->w, S = j.t->S;
    std::vector<uint32_t> raw(n_dead * S);
    gx_status rs = GX_OK;
    if (n_dead && hipMemcpy(raw.data(), j.t->eb.dead, raw.size() * sizeof(uint32_t),
                            hipMemcpyDeviceToHost) != hipSuccess)
      rs = GX_EDEVICE;
    std::vector<std::array<uint32_t, 4>> dl(n_dead);
    for (uint64_t i = 0; i < n_dead; ++i) {
      dl[i] = {0, 0, 0, 0};
      for (uint32_t x = 0; x < w; ++x) dl[i][x] = raw[i * S + x];
    }
    std::sort(dl.begin(), dl.end());
    uint64_t* L = static_cast<uint64_t*>(std::malloc(sizeof(uint64_t) * j.levels.size()));
    uint32_t* D = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (n_dead * w + 1)));
    uint32_t* V = nullptr;  // the table's contents, read before its block is released
    if (!L || !D) rs = GX_ENOMEM;
    if (rs == GX_OK && s->keep_states)
      rs = sorted_keys_malloc(j.t->words, j.t->n_buckets * j.t->B, S, w, &V);
    if (rs == GX_OK) {
      uint64_t total = 0;
      for (size_t l = 0; l < j.levels.size(); ++l) {
        L[l] = j.levels[l];
        total += L[l];
      }
      for (uint64_t i = 0; i < n_dead; ++i)
        for (uint32_t x = 0; x < w; ++x) D[i * w + x] = dl[i][x];
      r->result.n_states = total;
      r->result.n_transitions = transitions;
      r->result.words_per_state = w;
      r->result.n_levels = static_cast<uint32_t>(j.levels.size());
      r->result.level_counts = L;
      r->result.n_deadlocks = n_dead;
      r->result.deadlocks = D;
      r->result.violation_level = 0xFFFFFFFFu;  // no safety monitor in the server
      r->result.states = V;
      s->stats.states += total;
    } else {
      std::free(L);
      std::free(D);
      std::free(V);
    }
    complete(s, r, rs);
  }
  s->reserved -= j.reserved;
  s->free_slots.push_back(j.slot);
  s->buddy.release(j.block, j.reserved);
  delete j.t;  // a view: its memory stays in the arena
  s->active.erase(s->active.begin() + k);
}

void step_loop(gx_server* s) {
  std::vector<ServeJob> hjs[3];  // per slot-width class
  while (true) {
    {
      std::unique_lock<std::mutex> lock(s->mu);
      s->cv_work.wait(lock, [&] { return s->stop || !s->waiting.empty() || !s->active.empty(); });
      if (s->stop) return;
      admit(s);
      if (s->active.empty()) {
        // nothing admitted (budget held by nothing?) - wait for a new request
        if (!s->waiting.empty()) s->cv_work.wait_for(lock, std::chrono::milliseconds(1));
        continue;
      }
    }
    // one step over every active job, per slot-width class
    bool ok = true;
    for (uint32_t S : {1u, 2u, 4u}) {
      std::vector<ServeJob>& hj = hjs[S == 1 ? 0 : S == 2 ? 1 : 2];
      hj.clear();
      uint64_t tiles = 0;
      uint32_t img_max = 0;
      for (auto& j : s->active) {
        if (j.t->S != S) continue;
        ServeJob x;
        x.t = j.t->dev();
        x.img_off = j.slot * kImgMaxWords;
        x.img_words = static_cast<uint32_t>(j.r->img.size());
        x.frontier_in = j.t->eb.f[j.cur];
        x.n_in = j.n_in;
        x.frontier_out = j.t->eb.f[j.cur ^ 1];
        x.cap_out = j.t->eb.f_cap[j.cur ^ 1];
        x.dead = j.t->eb.dead;
        x.dead_cap = j.t->eb.dead_cap;
        x.ctr = s->d_ctr + kSlotCtrWords * j.slot;
        x.tile_begin = tiles;
        x.dead_ctr = nullptr;
        x.dead_tag = nullptr;
        x.tag = 0;
        x.pad = 0;
        tiles += (j.n_in + 255) / 256;
        img_max = std::max<uint32_t>(img_max, x.img_words);
        hj.push_back(x);
      }
      if (hj.empty()) continue;
      const uint32_t* c = s->cfg[S];
      ServeArgs a;
      a.jobs = s->d_jobs + (S == 1 ? 0 : S == 2 ? 1 : 2) * s->max_active;
      a.n_jobs = static_cast<uint32_t>(hj.size());
      a.img = s->d_img;
      a.img_stride = (img_max + 3) & ~3u;
      const size_t lds = (a.img_stride + kStageWords) * sizeof(uint32_t);
      // staged in pinned memory (one region per class, reused only after the
      // step's synchronisation) so the upload is a plain asynchronous copy
      ServeJob* staged = s->h_jobs + (S == 1 ? 0 : S == 2 ? 1 : 2) * s->max_active;
      std::copy(hj.begin(), hj.end(), staged);
      hipError_t e = hipMemcpyAsync(const_cast<ServeJob*>(a.jobs), staged,
                                    hj.size() * sizeof(ServeJob), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) {
        switch (S) {
          case 1: e = serve_launch<1>(c[0], c[1], c[2], a, static_cast<uint32_t>(tiles), lds, s->stream); break;
          case 2: e = serve_launch<2>(c[0], c[1], c[2], a, static_cast<uint32_t>(tiles), lds, s->stream); break;
          default: e = serve_launch<4>(c[0], c[1], c[2], a, static_cast<uint32_t>(tiles), lds, s->stream); break;
        }
      }
      if (e != hipSuccess) ok = false;
    }
    // one synchronisation per step: the classes' launches and the read-back
    // of the counters of slots 0 .. the highest active one follow each other
    // on the stream without host round trips
    uint32_t n_slots = 0;
    for (const auto& j : s->active) n_slots = std::max(n_slots, j.slot + 1);
    if (hipMemcpyAsync(s->h_ctr, s->d_ctr, kSlotCtrWords * n_slots * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      ok = false;
    const uint64_t* ctr = s->h_ctr;
    std::lock_guard<std::mutex> lock(s->mu);
    ++s->stats.steps;
    for (size_t k = s->active.size(); k-- > 0;) {
      gx_server::Job& j = s->active[k];
      if (!ok) {
        finish_job(s, k, GX_EDEVICE, 0, 0);
        continue;
      }
      const uint64_t* c = &ctr[kSlotCtrWords * j.slot];
      const uint64_t flags = c[kCtrFlags * kCtrSpread], n_next = c[kCtrTail * kCtrSpread];
      if (flags & kFlagTableFull) {
        finish_job(s, k, GX_ETABLEFULL, 0, 0);
      } else if (flags) {
        finish_job(s, k, GX_ENOMEM, 0, 0);
      } else if (n_next == 0) {
        finish_job(s, k, GX_OK, c[kCtrTrans * kCtrSpread], c[kCtrDead * kCtrSpread]);
      } else {
        j.levels.push_back(n_next);
        j.n_in = n_next;
        j.cur ^= 1;
      }
    }
    // clear the next-frontier tails of slots 0 .. n_slots - 1 in one strided
    // fill (finished or idle slots included: admission clears a slot's
    // counters anyway)
    if (ok && n_slots &&
        hipMemset2DAsync(s->d_ctr + kCtrTail * kCtrSpread, kSlotCtrWords * sizeof(uint64_t), 0,
                         sizeof(uint64_t), n_slots, s->stream) != hipSuccess) {
      for (size_t k = s->active.size(); k-- > 0;) finish_job(s, k, GX_EDEVICE, 0, 0);
    }
    s->cv_done.notify_all();
  }
}

void destroy_server(gx_server* s) {
  if (!s) return;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> lock(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->th.join();
  }
  (void)hipDeviceSynchronize();
  for (auto& j : s->active) delete j.t;
  for (auto& kv : s->reqs) gx_explore_result_free(&kv.second->result);
  if (s->d_jobs) (void)hipFree(s->d_jobs);
  if (s->d_img) (void)hipFree(s->d_img);
  if (s->d_ctr) (void)hipFree(s->d_ctr);
  if (s->h_ctr) (void)hipHostFree(s->h_ctr);
  if (s->h_jobs) (void)hipHostFree(s->h_jobs);
  if (s->arena) (void)hipFree(s->arena);
  if (s->d_hc) (void)hipFree(s->d_hc);
  if (s->d_small) (void)hipFree(s->d_small);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  s->cv_done.notify_all();
  delete s;
}

}  // namespace
}  // namespace gx

// ====================================================================== ABI
extern "C" {

gx_status gx_server_create(const gx_server_opts* opts, gx_server** out) {
  if (!opts || !out || opts->budget_bytes == 0) return GX_EINVAL;
  const double load = opts->load_factor > 0 ? opts->load_factor : 0.5;
  if (load > 0.95) return GX_EINVAL;
  if (opts->bucket_words && !(opts->bucket_words == 8 || opts->bucket_words == 16 ||
                              opts->bucket_words == 32 || opts->bucket_words == 64))
    return GX_EINVAL;
  if (opts->subgroup && !(opts->subgroup == 4 || opts->subgroup == 8 || opts->subgroup == 16))
    return GX_EINVAL;
  if (opts->subgroup == 4 && opts->bucket_words > 32) return GX_EINVAL;
  if (opts->keys_per_subgroup && !(opts->keys_per_subgroup == 1 || opts->keys_per_subgroup == 2))
    return GX_EINVAL;
  gx_server* s = new (std::nothrow) gx_server;
  if (!s) return GX_ENOMEM;
  s->budget = opts->budget_bytes;
  s->max_active = opts->max_active ? opts->max_active : 256;
  s->keep_states = opts->keep_states != 0;
  s->load = load;
  s->seed = opts->hash_seed ? opts->hash_seed : 0x1801058570ull;
  s->H = opts->max_hashes ? opts->max_hashes : 8;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return GX_EDEVICE;
  }
  for (uint32_t S : {1u, 2u, 4u}) {
    uint32_t B = opts->bucket_words, G = opts->subgroup, U = opts->keys_per_subgroup;
    if (!B || !G || !U) {
      uint32_t tb = 32, tg = 8, tu = 1;
      const gx_status st = gx_autotune(S, load, &tb, &tg, &tu);
      if (st != GX_OK) {
        delete s;
        return st;
      }
      B = B ? B : tb;
      G = G ? G : tg;
      // one key in flight per subgroup unless asked: the autotuner times the
      // isolated find-or-put, where more keys in flight pay off, but in the
      // exploration kernels they cost a wave per SIMD of occupancy
      (void)tu;
      U = U ? U : 1;
      gx::fit_subgroup(&B, &G, opts->bucket_words != 0);
    }
    if (B < 2 * S) B = 2 * S;
    s->cfg[S][0] = B;
    s->cfg[S][1] = G;
    s->cfg[S][2] = U;
  }
  s->cfg[3][0] = s->cfg[4][0];
  s->cfg[3][1] = s->cfg[4][1];
  s->cfg[3][2] = s->cfg[4][2];
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&s->d_jobs, 3ull * s->max_active * sizeof(gx::ServeJob)) != hipSuccess ||
      hipMalloc(&s->d_img, static_cast<uint64_t>(s->max_active) * gx::kImgMaxWords *
                               sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&s->d_ctr, gx::kSlotCtrWords * s->max_active * sizeof(uint64_t)) != hipSuccess ||
      hipHostMalloc(&s->h_ctr, gx::kSlotCtrWords * s->max_active * sizeof(uint64_t)) !=
          hipSuccess ||
      hipHostMalloc(&s->h_jobs, 3ull * s->max_active * sizeof(gx::ServeJob)) != hipSuccess) {
    (void)hipGetLastError();
    gx::destroy_server(s);
    return GX_ENOMEM;
  }
  // the arena (allocated once: admission allocates nothing), the hash
  // constants every job table shares, and each job slot's small state
  {
    const uint64_t arena_bytes = s->budget & ~((uint64_t(1) << gx::Buddy::kMinShift) - 1);
    std::vector<uint64_t> hc(2 * s->H);
    for (uint32_t j = 0; j < s->H; ++j) gx::hash_constants(s->seed, j, &hc[2 * j], &hc[2 * j + 1]);
    s->a0 = hc[0];
    s->c0 = hc[1];
    if (arena_bytes == 0 || hipMalloc(&s->arena, arena_bytes) != hipSuccess ||
        hipMalloc(&s->d_hc, hc.size() * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&s->d_small, gx::kSlotSmallBytes * s->max_active) != hipSuccess) {
      (void)hipGetLastError();
      gx::destroy_server(s);
      return GX_ENOMEM;
    }
    if (hipMemcpy(s->d_hc, hc.data(), hc.size() * sizeof(uint64_t), hipMemcpyHostToDevice) !=
        hipSuccess) {
      gx::destroy_server(s);
      return GX_EDEVICE;
    }
    s->arena_bytes = arena_bytes;
    s->buddy.init(arena_bytes);
  }
  for (uint32_t k = s->max_active; k-- > 0;) s->free_slots.push_back(k);
  try {
    s->th = std::thread(gx::step_loop, s);
  } catch (...) {
    gx::destroy_server(s);
    return GX_ENOMEM;
  }
  *out = s;
  return GX_OK;
}

gx_status gx_server_submit(gx_server* s, const gx_network* net, uint64_t declared_states,
                           uint64_t* request_id) {
  if (!s || !request_id || declared_states == 0) return GX_EINVAL;
  auto r = std::unique_ptr<gx::Request>(new (std::nothrow) gx::Request);
  if (!r) return GX_ENOMEM;
  uint64_t ms = 0;
  const gx_status st = gx::compile_network_image(net, &r->img, &r->w, &r->init, &ms);
  if (st != GX_OK) return st;
  r->declared = declared_states;
  r->arrival = gx::Clock::now();
  {
    std::lock_guard<std::mutex> lock(s->mu);
    r->id = s->next_id++;
    *request_id = r->id;
    s->waiting.push_back(r.get());
    s->reqs.emplace(r->id, std::move(r));
    ++s->stats.submitted;
  }
  s->cv_work.notify_all();
  return GX_OK;
}

gx_status gx_server_poll(gx_server* s, uint64_t id, int wait, gx_explore_result* out,
                         gx_status* request_status, uint64_t* latency_ns) {
  if (!s || !out || !request_status) return GX_EINVAL;
  std::unique_lock<std::mutex> lock(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return GX_EINVAL;
  if (!it->second->done) {
    if (!wait) return GX_EBUSY;
    s->cv_done.wait(lock, [&] { return it->second->done || s->stop; });
    if (!it->second->done) return GX_ECANCELED;
  }
  gx::Request* r = it->second.get();
  *out = r->result;
  r->result = gx_explore_result{};
  *request_status = r->status;
  if (latency_ns) *latency_ns = r->latency_ns;
  s->reqs.erase(it);
  return GX_OK;
}

gx_status gx_server_get_stats(gx_server* s, gx_server_stats* out) {
  if (!s || !out) return GX_EINVAL;
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->stats;
  out->reserved_now = s->reserved;
  out->pooled_bytes = s->arena_bytes - s->reserved;
  out->waiting = s->waiting.size();
  return GX_OK;
}

gx_status gx_server_destroy(gx_server* s) {
  gx::destroy_server(s);
  return GX_OK;
}

}  // extern "C"
