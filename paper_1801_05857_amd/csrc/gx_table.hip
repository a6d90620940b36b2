// Bucketed find-or-put table: storage management, the batch find-or-put
// kernel and the random-access bandwidth probe (Sec. 4.1, 4.2 and the isolated
// insert experiment of Sec. 5.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <mutex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gx_internal.hpp"

namespace gx {

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(256) void fill_kernel(uint4* p, uint64_t n16, uint32_t value,
                                                   uint64_t* counters, uint32_t n_counters) {
  const uint4 e = make_uint4(value, value, value, value);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
       i += stride) {
    p[i] = e;
  }
  if (counters)
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_counters;
         i += stride)
      counters[i] = 0;
}

// Random-access probe: subgroups of LANES lanes read LANES*4 contiguous bytes
// at a pseudo-random granule, 4 reads in flight per subgroup.
template <int LANES>
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint32_t* buf, uint64_t n_gran,
                                                           uint64_t n_reads, uint64_t seed,
                                                           uint64_t* sink) {
  constexpr int SUBS = 64 / LANES;
  constexpr int R = 4;
  const int lane = __lane_id();
  const int sg = lane / LANES;
  const int li = lane % LANES;
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  constexpr uint64_t per_round = static_cast<uint64_t>(SUBS) * R;
  uint32_t acc = 0;
  for (uint64_t base = wave * per_round; base < n_reads; base += n_waves * per_round) {
    uint32_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = base + static_cast<uint64_t>(r) * SUBS + sg;
      v[r] = 0;
      if (idx < n_reads) {
        const uint64_t g = mulhi64(fmix64(seed ^ (idx * kGolden)), n_gran);
        v[r] = buf[g * LANES + li];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc += v[r];
  }
  acc = wave_sum(acc);
  if (lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(sink), acc);
}

// Device-scope claim probe: n_ops operations at pseudo-random 64-byte
// granules, four in flight per lane.  Mode 1: one 64-bit compare-and-swap
// each.  Mode 2: an 8-byte read each and, for every other operation, a
// 64-bit compare-and-swap in the granule just read: the read-then-claim
// pattern of a find-or-put whose keys are half new.
__global__ __launch_bounds__(256) void claim_probe_kernel(uint64_t* buf, uint64_t n_gran,
                                                          uint64_t n_ops, uint32_t mode,
                                                          uint64_t seed, uint64_t* sink) {
  constexpr int R = 4;
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t n_threads = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t acc = 0;
  for (uint64_t base = tid * R; base < n_ops; base += n_threads * R) {
    uint64_t g[R], v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = base + r;
      g[r] = idx < n_ops ? mulhi64(fmix64(seed ^ (idx * kGolden)), n_gran) : 0;
      v[r] = 0;
    }
    if (mode == 2) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (base + r < n_ops) v[r] = buf[g[r] * 8];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = base + r;
      if (idx < n_ops && (mode == 1 || (idx & 1)))
        v[r] += atomicCAS(reinterpret_cast<unsigned long long*>(buf + g[r] * 8 + 1 + (v[r] & 1)),
                          ~0ull, static_cast<unsigned long long>(idx | 1));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc += v[r];
  }
  const uint32_t lo = wave_sum(static_cast<uint32_t>(acc));
  if (__lane_id() == 0) atomicAdd(reinterpret_cast<unsigned long long*>(sink), lo);
}

// ------------------------------------------------------------------ dispatch
uint32_t resident_grid(int device, uint32_t per_cu) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return static_cast<uint32_t>(cus) * per_cu;
}

hipError_t launch_find_or_put(const gx_table* t, const uint32_t* keys, uint64_t n,
                              uint8_t* status, uint64_t* n_new, hipStream_t stream) {
  FopArgs a{t->dev(), keys, t->w, n, status, n_new, resident_grid(t->device, 1), stream};
  switch (t->S) {
    case 1: return dispatch_b<1>(t->B, t->G, t->U, a);
    case 2: return dispatch_b<2>(t->B, t->G, t->U, a);
    case 4: return dispatch_b<4>(t->B, t->G, t->U, a);
  }
  return hipErrorInvalidValue;
}

hipError_t fill_words(uint32_t* p, uint64_t n_words, uint32_t value, int device,
                      hipStream_t stream) {
  if (n_words == 0) return hipSuccess;
  if (n_words % 4) return hipErrorInvalidValue;  // written as 16-byte vectors
  const uint64_t n16 = n_words / 4;
  const uint64_t want = (n16 + 255) / 256;
  const uint32_t grid = static_cast<uint32_t>(
      std::max<uint64_t>(1, std::min<uint64_t>(want, resident_grid(device, 8))));
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, stream, reinterpret_cast<uint4*>(p),
                     n16, value, static_cast<uint64_t*>(nullptr), 0u);
  return hipGetLastError();
}

namespace {

hipError_t clear_storage(const gx_table* t, hipStream_t stream) {
  const uint64_t n16 = t->n_buckets * t->B / 4;
  const uint64_t want = (n16 + 255) / 256;
  const uint32_t grid =
      static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(want, resident_grid(t->device, 8))));
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, stream,
                     reinterpret_cast<uint4*>(t->words), n16, kEmpty, t->counters,
                     t->ctr_slots * kNumCounters);
  return hipGetLastError();
}

bool pow2_in(uint32_t x, uint32_t lo, uint32_t hi) {
  return x >= lo && x <= hi && (x & (x - 1)) == 0;
}

void free_table(gx_table* t) {
  if (!t) return;
  if (t->words) (void)hipFree(t->words);
  if (t->hc) (void)hipFree(t->hc);
  if (t->counters) (void)hipFree(t->counters);
  gx_explore_buffers& e = t->eb;
  // (e.key and e.img live in e.ctr's allocation, the control block)
  for (void* p : {static_cast<void*>(e.f[0]), static_cast<void*>(e.f[1]),
                  static_cast<void*>(e.dead), static_cast<void*>(e.succ),
                  static_cast<void*>(e.ctr), static_cast<void*>(e.status),
                  static_cast<void*>(e.mon), static_cast<void*>(e.viol),
                  static_cast<void*>(e.viol_ctr), static_cast<void*>(e.img_global)})
    if (p) (void)hipFree(p);
  if (e.ctr_host) (void)hipHostFree(e.ctr_host);
  delete t;
}

}  // namespace
}  // namespace gx

// ====================================================================== ABI
using gx::kEmpty;

namespace gx {

gx_status sorted_keys(const uint32_t* dev_words, uint64_t total_words, uint32_t S, uint32_t w,
                      std::vector<uint32_t>* out, uint64_t* n_out) {
  std::vector<uint32_t> raw;
  try {
    raw.resize(total_words);
  } catch (...) {
    return GX_ENOMEM;
  }
  if (hipDeviceSynchronize() != hipSuccess ||
      (total_words && hipMemcpy(raw.data(), dev_words, total_words * sizeof(uint32_t),
                                hipMemcpyDeviceToHost) != hipSuccess))
    return GX_EDEVICE;
  const uint64_t n_slots = total_words / S;
  uint64_t count = 0;
  for (uint64_t s = 0; s < n_slots; ++s) count += raw[s * S] != kEmpty ? 1 : 0;
  try {
    out->resize(count * w);
  } catch (...) {
    return GX_ENOMEM;
  }
  if (w <= 2) {
    std::vector<uint64_t> v;
    v.reserve(count);
    for (uint64_t s = 0; s < n_slots; ++s) {
      if (raw[s * S] == kEmpty) continue;
      uint64_t x = w == 1 ? raw[s] : (static_cast<uint64_t>(raw[s * 2]) << 32) | raw[s * 2 + 1];
      v.push_back(x);  // word0 in the high half: numeric order is lexicographic
    }
    std::sort(v.begin(), v.end());
    for (uint64_t i = 0; i < count; ++i) {
      if (w == 1) {
        (*out)[i] = static_cast<uint32_t>(v[i]);
      } else {
        (*out)[2 * i] = static_cast<uint32_t>(v[i] >> 32);
        (*out)[2 * i + 1] = static_cast<uint32_t>(v[i]);
      }
    }
  } else {
    std::vector<std::array<uint32_t, 4>> v;
    v.reserve(count);
    for (uint64_t s = 0; s < n_slots; ++s) {
      if (raw[s * 4] == kEmpty) continue;
      v.push_back({raw[s * 4], raw[s * 4 + 1], raw[s * 4 + 2], w == 4 ? raw[s * 4 + 3] : 0u});
    }
    std::sort(v.begin(), v.end());
    for (uint64_t i = 0; i < count; ++i)
      for (uint32_t k = 0; k < w; ++k) (*out)[i * w + k] = v[i][k];
  }
  *n_out = count;
  return GX_OK;
}

size_t lds_per_workgroup(int device) {
  static std::atomic<int64_t> cached[64];
  static std::once_flag once;
  std::call_once(once, [] {
    for (auto& c : cached) c.store(-1);
  });
  if (device < 0 || device >= 64) return 65536;
  int64_t v = cached[device].load();
  if (v < 0) {
    int optin = 0, plain = 0;
    (void)hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device);
    (void)hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    (void)hipGetLastError();
    v = std::max<int64_t>(std::max(optin, plain), 32768) - 1024;  // room for static LDS
    cached[device].store(v);
  }
  return static_cast<size_t>(v);
}

gx_status sorted_keys_malloc(const uint32_t* dev_words, uint64_t total_words, uint32_t S,
                             uint32_t w, uint32_t** out) {
  std::vector<uint32_t> keys;
  uint64_t n = 0;
  const gx_status st = sorted_keys(dev_words, total_words, S, w, &keys, &n);
  if (st != GX_OK) return st;
  uint32_t* p = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (keys.size() + 1)));
  if (!p) return GX_ENOMEM;
  std::copy(keys.begin(), keys.end(), p);
  *out = p;
  return GX_OK;
}

}  // namespace gx

extern "C" {

const char* gx_status_str(gx_status s) {
  switch (s) {
    case GX_OK: return "GX_OK";
    case GX_EINVAL: return "GX_EINVAL: invalid argument";
    case GX_ENOMEM: return "GX_ENOMEM: out of memory or buffer too small";
    case GX_ETABLEFULL: return "GX_ETABLEFULL: hash functions exhausted";
    case GX_EDEVICE: return "GX_EDEVICE: HIP runtime error";
    case GX_EBUSY: return "GX_EBUSY";
    case GX_ECANCELED: return "GX_ECANCELED";
  }
  return "unknown gx_status";
}

gx_status gx_table_create(uint32_t w, uint32_t B, uint64_t capacity, const gx_table_opts* opts,
                          gx_table** out) {
  if (!out || w < 1 || w > 4 || !gx::pow2_in(B, 4, 64) || capacity == 0) return GX_EINVAL;
  const uint32_t S = gx::slot_words(w);
  uint32_t G = opts && opts->subgroup ? opts->subgroup : std::max<uint32_t>(8, std::min<uint32_t>(B, 64));
  uint32_t U = opts && opts->keys_per_subgroup ? opts->keys_per_subgroup : 1;
  uint32_t H = opts && opts->max_hashes ? opts->max_hashes : 8;
  uint64_t seed = opts && opts->hash_seed ? opts->hash_seed : 0x1801058570ull;
  if (!gx::pow2_in(G, 4, 64) || !gx::pow2_in(U, 1, 8) || U > G || H > 4096) return GX_EINVAL;
  if (B / std::min(G, B) > 8) return GX_EINVAL;  // at most 8 bucket words per lane
  const uint64_t slots_per_bucket = B / S;
  const uint64_t n_buckets = (capacity + slots_per_bucket - 1) / slots_per_bucket;
  if (n_buckets > (uint64_t(1) << 40)) return GX_EINVAL;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  gx_table* t = new (std::nothrow) gx_table;
  if (!t) return GX_ENOMEM;
  t->device = dev;
  t->w = w;
  t->S = S;
  t->B = B;
  t->G = G;
  t->U = U;
  t->H = H;
  t->seed = seed;
  t->n_buckets = n_buckets;
  std::vector<uint64_t> hc(2 * H);
  for (uint32_t j = 0; j < H; ++j) gx::hash_constants(seed, j, &hc[2 * j], &hc[2 * j + 1]);
  t->a0 = hc[0];
  t->c0 = hc[1];
  if (hipMalloc(&t->words, n_buckets * B * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&t->hc, hc.size() * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc(&t->counters, uint64_t(gx::kCtrSets) * gx::kNumCounters * sizeof(uint64_t)) !=
          hipSuccess) {
    (void)hipGetLastError();
    gx::free_table(t);
    return GX_ENOMEM;
  }
  t->ctr_slots = gx::kCtrSets;
  if (hipMemcpy(t->hc, hc.data(), hc.size() * sizeof(uint64_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      gx::clear_storage(t, nullptr) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
    gx::free_table(t);
    return GX_EDEVICE;
  }
  *out = t;
  return GX_OK;
}

gx_status gx_table_destroy(gx_table* t) {
  if (!t) return GX_OK;
  (void)hipDeviceSynchronize();
  gx::free_table(t);
  return GX_OK;
}

gx_status gx_table_clear(gx_table* t, void* stream) {
  if (!t) return GX_EINVAL;
  if (gx::clear_storage(t, static_cast<hipStream_t>(stream)) != hipSuccess) return GX_EDEVICE;
  t->holds_states = false;
  return GX_OK;
}

gx_status gx_find_or_put(gx_table* t, const uint32_t* keys, uint64_t n, uint8_t* status,
                         uint64_t* n_new, void* stream) {
  if (!t) return GX_EINVAL;
  if (n == 0) return GX_OK;
  if (!keys || !status) return GX_EINVAL;
  const uintptr_t align = t->S == 1 ? 4 : (t->S == 2 ? 8 : (t->w == 4 ? 16 : 4));
  if (reinterpret_cast<uintptr_t>(keys) % align != 0) return GX_EINVAL;
  if (n_new && reinterpret_cast<uintptr_t>(n_new) % 8 != 0) return GX_EINVAL;
  t->holds_states = true;
  return gx::launch_find_or_put(t, keys, n, status, n_new, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? GX_OK
             : GX_EDEVICE;
}

gx_status gx_table_get_info(const gx_table* t, gx_table_info* out) {
  if (!t || !out) return GX_EINVAL;
  out->words_per_state = t->w;
  out->slot_words = t->S;
  out->bucket_words = t->B;
  out->subgroup = t->G;
  out->keys_per_subgroup = t->U;
  out->max_hashes = t->H;
  out->n_buckets = t->n_buckets;
  out->n_slots = t->n_buckets * (t->B / t->S);
  out->hash_seed = t->seed;
  out->bytes = t->n_buckets * t->B * sizeof(uint32_t);
  return GX_OK;
}

gx_status gx_table_stats(gx_table* t, gx_stats* out) {
  if (!t || !out) return GX_EINVAL;
  std::vector<uint64_t> sets(static_cast<size_t>(t->ctr_slots) * gx::kNumCounters);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(sets.data(), t->counters, sets.size() * sizeof(uint64_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return GX_EDEVICE;
  uint64_t c[gx::kNumCounters] = {};
  for (uint32_t b = 0; b < t->ctr_slots; ++b)
    for (int k = 0; k < gx::kNumCounters; ++k) {
      const uint64_t v = sets[static_cast<size_t>(b) * gx::kNumCounters + k];
      c[k] = k == gx::kCntMaxJ ? std::max(c[k], v) : c[k] + v;
    }
  out->stored = c[gx::kCntStored];
  out->lookups = c[gx::kCntLookups];
  out->probes = c[gx::kCntProbes];
  out->full = c[gx::kCntFull];
  out->invalid = c[gx::kCntInvalid];
  out->max_hash_index = static_cast<uint32_t>(c[gx::kCntMaxJ]);
  out->reserved = 0;
  return GX_OK;
}

gx_status gx_table_read_raw(gx_table* t, uint32_t* host, uint64_t first, uint64_t n_words) {
  if (!t || (!host && n_words)) return GX_EINVAL;
  const uint64_t total = t->n_buckets * t->B;
  if (first > total || n_words > total - first) return GX_EINVAL;
  if (n_words == 0) return GX_OK;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(host, t->words + first, n_words * sizeof(uint32_t), hipMemcpyDeviceToHost) !=
          hipSuccess)
    return GX_EDEVICE;
  return GX_OK;
}

gx_status gx_table_copy_raw(gx_table* t, uint32_t* dev_words, uint64_t first, uint64_t n_words,
                            void* stream) {
  if (!t || (!dev_words && n_words)) return GX_EINVAL;
  const uint64_t total = t->n_buckets * t->B;
  if (first > total || n_words > total - first) return GX_EINVAL;
  if (n_words == 0) return GX_OK;
  if (hipMemcpyAsync(dev_words, t->words + first, n_words * sizeof(uint32_t),
                     hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)) != hipSuccess)
    return GX_EDEVICE;
  return GX_OK;
}

gx_status gx_table_dump(gx_table* t, uint32_t* host_keys, uint64_t cap, uint64_t* n_out) {
  if (!t || !n_out) return GX_EINVAL;
  std::vector<uint32_t> keys;
  uint64_t count = 0;
  const gx_status s = gx::sorted_keys(t->words, t->n_buckets * t->B, t->S, t->w, &keys, &count);
  if (s != GX_OK) return s;
  *n_out = count;
  if (!host_keys || cap < count) return GX_ENOMEM;
  std::copy(keys.begin(), keys.end(), host_keys);
  return GX_OK;
}

gx_status gx_hash_bucket(const uint32_t* key, uint32_t w, uint64_t seed, uint32_t j,
                         uint64_t n_buckets, uint64_t* bucket) {
  if (!key || !bucket || w < 1 || w > 4 || n_buckets == 0) return GX_EINVAL;
  if (seed == 0) seed = 0x1801058570ull;
  uint64_t a, c, mix;
  gx::hash_constants(seed, j, &a, &c);
  if (w == 1) {
    const uint32_t k[1] = {key[0]};
    mix = gx::key_mix<1>(k, seed);
  } else if (w == 2) {
    const uint32_t k[2] = {key[0], key[1]};
    mix = gx::key_mix<2>(k, seed);
  } else {
    const uint32_t k[4] = {key[0], key[1], key[2], w == 4 ? key[3] : 0u};
    mix = gx::key_mix<4>(k, seed);
  }
  *bucket = gx::bucket_of(mix, a, c, n_buckets);
  return GX_OK;
}

gx_status gx_claim_probe(uint64_t* buf, uint64_t buf_bytes, uint32_t mode, uint64_t n_ops,
                         uint64_t seed, uint64_t* sink, void* stream) {
  if (!buf || !sink || buf_bytes < 64 || (mode != 1 && mode != 2)) return GX_EINVAL;
  if (reinterpret_cast<uintptr_t>(buf) % 64 != 0) return GX_EINVAL;
  if (n_ops == 0) return GX_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  const uint32_t grid = static_cast<uint32_t>(std::max<uint64_t>(
      1, std::min<uint64_t>((n_ops + 1023) / 1024, gx::resident_grid(dev, 8))));
  hipLaunchKernelGGL(gx::claim_probe_kernel, dim3(grid), dim3(256), 0,
                     static_cast<hipStream_t>(stream), buf, buf_bytes / 64, n_ops, mode, seed, sink);
  return hipGetLastError() == hipSuccess ? GX_OK : GX_EDEVICE;
}

gx_status gx_gather_probe(const uint32_t* buf, uint64_t buf_bytes, uint32_t granule,
                          uint64_t n_reads, uint64_t seed, uint64_t* sink, void* stream) {
  if (!buf || !sink || !gx::pow2_in(granule, 4, 256) || buf_bytes < granule) return GX_EINVAL;
  if (reinterpret_cast<uintptr_t>(buf) % granule != 0) return GX_EINVAL;
  if (n_reads == 0) return GX_OK;
  const uint64_t n_gran = buf_bytes / granule;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GX_EDEVICE;
  const uint32_t lanes = granule / 4;
  const uint64_t per_block = 4ull * (64 / lanes) * 4;
  const uint32_t grid = static_cast<uint32_t>(std::max<uint64_t>(
      1, std::min<uint64_t>((n_reads + per_block - 1) / per_block, gx::resident_grid(dev, 8))));
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (lanes) {
#define GX_PROBE_CASE(L)                                                                     \
  case L:                                                                                    \
    hipLaunchKernelGGL(gx::gather_probe_kernel<L>, dim3(grid), dim3(256), 0, st, buf, n_gran, \
                       n_reads, seed, sink);                                                 \
    break;
    GX_PROBE_CASE(1)
    GX_PROBE_CASE(2)
    GX_PROBE_CASE(4)
    GX_PROBE_CASE(8)
    GX_PROBE_CASE(16)
    GX_PROBE_CASE(32)
    GX_PROBE_CASE(64)
#undef GX_PROBE_CASE
    default:
      return GX_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? GX_OK : GX_EDEVICE;
}

}  // extern "C"
