// Device core of the bucketed find-or-put table (Sec. 4.1 and 4.2 of
// "On the Scalability of the GPUexplore Explicit-State Model Checker").
//
// Table layout: n_buckets buckets of B 32-bit words, bucket b at words
// [b*B, b*B + B).  A key of w words lives in a slot of S words (S = w, or 4
// for w = 3 with the fourth word 0); a bucket holds B/S slots, slot s at
// bucket words [s*S, s*S + S).  Unused words hold kEmpty.  No key word may be
// kEmpty, so a slot is EMPTY (every word kEmpty), FINAL (no word kEmpty) or,
// transiently, PARTIAL.
//
// Probe (one subgroup of G lanes per key, G in {8,16,32,64}; the paper uses a
// warp of 32 per bucket of 32 integers, and groups of B threads for buckets of
// B integers, Sec. 4.2):
//   * the first GE = min(G, B) lanes each load K = B/GE consecutive words of
//     the bucket (one coalesced access of B*4 bytes per bucket);
//   * every lane compares its words with the key; ballots give per-slot
//     "match", "empty" and "partial" masks for the subgroup;
//   * match -> SEEN.  Otherwise the lane owning the lowest EMPTY slot tries a
//     compare-and-swap of the key into it (32-bit for S = 1, 64-bit for S = 2,
//     64-bit on words 0-1 for S = 4 followed by a store of words 2-3); a
//     failed CAS that returned the key -> SEEN, any other failure -> re-read
//     the bucket; no EMPTY slot -> next hash function (Sec. 4.1); after H
//     buckets -> FULL.
//
// Memory-model argument (why relaxed atomics are enough): every slot word is
// written exactly once, from kEmpty to its final value, and no reader derives
// anything from a slot except by comparing its words with a key.  A stale
// kEmpty from a plain load only costs a failed CAS, whose returned value is
// compared; a non-kEmpty value is final.  A PARTIAL slot (a head claimed and
// its tail not yet stored, or a torn read of a 64-bit slot) blocks claiming in
// its bucket until a re-read, done with agent-scope atomic loads, shows it
// EMPTY or FINAL.  Every inserter visits buckets in the same h_0, h_1, ...
// order and claims only the lowest EMPTY slot after comparing every FINAL
// slot, so a key is never stored twice.
//
// Forward progress: a lane that wins a head CAS stores the tail in the same
// straight-line step; waiting for someone else's tail is never a spin inside a
// branch but another pass of the outer loop, so lanes of one wavefront cannot
// wait on each other.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gx {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

enum : uint8_t { kSeen = 0, kNew = 1, kFull = 2, kInvalid = 3 };

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t fmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return static_cast<uint64_t>((static_cast<unsigned __int128>(a) * b) >> 64);
}

// 64-bit mix of a slot-format key (S words, the padding word of a 3-word key
// is 0) under the table seed.
template <int S>
__host__ __device__ inline uint64_t key_mix(const uint32_t (&k)[S], uint64_t seed) {
  uint64_t x = k[0];
  if constexpr (S >= 2) x |= static_cast<uint64_t>(k[1]) << 32;
  if constexpr (S == 4) {
    x = fmix64(x ^ seed) ^ (static_cast<uint64_t>(k[2]) | (static_cast<uint64_t>(k[3]) << 32));
  }
  return fmix64(x ^ seed);
}

// j-th set of hash constants (a_j odd, c_j) drawn from the seed.
__host__ __device__ inline void hash_constants(uint64_t seed, uint32_t j, uint64_t* a,
                                               uint64_t* c) {
  *a = fmix64(seed + (2ull * j + 1ull) * kGolden) | 1ull;
  *c = fmix64(seed + (2ull * j + 2ull) * kGolden);
}

__host__ __device__ inline uint64_t bucket_of(uint64_t mix, uint64_t a, uint64_t c,
                                              uint64_t n_buckets) {
  return mulhi64(a * mix + c, n_buckets);
}

// Counters kept with every table (one u64 each).
enum Counter : int {
  kCntStored = 0,
  kCntLookups = 1,
  kCntProbes = 2,
  kCntFull = 3,
  kCntInvalid = 4,
  kCntMaxJ = 5,
  kNumCounters = 8
};

// Statistics counter sets per table: workgroups add to set blockIdx % sets,
// so the adds at the end of a launch spread over many cache lines instead
// of all meeting on one (a launch of 2^20 keys spent most of its time
// there); readers sum the sets.
constexpr uint32_t kCtrSets = 2048;

struct TableDev {
  uint32_t* words;
  uint64_t n_buckets;
  const uint64_t* hc;  // 2*H hash constants: a_0, c_0, a_1, c_1, ...
  uint64_t seed;
  uint64_t a0, c0;     // first constant set, passed by value
  uint32_t H;
  uint64_t* counters;  // ctr_slots sets of kNumCounters words
  uint32_t ctr_slots = 1;  // workgroup b adds its statistics to set b % ctr_slots
};

// A value every lane of the wavefront holds the same copy of, moved to a
// scalar register (for table descriptors read from memory at run time, so
// they do not take vector registers in the probe loops).
__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return (static_cast<uint64_t>(uniform32(static_cast<uint32_t>(x >> 32))) << 32) |
         uniform32(static_cast<uint32_t>(x));
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform64(reinterpret_cast<uint64_t>(p)));
}
__device__ __forceinline__ TableDev uniform_table(const TableDev& t) {
  TableDev u;
  u.words = uniform_ptr(t.words);
  u.n_buckets = uniform64(t.n_buckets);
  u.hc = uniform_ptr(t.hc);
  u.seed = uniform64(t.seed);
  u.a0 = uniform64(t.a0);
  u.c0 = uniform64(t.c0);
  u.H = uniform32(t.H);
  u.counters = uniform_ptr(t.counters);
  u.ctr_slots = uniform32(t.ctr_slots);
  return u;
}

template <int S, int B, int G>
struct Geo {
  static_assert(S == 1 || S == 2 || S == 4, "slot words");
  static_assert(B == 4 || B == 8 || B == 16 || B == 32 || B == 64, "bucket words");
  static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "subgroup width");
  static_assert(B / (G < B ? G : B) <= 8, "at most 8 bucket words per lane");
  static constexpr int GE = G < B ? G : B;          // lanes holding bucket words
  static constexpr int K = B / GE;                  // words per lane
  static constexpr int L = K >= S ? 1 : S / K;      // lanes per slot
  static constexpr int SPL = K >= S ? K / S : 1;    // whole slots per lane
  static constexpr int SUBS = 64 / G;               // subgroups per wavefront
  static constexpr uint64_t GMASK = G == 64 ? ~0ull : ((1ull << G) - 1ull);
  // bits 0, L, 2L, ... below GE
  static constexpr uint64_t lead_mask() {
    uint64_t m = 0;
    for (int i = 0; i < GE; i += L) m |= 1ull << i;
    return m;
  }
};

template <int K>
__device__ inline void load_view(const uint32_t* p, uint32_t (&v)[K]) {
  if constexpr (K == 1) {
    v[0] = p[0];
  } else if constexpr (K == 2) {
    uint2 t = *reinterpret_cast<const uint2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else if constexpr (K == 4) {
    uint4 t = *reinterpret_cast<const uint4*>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
  } else {
    static_assert(K == 8, "words per lane");
    uint4 t0 = reinterpret_cast<const uint4*>(p)[0];
    uint4 t1 = reinterpret_cast<const uint4*>(p)[1];
    v[0] = t0.x;
    v[1] = t0.y;
    v[2] = t0.z;
    v[3] = t0.w;
    v[4] = t1.x;
    v[5] = t1.y;
    v[6] = t1.z;
    v[7] = t1.w;
  }
}

// Re-read with agent-scope atomic loads: never served from a stale cache line.
template <int K>
__device__ inline void load_view_fresh(uint32_t* p, uint32_t (&v)[K]) {
#pragma unroll
  for (int t = 0; t < K; ++t) {
    v[t] = __hip_atomic_load(p + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// k[idx] for a run-time idx, with mask arithmetic (see get_field in the
// exploration kernel: a select chain becomes a private-array indexed load).
template <int S>
__device__ __forceinline__ uint32_t key_word(const uint32_t (&k)[S], int idx) {
  uint32_t x = 0;
#pragma unroll
  for (int t = 0; t < S; ++t) x |= k[t] & (0u - static_cast<uint32_t>(idx == t));
  return x;
}

// Result of comparing one bucket view with a key, uniform over a subgroup.
struct Eval {
  bool match;     // a FINAL slot equals the key
  bool partial;   // some slot is PARTIAL
  int claim_lane; // lane (within the subgroup) owning the lowest EMPTY slot, -1 if none
  int claim_word; // on the claiming lane: offset of that slot within the lane's words
};

template <int S, int B, int G>
__device__ inline Eval evaluate(const uint32_t (&v)[Geo<S, B, G>::K], const uint32_t (&key)[S],
                                int li, int shift) {
  using Gm = Geo<S, B, G>;
  constexpr int K = Gm::K;
  Eval ev;
  if constexpr (Gm::L == 1) {
    uint32_t em = 0;
    bool mt = false, pt = false;
    if (li < Gm::GE) {
#pragma unroll
      for (int s = 0; s < Gm::SPL; ++s) {
        bool alle = true, alln = true, eq = true;
#pragma unroll
        for (int t = 0; t < S; ++t) {
          uint32_t x = v[s * S + t];
          alle &= (x == kEmpty);
          alln &= (x != kEmpty);
          eq &= (x == key[t]);
        }
        em |= static_cast<uint32_t>(alle) << s;
        mt |= alln && eq;
        pt |= !alle && !alln;
      }
    }
    const uint64_t M = (__ballot(mt) >> shift) & Gm::GMASK;
    const uint64_t P = (__ballot(pt) >> shift) & Gm::GMASK;
    const uint64_t E = (__ballot(em != 0) >> shift) & Gm::GMASK;
    ev.match = M != 0;
    ev.partial = P != 0;
    ev.claim_lane = E ? (__ffsll(static_cast<unsigned long long>(E)) - 1) : -1;
    ev.claim_word = em ? (__ffs(em) - 1) * S : 0;
  } else {
    constexpr int L = Gm::L;
    bool fe = false, ff = false, fq = false;
    if (li < Gm::GE) {
      fe = true;
      ff = true;
      fq = true;
      const int off = (li % L) * K;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        uint32_t x = v[t];
        fe &= (x == kEmpty);
        ff &= (x != kEmpty);
        fq &= (x == key_word<S>(key, off + t));
      }
    }
    const uint64_t E = (__ballot(fe) >> shift) & Gm::GMASK;
    const uint64_t F = (__ballot(ff) >> shift) & Gm::GMASK;
    const uint64_t Q = (__ballot(fq && ff) >> shift) & Gm::GMASK;
    uint64_t ae = E, af = F, aq = Q;
#pragma unroll
    for (int d = 1; d < L; ++d) {
      ae &= E >> d;
      af &= F >> d;
      aq &= Q >> d;
    }
    constexpr uint64_t lead = Gm::lead_mask();
    ae &= lead;
    af &= lead;
    aq &= lead;
    ev.match = aq != 0;
    ev.partial = (ae | af) != lead;
    ev.claim_lane = ae ? (__ffsll(static_cast<unsigned long long>(ae)) - 1) : -1;
    ev.claim_word = 0;
  }
  return ev;
}

// Statistics of a wavefront's find-or-puts.  The per-key outcomes (stored,
// lookups, full, invalid) are counted once per call with ballots, so they are
// wavefront-uniform and live in scalar registers; bucket reads and the
// longest hash chain are per lane (subgroup leaders), reduced at the end.
struct LaneStats {
  uint32_t stored = 0, lookups = 0, full = 0, invalid = 0;  // wavefront totals
  uint32_t probes = 0, max_j = 0;                            // per lane
};

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__device__ inline uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t y = __shfl_xor(x, d, 64);
    x = y > x ? y : x;
  }
  return x;
}

__device__ inline void flush_stats(const TableDev& t, const LaneStats& st, uint64_t* n_new) {
  const uint32_t stored = st.stored, lookups = st.lookups, full = st.full, invalid = st.invalid;
  const uint32_t probes = wave_sum(st.probes);
  const uint32_t mj = wave_max(st.max_j);
  if (__lane_id() != 0) return;
  if (stored && n_new) atomicAdd(reinterpret_cast<unsigned long long*>(n_new), stored);
  if (t.counters == nullptr) return;  // a table that keeps no statistics
  uint64_t* c = t.counters + static_cast<uint64_t>(blockIdx.x % t.ctr_slots) * kNumCounters;
  if (stored) atomicAdd(reinterpret_cast<unsigned long long*>(&c[kCntStored]), stored);
  if (lookups) atomicAdd(reinterpret_cast<unsigned long long*>(&c[kCntLookups]), lookups);
  if (probes) atomicAdd(reinterpret_cast<unsigned long long*>(&c[kCntProbes]), probes);
  if (full) atomicAdd(reinterpret_cast<unsigned long long*>(&c[kCntFull]), full);
  if (invalid) atomicAdd(reinterpret_cast<unsigned long long*>(&c[kCntInvalid]), invalid);
  if (mj) atomicMax(reinterpret_cast<unsigned long long*>(&c[kCntMaxJ]), mj);
}

// Find-or-put of U keys per subgroup.  Every lane of a subgroup holds the same
// U keys (slot format, no word kEmpty), their 64-bit mixes and first buckets.
// act[u] false: no key.  On return res[u] is kNew / kSeen / kFull for active
// keys.  Must be reached by the whole wavefront (it ballots across it).
template <int S, int B, int G, int U>
__device__ inline void find_or_put(const TableDev& t, const uint32_t (&key)[U][S],
                                   const uint64_t (&mix)[U], const uint64_t (&bkt0)[U],
                                   const bool (&act_in)[U], uint8_t (&res)[U], LaneStats& st) {
  using Gm = Geo<S, B, G>;
  constexpr int K = Gm::K;
  const int lane = __lane_id();
  const int li = lane % G;
  const int shift = (lane / G) * G;

  bool act[U];
  uint32_t j[U];
  uint64_t bkt[U];
  uint32_t view[U][K];

  // issue every first bucket read before looking at any of them
#pragma unroll
  for (int u = 0; u < U; ++u) {
    act[u] = act_in[u];
    res[u] = kSeen;
    j[u] = 0;
    bkt[u] = bkt0[u];
#pragma unroll
    for (int w = 0; w < K; ++w) view[u][w] = kEmpty;
    if (act[u]) {
      if (li < Gm::GE) load_view<K>(t.words + bkt[u] * B + li * K, view[u]);
      if (li == 0) ++st.probes;
    }
  }

  while (true) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < U; ++u) any |= act[u];
    if (!__any(any)) break;
    // Pass 1: compare every view; issue the compare-and-swaps and next-bucket
    // reads of all U keys before consuming any result, so the U round trips
    // of a subgroup overlap.
    bool claiming[U], reread[U];
    int cl[U], cw[U];
    uint64_t old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      claiming[u] = false;
      reread[u] = false;
      cl[u] = 0;
      cw[u] = 0;
      old[u] = ~0ull;
      if (!act[u]) continue;
      const Eval ev = evaluate<S, B, G>(view[u], key[u], li, shift);
      if (ev.match) {
        res[u] = kSeen;
        act[u] = false;
      } else if (ev.partial) {
        reread[u] = true;
      } else if (ev.claim_lane >= 0) {
        claiming[u] = true;
        cl[u] = ev.claim_lane;
        cw[u] = ev.claim_word;
        if (li == ev.claim_lane) {
          uint32_t* slot = t.words + bkt[u] * B + li * K + ev.claim_word;
          if constexpr (S == 1) {
            uint32_t exp = kEmpty;
            __hip_atomic_compare_exchange_strong(slot, &exp, key[u][0], __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            old[u] = 0xFFFFFFFF00000000ull | exp;
          } else {
            const uint64_t head =
                static_cast<uint64_t>(key[u][0]) | (static_cast<uint64_t>(key[u][1]) << 32);
            uint64_t exp = ~0ull;
            __hip_atomic_compare_exchange_strong(reinterpret_cast<uint64_t*>(slot), &exp, head,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            old[u] = exp;
          }
        }
      } else {
        // bucket full of other keys: next set of hash constants
        ++j[u];
        if (j[u] >= t.H) {
          res[u] = kFull;
          act[u] = false;
        } else {
          const uint64_t a = t.hc[2 * j[u]], c = t.hc[2 * j[u] + 1];
          bkt[u] = bucket_of(mix[u], a, c, t.n_buckets);
          if (li < Gm::GE) load_view<K>(t.words + bkt[u] * B + li * K, view[u]);
          if (li == 0) ++st.probes;
        }
      }
    }
    // Pass 2: consume the compare-and-swap results.  A CAS succeeded when it
    // returned the empty slot value.
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!claiming[u]) continue;
      bool won = false, same = false;
      uint32_t o0 = kEmpty, o1 = kEmpty, o2 = kEmpty, o3 = kEmpty;
      if (li == cl[u]) {
        uint32_t* slot = t.words + bkt[u] * B + li * K + cw[u];
        o0 = static_cast<uint32_t>(old[u]);
        o1 = static_cast<uint32_t>(old[u] >> 32);
        if constexpr (S == 1) {
          won = o0 == kEmpty;
          same = o0 == key[u][0];
        } else {
          const uint64_t head =
              static_cast<uint64_t>(key[u][0]) | (static_cast<uint64_t>(key[u][1]) << 32);
          won = old[u] == ~0ull;
          if constexpr (S == 2) {
            same = old[u] == head;
          } else {
            const uint64_t tail =
                static_cast<uint64_t>(key[u][2]) | (static_cast<uint64_t>(key[u][3]) << 32);
            if (won) {
              // publish the tail in the same step as the claim is known
              __hip_atomic_store(reinterpret_cast<uint64_t*>(slot + 2), tail, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
            } else if (old[u] == head) {
              // same head: the tail decides (still kEmpty while its owner has
              // not stored it, which leaves the slot PARTIAL)
              const uint64_t got = __hip_atomic_load(reinterpret_cast<uint64_t*>(slot + 2),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              same = got == tail;
              o2 = static_cast<uint32_t>(got);
              o3 = static_cast<uint32_t>(got >> 32);
            } else {
              // another key's head: the slot can never match; any non-kEmpty
              // placeholder for its tail keeps it FINAL in the view
              o2 = 0;
              o3 = 0;
            }
          }
        }
      }
      const uint64_t W = (__ballot(won) >> shift) & Gm::GMASK;
      const uint64_t Sm = (__ballot(same) >> shift) & Gm::GMASK;
      if (W) {
        res[u] = kNew;
        act[u] = false;
      } else if (Sm) {
        res[u] = kSeen;
        act[u] = false;
      } else {
        // Patch the view with what the CAS saw: that slot is no longer a
        // candidate, so every failed CAS retires one slot for good and the
        // loop makes progress whatever the plain loads returned.
        const int src = shift + cl[u];
        const uint32_t sv[4] = {__shfl(o0, src, 64), __shfl(o1, src, 64), __shfl(o2, src, 64),
                                __shfl(o3, src, 64)};
        const int c0 = cl[u] * K + __shfl(cw[u], src, 64);
#pragma unroll
        for (int x = 0; x < K; ++x) {
          const int d = li * K + x - c0;
          if (li < Gm::GE && d >= 0 && d < S) view[u][x] = key_word<4>(sv, d);
        }
      }
    }
    // Pass 3: re-read buckets that held a PARTIAL slot.
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (reread[u]) {
        if (li < Gm::GE) load_view_fresh<K>(t.words + bkt[u] * B + li * K, view[u]);
        if (li == 0) ++st.probes;
      }
      if (!act[u] && li == 0 && res[u] != kFull && j[u] > st.max_j) st.max_j = j[u];
    }
  }
}

// Find-or-put of one key per lane: lane l of the wavefront owns key `own`
// (slot format) when own_act.  Each lane hashes its own key (64 hashes per
// wavefront, no redundant work); subgroup g then probes the keys owned by its
// G lanes, U at a time, receiving key, mix and first bucket from the owner by
// lane shuffles; the result comes back to the owner lane.  Returns the owner's
// status (kNew / kSeen / kFull / kInvalid).  Must be reached by the whole
// wavefront.
template <int S, int B, int G, int U>
__device__ inline uint8_t find_or_put_lanes(const TableDev& t, const uint32_t (&own)[S],
                                            bool own_act, LaneStats& st) {
  static_assert(U >= 1 && U <= G && (G % U) == 0, "keys in flight per subgroup");
  const int lane = __lane_id();
  const int li = lane % G;
  const int first = lane - li;  // first lane of this subgroup
  uint8_t own_res = kSeen;
  bool bad = false;
#pragma unroll
  for (int w = 0; w < S; ++w) bad |= own[w] == kEmpty;
  if (own_act && bad) {
    own_res = kInvalid;
    own_act = false;
  }
  const uint64_t own_mix = key_mix<S>(own, t.seed);
  const uint64_t own_bkt = bucket_of(own_mix, t.a0, t.c0, t.n_buckets);
#pragma unroll 1
  for (int c = 0; c < G; c += U) {
    uint32_t key[U][S];
    uint64_t mix[U], bkt[U];
    bool act[U];
    uint8_t res[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int src = first + c + u;
#pragma unroll
      for (int w = 0; w < S; ++w) key[u][w] = __shfl(own[w], src, 64);
      mix[u] = (static_cast<uint64_t>(__shfl(static_cast<uint32_t>(own_mix >> 32), src, 64)) << 32) |
               __shfl(static_cast<uint32_t>(own_mix), src, 64);
      bkt[u] = (static_cast<uint64_t>(__shfl(static_cast<uint32_t>(own_bkt >> 32), src, 64)) << 32) |
               __shfl(static_cast<uint32_t>(own_bkt), src, 64);
      act[u] = __shfl(static_cast<int>(own_act), src, 64) != 0;
    }
    find_or_put<S, B, G, U>(t, key, mix, bkt, act, res, st);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (li == c + u && own_act) own_res = res[u];
  }
  st.lookups += static_cast<uint32_t>(__popcll(__ballot(own_act)));
  st.invalid += static_cast<uint32_t>(__popcll(__ballot(own_res == kInvalid)));
  st.stored += static_cast<uint32_t>(__popcll(__ballot(own_res == kNew)));
  st.full += static_cast<uint32_t>(__popcll(__ballot(own_res == kFull)));
  return own_res;
}

}  // namespace gx
