// Exploration level kernel and its (B, G, U) dispatch for one slot width S;
// each slot width is instantiated in a translation unit of its own.
#pragma once

#include <cstdint>
#include <type_traits>

#include "gx_internal.hpp"

namespace gx {

constexpr uint32_t kImgMaxWords = 11776;  // 46 KiB of LDS for the network image
constexpr uint32_t kStageWords = 4096;    // 16 KiB of LDS for staged successors

// ------------------------------------------------------------------ kernel

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

template <int S>
__device__ __forceinline__ void load_slot(const uint32_t* p, uint32_t (&k)[S]) {
  if constexpr (S == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    k[0] = v.x;
    k[1] = v.y;
    k[2] = v.z;
    k[3] = v.w;
  } else if constexpr (S == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    k[0] = v.x;
    k[1] = v.y;
  } else {
    k[0] = *p;
  }
}

// A three-word state's words without its slot's fourth (zero) word, and back.
template <int S>
__device__ __forceinline__ void store_words3(uint32_t* p, const uint32_t (&k)[S]) {
#pragma unroll
  for (int x = 0; x < 3 && x < S; ++x) p[x] = k[x];
}

template <int S>
__device__ __forceinline__ void load_words3(const uint32_t* p, uint32_t (&k)[S]) {
#pragma unroll
  for (int x = 0; x < S; ++x) k[x] = x < 3 ? p[x] : 0u;
}

template <int S>
__device__ __forceinline__ void store_slot(uint32_t* p, const uint32_t (&k)[S]) {
  if constexpr (S == 4) {
    *reinterpret_cast<uint4*>(p) = make_uint4(k[0], k[1], k[2], k[3]);
  } else if constexpr (S == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(k[0], k[1]);
  } else {
    *p = k[0];
  }
}

// The wavefront's successors, numbered in the order below, with numbers in
// [lo, hi) written to out[(k - lo) * S] (global memory or LDS) with
// coalesced stores.  The lanes walk their transitions in step: every loop
// runs until no lane has work left in it (its exit test is a ballot, so the
// wavefront never splits), and at each step the lanes that form a successor
// take consecutive numbers after those the wavefront has numbered so far.
// One store instruction thus covers a contiguous run of slots, where a run
// per lane would touch a cache line per lane.  kWindow: runs whose numbers
// all lie below lo are counted with one wavefront sum instead of walked, and
// the walk stops at hi (used to expand a wavefront's successors chunk by
// chunk); without it the window must be [0, total), or [0, hi) with hi at
// least the total.  Must be reached by the whole wavefront; a lane without a
// state passes has = false.  Optional outputs: *total, the wavefront's
// successors (without the window: all of them), and *mine, this lane's.
// kMaxGroup (1 or 4): the widest group of targets read per LDS round trip.
// out_words: words per successor in out (S; or 3 with S = 4, the three words
// of a three-word state without its slot's zero fourth word).
template <int S, bool kWindow, int kMaxGroup = 4>
__device__ __forceinline__ void emit_window(const uint32_t* img, const uint32_t (&sw)[S],
                                            bool has, uint32_t* out, uint32_t lo, uint32_t hi,
                                            uint32_t* total = nullptr, uint32_t* mine = nullptr,
                                            uint32_t out_words = S) {
  const uint32_t P = img[0], R = img[1];
  uint32_t cur = 0;  // successors the wavefront has numbered (the same in every lane)
  uint32_t own = 0;  // this lane's
  auto put = [&](bool act, const uint32_t (&succ)[S]) {
    const uint64_t m = __ballot(act);
    const uint32_t k = cur + __builtin_amdgcn_mbcnt_hi(
                                 static_cast<uint32_t>(m >> 32),
                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
    if (act && k >= lo && k < hi) {
      if (S == 4 && out_words == 3)
        store_words3<S>(out + static_cast<uint64_t>(k - lo) * 3, succ);
      else
        store_slot<S>(out + static_cast<uint64_t>(k - lo) * S, succ);
    }
    cur += static_cast<uint32_t>(__popcll(m));
    if (mine) own += act ? 1u : 0u;
  };
  // true when all n successors per lane still to come lie below the window:
  // then they are only counted
  auto below = [&](uint32_t n) -> bool {
    if constexpr (kWindow) {
      const uint32_t tot = __builtin_amdgcn_readfirstlane(wave_sum(n));
      if (cur + tot <= lo) {
        cur += tot;
        return true;
      }
    }
    return false;
  };
  // successors: `from` with field f set to each of img[s0 .. s0 + n); targets
  // are read from LDS g at a time before any successor of the group is
  // formed, so one LDS round trip serves up to g successors
  auto run_group = [&](auto g, const uint32_t (&from)[S], uint32_t f, uint32_t s0, uint32_t n) {
    constexpr int kG = decltype(g)::value;
    for (uint32_t t = 0; cur < hi && __ballot(t < n); t += kG) {
      uint32_t d[kG];
#pragma unroll
      for (int k = 0; k < kG; ++k) d[k] = t + k < n ? img[s0 + t + k] : 0u;
#pragma unroll
      for (int k = 0; k < kG; ++k) {
        uint32_t succ[S];
#pragma unroll
        for (int x = 0; x < S; ++x) succ[x] = from[x];
        set_field<S>(succ, f, d[k]);
        put(t + k < n, succ);
      }
    }
  };
  // the group is as wide as the wavefront's widest run needs, up to four: a
  // slot of a group that no lane fills still costs its wavefront-wide
  // numbering, and narrow runs (one or two targets) are the common case.
  // kMaxGroup = 1: always one (the latency-bound one-workgroup levels, where
  // the three inlined group widths cost more than wider groups save)
  auto run = [&](const uint32_t (&from)[S], uint32_t f, uint32_t s0, uint32_t n) {
    if (below(n)) return;
    if (kMaxGroup == 1 || !__ballot(n > 1)) run_group(std::integral_constant<int, 1>{}, from, f, s0, n);
    else if (!__ballot(n > 2)) run_group(std::integral_constant<int, 2>{}, from, f, s0, n);
    else run_group(std::integral_constant<int, 4>{}, from, f, s0, n);
  };
  for (uint32_t p = 0; p < P && cur < hi; ++p) {
    const uint32_t f = img[4 + p];
    const uint32_t l = get_field<S>(sw, f);
    const uint32_t ob = img[4 + P + p];
    const uint32_t s0 = img[ob + l];
    run(sw, f, s0, has ? img[ob + l + 1] - s0 : 0u);
  }
  for (uint32_t r = 0; r < R && cur < hi; ++r) {
    const uint32_t rb = img[4 + 2 * P + r];
    const uint32_t np = img[rb];
    if (np == 2) {
      // two participants (the common rendezvous): their target ranges are
      // read once, the combinations enumerated by two nested loops
      const uint32_t f0 = img[4 + img[rb + 1]], ob0 = img[rb + 2];
      const uint32_t f1 = img[4 + img[rb + 3]], ob1 = img[rb + 4];
      const uint32_t l0 = get_field<S>(sw, f0), l1 = get_field<S>(sw, f1);
      const uint32_t a0 = img[ob0 + l0], e0 = img[ob0 + l0 + 1];
      const uint32_t a1 = img[ob1 + l1], n1 = img[ob1 + l1 + 1] - a1;
      const uint32_t n0 = has && n1 ? e0 - a0 : 0u;
      if (below(n0 * n1)) continue;
      for (uint32_t t0 = 0; cur < hi && __ballot(t0 < n0); ++t0) {
        const bool act = t0 < n0;
        uint32_t mid[S];
#pragma unroll
        for (int x = 0; x < S; ++x) mid[x] = sw[x];
        set_field<S>(mid, f0, act ? img[a0 + t0] : 0u);
        run(mid, f1, a1, act ? n1 : 0u);
      }
      continue;
    }
    uint32_t prod = has ? 1u : 0u;
    for (uint32_t i = 0; i < np && prod; ++i) {
      const uint32_t q = img[rb + 1 + 2 * i], ob = img[rb + 2 + 2 * i];
      const uint32_t l = get_field<S>(sw, img[4 + q]);
      prod *= img[ob + l + 1] - img[ob + l];
    }
    if (below(prod)) continue;
    for (uint32_t c = 0; cur < hi && __ballot(c < prod); ++c) {
      const bool act = c < prod;
      uint32_t succ[S];
#pragma unroll
      for (int x = 0; x < S; ++x) succ[x] = sw[x];
      if (act) {
        uint32_t rem = c;
        for (uint32_t i = 0; i < np; ++i) {
          const uint32_t q = img[rb + 1 + 2 * i], ob = img[rb + 2 + 2 * i];
          const uint32_t fq = img[4 + q];
          const uint32_t l = get_field<S>(sw, fq);
          const uint32_t b0 = img[ob + l], cnt = img[ob + l + 1] - b0;
          set_field<S>(succ, fq, img[b0 + rem % cnt]);
          rem /= cnt;
        }
      }
      put(act, succ);
    }
  }
  if (total) *total = cur;
  if (mine) *mine = own;
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

// An exploration's counters live kCtrSpread words apart, each on a cache
// line of its own: every wavefront of a level updates some of them, and
// counters sharing a line would serialise at one L2 atomic unit.
constexpr uint32_t kCtrSpread = 16;
enum : uint32_t { kCtrTail = 0, kCtrDead = 1, kCtrTrans = 2, kCtrFlags = 3, kCtrDups = 4,
                  kCtrSucc = 5, kCtrSuccAlt = 6, kCtrCount = 7 };

__device__ __forceinline__ unsigned long long* ctr_at(uint64_t* ctr, uint32_t k) {
  return reinterpret_cast<unsigned long long*>(ctr + k * kCtrSpread);
}

// One wavefront's share of a BFS level: frontier states [first, first + 64)
// (those below n_in) of one exploration.  Counters of that exploration:
// Counters of that exploration: ctr_at(ctr, kCtrTail / kCtrDead / kCtrTrans /
// kCtrFlags / kCtrDups).
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

// Local duplicate filter (the block-local state cache of the tool, Sec. 3):
// the first occurrence of a successor among the n_st staged in this chunk
// claims an entry of the wavefront's LDS set `dtab`; later occurrences find it
// and are marked in *dupmask (bit r: this lane's staged index of round r,
// r0 = 64 r).  Returns the wavefront's number of marked successors.  Must be
// reached by the whole wavefront; the staged chunk is only read.
template <int S>
__device__ inline uint32_t dedup_chunk(uint32_t* dtab, const uint32_t* stage, uint32_t n_st,
                                       uint32_t* dupmask) {
  constexpr uint32_t D = dedup_entries<S>();
  const int lane = __lane_id();
  for (uint32_t e = lane; e < D; e += 64) dtab[e] = kEmpty;
  wave_lds_sync();
  uint32_t dups = 0, mask = 0;
  for (uint32_t r0 = 0, r = 0; r0 < n_st; r0 += 64, ++r) {
    const uint32_t idx = r0 + lane;
    if (idx < n_st) {
      uint32_t key[S];
#pragma unroll
      for (int x = 0; x < S; ++x) key[x] = stage[idx * S + x];
      uint32_t h = dedup_hash<S>(key) & (D - 1);
      while (true) {
        uint32_t prev = kEmpty;
        if (__hip_atomic_compare_exchange_strong(&dtab[h], &prev, idx, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT))
          break;  // first occurrence
        bool same = true;
#pragma unroll
        for (int x = 0; x < S; ++x) same &= stage[prev * S + x] == key[x];
        if (same) {
          mask |= 1u << r;
          ++dups;
          break;
        }
        h = (h + 1) & (D - 1);
      }
    }
  }
  wave_lds_sync();
  *dupmask = mask;
  return wave_sum(dups);
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
  uint32_t total = 0;
  {
    uint32_t sw[S];
#pragma unroll
    for (int x = 0; x < S; ++x) sw[x] = has ? j.frontier_in[i * S + x] : 0u;
    const uint32_t c = has ? count_successors<S>(j.img, sw) : 0u;
    if (has && c == 0) {
      const uint64_t d = atomicAdd(reinterpret_cast<unsigned long long*>(j.dead_ctr), 1ull);
      if (j.dead_ctr != reinterpret_cast<uint64_t*>(ctr_at(j.ctr, kCtrDead)))
        atomicAdd(ctr_at(j.ctr, kCtrDead), 1ull);
      if (d < j.dead_cap) {
#pragma unroll
        for (int x = 0; x < S; ++x) j.dead[d * S + x] = sw[x];
        if (j.dead_tag) j.dead_tag[d] = j.tag;
      }
    }
    (void)wave_exclusive_scan(c, &total);
    if (lane == 0 && total)
      atomicAdd(ctr_at(j.ctr, kCtrTrans),
                static_cast<unsigned long long>(total));
  }

  for (uint32_t lo = 0; lo < total; lo += CAP) {
    const uint32_t hi = min(total, lo + CAP);
    {
      // The state is reloaded for every chunk rather than kept: nothing of
      // the generation stays live in registers while the chunk is probed,
      // which keeps the probe phase at the find-or-put kernel's register
      // budget.
      uint32_t sw[S];
#pragma unroll
      for (int x = 0; x < S; ++x) sw[x] = has ? j.frontier_in[i * S + x] : 0u;
      emit_window<S, true>(j.img, sw, has, stage, lo, hi);
    }
    wave_lds_sync();
    const uint32_t n_st = hi - lo;
    uint32_t dupmask = 0;
    if (j.dtab) {
      const uint32_t wd = dedup_chunk<S>(j.dtab, stage, n_st, &dupmask);
      if (lane == 0 && wd) atomicAdd(ctr_at(j.ctr, kCtrDups), static_cast<unsigned long long>(wd));
    }
    // NEW keys are compacted in place to the front of the staging area (a
    // round writes below the end of the keys it has read), then moved to the
    // next frontier with one atomic add and coalesced stores per chunk.
    uint32_t n_new = 0;
    bool full = false;
    for (uint32_t r0 = 0, r = 0; r0 < n_st; r0 += 64, ++r) {
      const uint32_t idx = r0 + lane;
      const bool act = idx < n_st && !((dupmask >> r) & 1u);
      uint32_t key[S];
#pragma unroll
      for (int x = 0; x < S; ++x) key[x] = act ? stage[idx * S + x] : 0u;
      const uint8_t res = find_or_put_lanes<S, B, G, U>(j.t, key, act, st);
      const bool is_new = act && res == kNew;
      full |= act && res == kFull;
      const uint64_t m = __ballot(is_new);
      wave_lds_sync();  // every lane's key of this round is read before any write
      if (is_new) {
        const uint32_t pos = n_new + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
#pragma unroll
        for (int x = 0; x < S; ++x) stage[pos * S + x] = key[x];
      }
      n_new += static_cast<uint32_t>(__popcll(m));
    }
    if (__ballot(full) && lane == 0)
      atomicOr(ctr_at(j.ctr, kCtrFlags), kFlagTableFull);
    wave_lds_sync();
    if (n_new) {
      unsigned long long base = 0;
      if (lane == 0)
        base = atomicAdd(ctr_at(j.ctr, kCtrTail),
                         static_cast<unsigned long long>(n_new));
      base = __shfl(base, 0, 64);
      if (lane == 0 && base + n_new > j.cap_out)
        atomicOr(ctr_at(j.ctr, kCtrFlags), kFlagFrontierOverflow);
      for (uint32_t k = lane; k < n_new * S; k += 64)
        if (base * S + k < j.cap_out * S) j.frontier_out[base * S + k] = stage[k];
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------- two-kernel BFS level
// A level (or a slice of it) of a single exploration runs as two kernels:
//   gen_level_kernel<S>: every wavefront expands 64 frontier states from the
//     LDS network image (counts, deadlocks, transitions) and writes their
//     successors to a successor buffer: each lane its own contiguous run, or,
//     with the duplicate filter, chunk by chunk through LDS staging without
//     in-chunk duplicates;
//   append_kernel<S,B,G,U>: find-or-put of that buffer (one key per lane,
//     grid-stride, as the isolated find-or-put) that appends the NEW keys to
//     the next frontier.
// Splitting keeps the table probes in a kernel with the register budget and
// occupancy of the isolated find-or-put instead of sharing waves with the
// successor generation.

struct GenArgs {
  const uint32_t* img;  // global memory (copied to LDS unless global_img)
  uint32_t img_words;
  uint32_t img_stride;  // LDS words of the image: img_words rounded up to 4, 0 with global_img
  uint32_t global_img;  // the image is read from global memory (too large for LDS)
  const uint32_t* frontier_in;
  uint64_t n_in;
  uint32_t* succ;       // successor keys, S words each
  uint64_t succ_cap;    // keys
  uint32_t* dead;
  uint64_t dead_cap;
  uint64_t* ctr;  // kCtrCount counters, kCtrSpread words apart (see ctr_at)
  uint32_t dedup;
  // Successor counts alternate between kCtrSucc and kCtrSuccAlt from slice
  // to slice: this slice reserves room on succ_ctr, and the kernel's first
  // thread zeroes the other one for the next slice (the previous slice's
  // append kernel, its last reader, has finished) and, with reset_tail, the
  // next-frontier tail at the first slice of a level.  No host-side clears.
  uint32_t succ_ctr;
  uint32_t reset_tail;
  uint32_t succ_words;  // words per successor in succ (S, or 3: see emit_window)
  uint32_t pad;
};

// Load, count and deadlock-check this lane's frontier state.
template <int S>
__device__ __forceinline__ uint32_t gen_count(const GenArgs& a, const uint32_t* img, uint64_t i,
                                              uint32_t (&sw)[S]) {
  const bool has = i < a.n_in;
#pragma unroll
  for (int x = 0; x < S; ++x) sw[x] = 0;
  if (has) load_slot<S>(a.frontier_in + i * S, sw);
  const uint32_t c = has ? count_successors<S>(img, sw) : 0u;
  if (has && c == 0) {
    const uint64_t d = atomicAdd(ctr_at(a.ctr, kCtrDead), 1ull);
    if (d < a.dead_cap) store_slot<S>(a.dead + d * S, sw);
  }
  return c;
}

// With the duplicate filter: 64 frontier states [first, first + 64) expanded
// chunk by chunk through the wavefront's LDS staging; repeats within a chunk
// are dropped, the rest copied out with coalesced stores.
template <int S>
__device__ inline void gen_wave_filtered(const GenArgs& a, const uint32_t* img, uint32_t* stage,
                                         uint32_t* dtab, uint64_t first) {
  constexpr uint32_t CAP = kStageWords / 4 / S;  // staged successors per chunk
  const int lane = __lane_id();
  uint32_t sw[S];
  const uint32_t c = gen_count<S>(a, img, first + lane, sw);
  uint32_t total = 0;
  (void)wave_exclusive_scan(c, &total);
  if (lane == 0 && total)
    atomicAdd(ctr_at(a.ctr, kCtrTrans), static_cast<unsigned long long>(total));
  const bool has = first + lane < a.n_in;
  for (uint32_t lo = 0; lo < total; lo += CAP) {
    const uint32_t hi = min(total, lo + CAP);
    emit_window<S, true>(img, sw, has, stage, lo, hi);
    wave_lds_sync();
    const uint32_t n_st = hi - lo;
    uint32_t dupmask = 0;
    const uint32_t wd = dedup_chunk<S>(dtab, stage, n_st, &dupmask);
    if (lane == 0 && wd) atomicAdd(ctr_at(a.ctr, kCtrDups), static_cast<unsigned long long>(wd));
    const uint32_t n_keep = n_st - wd;
    unsigned long long base = 0;
    if (lane == 0 && n_keep)
      base = atomicAdd(ctr_at(a.ctr, a.succ_ctr), static_cast<unsigned long long>(n_keep));
    base = __shfl(base, 0, 64);
    if (base + n_keep > a.succ_cap) {
      // cannot happen with the host's bound; refuse rather than overrun
      if (lane == 0) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagFrontierOverflow);
    } else {
      uint32_t kept = 0;  // kept successors of earlier rounds
      for (uint32_t r0 = 0, r = 0; r0 < n_st; r0 += 64, ++r) {
        const uint32_t idx = r0 + lane;
        const bool keep = idx < n_st && !((dupmask >> r) & 1u);
        const uint64_t m = __ballot(keep);
        if (keep) {
          uint32_t key[S];
          load_slot<S>(stage + idx * S, key);
          const uint64_t pos = base + kept + __popcll(m & ((1ull << lane) - 1ull));
          store_slot<S>(a.succ + pos * S, key);
        }
        kept += static_cast<uint32_t>(__popcll(m));
      }
    }
    wave_lds_sync();
  }
}

// kFilter (a.dedup set): the chunked path with the duplicate filter, built as
// its own kernel so its registers do not lower the plain path's occupancy.
// kGlobalImg (a.global_img set): the image is read where it is, in global
// memory (through the caches), for networks whose image exceeds the LDS
// budget; a kernel of its own, so the LDS path keeps its LDS loads.
template <int S, bool kFilter, bool kGlobalImg>
__global__ __launch_bounds__(256) void gen_level_kernel(GenArgs a) {
  extern __shared__ uint32_t smem[];
  __shared__ uint32_t wave_total[4];
  __shared__ unsigned long long group_base;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *ctr_at(a.ctr, a.succ_ctr == kCtrSucc ? kCtrSuccAlt : kCtrSucc) = 0;
    if (a.reset_tail) *ctr_at(a.ctr, kCtrTail) = 0;
  }
  const uint32_t* img;
  if constexpr (kGlobalImg) {
    img = a.img;
  } else {
    for (uint32_t k = threadIdx.x; k < a.img_words; k += 256) smem[k] = a.img[k];
    img = smem;
  }
  __syncthreads();
  const int wave = static_cast<int>(threadIdx.x >> 6);
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * 256 + (threadIdx.x & ~63u);
  if constexpr (kFilter) {
    // staging and filter space only with the duplicate filter
    uint32_t* stage = smem + a.img_stride + wave * (kStageWords / 4);
    uint32_t* dtab = smem + a.img_stride + kStageWords + wave * dedup_entries<S>();
    if (first < a.n_in) gen_wave_filtered<S>(a, img, stage, dtab, first);
    return;
  }
  // No filter: one atomic add per workgroup reserves the room of all its
  // successors; every wavefront then writes its own with coalesced stores
  // in one pass over its lanes' transitions.
  const int lane = __lane_id();
  uint32_t sw[S];
  const uint32_t c = gen_count<S>(a, img, first + lane, sw);
  uint32_t total = 0;
  (void)wave_exclusive_scan(c, &total);
  if (lane == 0) wave_total[wave] = total;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t t = static_cast<uint64_t>(wave_total[0]) + wave_total[1] + wave_total[2] +
                       wave_total[3];
    unsigned long long b = 0;
    if (t) {
      // (the slice's transition count is its successor count: the append
      // kernel adds it once)
      b = atomicAdd(ctr_at(a.ctr, a.succ_ctr), static_cast<unsigned long long>(t));
      if (b + t > a.succ_cap) {
        // cannot happen with the host's bound; refuse rather than overrun
        atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagFrontierOverflow);
        b = ~0ull;
      }
    }
    group_base = b;
  }
  __syncthreads();
  uint64_t base = group_base;
  if (base == ~0ull || total == 0) return;
  for (int w = 0; w < wave; ++w) base += wave_total[w];
  emit_window<S, false>(img, sw, first + lane < a.n_in, a.succ + base * a.succ_words, 0, total,
                        nullptr, nullptr, a.succ_words);
}

struct AppendArgs {
  TableDev t;
  const uint32_t* keys;    // S words per key
  uint64_t keys_cap;       // keys the buffer holds
  const uint64_t* n_keys;  // device memory: the number of keys (clamped to keys_cap)
  uint32_t* frontier_out;
  uint64_t cap_out;        // states
  uint64_t* ctr;           // the level's counters (see ctr_at)
  uint32_t count_trans;    // add n_keys to the transition count (unfiltered slices)
  uint32_t key_words;      // words per key in keys (S, or 3: see emit_window)
};

constexpr uint32_t kAppendKeys = 256;  // NEW keys a wavefront gathers in LDS

// Move a wavefront's cnt gathered NEW keys from LDS to the next frontier:
// one atomic add reserves the room, the copy is coalesced.
template <int S>
__device__ inline void append_flush(const AppendArgs& a, const uint32_t* buf, uint32_t cnt) {
  if (cnt == 0) return;
  const int lane = __lane_id();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(ctr_at(a.ctr, kCtrTail), static_cast<unsigned long long>(cnt));
  base = __shfl(base, 0, 64);
  if (lane == 0 && base + cnt > a.cap_out) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagFrontierOverflow);
  for (uint32_t k = lane; k < cnt; k += 64) {
    if (base + k < a.cap_out) {
      uint32_t key[S];
      load_slot<S>(buf + k * S, key);
      store_slot<S>(a.frontier_out + (base + k) * S, key);
    }
  }
}

template <int S, int B, int G, int U>
__global__ __launch_bounds__(256) void append_kernel(AppendArgs a) {
  __shared__ __align__(16) uint32_t sbuf[4][kAppendKeys * S];
  uint32_t* buf = sbuf[threadIdx.x >> 6];
  const int lane = __lane_id();
  // a generation that overran the buffer has flagged it; never read past it
  const uint64_t n = min(*a.n_keys, a.keys_cap);
  if (a.count_trans && blockIdx.x == 0 && threadIdx.x == 0 && n)
    atomicAdd(ctr_at(a.ctr, kCtrTrans), static_cast<unsigned long long>(n));
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  LaneStats st;
  uint32_t cnt = 0;  // gathered NEW keys (wavefront-uniform)
  bool full = false;
  for (uint64_t base = wave * 64; base < n; base += n_waves * 64) {
    const uint64_t idx = base + lane;
    const bool act = idx < n;
    uint32_t key[S];
#pragma unroll
    for (int x = 0; x < S; ++x) key[x] = 0;
    if (act) {
      if (S == 4 && a.key_words == 3)
        load_words3<S>(a.keys + idx * 3, key);
      else
        load_slot<S>(a.keys + idx * S, key);
    }
    const uint8_t r = find_or_put_lanes<S, B, G, U>(a.t, key, act, st);
    const bool is_new = act && r == kNew;
    full |= act && r == kFull;
    const uint64_t m = __ballot(is_new);
    if (is_new) store_slot<S>(buf + (cnt + __popcll(m & ((1ull << lane) - 1ull))) * S, key);
    cnt += static_cast<uint32_t>(__popcll(m));
    if (cnt > kAppendKeys - 64) {
      wave_lds_sync();
      append_flush<S>(a, buf, cnt);
      wave_lds_sync();
      cnt = 0;
    }
  }
  wave_lds_sync();
  append_flush<S>(a, buf, cnt);
  if (__ballot(full) && lane == 0) atomicOr(ctr_at(a.ctr, kCtrFlags), kFlagTableFull);
  flush_stats(a.t, st, nullptr);
}

template <int S, int B, int G, int U>
hipError_t launch_append(const AppendArgs& a, uint32_t cus, hipStream_t s) {
  // as many workgroups as can be resident at once (grid-stride over rounds)
  static int per_cu = 0;
  if (per_cu == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, append_kernel<S, B, G, U>, 256, 0) !=
            hipSuccess ||
        b <= 0)
      b = 2;
    per_cu = b;
  }
  hipLaunchKernelGGL((append_kernel<S, B, G, U>), dim3(cus * static_cast<uint32_t>(per_cu)),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int S, bool kFilter, bool kGlobalImg>
hipError_t launch_gen_k(const GenArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  if (lds > 65536) {  // more than the default per-workgroup LDS: ask for it
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&gen_level_kernel<S, kFilter, kGlobalImg>),
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gen_level_kernel<S, kFilter, kGlobalImg>), dim3(grid), dim3(256), lds, s,
                     a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_gen(const GenArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  if (a.global_img)
    return a.dedup ? launch_gen_k<S, true, true>(a, grid, lds, s)
                   : launch_gen_k<S, false, true>(a, grid, lds, s);
  return a.dedup ? launch_gen_k<S, true, false>(a, grid, lds, s)
                 : launch_gen_k<S, false, false>(a, grid, lds, s);
}

template <int S, int B, int G>
hipError_t append_u(uint32_t U, const AppendArgs& a, uint32_t cus, hipStream_t s) {
  switch (U) {
    case 1: return launch_append<S, B, G, 1>(a, cus, s);
    case 2: return launch_append<S, B, G, 2>(a, cus, s);
    case 4: return launch_append<S, B, G, 4>(a, cus, s);
    case 8:
      if constexpr (G >= 8) return launch_append<S, B, G, 8>(a, cus, s);
      break;
  }
  return hipErrorInvalidValue;
}

template <int S, int B>
hipError_t append_g(uint32_t G, uint32_t U, const AppendArgs& a, uint32_t cus, hipStream_t s) {
  switch (G) {
    case 4:
      if constexpr (B <= 32) return append_u<S, B, 4>(U, a, cus, s);
      break;
    case 8: return append_u<S, B, 8>(U, a, cus, s);
    case 16: return append_u<S, B, 16>(U, a, cus, s);
    case 32: return append_u<S, B, 32>(U, a, cus, s);
    case 64: return append_u<S, B, 64>(U, a, cus, s);
  }
  return hipErrorInvalidValue;
}

// Find-or-put-and-append dispatch over (B, G, U) for slot width S.
template <int S>
hipError_t append_b(uint32_t B, uint32_t G, uint32_t U, const AppendArgs& a, uint32_t cus,
                    hipStream_t s) {
  switch (B) {
    case 4: return append_g<S, 4>(G, U, a, cus, s);
    case 8: return append_g<S, 8>(G, U, a, cus, s);
    case 16: return append_g<S, 16>(G, U, a, cus, s);
    case 32: return append_g<S, 32>(G, U, a, cus, s);
    case 64: return append_g<S, 64>(G, U, a, cus, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gx
