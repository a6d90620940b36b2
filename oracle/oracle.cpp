// Oracle for the GPUexplore-style exploration path (arXiv 1801.05857).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct CPU
// model of what the GPU library computes.  Only the test suite, the smoke check
// and the CPU-baseline leg of the benchmark may load it.  It shares no code,
// header, constant or helper with the GPU library, and it includes nothing from
// the package.
//
// What it computes, and where the paper defines it:
//   * find-or-put (Sec. 4.1): inserting a vector either finds it already stored
//     or stores it.  Sequentially that is set insertion; the oracle is
//     std::unordered_set::insert, and a key is NEW exactly at its first
//     occurrence in the stream.
//   * exploration (Sec. 3, Fig. 1): breadth-first construction of the reachable
//     part of the synchronous product of a network of LTSs, layer by layer,
//     with deadlock detection (states without an outgoing product transition).
//   * safety checking (Sec. 3): the negation of a safety property is an
//     automaton added to the network as one more process; a reachable state
//     whose monitor process sits in a bad local state is a violation.
//   * packing (Sec. 3 and Sec. 5.2): process states are packed into 32-bit
//     integers; a vector that needs more than one integer spans several words.
//
// Readings of points the paper leaves open (each is listed with its reason in
// the design notes of the repository):
//   * A transition of process p whose label is named at position p of some
//     synchronisation rule fires only through such rules, all participants of
//     the rule stepping together; every other transition fires alone.  (Fig. 1
//     and its count of 8 states and 24 transitions, Sec. 3.)
//   * One product transition per local transition fired alone, and one per
//     choice of one matching transition for every participant of a rule.  No
//     merging of parallel product transitions.
//   * Field width of process p: max(1, ceil(log2 n_p)) bits; fields are laid
//     out in process order from the least significant bit, never straddle a
//     word, and only bits 0..30 of a word are used, so bit 31 is always 0.
//   * Level k holds the states at BFS distance k; level 0 is the initial state.
//   * Deadlocks and set dumps are sorted lexicographically by (word0, word1,
//     ...) as unsigned integers.
//
// Parity pins (tests/test_oracle_pins.py): Fig. 1 counts, the Token Ring state
// counts of Table 1, closed forms for products of independent cycles and for
// the tiny four-process network, hand-packed vectors, and the brute-force
// fixpoint enumerator below (a different algorithm and data structure).

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <thread>
#include <unordered_set>
#include <vector>

namespace {

constexpr uint32_t kMaxWords = 4;
using Vec = std::array<uint32_t, kMaxWords>;  // unused words stay 0

struct VecHash {
  // FNV-1a over the four words: a plain hash for std::unordered_set.
  size_t operator()(const Vec& v) const noexcept {
    uint64_t h = 1469598103934665603ULL;
    for (uint32_t x : v) {
      for (int b = 0; b < 4; ++b) {
        h ^= (x >> (8 * b)) & 0xFFu;
        h *= 1099511628211ULL;
      }
    }
    return static_cast<size_t>(h);
  }
};

using VecSet = std::unordered_set<Vec, VecHash>;

bool vec_less(const Vec& a, const Vec& b) {
  for (uint32_t i = 0; i < kMaxWords; ++i) {
    if (a[i] != b[i]) return a[i] < b[i];
  }
  return false;
}

// ---------------------------------------------------------------- packing
struct Plan {
  uint32_t words = 0;
  std::vector<uint32_t> word_of, shift_of, width_of;
};

uint32_t field_width(uint32_t n_states) {
  // smallest b >= 1 with 2^b >= n_states
  uint32_t b = 1;
  while (b < 32 && (uint64_t(1) << b) < n_states) ++b;
  return b;
}

bool make_plan(uint32_t P, const uint32_t* n_states, Plan* plan) {
  plan->word_of.assign(P, 0);
  plan->shift_of.assign(P, 0);
  plan->width_of.assign(P, 0);
  uint32_t word = 0, used = 0;
  for (uint32_t p = 0; p < P; ++p) {
    if (n_states[p] == 0) return false;
    uint32_t b = field_width(n_states[p]);
    if (b > 31) return false;
    if (used + b > 31) {  // would straddle: start a fresh word
      ++word;
      used = 0;
    }
    plan->word_of[p] = word;
    plan->shift_of[p] = used;
    plan->width_of[p] = b;
    used += b;
  }
  plan->words = (P == 0) ? 0 : word + 1;
  return true;
}

Vec pack(const Plan& plan, const std::vector<uint32_t>& local) {
  Vec v{};
  for (size_t p = 0; p < local.size(); ++p) {
    v[plan.word_of[p]] |= local[p] << plan.shift_of[p];
  }
  return v;
}

std::vector<uint32_t> unpack(const Plan& plan, const Vec& v) {
  std::vector<uint32_t> local(plan.word_of.size());
  for (size_t p = 0; p < local.size(); ++p) {
    uint32_t mask = (plan.width_of[p] == 32) ? 0xFFFFFFFFu : ((1u << plan.width_of[p]) - 1u);
    local[p] = (v[plan.word_of[p]] >> plan.shift_of[p]) & mask;
  }
  return local;
}

// ---------------------------------------------------------------- network
struct Trans {
  uint32_t label, dst;
};

struct Net {
  uint32_t P = 0, n_labels = 0, R = 0;
  std::vector<uint32_t> n_states, initial;
  // out[p][s] = transitions leaving local state s of process p
  std::vector<std::vector<std::vector<Trans>>> out;
  std::vector<int32_t> rules;  // R x P, label or -1
  // governed[p][a]: label a is named at position p by some rule
  std::vector<std::vector<bool>> governed;
};

bool load_net(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
              const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
              const uint32_t* dst, uint32_t n_labels, uint32_t R, const int32_t* rules,
              Net* net) {
  net->P = P;
  net->n_labels = n_labels;
  net->R = R;
  net->n_states.assign(n_states, n_states + P);
  net->initial.assign(initial, initial + P);
  net->out.assign(P, {});
  net->governed.assign(P, std::vector<bool>(n_labels, false));
  uint64_t base = 0;
  for (uint32_t p = 0; p < P; ++p) {
    if (n_states[p] == 0 || initial[p] >= n_states[p]) return false;
    net->out[p].assign(n_states[p], {});
    for (uint32_t t = 0; t < n_trans[p]; ++t) {
      uint32_t s = src[base + t], a = label[base + t], d = dst[base + t];
      if (s >= n_states[p] || d >= n_states[p] || a >= n_labels) return false;
      net->out[p][s].push_back({a, d});
    }
    base += n_trans[p];
  }
  net->rules.assign(rules, rules + size_t(R) * P);
  for (uint32_t r = 0; r < R; ++r) {
    uint32_t parts = 0;
    for (uint32_t p = 0; p < P; ++p) {
      int32_t a = net->rules[size_t(r) * P + p];
      if (a < -1 || a >= int32_t(n_labels)) return false;
      if (a >= 0) {
        net->governed[p][a] = true;
        ++parts;
      }
    }
    if (parts == 0) return false;
  }
  return true;
}

// All product successors of the unpacked state `local`, with multiplicity.
// With `actions`, also the action each one performs: a transition that fires
// alone performs action R + its label, rule r performs action r.
void successors(const Net& net, const std::vector<uint32_t>& local,
                std::vector<std::vector<uint32_t>>* succ,
                std::vector<uint32_t>* actions = nullptr) {
  succ->clear();
  if (actions) actions->clear();
  // transitions that fire alone
  for (uint32_t p = 0; p < net.P; ++p) {
    for (const Trans& t : net.out[p][local[p]]) {
      if (net.governed[p][t.label]) continue;
      std::vector<uint32_t> s = local;
      s[p] = t.dst;
      succ->push_back(std::move(s));
      if (actions) actions->push_back(net.R + t.label);
    }
  }
  // synchronisation rules: every participant takes one matching transition
  for (uint32_t r = 0; r < net.R; ++r) {
    std::vector<uint32_t> parts;
    for (uint32_t p = 0; p < net.P; ++p) {
      if (net.rules[size_t(r) * net.P + p] >= 0) parts.push_back(p);
    }
    std::vector<uint32_t> cur = local;
    std::function<void(size_t)> choose = [&](size_t i) {
      if (i == parts.size()) {
        succ->push_back(cur);
        if (actions) actions->push_back(r);
        return;
      }
      uint32_t q = parts[i];
      uint32_t want = uint32_t(net.rules[size_t(r) * net.P + q]);
      for (const Trans& t : net.out[q][local[q]]) {
        if (t.label != want) continue;
        cur[q] = t.dst;
        choose(i + 1);
      }
      cur[q] = local[q];
    };
    choose(0);
  }
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

// ---- set (find-or-put oracle) ----------------------------------------
struct oracle_set {
  uint32_t w;
  VecSet set;
};

oracle_set* oracle_set_new(uint32_t w) {
  if (w == 0 || w > kMaxWords) return nullptr;
  oracle_set* s = new oracle_set;
  s->w = w;
  return s;
}

void oracle_set_free(oracle_set* s) { delete s; }

uint64_t oracle_set_size(const oracle_set* s) { return s->set.size(); }

// Insert keys[0..n) (row-major, w words each) in order.  status[i] = 1 when
// key i was not in the set before its insertion, else 0.  Returns the number
// of keys that were new.
uint64_t oracle_set_insert(oracle_set* s, const uint32_t* keys, uint64_t n, uint8_t* status) {
  uint64_t fresh = 0;
  for (uint64_t i = 0; i < n; ++i) {
    Vec v{};
    for (uint32_t k = 0; k < s->w; ++k) v[k] = keys[i * s->w + k];
    bool inserted = s->set.insert(v).second;
    if (status) status[i] = inserted ? 1 : 0;
    fresh += inserted ? 1 : 0;
  }
  return fresh;
}

int oracle_set_contains(const oracle_set* s, const uint32_t* key) {
  Vec v{};
  for (uint32_t k = 0; k < s->w; ++k) v[k] = key[k];
  return s->set.count(v) ? 1 : 0;
}

// Write the set, sorted lexicographically, as size*w words.
void oracle_set_dump(const oracle_set* s, uint32_t* out) {
  std::vector<Vec> all(s->set.begin(), s->set.end());
  std::sort(all.begin(), all.end(), vec_less);
  for (size_t i = 0; i < all.size(); ++i) {
    for (uint32_t k = 0; k < s->w; ++k) out[i * s->w + k] = all[i][k];
  }
}

// ---- packing plan -----------------------------------------------------
// Returns 0 and the number of words on success, -1 when a process has no
// states or a field would need more than 31 bits.
int oracle_pack_plan(uint32_t P, const uint32_t* n_states, uint32_t* word_of,
                     uint32_t* shift_of, uint32_t* width_of, uint32_t* words) {
  Plan plan;
  if (!make_plan(P, n_states, &plan)) return -1;
  for (uint32_t p = 0; p < P; ++p) {
    if (word_of) word_of[p] = plan.word_of[p];
    if (shift_of) shift_of[p] = plan.shift_of[p];
    if (width_of) width_of[p] = plan.width_of[p];
  }
  *words = plan.words;
  return 0;
}

// Pack n unpacked states (n x P local states) into n x words words.
int oracle_pack(uint32_t P, const uint32_t* n_states, const uint32_t* local, uint64_t n,
                uint32_t* out) {
  Plan plan;
  if (!make_plan(P, n_states, &plan)) return -1;
  for (uint64_t i = 0; i < n; ++i) {
    std::vector<uint32_t> l(local + i * P, local + (i + 1) * P);
    Vec v = pack(plan, l);
    for (uint32_t k = 0; k < plan.words; ++k) out[i * plan.words + k] = v[k];
  }
  return 0;
}

// ---- exploration --------------------------------------------------------
struct oracle_result {
  uint32_t words;
  uint32_t n_levels;
  uint64_t n_states;
  uint64_t n_transitions;
  uint64_t* levels;       // n_levels
  uint64_t n_deadlocks;
  uint32_t* deadlocks;    // n_deadlocks x words, sorted
  uint32_t* visited;      // n_states x words, sorted (only when requested)
  uint64_t n_violations;  // reachable states whose monitor process is in a bad state
  uint32_t* violations;   // n_violations x words, sorted
  uint32_t violation_level;  // first level holding one; 0xFFFFFFFF when none
};

void oracle_result_free(oracle_result* r) {
  if (!r) return;
  std::free(r->levels);
  std::free(r->deadlocks);
  std::free(r->visited);
  std::free(r->violations);
  r->levels = nullptr;
  r->deadlocks = nullptr;
  r->visited = nullptr;
  r->violations = nullptr;
}

static void set_violations(const Plan& plan, std::vector<Vec>& viol, uint32_t level,
                           oracle_result* out) {
  std::sort(viol.begin(), viol.end(), vec_less);
  out->n_violations = viol.size();
  out->violations =
      static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (viol.size() * plan.words + 1)));
  for (size_t i = 0; i < viol.size(); ++i)
    for (uint32_t k = 0; k < plan.words; ++k) out->violations[i * plan.words + k] = viol[i][k];
  out->violation_level = level;
}

static void fill_result(const Plan& plan, const std::vector<uint64_t>& levels,
                        uint64_t n_states, uint64_t n_transitions, std::vector<Vec>& dead,
                        std::vector<Vec>* visited, oracle_result* out) {
  std::sort(dead.begin(), dead.end(), vec_less);
  out->words = plan.words;
  out->n_levels = uint32_t(levels.size());
  out->n_states = n_states;
  out->n_transitions = n_transitions;
  out->levels = static_cast<uint64_t*>(std::malloc(sizeof(uint64_t) * (levels.size() + 1)));
  for (size_t i = 0; i < levels.size(); ++i) out->levels[i] = levels[i];
  out->n_deadlocks = dead.size();
  out->deadlocks =
      static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (dead.size() * plan.words + 1)));
  for (size_t i = 0; i < dead.size(); ++i)
    for (uint32_t k = 0; k < plan.words; ++k) out->deadlocks[i * plan.words + k] = dead[i][k];
  out->visited = nullptr;
  out->n_violations = 0;
  out->violations = nullptr;
  out->violation_level = 0xFFFFFFFFu;
  if (visited) {
    std::sort(visited->begin(), visited->end(), vec_less);
    out->visited = static_cast<uint32_t*>(
        std::malloc(sizeof(uint32_t) * (visited->size() * plan.words + 1)));
    for (size_t i = 0; i < visited->size(); ++i)
      for (uint32_t k = 0; k < plan.words; ++k)
        out->visited[i * plan.words + k] = (*visited)[i][k];
  }
}

using SuccFn =
    std::function<void(const std::vector<uint32_t>&, std::vector<std::vector<uint32_t>>*)>;

// Plain breadth-first search over std::unordered_set from the unpacked state
// `init`, with the product successors given by succ_fn.  Returns 0, or -2 when
// more than max_states states are reachable (max_states == 0: no limit).  With
// max_levels > 0 the search stops once levels 0 .. max_levels-1 are known (a
// BFS prefix: level counts of those levels, the states at distance below
// max_levels, and transitions and deadlocks of the levels expanded so far).
//
// Safety monitor (Sec. 3: the negation of a safety property is an automaton
// added to the network): with monitor_proc >= 0, a state violates the
// property when the local state of process monitor_proc is marked in
// monitor_bad (one byte per local state).  Every level is checked as soon as
// it is complete; the violating states and the first level that holds one
// are returned.  With stop_on_violation the search ends there: that level is
// counted but not expanded.
static int bfs(const Plan& plan, const std::vector<uint32_t>& init_local, const SuccFn& succ_fn,
        uint64_t max_states, uint32_t max_levels, int want_visited, int32_t monitor_proc,
        const uint8_t* monitor_bad, int stop_on_violation, oracle_result* out) {
  VecSet visited;
  std::vector<Vec> frontier, next, dead, viol;
  std::vector<uint64_t> levels;
  uint64_t transitions = 0;
  uint32_t viol_level = 0xFFFFFFFFu;
  std::vector<std::vector<uint32_t>> succ;
  auto violates = [&](const Vec& v) {
    return monitor_proc >= 0 && monitor_bad[unpack(plan, v)[monitor_proc]] != 0;
  };
  // record the violating states of the level just completed
  auto check_level = [&](const std::vector<Vec>& level) {
    for (const Vec& v : level) {
      if (violates(v)) {
        viol.push_back(v);
        if (viol_level == 0xFFFFFFFFu) viol_level = uint32_t(levels.size() - 1);
      }
    }
  };

  Vec init = pack(plan, init_local);
  visited.insert(init);
  frontier.push_back(init);
  levels.push_back(1);
  check_level(frontier);
  while (!frontier.empty()) {
    if (stop_on_violation && !viol.empty()) break;
    if (max_levels && levels.size() >= max_levels) break;
    next.clear();
    for (const Vec& s : frontier) {
      succ_fn(unpack(plan, s), &succ);
      transitions += succ.size();
      if (succ.empty()) dead.push_back(s);
      for (const auto& t : succ) {
        Vec v = pack(plan, t);
        if (visited.insert(v).second) next.push_back(v);
      }
      if (max_states && visited.size() > max_states) return -2;
    }
    if (!next.empty()) {
      levels.push_back(next.size());
      check_level(next);
    }
    frontier.swap(next);
  }
  std::vector<Vec> vis;
  if (want_visited) vis.assign(visited.begin(), visited.end());
  fill_result(plan, levels, visited.size(), transitions, dead, want_visited ? &vis : nullptr,
              out);
  set_violations(plan, viol, viol_level, out);
  return 0;
}

// Plain breadth-first search of the network's synchronous product (Sec. 3).
// Returns 0 on success, -1 on an invalid network, -2 when more than
// max_states states are reachable; max_levels and the monitor as for bfs().
int oracle_explore_monitored(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                             const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                             const uint32_t* dst, uint32_t n_labels, uint32_t R,
                             const int32_t* rules, uint64_t max_states, uint32_t max_levels,
                             int want_visited, int32_t monitor_proc, const uint8_t* monitor_bad,
                             int stop_on_violation, oracle_result* out) {
  Net net;
  Plan plan;
  if (P == 0 || !load_net(P, n_states, initial, n_trans, src, label, dst, n_labels, R, rules,
                          &net))
    return -1;
  if (!make_plan(P, n_states, &plan) || plan.words > kMaxWords) return -1;
  if (monitor_proc >= 0 && (uint32_t(monitor_proc) >= P || !monitor_bad)) return -1;
  SuccFn fn = [&](const std::vector<uint32_t>& local, std::vector<std::vector<uint32_t>>* succ) {
    successors(net, local, succ);
  };
  return bfs(plan, net.initial, fn, max_states, max_levels, want_visited, monitor_proc,
             monitor_bad, stop_on_violation, out);
}

// Exploration of a network watched by the automaton of a negated safety
// property (Sec. 3), straight from the meaning of "the automaton observes the
// network's actions", without composing a new network: the state is the
// network's state plus the automaton's state (packed as one more process
// after the network's); each product transition of the network (action r for
// rule r, action R + l for label l fired alone) moves the automaton along each
// of its transitions on that action when it observes the action (any of its
// transitions carries it), stays put when it observes the action but has no
// transition on it in its current state, and stays put for unobserved
// actions.  A state whose automaton state is bad is a violation; max_levels,
// stop_on_violation and the result as for bfs().
int oracle_explore_automaton(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                             const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                             const uint32_t* dst, uint32_t n_labels, uint32_t R,
                             const int32_t* rules, uint32_t mon_states, uint32_t mon_initial,
                             uint32_t mon_n_trans, const uint32_t* mon_src,
                             const uint32_t* mon_action, const uint32_t* mon_dst,
                             const uint8_t* mon_bad, uint32_t max_levels, int want_visited,
                             int stop_on_violation, oracle_result* out) {
  Net net;
  if (P == 0 || !load_net(P, n_states, initial, n_trans, src, label, dst, n_labels, R, rules,
                          &net))
    return -1;
  if (mon_states == 0 || mon_initial >= mon_states || !mon_bad) return -1;
  const uint32_t n_actions = R + n_labels;
  std::vector<std::vector<std::vector<uint32_t>>> moves(
      mon_states, std::vector<std::vector<uint32_t>>(n_actions));
  std::vector<bool> observed(n_actions, false);
  for (uint32_t t = 0; t < mon_n_trans; ++t) {
    if (mon_src[t] >= mon_states || mon_dst[t] >= mon_states || mon_action[t] >= n_actions)
      return -1;
    moves[mon_src[t]][mon_action[t]].push_back(mon_dst[t]);
    observed[mon_action[t]] = true;
  }
  std::vector<uint32_t> sizes(n_states, n_states + P);
  sizes.push_back(mon_states);
  Plan plan;
  if (!make_plan(P + 1, sizes.data(), &plan) || plan.words > kMaxWords) return -1;
  std::vector<uint32_t> init = net.initial;
  init.push_back(mon_initial);
  std::vector<std::vector<uint32_t>> net_succ;
  std::vector<uint32_t> acts;
  SuccFn fn = [&](const std::vector<uint32_t>& local, std::vector<std::vector<uint32_t>>* succ) {
    succ->clear();
    const std::vector<uint32_t> net_local(local.begin(), local.begin() + P);
    const uint32_t m = local[P];
    successors(net, net_local, &net_succ, &acts);
    for (size_t i = 0; i < net_succ.size(); ++i) {
      std::vector<uint32_t> t = net_succ[i];
      t.push_back(m);
      const std::vector<uint32_t>& to = moves[m][acts[i]];
      if (!observed[acts[i]] || to.empty()) {
        succ->push_back(t);
        continue;
      }
      for (uint32_t m2 : to) {
        t[P] = m2;
        succ->push_back(t);
      }
    }
  };
  return bfs(plan, init, fn, 0, max_levels, want_visited, int32_t(P), mon_bad,
             stop_on_violation, out);
}

int oracle_explore(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                   const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                   const uint32_t* dst, uint32_t n_labels, uint32_t R, const int32_t* rules,
                   uint64_t max_states, uint32_t max_levels, int want_visited,
                   oracle_result* out) {
  return oracle_explore_monitored(P, n_states, initial, n_trans, src, label, dst, n_labels, R,
                                  rules, max_states, max_levels, want_visited, -1, nullptr, 0,
                                  out);
}

// Product successors (Sec. 3), with multiplicity, of n packed states
// (n x words).  counts[i] receives the number of successors of state i; *out
// receives a malloc'd array of all successors, packed, state by state in the
// order successors() lists them (free with oracle_free).  Returns 0, or -1 on
// an invalid network or a state with a field outside its process's states.
int oracle_successors(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                      const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                      const uint32_t* dst, uint32_t n_labels, uint32_t R, const int32_t* rules,
                      const uint32_t* states, uint64_t n, uint64_t* counts, uint32_t** out,
                      uint64_t* n_out) {
  Net net;
  Plan plan;
  if (P == 0 || !load_net(P, n_states, initial, n_trans, src, label, dst, n_labels, R, rules,
                          &net))
    return -1;
  if (!make_plan(P, n_states, &plan) || plan.words > kMaxWords) return -1;
  std::vector<uint32_t> all;
  std::vector<std::vector<uint32_t>> succ;
  for (uint64_t i = 0; i < n; ++i) {
    Vec v{};
    for (uint32_t k = 0; k < plan.words; ++k) v[k] = states[i * plan.words + k];
    std::vector<uint32_t> local = unpack(plan, v);
    for (uint32_t p = 0; p < P; ++p)
      if (local[p] >= n_states[p]) return -1;
    successors(net, local, &succ);
    counts[i] = succ.size();
    for (const auto& t : succ) {
      Vec w = pack(plan, t);
      for (uint32_t k = 0; k < plan.words; ++k) all.push_back(w[k]);
    }
  }
  *n_out = all.size() / plan.words;
  *out = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (all.size() + 1)));
  std::copy(all.begin(), all.end(), *out);
  return 0;
}

void oracle_free(void* p) { std::free(p); }

// Brute-force fixpoint over a dense bitmap of every vector of local states
// (mixed-radix index over n_p), a different algorithm and data structure from
// the BFS above: R_0 = {init}, R_{k+1} = R_k  union  post(R_k), recomputing post of
// the whole set at every step.  Level k = |R_k \ R_{k-1}|.  Requires
// prod n_p <= 2^24.  Same return codes as oracle_explore (-2: too large).
int oracle_bruteforce(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                      const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                      const uint32_t* dst, uint32_t n_labels, uint32_t R, const int32_t* rules,
                      int want_visited, oracle_result* out) {
  Plan plan;
  if (P == 0 || !make_plan(P, n_states, &plan) || plan.words > kMaxWords) return -1;
  uint64_t total = 1;
  for (uint32_t p = 0; p < P; ++p) {
    if (n_states[p] == 0 || initial[p] >= n_states[p]) return -1;
    total *= n_states[p];
    if (total > (uint64_t(1) << 24)) return -2;
  }
  // flat transition list per process, scanned in full for every state
  std::vector<uint64_t> first(P + 1, 0);
  for (uint32_t p = 0; p < P; ++p) first[p + 1] = first[p] + n_trans[p];
  for (uint32_t p = 0; p < P; ++p)
    for (uint64_t t = first[p]; t < first[p + 1]; ++t)
      if (src[t] >= n_states[p] || dst[t] >= n_states[p] || label[t] >= n_labels) return -1;
  auto named_at = [&](uint32_t p, uint32_t a) {
    for (uint32_t r = 0; r < R; ++r)
      if (rules[size_t(r) * P + p] == int32_t(a)) return true;
    return false;
  };
  for (uint32_t r = 0; r < R; ++r) {
    bool any = false;
    for (uint32_t p = 0; p < P; ++p) {
      int32_t a = rules[size_t(r) * P + p];
      if (a < -1 || a >= int32_t(n_labels)) return -1;
      any |= a >= 0;
    }
    if (!any) return -1;
  }
  std::vector<uint64_t> radix(P, 1);
  for (uint32_t p = 1; p < P; ++p) radix[p] = radix[p - 1] * n_states[p - 1];
  auto digit = [&](uint64_t idx, uint32_t p) { return (idx / radix[p]) % n_states[p]; };

  // post(idx): all successor indices with multiplicity
  auto post = [&](uint64_t idx, std::vector<uint64_t>* res) {
    res->clear();
    for (uint32_t p = 0; p < P; ++p) {
      uint64_t cur = digit(idx, p);
      for (uint64_t t = first[p]; t < first[p + 1]; ++t) {
        if (src[t] != cur || named_at(p, label[t])) continue;
        res->push_back(idx - cur * radix[p] + uint64_t(dst[t]) * radix[p]);
      }
    }
    for (uint32_t r = 0; r < R; ++r) {
      // iterative odometer over the participants' matching transitions
      std::vector<uint32_t> parts;
      std::vector<std::vector<uint64_t>> choices;
      bool blocked = false;
      for (uint32_t p = 0; p < P && !blocked; ++p) {
        int32_t a = rules[size_t(r) * P + p];
        if (a < 0) continue;
        std::vector<uint64_t> c;
        uint64_t cur = digit(idx, p);
        for (uint64_t t = first[p]; t < first[p + 1]; ++t)
          if (src[t] == cur && label[t] == uint32_t(a)) c.push_back(t);
        if (c.empty()) blocked = true;
        parts.push_back(p);
        choices.push_back(std::move(c));
      }
      if (blocked) continue;
      std::vector<size_t> pick(parts.size(), 0);
      while (true) {
        uint64_t v = idx;
        for (size_t i = 0; i < parts.size(); ++i) {
          uint32_t p = parts[i];
          v = v - digit(idx, p) * radix[p] + uint64_t(dst[choices[i][pick[i]]]) * radix[p];
        }
        res->push_back(v);
        size_t i = 0;
        while (i < parts.size() && ++pick[i] == choices[i].size()) pick[i++] = 0;
        if (i == parts.size()) break;
      }
    }
  };

  uint64_t init = 0;
  for (uint32_t p = 0; p < P; ++p) init += uint64_t(initial[p]) * radix[p];
  std::vector<uint8_t> in(total, 0), nxt;
  in[init] = 1;
  std::vector<uint64_t> levels{1};
  std::vector<uint64_t> res;
  while (true) {
    nxt = in;
    for (uint64_t i = 0; i < total; ++i) {
      if (!in[i]) continue;
      post(i, &res);
      for (uint64_t v : res) nxt[v] = 1;
    }
    uint64_t added = 0;
    for (uint64_t i = 0; i < total; ++i) added += (nxt[i] && !in[i]) ? 1 : 0;
    if (added == 0) break;
    levels.push_back(added);
    in.swap(nxt);
  }
  uint64_t n_reach = 0, transitions = 0;
  std::vector<Vec> dead, vis;
  std::vector<uint32_t> local(P);
  for (uint64_t i = 0; i < total; ++i) {
    if (!in[i]) continue;
    ++n_reach;
    post(i, &res);
    transitions += res.size();
    for (uint32_t p = 0; p < P; ++p) local[p] = uint32_t(digit(i, p));
    Vec v = pack(plan, local);
    if (res.empty()) dead.push_back(v);
    if (want_visited) vis.push_back(v);
  }
  fill_result(plan, levels, n_reach, transitions, dead, want_visited ? &vis : nullptr, out);
  return 0;
}


// ---- set digest -----------------------------------------------------------
// Order-independent digest of a set of packed states, for comparing sets too
// large to list (billions of states).  It is test bookkeeping, not part of the
// method: two sums, modulo the Mersenne prime p = 2^31 - 1, of f_k = u^3 + u
// mod p, where u = c_k + sum_i (x_i mod p) * a_k[i] mod p over the state's
// words x_i.  The tests evaluate the same formula over a table's contents.
namespace {
constexpr uint64_t kDigestP = 0x7FFFFFFFULL;
constexpr uint64_t kDigestA[2][4] = {{1103515245ULL, 1664525013ULL, 22695477ULL, 134775813ULL},
                                     {1013904223ULL, 69069ULL, 2147483629ULL, 1566083941ULL}};
constexpr uint64_t kDigestC[2] = {12345ULL, 987654321ULL};

void digest_add(const Vec& v, uint32_t words, uint64_t* d) {
  for (int k = 0; k < 2; ++k) {
    uint64_t u = kDigestC[k];
    for (uint32_t i = 0; i < words; ++i)
      u = (u + (v[i] % kDigestP) * kDigestA[k][i] % kDigestP) % kDigestP;
    const uint64_t f = (u * u % kDigestP * u + u) % kDigestP;
    d[k] = (d[k] + f) % kDigestP;
  }
}
}  // namespace

// Digest of n packed states (n x words), written to digest[0..1].
void oracle_digest(uint32_t words, const uint32_t* states, uint64_t n, uint64_t* digest) {
  digest[0] = digest[1] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    Vec v{};
    for (uint32_t k = 0; k < words; ++k) v[k] = states[i * words + k];
    digest_add(v, words, digest);
  }
}

// ---- exploration over dense bitmaps ----------------------------------------
struct oracle_dense_result {
  uint32_t words;
  uint32_t n_levels;
  uint64_t n_states;
  uint64_t n_transitions;
  uint64_t* levels;            // n_levels
  uint64_t n_deadlocks;
  uint64_t n_deadlocks_listed; // n_deadlocks when it is at most the cap, else 0
  uint32_t* deadlocks;         // n_deadlocks_listed x words, sorted
  uint64_t digest[2];          // digest of the reachable set
  uint64_t dead_digest[2];     // digest of the deadlock set
  uint64_t index_space;        // product of the locally reachable state counts
  uint32_t* visited;           // n_states x words, sorted (only when requested)
};

void oracle_dense_result_free(oracle_dense_result* r) {
  if (!r) return;
  std::free(r->levels);
  std::free(r->deadlocks);
  std::free(r->visited);
  r->levels = nullptr;
  r->deadlocks = nullptr;
  r->visited = nullptr;
}

// The same level-synchronous breadth-first search as oracle_explore (Sec. 3),
// for state spaces too large for a hash set: the visited set, the current
// level and the next level are dense bitmaps over the product of the
// processes' locally reachable states (every reachable product state lies in
// that product), indexed mixed-radix, and the states of a level are expanded
// by n_threads threads.  A level holds exactly the states at distance k
// whatever order the threads take, so every result is deterministic.
// Successors follow the same semantics as successors() above: a transition
// whose label a rule names at its process fires only through rules, all
// participants stepping together; every other transition fires alone.
//
// Returns 0, -1 on an invalid network, -2 when the index space exceeds
// max_index_space, -3 when the bitmaps cannot be allocated.
int oracle_explore_dense(uint32_t P, const uint32_t* n_states, const uint32_t* initial,
                         const uint32_t* n_trans, const uint32_t* src, const uint32_t* label,
                         const uint32_t* dst, uint32_t n_labels, uint32_t R,
                         const int32_t* rules, uint32_t n_threads, uint64_t max_index_space,
                         uint64_t dead_cap, int want_visited, oracle_dense_result* out) {
  Net net;
  Plan plan;
  if (P == 0 || !load_net(P, n_states, initial, n_trans, src, label, dst, n_labels, R, rules,
                          &net))
    return -1;
  if (!make_plan(P, n_states, &plan) || plan.words > kMaxWords) return -1;
  if (n_threads == 0) n_threads = std::max(1u, std::thread::hardware_concurrency());

  // Locally reachable states of each process: the closure of its initial state
  // under all of its transitions.  digit d of process p stands for local state
  // reach[p][d].
  std::vector<std::vector<uint32_t>> reach(P);
  std::vector<std::vector<int64_t>> digit_of(P);
  for (uint32_t p = 0; p < P; ++p) {
    std::vector<bool> seen(net.n_states[p], false);
    std::vector<uint32_t> stack{net.initial[p]};
    seen[net.initial[p]] = true;
    while (!stack.empty()) {
      uint32_t s = stack.back();
      stack.pop_back();
      for (const Trans& t : net.out[p][s])
        if (!seen[t.dst]) {
          seen[t.dst] = true;
          stack.push_back(t.dst);
        }
    }
    digit_of[p].assign(net.n_states[p], -1);
    for (uint32_t s = 0; s < net.n_states[p]; ++s)
      if (seen[s]) {
        digit_of[p][s] = int64_t(reach[p].size());
        reach[p].push_back(s);
      }
  }
  std::vector<uint64_t> radix(P, 1);
  uint64_t total = 1;
  for (uint32_t p = 0; p < P; ++p) {
    radix[p] = total;
    if (total > max_index_space / reach[p].size()) return -2;
    total *= reach[p].size();
  }
  // Per process and digit: the targets (as digits) of the transitions that
  // fire alone; per rule and participant: the targets of its matching ones.
  std::vector<std::vector<std::vector<uint32_t>>> alone(P);
  for (uint32_t p = 0; p < P; ++p) {
    alone[p].resize(reach[p].size());
    for (size_t d = 0; d < reach[p].size(); ++d)
      for (const Trans& t : net.out[p][reach[p][d]])
        if (!net.governed[p][t.label]) alone[p][d].push_back(uint32_t(digit_of[p][t.dst]));
  }
  struct Part {
    uint32_t p;
    std::vector<std::vector<uint32_t>> to;  // digit -> target digits
  };
  std::vector<std::vector<Part>> rule_parts(R);
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t p = 0; p < P; ++p) {
      const int32_t a = net.rules[size_t(r) * P + p];
      if (a < 0) continue;
      Part part{p, std::vector<std::vector<uint32_t>>(reach[p].size())};
      for (size_t d = 0; d < reach[p].size(); ++d)
        for (const Trans& t : net.out[p][reach[p][d]])
          if (t.label == uint32_t(a)) part.to[d].push_back(uint32_t(digit_of[p][t.dst]));
      rule_parts[r].push_back(std::move(part));
    }

  const uint64_t n_words = (total + 63) / 64;
  auto alloc = [&](void) {
    return static_cast<uint64_t*>(std::calloc(n_words, sizeof(uint64_t)));
  };
  std::unique_ptr<uint64_t, decltype(&std::free)> visited(alloc(), &std::free),
      cur(alloc(), &std::free), nxt(alloc(), &std::free);
  if (!visited || !cur || !nxt) return -3;
  uint64_t* V = visited.get();
  uint64_t* F = cur.get();
  uint64_t* N = nxt.get();

  uint64_t init = 0;
  for (uint32_t p = 0; p < P; ++p) init += uint64_t(digit_of[p][net.initial[p]]) * radix[p];
  V[init / 64] |= uint64_t(1) << (init % 64);
  F[init / 64] |= uint64_t(1) << (init % 64);

  auto digits_of = [&](uint64_t idx, uint32_t* d) {
    for (uint32_t p = 0; p < P; ++p) {
      d[p] = uint32_t(idx % reach[p].size());
      idx /= reach[p].size();
    }
  };
  auto packed = [&](const uint32_t* d) {
    std::vector<uint32_t> local(P);
    for (uint32_t p = 0; p < P; ++p) local[p] = reach[p][d[p]];
    return pack(plan, local);
  };

  struct Acc {
    uint64_t fresh = 0, trans = 0, dead = 0;
    uint64_t dead_digest[2] = {0, 0};
    std::vector<uint64_t> dead_idx;
  };
  std::vector<Acc> acc(n_threads);
  std::vector<uint64_t> levels{1};
  constexpr uint64_t kChunk = 1024;  // bitmap words per unit of work

  auto expand_level = [&](uint32_t tid, std::atomic<uint64_t>* next_chunk) {
    Acc& a = acc[tid];
    std::vector<uint32_t> d(P);
    std::vector<size_t> pick;
    auto visit = [&](uint64_t s) {
      ++a.trans;
      uint64_t* wv = V + s / 64;
      const uint64_t bit = uint64_t(1) << (s % 64);
      if (__atomic_load_n(wv, __ATOMIC_RELAXED) & bit) return;
      if (__atomic_fetch_or(wv, bit, __ATOMIC_RELAXED) & bit) return;
      __atomic_fetch_or(N + s / 64, bit, __ATOMIC_RELAXED);
      ++a.fresh;
    };
    while (true) {
      const uint64_t c = next_chunk->fetch_add(1);
      if (c * kChunk >= n_words) break;
      const uint64_t end = std::min(n_words, (c + 1) * kChunk);
      for (uint64_t wi = c * kChunk; wi < end; ++wi) {
        uint64_t x = F[wi];
        if (!x) continue;
        F[wi] = 0;  // consumed: this bitmap is the next level's after the swap
        while (x) {
          const uint64_t idx = wi * 64 + uint64_t(__builtin_ctzll(x));
          x &= x - 1;
          digits_of(idx, d.data());
          const uint64_t before = a.trans;
          for (uint32_t p = 0; p < P; ++p)
            for (uint32_t t : alone[p][d[p]])
              visit(idx - uint64_t(d[p]) * radix[p] + uint64_t(t) * radix[p]);
          for (uint32_t r = 0; r < R; ++r) {
            const std::vector<Part>& parts = rule_parts[r];
            bool blocked = false;
            for (const Part& q : parts) blocked |= q.to[d[q.p]].empty();
            if (blocked) continue;
            pick.assign(parts.size(), 0);
            while (true) {  // every choice of one matching transition per participant
              uint64_t s = idx;
              for (size_t i = 0; i < parts.size(); ++i) {
                const Part& q = parts[i];
                s = s - uint64_t(d[q.p]) * radix[q.p] +
                    uint64_t(q.to[d[q.p]][pick[i]]) * radix[q.p];
              }
              visit(s);
              size_t i = 0;
              while (i < parts.size() && ++pick[i] == parts[i].to[d[parts[i].p]].size())
                pick[i++] = 0;
              if (i == parts.size()) break;
            }
          }
          if (a.trans == before) {  // no product transition: a deadlock
            ++a.dead;
            digest_add(packed(d.data()), plan.words, a.dead_digest);
            if (a.dead_idx.size() <= dead_cap) a.dead_idx.push_back(idx);
          }
        }
      }
    }
  };

  while (true) {
    std::atomic<uint64_t> next_chunk{0};
    for (Acc& a : acc) a.fresh = 0;
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < n_threads; ++t) pool.emplace_back(expand_level, t, &next_chunk);
    for (std::thread& th : pool) th.join();
    uint64_t fresh = 0;
    for (const Acc& a : acc) fresh += a.fresh;
    if (fresh == 0) break;
    levels.push_back(fresh);
    std::swap(F, N);
  }

  // Count, digest (and optionally list) the visited set.
  struct Scan {
    uint64_t n = 0;
    uint64_t digest[2] = {0, 0};
    std::vector<Vec> vis;
  };
  std::vector<Scan> scans(n_threads);
  {
    std::atomic<uint64_t> next_chunk{0};
    auto scan = [&](uint32_t tid) {
      Scan& sc = scans[tid];
      std::vector<uint32_t> d(P);
      while (true) {
        const uint64_t c = next_chunk.fetch_add(1);
        if (c * kChunk >= n_words) break;
        const uint64_t end = std::min(n_words, (c + 1) * kChunk);
        for (uint64_t wi = c * kChunk; wi < end; ++wi)
          for (uint64_t x = V[wi]; x; x &= x - 1) {
            digits_of(wi * 64 + uint64_t(__builtin_ctzll(x)), d.data());
            const Vec v = packed(d.data());
            ++sc.n;
            digest_add(v, plan.words, sc.digest);
            if (want_visited) sc.vis.push_back(v);
          }
      }
    };
    std::vector<std::thread> pool;
    for (uint32_t t = 0; t < n_threads; ++t) pool.emplace_back(scan, t);
    for (std::thread& th : pool) th.join();
  }

  uint64_t n_reach = 0, transitions = 0, n_dead = 0;
  uint64_t digest[2] = {0, 0}, dead_digest[2] = {0, 0};
  std::vector<Vec> dead, vis;
  for (const Scan& sc : scans) {
    n_reach += sc.n;
    for (int k = 0; k < 2; ++k) digest[k] = (digest[k] + sc.digest[k]) % kDigestP;
    if (want_visited) vis.insert(vis.end(), sc.vis.begin(), sc.vis.end());
  }
  for (const Acc& a : acc) {
    transitions += a.trans;
    n_dead += a.dead;
    for (int k = 0; k < 2; ++k) dead_digest[k] = (dead_digest[k] + a.dead_digest[k]) % kDigestP;
  }
  if (n_dead <= dead_cap) {
    std::vector<uint32_t> d(P);
    for (const Acc& a : acc)
      for (uint64_t idx : a.dead_idx) {
        digits_of(idx, d.data());
        dead.push_back(packed(d.data()));
      }
  }
  uint64_t level_sum = 0;
  for (uint64_t l : levels) level_sum += l;
  if (level_sum != n_reach) return -4;  // cannot happen: every visited bit is counted once

  oracle_result base{};
  fill_result(plan, levels, n_reach, transitions, dead, want_visited ? &vis : nullptr, &base);
  out->words = base.words;
  out->n_levels = base.n_levels;
  out->n_states = base.n_states;
  out->n_transitions = base.n_transitions;
  out->levels = base.levels;
  out->n_deadlocks = n_dead;
  out->n_deadlocks_listed = base.n_deadlocks;
  out->deadlocks = base.deadlocks;
  out->visited = base.visited;
  for (int k = 0; k < 2; ++k) {
    out->digest[k] = digest[k];
    out->dead_digest[k] = dead_digest[k];
  }
  out->index_space = total;
  return 0;
}

}  // extern "C"
