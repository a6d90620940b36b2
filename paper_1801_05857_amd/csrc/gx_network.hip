// Composition of a network of LTSs with the automaton of a negated safety
// property (Sec. 3: such an automaton can be added to the network and the
// property checked during exploration).  Host code only.
#include <algorithm>
#include <cstdint>
#include <new>
#include <set>
#include <vector>

#include "../../include/gx.h"

namespace {

// Storage behind a gx_monitored_network.
struct Composed {
  std::vector<gx_lts> procs;
  std::vector<std::vector<uint32_t>> src, label, dst;
  std::vector<int32_t> rules;
  std::vector<uint8_t> bad;
};

}  // namespace

extern "C" {

gx_status gx_network_add_monitor(const gx_network* net, const gx_monitor* mon,
                                 gx_monitored_network* out) {
  if (!net || !mon || !out) return GX_EINVAL;
  uint32_t w = 0;
  if (gx_network_words(net, &w) != GX_OK) return GX_EINVAL;  // validates the network
  const uint32_t P = net->n_procs, R = net->n_rules, L = net->n_labels;
  const uint64_t n_actions = uint64_t(R) + L;
  if (mon->n_states == 0 || mon->initial >= mon->n_states || !mon->bad ||
      (mon->n_trans && (!mon->src || !mon->action || !mon->dst)))
    return GX_EINVAL;
  for (uint32_t t = 0; t < mon->n_trans; ++t)
    if (mon->src[t] >= mon->n_states || mon->dst[t] >= mon->n_states ||
        mon->action[t] >= n_actions)
      return GX_EINVAL;

  // governed[p][l]: some rule names label l at process p
  std::vector<std::vector<bool>> governed(P, std::vector<bool>(L, false));
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t p = 0; p < P; ++p) {
      const int32_t a = net->rules[uint64_t(r) * P + p];
      if (a >= 0) governed[p][a] = true;
    }
  std::vector<bool> observed(n_actions, false);
  for (uint32_t t = 0; t < mon->n_trans; ++t) observed[mon->action[t]] = true;

  // Actions the network performs and the automaton observes get one fresh
  // label each (after the network's own labels): every observed rule, and
  // every observed label that some process fires alone.
  std::vector<int64_t> fresh(n_actions, -1);
  uint32_t n_new = 0;
  for (uint32_t r = 0; r < R; ++r)
    if (observed[r]) fresh[r] = L + n_new++;
  std::vector<std::set<uint32_t>> alone(P);  // labels p fires alone
  for (uint32_t p = 0; p < P; ++p)
    for (uint32_t t = 0; t < net->procs[p].n_trans; ++t) {
      const uint32_t l = net->procs[p].label[t];
      if (!governed[p][l]) alone[p].insert(l);
    }
  for (uint32_t l = 0; l < L; ++l) {
    if (!observed[R + l]) continue;
    bool performed = false;
    for (uint32_t p = 0; p < P && !performed; ++p) performed = alone[p].count(l) != 0;
    if (performed) fresh[R + l] = L + n_new++;
  }

  Composed* c = new (std::nothrow) Composed;
  if (!c) return GX_ENOMEM;
  try {
    // rules: each existing rule, with the automaton taking part when it
    // observes the rule; then one rule (l at p, the automaton) for every
    // observed label l that process p fires alone
    for (uint32_t r = 0; r < R; ++r) {
      for (uint32_t p = 0; p < P; ++p) c->rules.push_back(net->rules[uint64_t(r) * P + p]);
      c->rules.push_back(static_cast<int32_t>(fresh[r]));
    }
    for (uint32_t p = 0; p < P; ++p)
      for (uint32_t l : alone[p]) {
        if (fresh[R + l] < 0) continue;
        for (uint32_t q = 0; q <= P; ++q) c->rules.push_back(-1);
        c->rules[c->rules.size() - (P + 1) + p] = static_cast<int32_t>(l);
        c->rules.back() = static_cast<int32_t>(fresh[R + l]);
      }
    // the automaton: its transitions on performed actions, completed with a
    // self-loop wherever it leaves a performed action unspecified (so it
    // never blocks the network); actions the network never performs drop out
    std::vector<uint32_t> ms, ml, md;
    std::set<std::pair<uint32_t, uint32_t>> has;
    for (uint32_t t = 0; t < mon->n_trans; ++t) {
      const int64_t f = fresh[mon->action[t]];
      if (f < 0) continue;
      ms.push_back(mon->src[t]);
      ml.push_back(static_cast<uint32_t>(f));
      md.push_back(mon->dst[t]);
      has.insert({mon->src[t], static_cast<uint32_t>(f)});
    }
    for (uint32_t m = 0; m < mon->n_states; ++m)
      for (uint64_t a = 0; a < n_actions; ++a) {
        if (fresh[a] < 0 || has.count({m, static_cast<uint32_t>(fresh[a])})) continue;
        ms.push_back(m);
        ml.push_back(static_cast<uint32_t>(fresh[a]));
        md.push_back(m);
      }
    c->src.resize(P + 1);
    c->label.resize(P + 1);
    c->dst.resize(P + 1);
    c->procs.resize(P + 1);
    for (uint32_t p = 0; p < P; ++p) {
      const gx_lts& l = net->procs[p];
      c->src[p].assign(l.src, l.src + l.n_trans);
      c->label[p].assign(l.label, l.label + l.n_trans);
      c->dst[p].assign(l.dst, l.dst + l.n_trans);
    }
    c->src[P] = ms;
    c->label[P] = ml;
    c->dst[P] = md;
    for (uint32_t p = 0; p <= P; ++p) {
      c->procs[p].n_states = p < P ? net->procs[p].n_states : mon->n_states;
      c->procs[p].initial = p < P ? net->procs[p].initial : mon->initial;
      c->procs[p].n_trans = static_cast<uint32_t>(c->src[p].size());
      c->procs[p].src = c->src[p].data();
      c->procs[p].label = c->label[p].data();
      c->procs[p].dst = c->dst[p].data();
    }
    c->bad.assign(mon->bad, mon->bad + mon->n_states);
  } catch (...) {
    delete c;
    return GX_ENOMEM;
  }
  out->net.n_procs = P + 1;
  out->net.procs = c->procs.data();
  out->net.n_labels = std::max<uint32_t>(1, L + n_new);
  out->net.n_rules = static_cast<uint32_t>(c->rules.size() / (P + 1));
  out->net.rules = c->rules.empty() ? nullptr : c->rules.data();
  out->monitor_proc = P;
  out->monitor_bad = c->bad.data();
  out->owner = c;
  return GX_OK;
}

void gx_monitored_network_free(gx_monitored_network* m) {
  if (!m) return;
  delete static_cast<Composed*>(m->owner);
  m->owner = nullptr;
  m->net = gx_network{};
  m->monitor_bad = nullptr;
}

}  // extern "C"
