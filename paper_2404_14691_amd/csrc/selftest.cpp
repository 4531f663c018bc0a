// Host-only randomized checks of the block pool and its fingerprint index
// against a plain model, invariants checked after every operation (no GPU:
// the pool's arena is a host stand-in whose slot addresses are never
// dereferenced).  Built into libsage.so and into the sanitizer test driver.
#include <algorithm>
#include <cstring>
#include <random>
#include <unordered_map>

#include "internal.h"

namespace sage {
namespace {

struct ModelClass {
  uint64_t fp;
  bool resident;
  uint32_t active;
};

// The operations the registration, setup, release, reload and unregister
// paths apply to the pool, drawn at random.  Returns the number of the first
// operation after which an invariant fails (message in `why`), or n_ops.
uint32_t pool_stress(uint64_t seed, uint32_t n_ops, uint32_t budget, std::string& why) {
  std::mt19937_64 rng(seed);
  Pool P;
  P.init(budget, std::min<uint32_t>(budget, 16384), /*host_standin=*/true);
  std::unordered_map<uint32_t, ModelClass> model;
  std::vector<uint32_t> lru;  // model eviction order (front = first victim)
  uint32_t resident = 0;
  double now = 0;
  auto pick = [&](auto pred) -> uint32_t {
    std::vector<uint32_t> c;
    for (auto& kv : model)
      if (pred(kv.second)) c.push_back(kv.first);
    if (c.empty()) return kNone;
    std::sort(c.begin(), c.end());
    return c[rng() % c.size()];
  };
  auto lru_drop = [&](uint32_t c) { lru.erase(std::remove(lru.begin(), lru.end(), c), lru.end()); };
  // a slot as alloc_slot gives it: a free one while below the budget, else
  // the front unreferenced class is evicted; kNone when none is left
  auto slot_for = [&](uint32_t* out) -> bool {
    const bool full = resident >= budget;
    if (full && lru.empty()) {
      if (P.alloc_slot([](uint32_t) { return false; }) != kNone) {
        why = "alloc_slot gave a slot with every slot referenced";
        return false;
      }
      *out = kNone;
      return true;
    }
    if (full) {
      const uint32_t v = lru.front();
      lru.erase(lru.begin());
      model[v].resident = false;
      resident--;
    }
    *out = P.alloc_slot([](uint32_t) { return false; });
    if (*out == kNone) {
      why = "alloc_slot found no slot although one was free or evictable";
      return false;
    }
    resident++;
    return true;
  };
  auto check = [&]() -> bool {
    std::vector<uint32_t> slots;
    uint32_t indexed = 0;
    for (auto& kv : model) {
      const Class& k = P.cls[kv.first];
      if (!k.alive) return why = "model class not alive in the pool", false;
      if ((k.slot != kNone) != kv.second.resident) return why = "residency differs from the model", false;
      if (k.slot != kNone) slots.push_back(k.slot);
      if (k.indexed != kv.second.resident) return why = "index membership differs from residency", false;
      indexed += k.indexed;
    }
    if (P.live_classes != model.size()) return why = "live class count differs", false;
    if (P.used_ != resident || slots.size() != resident) return why = "used slots differ from resident classes", false;
    std::sort(slots.begin(), slots.end());
    if (std::adjacent_find(slots.begin(), slots.end()) != slots.end()) return why = "two classes share a slot", false;
    if (!slots.empty() && slots.back() >= budget) return why = "slot beyond the budget", false;
    // eviction order
    std::vector<uint32_t> walk;
    for (uint32_t c = P.lru_front(); c != kNone; c = P.cls[c].lru_next) {
      walk.push_back(c);
      if (walk.size() > model.size()) return why = "eviction list has a cycle", false;
    }
    if (walk != lru) return why = "eviction order differs from the model", false;
    // fingerprint chains: each holds exactly the indexed classes of its fp
    uint32_t chained = 0;
    std::vector<uint64_t> fps;
    for (auto& kv : model) fps.push_back(kv.second.fp);
    std::sort(fps.begin(), fps.end());
    fps.erase(std::unique(fps.begin(), fps.end()), fps.end());
    for (uint64_t fp : fps) {
      for (uint32_t c = P.chain_head(fp); c != kNone; c = P.cls[c].next) {
        auto it = model.find(c);
        if (it == model.end() || it->second.fp != fp || !it->second.resident)
          return why = "fingerprint chain holds a wrong class", false;
        if (++chained > model.size()) return why = "fingerprint chain has a cycle", false;
      }
    }
    if (chained != indexed) return why = "an indexed class is missing from its chain", false;
    return true;
  };
  for (uint32_t op = 0; op < n_ops; op++) {
    now += 1.0;
    const uint32_t r = (uint32_t)(rng() % 100);
    if (r < 40) {  // registration: a new class in a fresh slot, unreferenced
      uint32_t s;
      if (!slot_for(&s)) return op;
      if (s != kNone) {
        const uint64_t fp = rng() % 48;
        const uint32_t c = P.new_class(fp, 1 + (uint32_t)(rng() % kBlock));
        P.cls[c].slot = s;
        P.index_add(c);
        P.lru_back(c, now);
        model[c] = ModelClass{fp, true, 0};
        lru.push_back(c);
      }
    } else if (r < 65) {  // setup: one more reference on a resident class
      const uint32_t c = pick([](const ModelClass& m) { return m.resident; });
      if (c != kNone) {
        if (model[c].active++ == 0) {
          P.lru_remove(c);
          lru_drop(c);
        }
        P.cls[c].active++;
      }
    } else if (r < 85) {  // release
      const uint32_t c = pick([](const ModelClass& m) { return m.active > 0; });
      if (c != kNone) {
        P.cls[c].active--;
        if (--model[c].active == 0) {
          P.lru_back(c, now);
          lru.push_back(c);
        }
      }
    } else if (r < 95) {  // reload of an evicted class
      const uint32_t c = pick([](const ModelClass& m) { return !m.resident; });
      if (c != kNone) {
        uint32_t s;
        if (!slot_for(&s)) return op;
        if (s != kNone) {
          P.cls[c].slot = s;
          P.index_add(c);
          P.lru_back(c, now);
          model[c].resident = true;
          lru.push_back(c);
        }
      }
    } else {  // unregister of the class's last member
      const uint32_t c = pick([](const ModelClass& m) { return m.active == 0; });
      if (c != kNone) {
        if (model[c].resident) resident--;
        P.drop_class(c);
        lru_drop(c);
        model.erase(c);
      }
    }
    if (!check()) return op;
  }
  // creation order sort of every live class, of the same classes shuffled,
  // of an already ascending list and of a sparse subset (every path of the
  // sort: ascending, direct placement, radix); each against std::sort
  std::vector<uint32_t> ids;
  for (auto& kv : model) ids.push_back(kv.first);
  auto by_seq = [&](std::vector<uint32_t> v) {
    std::sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) { return P.cls[a].seq < P.cls[b].seq; });
    return v;
  };
  std::vector<std::vector<uint32_t>> cases{ids};
  std::shuffle(cases[0].begin(), cases[0].end(), rng);
  cases.push_back(by_seq(ids));
  std::vector<uint32_t> sparse;
  for (size_t i = 0; i < cases[1].size(); i += 97) sparse.push_back(cases[1][i]);
  std::reverse(sparse.begin(), sparse.end());
  cases.push_back(sparse);
  cases.push_back(ids);
  for (auto& v : cases) {
    const std::vector<uint32_t> want = by_seq(v);
    P.sort_by_seq(v);
    if (v != want) return why = "sort_by_seq: not the creation order of its input", n_ops - 1;
  }
  P.destroy();
  // classes spread over a wide range of sequence numbers (the radix path)
  Pool Q;
  Q.init(1, 1, /*host_standin=*/true);
  std::vector<uint32_t> wide;
  for (uint32_t i = 0; i < 40000; i++) {
    const uint32_t c = Q.new_class(rng(), 1);
    if (rng() % 64 == 0) wide.push_back(c);
  }
  std::shuffle(wide.begin(), wide.end(), rng);
  std::vector<uint32_t> want = wide;
  std::sort(want.begin(), want.end(), [&](uint32_t a, uint32_t b) { return Q.cls[a].seq < Q.cls[b].seq; });
  Q.sort_by_seq(wide);
  Q.destroy();
  if (wide != want) return why = "sort_by_seq: not the creation order of a sparse input", n_ops - 1;
  return n_ops;
}

// FpIndex against std::unordered_map under random inserts, overwrites and
// backward-shift deletions.
uint32_t index_stress(uint64_t seed, uint32_t n_ops, std::string& why) {
  std::mt19937_64 rng(seed ^ 0x5bd1e995u);
  FpIndex ix;
  std::unordered_map<uint64_t, uint32_t> m;
  const uint64_t keys = 1 + n_ops / 3;
  for (uint32_t op = 0; op < n_ops; op++) {
    const uint64_t k = (rng() % keys) * 0x9E3779B97F4A7C15ull;  // clustered home buckets after hashing
    const uint32_t r = (uint32_t)(rng() % 6);
    if (r < 3) {
      const uint32_t v = (uint32_t)(rng() % 1000000);
      ix.set(k, v);
      m[k] = v;
    } else if (r == 3) {  // insert only if absent: returns what was there
      const uint32_t v = (uint32_t)(rng() % 1000000);
      auto it = m.find(k);
      const uint32_t had = it == m.end() ? kNone : it->second;
      if (ix.insert_if_absent(k, v) != had) return why = "fingerprint index insert_if_absent differs", op;
      if (had == kNone) m[k] = v;
    } else if (r == 4) {  // replace or drop the value if it is the expected one
      auto it = m.find(k);
      const uint32_t had = it == m.end() ? kNone : it->second;
      const uint32_t expect = rng() % 2 && had != kNone ? had : (uint32_t)(rng() % 1000000);
      const uint32_t next = rng() % 2 ? kNone : (uint32_t)(rng() % 1000000);
      if (ix.pop_head(k, expect, next) != had) return why = "fingerprint index pop_head differs", op;
      if (had != kNone && had == expect) {
        if (next == kNone) m.erase(k);
        else m[k] = next;
      }
    } else {
      ix.erase(k);
      m.erase(k);
    }
    const uint64_t q = (rng() % keys) * 0x9E3779B97F4A7C15ull;
    auto it = m.find(q);
    if (ix.find(q) != (it == m.end() ? kNone : it->second)) return why = "fingerprint index lookup differs", op;
  }
  for (auto& kv : m)
    if (ix.find(kv.first) != kv.second) return why = "fingerprint index lost a key", n_ops - 1;
  return n_ops;
}

}  // namespace
}  // namespace sage

using namespace sage;

extern "C" sage_status sage_selftest_pool(uint64_t seed, uint32_t n_ops, uint32_t budget_slots,
                                          uint32_t* failed_op) {
  return guard([&] {
    if (!failed_op || budget_slots < 1 || n_ops < 1) fail(SAGE_EINVAL, "bad argument");
    std::string why;
    uint32_t at = pool_stress(seed, n_ops, budget_slots, why);
    if (at == n_ops) at = index_stress(seed, n_ops, why);
    *failed_op = at;
    if (at != n_ops) fail(SAGE_EINVAL, "operation %u: %s", at, why.c_str());
  });
}
