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
  // creation order sort of every live class
  std::vector<uint32_t> ids;
  for (auto& kv : model) ids.push_back(kv.first);
  P.sort_by_seq(ids);
  for (size_t i = 1; i < ids.size(); i++)
    if (P.cls[ids[i - 1]].seq >= P.cls[ids[i]].seq) return why = "sort_by_seq out of order", n_ops - 1;
  P.destroy();
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
    if (rng() % 3) {
      const uint32_t v = (uint32_t)(rng() % 1000000);
      ix.set(k, v);
      m[k] = v;
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
