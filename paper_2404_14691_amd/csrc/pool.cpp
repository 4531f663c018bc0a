// Shared block pool: an arena of 64 KiB slots, the fingerprint index of
// resident classes, references and the eviction order of unreferenced
// classes (front = least recently released).
#include "internal.h"

namespace sage {

void Pool::init(uint64_t budget_slots, size_t seg_slots) {
  budget = budget_slots;
  seg_slots_ = seg_slots;
}

void Pool::destroy() {
  for (uint8_t* s : segs_) (void)hipFree(s);
  segs_.clear();
  free_.clear();
  index_.clear();
  lru.clear();
  cls.clear();
  used_ = 0;
}

uint32_t Pool::alloc_slot(const std::function<bool(uint32_t)>& protect) {
  const uint64_t cap = (uint64_t)segs_.size() * seg_slots_;
  if (free_.empty() && used_ < budget && cap < budget) {
    const uint64_t n = std::min<uint64_t>(seg_slots_, budget - cap);
    uint8_t* p = nullptr;
    if (hipMalloc(&p, n * kBlock) == hipSuccess) {
      const uint32_t base = (uint32_t)cap;
      segs_.push_back(p);
      for (uint64_t i = n; i-- > 0;) free_.push_back(base + (uint32_t)i);
    } else {
      (void)hipGetLastError();
      budget = used_;  // the device is full: the budget stops at what is held
    }
  }
  if (free_.empty() || used_ >= budget) {
    uint32_t victim = kNone;
    for (uint32_t c : lru)
      if (!protect(c)) {
        victim = c;
        break;
      }
    if (victim == kNone) return kNone;
    evict(victim);
  }
  if (free_.empty()) return kNone;
  const uint32_t s = free_.back();
  free_.pop_back();
  used_++;
  return s;
}

uint32_t Pool::new_class(uint64_t fp, uint32_t len) {
  Class c;
  c.fp = fp;
  c.len = len;
  c.alive = true;
  cls.push_back(c);
  return (uint32_t)cls.size() - 1;
}

void Pool::index_add(uint32_t c) {
  cls[c].next = kNone;
  auto it = index_.find(cls[c].fp);
  if (it == index_.end()) {
    index_.emplace(cls[c].fp, c);
  } else {
    uint32_t t = it->second;
    while (cls[t].next != kNone) t = cls[t].next;
    cls[t].next = c;
  }
  cls[c].indexed = true;
}

void Pool::index_remove(uint32_t c) {
  if (!cls[c].indexed) return;
  auto it = index_.find(cls[c].fp);
  if (it != index_.end()) {
    if (it->second == c) {
      if (cls[c].next == kNone) index_.erase(it);
      else it->second = cls[c].next;
    } else {
      uint32_t t = it->second;
      while (t != kNone && cls[t].next != c) t = cls[t].next;
      if (t != kNone) cls[t].next = cls[c].next;
    }
  }
  cls[c].next = kNone;
  cls[c].indexed = false;
}

uint32_t Pool::chain_head(uint64_t fp) const {
  auto it = index_.find(fp);
  return it == index_.end() ? kNone : it->second;
}

void Pool::lru_back(uint32_t c) {
  Class& k = cls[c];
  if (k.in_lru) lru.erase(k.lru_it);
  lru.push_back(c);
  k.lru_it = std::prev(lru.end());
  k.in_lru = true;
}

void Pool::lru_remove(uint32_t c) {
  Class& k = cls[c];
  if (!k.in_lru) return;
  lru.erase(k.lru_it);
  k.in_lru = false;
}

void Pool::evict(uint32_t c) {
  Class& k = cls[c];
  lru_remove(c);
  index_remove(c);
  if (k.slot != kNone) {
    free_slot(k.slot);
    k.slot = kNone;
  }
  evictions++;
  epoch++;
}

void Pool::drop_class(uint32_t c) {
  Class& k = cls[c];
  lru_remove(c);
  index_remove(c);
  if (k.slot != kNone) {
    free_slot(k.slot);
    k.slot = kNone;
  }
  k.alive = false;
  k.pending = nullptr;
}

}  // namespace sage
