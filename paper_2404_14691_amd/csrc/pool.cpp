// Shared block pool: an arena of 64 KiB slots, the fingerprint index of
// resident classes, references and the eviction order of unreferenced
// classes (front = least recently released).  All lists are intrusive in
// the class records, so the steady state allocates nothing.
#include "internal.h"

namespace sage {

// ---------------------------------------------------------------- FpIndex
static inline size_t fp_hash(uint64_t fp) { return (size_t)(fp ^ (fp >> 29)) * 0x9E3779B97F4A7C15ull >> 7; }

uint32_t FpIndex::find(uint64_t fp) const {
  if (!n_) return kNone;
  for (size_t i = fp_hash(fp) & mask_;; i = (i + 1) & mask_) {
    if (val_[i] == kNone) return kNone;
    if (key_[i] == fp) return val_[i];
  }
}

void FpIndex::grow() {
  std::vector<uint64_t> k = std::move(key_);
  std::vector<uint32_t> v = std::move(val_);
  const size_t cap = k.empty() ? 1024 : k.size() * 2;
  key_.assign(cap, 0);
  val_.assign(cap, kNone);
  mask_ = cap - 1;
  n_ = 0;
  for (size_t i = 0; i < k.size(); i++)
    if (v[i] != kNone) set(k[i], v[i]);
}

void FpIndex::set(uint64_t fp, uint32_t head) {
  if ((n_ + 1) * 2 > key_.size()) grow();
  for (size_t i = fp_hash(fp) & mask_;; i = (i + 1) & mask_) {
    if (val_[i] == kNone) {
      key_[i] = fp;
      val_[i] = head;
      n_++;
      return;
    }
    if (key_[i] == fp) {
      val_[i] = head;
      return;
    }
  }
}

uint32_t FpIndex::insert_if_absent(uint64_t fp, uint32_t head) {
  if ((n_ + 1) * 2 > key_.size()) grow();
  for (size_t i = fp_hash(fp) & mask_;; i = (i + 1) & mask_) {
    if (val_[i] == kNone) {
      key_[i] = fp;
      val_[i] = head;
      n_++;
      return kNone;
    }
    if (key_[i] == fp) return val_[i];
  }
}

// Linear probing with backward-shift deletion (no tombstones).
void FpIndex::erase(uint64_t fp) {
  if (!n_) return;
  for (size_t i = fp_hash(fp) & mask_;; i = (i + 1) & mask_) {
    if (val_[i] == kNone) return;
    if (key_[i] == fp) return erase_at(i);
  }
}

void FpIndex::erase_at(size_t i) {
  for (size_t j = (i + 1) & mask_;; j = (j + 1) & mask_) {
    if (val_[j] == kNone) break;
    const size_t home = fp_hash(key_[j]) & mask_;
    // move j back to i when its home is not in the cyclic range (i, j]
    const bool in_range = i <= j ? (home > i && home <= j) : (home > i || home <= j);
    if (!in_range) {
      key_[i] = key_[j];
      val_[i] = val_[j];
      i = j;
    }
  }
  val_[i] = kNone;
  n_--;
}

uint32_t FpIndex::pop_head(uint64_t fp, uint32_t head, uint32_t next) {
  if (!n_) return kNone;
  for (size_t i = fp_hash(fp) & mask_;; i = (i + 1) & mask_) {
    if (val_[i] == kNone) return kNone;
    if (key_[i] != fp) continue;
    const uint32_t h = val_[i];
    if (h == head) {
      if (next != kNone) val_[i] = next;
      else erase_at(i);
    }
    return h;
  }
}

void FpIndex::clear() {
  key_.clear();
  val_.clear();
  mask_ = n_ = 0;
}

// ---------------------------------------------------------------- Pool
void Pool::init(uint64_t budget_slots, size_t seg_slots, bool host_standin) {
  budget = budget_slots;
  standin_ = host_standin;
  // a power-of-two stride, so that a slot's segment and offset are a shift
  // and a mask; a segment still holds no more slots than the budget leaves
  seg_shift_ = 0;
  while (((size_t)1 << seg_shift_) < std::max<size_t>(seg_slots, 1)) seg_shift_++;
  seg_slots_ = (size_t)1 << seg_shift_;
}

void Pool::destroy() {
  if (!standin_)
    for (uint8_t* s : segs_) (void)hipFree(s);
  for (HostBuf& h : hbufs)
    if (h.p) (void)hipHostFree(h.p);
  for (auto& kv : spare_host_) (void)hipHostFree(kv.second);
  spare_host_.clear();
  spare_bytes_ = 0;
  hbufs.clear();
  free_hbufs_.clear();
  host_lru.clear();
  host_bytes = 0;
  segs_.clear();
  free_.clear();
  free_cls_.clear();
  index_.clear();
  cls.clear();
  lru_head_ = lru_tail_ = kNone;
  used_ = live_classes = 0;
}

bool Pool::grow_arena() {
  const uint64_t cap = (uint64_t)segs_.size() * seg_slots_;
  if (cap >= budget) return false;
  const uint64_t n = std::min<uint64_t>(seg_slots_, budget - cap);
  uint8_t* p = nullptr;
  if (standin_) {
    // host self-test: distinct, never dereferenced segment addresses
    p = reinterpret_cast<uint8_t*>((uint64_t)(segs_.size() + 1) << 40);
  } else if ((fault && fault->fail_now()) || hipMalloc(&p, n * kBlock) != hipSuccess) {
    (void)hipGetLastError();
    budget = used_;  // the device is full: the budget stops at what is held
    return false;
  }
  const uint32_t base = (uint32_t)cap;
  segs_.push_back(p);
  for (uint64_t i = n; i-- > 0;) free_.push_back(base + (uint32_t)i);
  return true;
}

uint32_t Pool::new_class(uint64_t fp, uint32_t len) {
  uint32_t c;
  if (!free_cls_.empty()) {
    c = free_cls_.back();
    free_cls_.pop_back();
  } else {
    cls.emplace_back();
    c = (uint32_t)cls.size() - 1;
  }
  Class& k = cls[c];
  k = Class{};
  k.fp = fp;
  k.len = len;
  k.seq = seq_++;
  k.alive = true;
  live_classes++;
  return c;
}

void Pool::index_add(uint32_t c) {
  cls[c].next = kNone;
  const uint32_t h = index_.insert_if_absent(cls[c].fp, c);
  if (h != kNone) {
    uint32_t t = h;
    while (cls[t].next != kNone) t = cls[t].next;
    cls[t].next = c;
  }
  cls[c].indexed = true;
}

void Pool::index_remove(uint32_t c) {
  if (!cls[c].indexed) return;
  const uint32_t h = index_.pop_head(cls[c].fp, c, cls[c].next);
  if (h != c && h != kNone) {
    uint32_t t = h;
    while (t != kNone && cls[t].next != c) t = cls[t].next;
    if (t != kNone) cls[t].next = cls[c].next;
  }
  cls[c].next = kNone;
  cls[c].indexed = false;
}

void Pool::lru_remove(uint32_t c) {
  Class& k = cls[c];
  if (!k.in_lru) return;
  if (k.lru_prev != kNone) cls[k.lru_prev].lru_next = k.lru_next;
  else lru_head_ = k.lru_next;
  if (k.lru_next != kNone) cls[k.lru_next].lru_prev = k.lru_prev;
  else lru_tail_ = k.lru_prev;
  k.lru_prev = k.lru_next = kNone;
  k.in_lru = false;
}

void Pool::lru_back(uint32_t c, double now) {
  lru_remove(c);
  Class& k = cls[c];
  k.lru_prev = lru_tail_;
  k.lru_next = kNone;
  if (lru_tail_ != kNone) cls[lru_tail_].lru_next = c;
  else lru_head_ = c;
  lru_tail_ = c;
  k.in_lru = true;
  k.idle_since = now;
}

void Pool::evict(uint32_t c, bool demotion) {
  Class& k = cls[c];
  lru_remove(c);
  index_remove(c);
  if (k.slot != kNone) {
    free_slot(k.slot);
    k.slot = kNone;
  }
  if (demotion) demotions++;
  else evictions++;
  epoch++;
}

void Pool::drop_class(uint32_t c) {
  Class& k = cls[c];
  if (!k.alive) return;
  lru_remove(c);
  index_remove(c);
  if (k.slot != kNone) {
    free_slot(k.slot);
    k.slot = kNone;
  }
  host_release(c);
  k.alive = false;
  k.pending = nullptr;
  live_classes--;
  free_cls_.push_back(c);
}

uint32_t Pool::host_buffer(uint32_t blocks, uint64_t budget_bytes) {
  uint64_t bytes = (uint64_t)blocks * kBlock;
  if (budget_bytes && host_bytes + bytes > budget_bytes) return kNone;
  uint8_t* p = nullptr;
  // a spare pinned buffer of the same size first: pinning and unpinning cost
  // milliseconds per buffer, more than moving its bytes over the link
  auto it = spare_host_.find(blocks);
  if (it != spare_host_.end()) {
    p = it->second;
    spare_host_.erase(it);
    spare_bytes_ -= bytes;
  } else if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return kNone;
  }
  uint32_t h;
  if (!free_hbufs_.empty()) {
    h = free_hbufs_.back();
    free_hbufs_.pop_back();
  } else {
    hbufs.emplace_back();
    h = (uint32_t)hbufs.size() - 1;
  }
  hbufs[h] = HostBuf{p, blocks, 0};
  host_bytes += bytes;
  return h;
}

void Pool::host_release(uint32_t c) {
  Class& k = cls[c];
  if (k.hbuf == kNone) return;
  HostBuf& h = hbufs[k.hbuf];
  if (--h.live == 0) {
    const uint64_t bytes = (uint64_t)h.blocks * kBlock;
    if (spare_bytes_ + bytes <= kSpareHostBytes) {
      spare_host_.emplace(h.blocks, h.p);
      spare_bytes_ += bytes;
    } else {
      (void)hipHostFree(h.p);
    }
    host_bytes -= bytes;
    h = HostBuf{};
    free_hbufs_.push_back(k.hbuf);
  }
  k.hbuf = kNone;
  k.hoff = 0;
}

void Pool::sort_by_seq(std::vector<uint32_t>& ids) const {
  if (ids.size() < 2) return;
  // sequence numbers are unique: already ascending, or spread over few
  // values (a registration's classes were mostly created recently), a
  // direct placement by seq - min is one pass
  uint64_t mn = ~0ull, mx = 0;
  bool sorted = true;
  for (size_t i = 0; i < ids.size(); i++) {
    const uint64_t q = cls[ids[i]].seq;
    if (i && q < cls[ids[i - 1]].seq) sorted = false;
    mn = std::min(mn, q);
    mx = std::max(mx, q);
  }
  if (sorted) return;
  if (mx - mn < 8 * (uint64_t)ids.size() + 4096) {
    std::vector<uint32_t> at(mx - mn + 1, kNone);
    for (uint32_t id : ids) at[cls[id].seq - mn] = id;
    size_t k = 0;
    for (uint32_t id : at)
      if (id != kNone) ids[k++] = id;
    return;
  }
  std::vector<std::pair<uint64_t, uint32_t>> a(ids.size()), b(ids.size());
  for (size_t i = 0; i < ids.size(); i++) a[i] = {cls[ids[i]].seq, ids[i]};
  for (unsigned shift = 0; shift < 64 && (mx >> shift) != 0; shift += 8) {
    size_t cnt[257] = {0};
    for (const auto& e : a) cnt[((e.first >> shift) & 255) + 1]++;
    for (int k = 0; k < 256; k++) cnt[k + 1] += cnt[k];
    for (const auto& e : a) b[cnt[(e.first >> shift) & 255]++] = e;
    a.swap(b);
  }
  for (size_t i = 0; i < ids.size(); i++) ids[i] = a[i].second;
}

}  // namespace sage
