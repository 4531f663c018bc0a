// Multi-stage exit of idle read-only data and code (section "Multi-stage
// Resource Exit"; Table 4 gives the per-stage latency breakdown).  With the
// interval T = exit_stage_ms, an invocation's resources are released in
// order, each stage one interval long:
//   first stage  (idle < T):      blocks resident in HBM, code object loaded;
//   second stage (T <= idle < 2T): blocks moved to a pinned host cache;
//   third stage  (2T <= idle < 3T): code object unloaded as well;
//   fourth stage (idle >= 3T):     host copies dropped, only the function's
//                                  registered source remains.
// A block's idle time runs from when its last reference went (LRU order);
// a code object's from the last setup or release of one of its functions.
// Any setup ends the exit for what it uses: it reloads from where the bytes
// are and loads the code object again, the two in parallel.
#include <cstring>

#include "internal.h"

namespace sage {


// Second stage for `due` (unreferenced, resident, oldest first): gather each
// batch of blocks into the device staging buffer, one DMA to a new pinned
// host buffer, then free the HBM slots.  Without host budget the blocks are
// simply evicted (the source stays).
static void demote(Ctx& c, const std::vector<uint32_t>& due) {
  Pool& P = c.pool;
  Ring& R = c.ring;
  const size_t per = std::min<size_t>(R.chunk / kBlock, R.cap[0]);
  HIPX(hipEventSynchronize(R.ev[0]));    // slot 0's last batch (e.g. of a reload) has read its buffers
  HIPX(hipEventSynchronize(R.ev_c[0]));  // slot 0's last registration COPY has read its buffers
  for (size_t i = 0; i < due.size(); i += per) {
    const size_t n = std::min(per, due.size() - i);
    const uint32_t h = P.host_buffer((uint32_t)n, c.cfg.host_cache_bytes);
    if (h != kNone) {
      BlkOp* ops = R.hops[0];
      for (size_t j = 0; j < n; j++) {
        const Class& k = P.cls[due[i + j]];
        ops[j] = BlkOp{(uint64_t)P.addr(k.slot), (uint64_t)(R.dev[0] + j * kBlock), k.len, 0};
      }
      // on the control stream: behind any copy still filling these slots
      HIPX(hipMemcpyAsync(R.dops[0], ops, n * sizeof(BlkOp), hipMemcpyHostToDevice, c.ctl));
      HIPX(launch_blkcopy(R.dops[0], (uint32_t)n, R.dres[0], c.max_groups_copy(), c.ctl));
      HIPX(hipMemcpyAsync(P.hbufs[h].p, R.dev[0], n * kBlock, hipMemcpyDeviceToHost, c.ctl));
      HIPX(hipStreamSynchronize(c.ctl));
    }
    for (size_t j = 0; j < n; j++) {
      const uint32_t cl = due[i + j];
      P.evict(cl, h != kNone);
      if (h == kNone) continue;
      Class& k = P.cls[cl];
      P.host_release(cl);  // an older host copy not yet released after its reload
      k.hbuf = h;
      k.hoff = (uint32_t)j;
      k.hgen = P.demotions;
      P.hbufs[h].live++;
      P.host_lru.push_back({cl, k.hgen});
    }
  }
}

void unload_module(Ctx& c, Module& m) {
  flights_drop_graphs(c);  // captured graphs hold the code object's kernels
  std::lock_guard<std::mutex> lk(c.module_mu);
  if (!m.mod) return;
  HIPX(hipModuleUnload(m.mod));
  m.mod = nullptr;
  m.fn.clear();
  c.module_unloads++;
}

void advance_exit(Ctx& c) {
  const double T = c.cfg.exit_stage_ms;
  if (!(T > 0)) return;
  const double now = now_ms();
  Pool& P = c.pool;
  if (c.cfg.share) {
    settle_reloads(c, false);
    std::vector<uint32_t> due;
    for (uint32_t cl = P.lru_front(); cl != kNone; cl = P.cls[cl].lru_next) {
      if (now - P.cls[cl].idle_since < T) break;  // the LRU list is in idle order
      due.push_back(cl);
    }
    if (!due.empty()) demote(c, due);
    while (!P.host_lru.empty()) {
      const auto [cl, gen] = P.host_lru.front();
      const Class& k = P.cls[cl];
      const bool held = k.alive && k.hbuf != kNone && k.slot == kNone && k.hgen == gen;
      if (held && now - k.idle_since < 3 * T) break;
      P.host_lru.pop_front();
      if (held) P.host_release(cl);
    }
  }
  for (auto& kv : c.modules) {
    Module& m = *kv.second;
    if (!m.mod || now - m.last_use < 2 * T) continue;
    bool live = false;
    for (auto& f : c.fns) live |= f.second->mod == &m && f.second->live > 0;
    if (!live) unload_module(c, m);
  }
}

}  // namespace sage
