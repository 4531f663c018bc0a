// Data preparation: the staging ring, the chunked fingerprint + dedup commit
// of fn_register, private copies (share=0), reloads of evicted classes and
// the per-function block tables.
#include <dlfcn.h>

#include <algorithm>
#include <cstring>
#include <unordered_set>

#include "internal.h"

namespace sage {

// ----------------------------------------------------------------- ring
void ring_init(Ctx& c) {
  Ring& R = c.ring;
  R.slots = c.cfg.ring_slots;
  R.chunk = c.cfg.chunk_bytes;
  const size_t nblk = R.chunk / kBlock;
  R.ops_cap = nblk;
  R.cap.assign(R.slots, nblk);
  for (size_t i = 0; i < R.slots; i++) {
    uint8_t *h = nullptr, *d = nullptr;
    uint64_t *dfp = nullptr, *hfp = nullptr;
    BlkOp *dops = nullptr, *hops = nullptr;
    uint32_t *dres = nullptr, *hres = nullptr;
    hipEvent_t ev, ev_c;
    HIPX(hipHostMalloc((void**)&h, R.chunk, hipHostMallocDefault));
    HIPX(hipMalloc((void**)&d, R.chunk));
    HIPX(hipMalloc((void**)&dfp, nblk * 8));
    HIPX(hipHostMalloc((void**)&hfp, nblk * 8, hipHostMallocDefault));
    HIPX(hipMalloc((void**)&dops, nblk * sizeof(BlkOp)));
    HIPX(hipHostMalloc((void**)&hops, nblk * sizeof(BlkOp), hipHostMallocDefault));
    HIPX(hipMalloc((void**)&dres, nblk * 4));
    HIPX(hipHostMalloc((void**)&hres, nblk * 4, hipHostMallocDefault));
    HIPX(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&ev_c, hipEventDisableTiming));
    R.host.push_back(h);
    R.dev.push_back(d);
    R.dfp.push_back(dfp);
    R.hfp.push_back(hfp);
    R.dops.push_back(dops);
    R.hops.push_back(hops);
    R.dres.push_back(dres);
    R.hres.push_back(hres);
    R.ev.push_back(ev);
    R.ev_c.push_back(ev_c);
    R.dops_c.push_back(nullptr);
    R.hops_c.push_back(nullptr);
    R.dres_c.push_back(nullptr);
    HIPX(hipMalloc((void**)&R.dops_c.back(), nblk * sizeof(BlkOp)));
    HIPX(hipHostMalloc((void**)&R.hops_c.back(), nblk * sizeof(BlkOp), hipHostMallocDefault));
    HIPX(hipMalloc((void**)&R.dres_c.back(), nblk * 4));
  }
}

void ring_destroy(Ctx& c) {
  Ring& R = c.ring;
  for (size_t i = 0; i < R.host.size(); i++) {
    (void)hipHostFree(R.host[i]);
    (void)hipFree(R.dev[i]);
    (void)hipFree(R.dfp[i]);
    (void)hipHostFree(R.hfp[i]);
    (void)hipFree(R.dops[i]);
    (void)hipHostFree(R.hops[i]);
    (void)hipFree(R.dres[i]);
    (void)hipHostFree(R.hres[i]);
    (void)hipEventDestroy(R.ev[i]);
    (void)hipEventDestroy(R.ev_c[i]);
    (void)hipFree(R.dops_c[i]);
    (void)hipHostFree(R.hops_c[i]);
    (void)hipFree(R.dres_c[i]);
  }
  R = Ring{};
}

// Grow the per-slot fingerprint / operation / result buffers of `slot` to
// hold `nblk` blocks (device-resident sources are fingerprinted whole).
static void ring_reserve(Ctx& c, int slot, size_t nblk) {
  Ring& R = c.ring;
  if (R.cap[slot] >= nblk) return;
  HIPX(hipEventSynchronize(R.ev_c[slot]));  // an in-flight COPY may still read the old op buffers
  (void)hipFree(R.dops_c[slot]);
  (void)hipHostFree(R.hops_c[slot]);
  (void)hipFree(R.dres_c[slot]);
  R.dops_c[slot] = R.hops_c[slot] = nullptr;
  R.dres_c[slot] = nullptr;
  (void)hipFree(R.dfp[slot]);
  (void)hipHostFree(R.hfp[slot]);
  (void)hipFree(R.dops[slot]);
  (void)hipHostFree(R.hops[slot]);
  (void)hipFree(R.dres[slot]);
  (void)hipHostFree(R.hres[slot]);
  R.dfp[slot] = R.hfp[slot] = nullptr;
  R.dops[slot] = R.hops[slot] = nullptr;
  R.dres[slot] = R.hres[slot] = nullptr;
  R.cap[slot] = 0;
  HIPX(hipMalloc((void**)&R.dfp[slot], nblk * 8));
  HIPX(hipHostMalloc((void**)&R.hfp[slot], nblk * 8, hipHostMallocDefault));
  HIPX(hipMalloc((void**)&R.dops[slot], nblk * sizeof(BlkOp)));
  HIPX(hipHostMalloc((void**)&R.hops[slot], nblk * sizeof(BlkOp), hipHostMallocDefault));
  HIPX(hipMalloc((void**)&R.dres[slot], nblk * 4));
  HIPX(hipHostMalloc((void**)&R.hres[slot], nblk * 4, hipHostMallocDefault));
  HIPX(hipMalloc((void**)&R.dops_c[slot], nblk * sizeof(BlkOp)));
  HIPX(hipHostMalloc((void**)&R.hops_c[slot], nblk * sizeof(BlkOp), hipHostMallocDefault));
  HIPX(hipMalloc((void**)&R.dres_c[slot], nblk * 4));
  R.cap[slot] = nblk;
}

// Host copy of a pageable source into pinned staging, split over threads.
void fill_parallel(Ctx& c, uint8_t* dst, const uint8_t* src, size_t n) {
  const size_t nt = std::max<uint32_t>(1, c.cfg.fill_threads);
  if (nt == 1 || n < (1u << 20)) {
    std::memcpy(dst, src, n);
    return;
  }
  const size_t part = (n / nt + 4095) & ~size_t(4095);
  std::vector<std::thread> th;
  for (size_t i = 1; i < nt; i++) {
    const size_t o = i * part;
    if (o >= n) break;
    th.emplace_back([=] { std::memcpy(dst + o, src + o, std::min(part, n - o)); });
  }
  std::memcpy(dst, src, std::min(part, n));
  for (auto& t : th) t.join();
}

// --------------------------------------------------------------- modules
static std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&lib_dir, &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    const size_t k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k);
  }
  return ".";
}

hipFunction_t Module::get(const char* name) {
  auto it = fn.find(name);
  if (it != fn.end()) return it->second;
  if (!mod) fail(SAGE_ESTATE, "code object %s is not loaded", path.c_str());
  hipFunction_t f = nullptr;
  const hipError_t e = hipModuleGetFunction(&f, mod, name);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(SAGE_EIO, "kernel %s not found in code object", name);
  }
  fn[name] = f;
  return f;
}

// The code of a kind is loaded once per context and shared by all its
// functions and invocations (section "Context Memory Sharing").
Module* load_module(Ctx& c, int kind) {
  std::lock_guard<std::mutex> lk(c.module_mu);
  const int key = is_grid(kind) ? SAGE_STENCIL7_F32 : SAGE_MLP_BF16;
  std::unique_ptr<Module>& slot = c.modules[key];
  if (!slot) {
    slot = std::make_unique<Module>();
    slot->key = key;
    slot->path = lib_dir() + (key == SAGE_STENCIL7_F32 ? "/sage_stencil.hsaco" : "/sage_mlp.hsaco");
  }
  Module* m = slot.get();
  if (m->mod) return m;
  const double t0 = now_ms();
  HIPX(hipSetDevice(c.device));
  const hipError_t e = hipModuleLoad(&m->mod, m->path.c_str());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    m->mod = nullptr;
    fail(SAGE_EIO, "hipModuleLoad(%s): %s", m->path.c_str(), hipGetErrorString(e));
  }
  if (key == SAGE_STENCIL7_F32) {
    m->get("stencil7_sweep2");
  } else {
    m->get("mlp_f32_layer");
    m->get("ggemm_bf16_128x128");
  }
  m->last_use = now_ms();
  c.module_loads++;
  c.t_module += now_ms() - t0;
  return m;
}

// --------------------------------------------------------------- blocks
uint32_t Fn::block_len(uint32_t b) const {
  size_t i = std::upper_bound(blob_first.begin(), blob_first.end(), b) - blob_first.begin() - 1;
  const uint64_t off = (uint64_t)(b - blob_first[i]) * kBlock;
  return (uint32_t)std::min<uint64_t>(kBlock, srcs[i].n - off);
}

const uint8_t* Fn::block_src(uint32_t b, bool* dev) const {
  size_t i = std::upper_bound(blob_first.begin(), blob_first.end(), b) - blob_first.begin() - 1;
  *dev = srcs[i].dev;
  return srcs[i].p + (uint64_t)(b - blob_first[i]) * kBlock;
}

// ------------------------------------------------------- register (shared)
namespace {
struct Chunk {
  uint32_t blob;
  uint64_t off, bytes;
  uint32_t first, nblk;
  int slot;
  const uint8_t* data;  // device address of the chunk's bytes
};
}  // namespace

// The data branch of fn_register with sharing on.  Chunks stream through
// the ring: H2D (or the device source in place) -> fingerprints -> D2H, up
// to `ring_slots` chunks ahead, while the host commits earlier chunks in
// order: each block either joins the first indexed class with the same
// fingerprint whose bytes verify equal, or becomes a new class copied into
// a fresh slot.  Fingerprints are only an index; equality is decided by
// the VERIFY kernel, so a collision costs a slot, never a wrong byte.
//
// Pool writes are ordered on the control stream: a chunk's VERIFY launch
// runs there and is waited for; its COPY launch follows and is left in
// flight, overlapping the next chunk's (or registration's) host work.
// Everything that reads pool slots later is ordered behind it: VERIFYs and
// reloads on the same stream, bodies through the function's ready event
// (recorded on the control stream), a ring slot's next fill through the
// slot's copy event.
void register_shared(Ctx& c, Fn& f) {
  Pool& P = c.pool;
  Ring& R = c.ring;
  std::vector<Chunk> chunks;
  for (uint32_t b = 0; b < f.srcs.size(); b++) {
    // device sources need no staging: fingerprint and commit them whole
    const uint64_t step = f.srcs[b].dev ? std::max<uint64_t>(f.srcs[b].n, 1) : R.chunk;
    for (uint64_t off = 0; off < f.srcs[b].n; off += step) {
      Chunk ch{};
      ch.blob = b;
      ch.off = off;
      ch.bytes = std::min<uint64_t>(step, f.srcs[b].n - off);
      ch.first = f.blob_first[b] + (uint32_t)(off / kBlock);
      ch.nblk = (uint32_t)((ch.bytes + kBlock - 1) / kBlock);
      ch.slot = -1;
      chunks.push_back(ch);
    }
  }
  f.cls.assign(f.n_blocks, kNone);
  f.fps.assign(f.n_blocks, 0);
  std::vector<uint32_t> created;
  // classes this registration joined, created or is verifying against are
  // stamped and never chosen as eviction victims while it runs
  const uint32_t mark = P.new_mark();
  auto protect = [&](uint32_t cl) { return P.cls[cl].mark == mark; };
  std::vector<int> free_slots;
  for (int s = (int)R.slots; s-- > 0;) free_slots.push_back(s);

  auto stream_of = [&](int slot) { return c.streams[slot % c.streams.size()]; };

  auto issue = [&](Chunk& ch) {
    ch.slot = free_slots.back();
    free_slots.pop_back();
    ring_reserve(c, ch.slot, ch.nblk);
    hipStream_t s = stream_of(ch.slot);
    const Src& src = f.srcs[ch.blob];
    if (src.dev) {
      ch.data = src.p + ch.off;
    } else {
      HIPX(hipStreamWaitEvent(s, R.ev_c[ch.slot], 0));  // the slot's last COPY has read its data
      const uint8_t* hsrc = src.p + ch.off;
      if (!src.pinned) {
        fill_parallel(c, R.host[ch.slot], hsrc, ch.bytes);
        hsrc = R.host[ch.slot];
      }
      HIPX(hipMemcpyAsync(R.dev[ch.slot], hsrc, ch.bytes, hipMemcpyHostToDevice, s));
      ch.data = R.dev[ch.slot];
    }
    const int tok = c.timer.start("fp64k", s, 1);
    HIPX(launch_fp64k(ch.data, ch.bytes, R.dfp[ch.slot], c.max_groups_stream(), s));
    c.timer.stop(tok, s);
    HIPX(hipMemcpyAsync(R.hfp[ch.slot], R.dfp[ch.slot], ch.nblk * 8, hipMemcpyDeviceToHost, s));
    HIPX(hipEventRecord(R.ev[ch.slot], s));
  };

  auto process = [&](Chunk& ch) {
    const int slot = ch.slot;
    hipStream_t s = c.ctl;
    double t0 = now_ms();
    HIPX(hipEventSynchronize(R.ev[slot]));
    HIPX(hipEventSynchronize(R.ev_c[slot]));  // the slot's previous COPY has read its op buffer
    double t1 = now_ms();
    c.t_fp_wait += t1 - t0;
    BlkOp* ops = R.hops[slot];
    BlkOp* cops = R.hops_c[slot];
    uint32_t nops = 0, ncops = 0;
    struct Pend {
      uint32_t i, cand, op;
    };
    std::vector<Pend> pend;
    std::vector<uint32_t> chunk_new;
    auto ref_addr = [&](uint32_t cl) -> uint64_t {
      const Class& k = P.cls[cl];
      return (uint64_t)(k.pending ? k.pending : P.addr(k.slot));
    };
    auto make_new = [&](uint32_t i) {
      const uint32_t gb = ch.first + i, len = f.block_len(gb);
      const uint32_t slotid = P.alloc_slot(protect);
      if (slotid == kNone)
        fail(SAGE_ENOMEM, "pool full: no unreferenced block to evict (budget %llu slots)",
             (unsigned long long)P.budget);
      const uint32_t cl = P.new_class(f.fps[gb], len);
      P.cls[cl].slot = slotid;
      P.cls[cl].pending = ch.data + (uint64_t)i * kBlock;
      P.index_add(cl);
      created.push_back(cl);
      chunk_new.push_back(cl);
      P.cls[cl].mark = mark;
      f.cls[gb] = cl;
      cops[ncops++] = BlkOp{(uint64_t)(ch.data + (uint64_t)i * kBlock), (uint64_t)P.addr(slotid), len, 0};
    };
    // first candidate after `after` (or the first one) with the block's length
    auto next_cand = [&](uint64_t fp, uint32_t len, uint32_t after) -> uint32_t {
      uint32_t k = after == kNone ? P.chain_head(fp) : P.cls[after].next;
      for (; k != kNone; k = P.cls[k].next) {
        P.cls[k].mark = mark;
        if (P.cls[k].len == len) return k;
      }
      return kNone;
    };
    for (uint32_t i = 0; i < ch.nblk; i++) {
      const uint32_t gb = ch.first + i;
      const uint64_t fp = c.test_fp_const ? c.test_fp_value : R.hfp[slot][i];
      f.fps[gb] = fp;
      const uint32_t len = f.block_len(gb);
      const uint32_t cand = next_cand(fp, len, kNone);
      if (cand != kNone) {
        pend.push_back({i, cand, nops});
        ops[nops++] = BlkOp{(uint64_t)(ch.data + (uint64_t)i * kBlock), ref_addr(cand), len, 1};
      } else {
        make_new(i);
      }
    }
    while (nops > 0) {
      const double tv = now_ms();
      c.t_dedup += tv - t1;
      HIPX(hipMemcpyAsync(R.dops[slot], ops, nops * sizeof(BlkOp), hipMemcpyHostToDevice, s));
      const int tok = c.timer.start("blkcopy", s, 1);
      HIPX(launch_blkcopy(R.dops[slot], nops, R.dres[slot], c.max_groups_copy(), s));
      c.timer.stop(tok, s);
      HIPX(hipMemcpyAsync(R.hres[slot], R.dres[slot], nops * 4, hipMemcpyDeviceToHost, s));
      HIPX(hipEventRecord(R.ev[slot], s));
      HIPX(hipEventSynchronize(R.ev[slot]));
      t1 = now_ms();
      c.t_verify += t1 - tv;
      std::vector<uint32_t> res(R.hres[slot], R.hres[slot] + nops);
      nops = 0;
      std::vector<Pend> again;
      for (const Pend& p : pend) {
        const uint32_t gb = ch.first + p.i;
        if (res[p.op] == 0) {
          f.cls[gb] = p.cand;
          continue;
        }
        c.mismatches++;
        const uint32_t nxt = next_cand(f.fps[gb], f.block_len(gb), p.cand);
        if (nxt != kNone) {
          again.push_back({p.i, nxt, nops});
          ops[nops++] = BlkOp{(uint64_t)(ch.data + (uint64_t)p.i * kBlock), ref_addr(nxt), f.block_len(gb), 1};
        } else {
          make_new(p.i);
        }
      }
      pend.swap(again);
    }
    if (ncops > 0) {
      // new classes: copy into their slots, left in flight on the control stream
      HIPX(hipMemcpyAsync(R.dops_c[slot], cops, ncops * sizeof(BlkOp), hipMemcpyHostToDevice, s));
      const int tok = c.timer.start("blkcopy", s, 1);
      HIPX(launch_blkcopy(R.dops_c[slot], ncops, R.dres_c[slot], c.max_groups_copy(), s));
      c.timer.stop(tok, s);
      HIPX(hipEventRecord(R.ev_c[slot], s));
    }
    for (uint32_t cl : chunk_new) P.cls[cl].pending = nullptr;
    c.t_dedup += now_ms() - t1;
  };

  try {
    std::deque<size_t> inflight;
    size_t next = 0;
    while (next < chunks.size() || !inflight.empty()) {
      while (next < chunks.size() && !free_slots.empty()) {
        issue(chunks[next]);
        inflight.push_back(next++);
      }
      Chunk& ch = chunks[inflight.front()];
      inflight.pop_front();
      process(ch);
      free_slots.push_back(ch.slot);
    }
  } catch (...) {
    for (hipStream_t s : c.streams) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(c.ctl);
    for (uint32_t cl : created) P.drop_class(cl);
    throw;
  }
  for (uint32_t cl : f.cls) P.cls[cl].members++;
  // distinct classes in creation order (the order ties are broken in)
  const uint32_t dmark = P.new_mark();
  f.distinct.clear();
  for (uint32_t cl : f.cls)
    if (P.cls[cl].mark != dmark) {
      P.cls[cl].mark = dmark;
      f.distinct.push_back(cl);
    }
  P.sort_by_seq(f.distinct);
  const double now = now_ms();
  for (uint32_t cl : f.distinct)
    if (P.cls[cl].active == 0) P.lru_back(cl, now);
  c.h2d += f.ro_bytes;
}

// ------------------------------------------------------ private copies
// share=0: the whole read-only data goes to `dst` (blob i at its first
// block), through the same staging ring for pageable host sources.
void copy_private(Ctx& c, Fn& f, uint8_t* dst, hipStream_t s) {
  Ring& R = c.ring;
  size_t k = 0;
  for (size_t b = 0; b < f.srcs.size(); b++) {
    const Src& src = f.srcs[b];
    uint8_t* d = dst + (uint64_t)f.blob_first[b] * kBlock;
    if (src.dev) {
      HIPX(hipMemcpyAsync(d, src.p, src.n, hipMemcpyDeviceToDevice, s));
    } else if (src.pinned) {
      for (uint64_t off = 0; off < src.n; off += R.chunk, k++) {
        hipStream_t cs = c.streams[k % c.streams.size()];
        HIPX(hipMemcpyAsync(d + off, src.p + off, std::min<uint64_t>(R.chunk, src.n - off),
                            hipMemcpyHostToDevice, cs));
      }
    } else {
      for (uint64_t off = 0; off < src.n; off += R.chunk, k++) {
        const int slot = (int)(k % R.slots);
        hipStream_t cs = c.streams[slot % c.streams.size()];
        if (k >= R.slots) HIPX(hipEventSynchronize(R.ev[slot]));  // slot's previous copy done
        const uint64_t n = std::min<uint64_t>(R.chunk, src.n - off);
        fill_parallel(c, R.host[slot], src.p + off, n);
        HIPX(hipMemcpyAsync(d + off, R.host[slot], n, hipMemcpyHostToDevice, cs));
        HIPX(hipEventRecord(R.ev[slot], cs));
      }
    }
  }
  for (hipStream_t cs : c.streams) HIPX(hipStreamSynchronize(cs));
  c.h2d += f.ro_bytes;
}

// ------------------------------------------------------------ reloads
// Bring evicted classes of `f` back: a demoted class from its host-cache
// copy, any other from the source block of `f` that first referenced it (the
// source is read-only and was verified equal at registration).  Pinned host
// bytes reach the device staging buffer in one DMA per contiguous run.
void reload_classes(Ctx& c, Fn& f, const std::vector<uint32_t>& missing) {
  if (missing.empty()) return;
  const double t_start = now_ms();
  Pool& P = c.pool;
  Ring& R = c.ring;
  std::unordered_map<uint32_t, uint32_t> first;
  for (uint32_t b = 0; b < f.n_blocks; b++) first.emplace(f.cls[b], b);
  const uint32_t mark = P.new_mark();
  for (uint32_t cl : f.distinct) P.cls[cl].mark = mark;
  auto protect = [&](uint32_t cl) { return P.cls[cl].mark == mark; };
  // Batches go round the staging ring on the copy streams, so staging of one
  // overlaps the copies of the others.  Every stream first waits for the
  // control stream: a freed slot may still be the target of a registration
  // copy in flight there.
  HIPX(hipEventRecord(c.ctl_ev, c.ctl));
  for (size_t k = 0; k < R.slots; k++) HIPX(hipEventSynchronize(R.ev_c[k]));
  for (hipStream_t cs : c.streams) HIPX(hipStreamWaitEvent(cs, c.ctl_ev, 0));
  size_t i = 0, batch = 0;
  std::vector<uint32_t> from_host;
  while (i < missing.size()) {
    const int slot = (int)(batch % R.slots);
    hipStream_t s = c.streams[slot % c.streams.size()];
    if (batch >= R.slots) HIPX(hipEventSynchronize(R.ev[slot]));  // the slot's previous batch is done
    batch++;
    const size_t per_slot = std::min<size_t>(R.chunk / kBlock, R.cap[slot]);
    BlkOp* ops = R.hops[slot];
    uint32_t nops = 0;
    size_t staged = 0;
    // runs of contiguous pinned host blocks reach the staging buffer in one DMA each
    const uint8_t* run_src = nullptr;
    size_t run_at = 0, run_n = 0;
    auto flush_run = [&] {
      if (run_n)
        HIPX(hipMemcpyAsync(R.dev[slot] + run_at * kBlock, run_src, run_n * kBlock, hipMemcpyHostToDevice, s));
      run_n = 0;
    };
    while (i < missing.size() && nops < per_slot) {
      const uint32_t cl = missing[i++];
      Class& k = P.cls[cl];
      const uint32_t len = k.len;
      const uint32_t slotid = P.alloc_slot(protect);
      if (slotid == kNone) fail(SAGE_ENOMEM, "pool full during reload");
      k.slot = slotid;
      P.index_add(cl);
      bool dev = false;
      const uint8_t* hsrc = nullptr;  // pinned host bytes to stage, if any
      if (k.hbuf != kNone) {
        // the bytes wait in the pinned host cache (second or third stage)
        hsrc = P.hbufs[k.hbuf].p + (uint64_t)k.hoff * kBlock;
        from_host.push_back(cl);
        c.host_reloads++;
      } else {
        const uint8_t* src = f.block_src(first.at(cl), &dev);
        if (dev) {
          ops[nops++] = BlkOp{(uint64_t)src, (uint64_t)P.addr(slotid), len, 0};
        } else {
          std::memcpy(R.host[slot] + staged * kBlock, src, len);
          hsrc = R.host[slot] + staged * kBlock;
        }
      }
      if (hsrc) {
        if (!(run_n && hsrc == run_src + run_n * kBlock)) {
          flush_run();
          run_src = hsrc;
          run_at = staged;
        }
        run_n++;
        ops[nops++] = BlkOp{(uint64_t)(R.dev[slot] + staged * kBlock), (uint64_t)P.addr(slotid), len, 0};
        staged++;
      }
      c.h2d += len;
      c.reloads++;
    }
    flush_run();
    HIPX(hipMemcpyAsync(R.dops[slot], ops, nops * sizeof(BlkOp), hipMemcpyHostToDevice, s));
    const int tok = c.timer.start("blkcopy", s, 1);
    HIPX(launch_blkcopy(R.dops[slot], nops, R.dres[slot], c.max_groups_copy(), s));
    c.timer.stop(tok, s);
    HIPX(hipEventRecord(R.ev[slot], s));
  }
  for (hipStream_t cs : c.streams) HIPX(hipStreamSynchronize(cs));
  for (uint32_t cl : from_host) P.host_release(cl);  // back in HBM: the host copy goes
  c.t_reload += now_ms() - t_start;
}

// Rebuild the device block table of `f` when any of its classes moved.
void refresh_table(Ctx& c, Fn& f) {
  if (f.table_epoch == c.pool.epoch && !f.h_table.empty()) return;
  std::vector<uint64_t> t(f.n_blocks);
  for (uint32_t b = 0; b < f.n_blocks; b++) t[b] = (uint64_t)c.pool.addr(c.pool.cls[f.cls[b]].slot);
  if (t != f.h_table) {
    HIPX(hipEventSynchronize(c.stage_ev));  // the previous upload has read the staging buffer
    if (c.h_stage_cap < t.size()) {
      if (c.h_stage) HIPX(hipHostFree(c.h_stage));
      c.h_stage = nullptr;
      c.h_stage_cap = 0;
      HIPX(hipHostMalloc((void**)&c.h_stage, std::max<size_t>(t.size(), 65536) * 8, hipHostMallocDefault));
      c.h_stage_cap = std::max<size_t>(t.size(), 65536);
    }
    std::memcpy(c.h_stage, t.data(), t.size() * 8);
    HIPX(hipMemcpyAsync(f.d_table, c.h_stage, t.size() * 8, hipMemcpyHostToDevice, c.ctl));
    HIPX(hipEventRecord(c.stage_ev, c.ctl));
    HIPX(hipEventRecord(f.ready, c.ctl));  // bodies of f wait for the new table
    f.h_table.swap(t);
  }
  f.table_epoch = c.pool.epoch;
}

}  // namespace sage
