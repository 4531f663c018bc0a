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
  R.held.assign(R.slots, 0);
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
  HIPX(hipEventSynchronize(R.ev[slot]));
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

// Host copy of a pageable source into pinned staging, over the copy threads.
void fill_parallel(Ctx& c, uint8_t* dst, const uint8_t* src, size_t n) { copy_parallel(c, {HostCopy{dst, src, n}}); }

// Many host copies (a pageable source into staging, a batched launch's host
// inputs into pinned staging or its outputs out of it), cut into pieces of
// at most 1 MiB that the context's copy threads and the caller take round
// robin.  Below 1 MiB in all, the caller copies alone.
void copy_parallel(Ctx& c, const std::vector<HostCopy>& items) {
  size_t total = 0;
  for (const HostCopy& it : items) total += it.n;
  if (total < (1u << 20)) {
    for (const HostCopy& it : items) std::memcpy(it.dst, it.src, it.n);
    return;
  }
  constexpr size_t kPiece = 1u << 20;
  std::vector<HostCopy> pieces;
  pieces.reserve(total / kPiece + items.size());
  for (const HostCopy& it : items)
    for (size_t o = 0; o < it.n; o += kPiece) pieces.push_back({it.dst + o, it.src + o, std::min(kPiece, it.n - o)});
  c.copier.run(pieces);
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

const uint8_t* Fn::block_src(uint32_t b, bool* dev, bool* pinned) const {
  size_t i = std::upper_bound(blob_first.begin(), blob_first.end(), b) - blob_first.begin() - 1;
  *dev = srcs[i].dev;
  if (pinned) *pinned = srcs[i].pinned;
  return srcs[i].p + (uint64_t)(b - blob_first[i]) * kBlock;
}

// ------------------------------------------------------- register (shared)
using Chunk = RegChunk;

// The chunks of a registration: device sources in chunks of up to
// `dev_chunk` bytes (fingerprinted in place; their VERIFY / COPY work waits
// for the whole registration), host sources in ring-slot chunks.
static std::vector<Chunk> make_chunks(const Ctx& c, const Fn& f) {
  std::vector<Chunk> chunks;
  for (uint32_t b = 0; b < f.srcs.size(); b++) {
    const uint64_t step = f.srcs[b].dev ? std::max<uint64_t>(std::min<uint64_t>(f.srcs[b].n, c.dev_chunk), 1)
                                        : c.ring.chunk;
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
  return chunks;
}

// Fingerprints of a device-source chunk into ring slot `slot`, in place, on
// the control stream: one after another and after the previous
// registration's COPY, so the HBM-bound kernels run one at a time at full
// bandwidth instead of sharing it.
static void issue_dev_chunk(Ctx& c, const Fn& f, Chunk& ch, int slot) {
  Ring& R = c.ring;
  ch.slot = slot;
  HIPX(hipEventSynchronize(R.ev[slot]));  // e.g. a progressive reload still reading the slot
  ring_reserve(c, slot, ch.nblk);
  ch.data = f.srcs[ch.blob].p + ch.off;
  hipStream_t s = c.ctl;
  const int tok = c.timer.start("fp64k", s, 1);
  HIPX(launch_fp64k(ch.data, ch.bytes, R.dfp[slot], c.max_groups_stream(), s));
  c.timer.stop(tok, s);
  HIPX(hipMemcpyAsync(R.hfp[slot], R.dfp[slot], ch.nblk * 8, hipMemcpyDeviceToHost, s));
  HIPX(hipEventRecord(R.ev[slot], s));
}

bool register_prefetch(Ctx& c, Fn& f) {
  Ring& R = c.ring;
  if (!c.cfg.share || f.srcs.empty() || !f.pre.empty()) return false;
  for (const Src& sr : f.srcs)
    if (!sr.dev) return false;
  std::vector<Chunk> chunks = make_chunks(c, f);
  std::vector<int> avail;
  for (int s = (int)R.slots; s-- > 0;)
    if (!R.held[s]) avail.push_back(s);
  // one slot stays free for the registration that runs meanwhile
  if (chunks.empty() || chunks.size() + 1 > avail.size()) return false;
  try {
    for (Chunk& ch : chunks) {
      const int slot = avail.back();
      avail.pop_back();
      R.held[slot] = 1;
      issue_dev_chunk(c, f, ch, slot);
    }
  } catch (...) {
    (void)hipStreamSynchronize(c.ctl);
    for (const Chunk& ch : chunks)
      if (ch.slot >= 0) R.held[ch.slot] = 0;
    throw;
  }
  f.pre = std::move(chunks);
  return true;
}

void register_drop_prefetch(Ctx& c, Fn& f) {
  if (f.pre.empty()) return;
  (void)hipStreamSynchronize(c.ctl);  // the fingerprints write the slots' buffers
  for (const Chunk& ch : f.pre) c.ring.held[ch.slot] = 0;
  f.pre.clear();
}

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
  // chunks fingerprinted ahead (register_prefetch) are already in flight,
  // each in the slot it holds
  const size_t n_pre = f.pre.size();
  std::vector<Chunk> chunks = n_pre ? std::move(f.pre) : make_chunks(c, f);
  f.pre.clear();
  f.cls.assign(f.n_blocks, kNone);
  f.fps.assign(f.n_blocks, 0);
  std::vector<uint32_t> created;
  // classes this registration joined, created or is verifying against are
  // stamped and never chosen as eviction victims while it runs
  const uint32_t mark = P.new_mark();
  auto protect = [&](uint32_t cl) { return P.cls[cl].mark == mark; };
  std::vector<int> free_slots;  // not held by a chunk fingerprinted ahead (this function's or the next one's)
  for (int s = (int)R.slots; s-- > 0;)
    if (!R.held[s]) free_slots.push_back(s);

  auto stream_of = [&](int slot) { return c.streams[slot % c.streams.size()]; };

  // bytes a VERIFY compares against: the first block of a class still being
  // copied (its source), else its pool slot
  auto ref_addr = [&](uint32_t cl) -> uint64_t {
    const Class& k = P.cls[cl];
    return (uint64_t)(k.pending ? k.pending : P.addr(k.slot));
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
  // a new class for block gb whose bytes are at `data`, in a fresh slot
  auto new_class_for = [&](uint32_t gb, const uint8_t* data) -> uint32_t {
    const uint32_t slotid = P.alloc_slot(protect);
    if (slotid == kNone)
      fail(SAGE_ENOMEM, "pool full: no unreferenced block to evict (budget %llu slots)", (unsigned long long)P.budget);
    const uint32_t cl = P.new_class(f.fps[gb], f.block_len(gb));
    P.cls[cl].slot = slotid;
    P.cls[cl].pending = data;
    P.index_add(cl);
    created.push_back(cl);
    P.cls[cl].mark = mark;
    f.cls[gb] = cl;
    return cl;
  };
  // device-source chunks: VERIFY and COPY operations gathered over the whole
  // registration and run once at its end (one device round trip instead of
  // one per chunk); the classes they create keep their source as `pending`
  struct DPend {
    uint32_t gb, cand, op;
    const uint8_t* data;
  };
  std::vector<BlkOp> dv, dc;
  std::vector<DPend> dpend;
  std::vector<uint32_t> dnew;
  bool any_dev = false;
  for (const Src& sr : f.srcs) any_dev |= sr.dev;
  if (any_dev) {
    dv.reserve(f.n_blocks);
    dc.reserve(f.n_blocks);
    dpend.reserve(f.n_blocks);
  }

  auto issue = [&](Chunk& ch) {
    const int slot = free_slots.back();
    free_slots.pop_back();
    const Src& src = f.srcs[ch.blob];
    if (src.dev) {
      issue_dev_chunk(c, f, ch, slot);
      return;
    }
    ch.slot = slot;
    HIPX(hipEventSynchronize(R.ev[ch.slot]));  // e.g. a progressive reload still reading the slot
    ring_reserve(c, ch.slot, ch.nblk);
    // staged chunks keep their slot's stream for the host-to-device copies
    hipStream_t s = stream_of(ch.slot);
    HIPX(hipStreamWaitEvent(s, R.ev_c[ch.slot], 0));  // the slot's last COPY has read its data
    const uint8_t* hsrc = src.p + ch.off;
    if (!src.pinned) {
      fill_parallel(c, R.host[ch.slot], hsrc, ch.bytes);
      hsrc = R.host[ch.slot];
    }
    HIPX(hipMemcpyAsync(R.dev[ch.slot], hsrc, ch.bytes, hipMemcpyHostToDevice, s));
    ch.data = R.dev[ch.slot];
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
    const bool deferred = f.srcs[ch.blob].dev;
    auto make_new = [&](uint32_t i) {
      const uint32_t gb = ch.first + i;
      const uint8_t* data = ch.data + (uint64_t)i * kBlock;
      const uint32_t cl = new_class_for(gb, data);
      const BlkOp op{(uint64_t)data, (uint64_t)P.addr(P.cls[cl].slot), f.block_len(gb), 0};
      if (deferred) {
        dc.push_back(op);
        dnew.push_back(cl);
      } else {
        cops[ncops++] = op;
        chunk_new.push_back(cl);
      }
    };
    for (uint32_t i = 0; i < ch.nblk; i++) {
      const uint32_t gb = ch.first + i;
      const uint64_t fp = c.test_fp_const ? c.test_fp_value : R.hfp[slot][i];
      f.fps[gb] = fp;
      const uint32_t len = f.block_len(gb);
      const uint32_t cand = next_cand(fp, len, kNone);
      const uint8_t* data = ch.data + (uint64_t)i * kBlock;
      if (cand != kNone && deferred) {
        f.cls[gb] = cand;  // until its VERIFY says otherwise
        dpend.push_back({gb, cand, (uint32_t)dv.size(), data});
        dv.push_back(BlkOp{(uint64_t)data, ref_addr(cand), len, 1});
      } else if (cand != kNone) {
        pend.push_back({i, cand, nops});
        ops[nops++] = BlkOp{(uint64_t)data, ref_addr(cand), len, 1};
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

  // Device-source chunks, at the end of the registration: every gathered
  // VERIFY and the COPY of the classes created so far go out at once (op
  // list up, VERIFY, its results down, COPY left in flight), and the
  // blocks are counted into their candidates' classes before the results
  // are back.  A failed VERIFY (a fingerprint collision) takes the counts
  // back, settles the blocks round by round as the staged chunks do, copies
  // the classes that split off and counts again.
  auto reg_reserve = [&](size_t need) {
    if (c.reg_cap >= need) return;
    HIPX(hipStreamSynchronize(c.ctl));
    if (c.reg_hops) HIPX(hipHostFree(c.reg_hops));
    if (c.reg_hres) HIPX(hipHostFree(c.reg_hres));
    if (c.reg_dops) HIPX(hipFree(c.reg_dops));
    if (c.reg_dres) HIPX(hipFree(c.reg_dres));
    c.reg_hops = c.reg_dops = nullptr;
    c.reg_hres = c.reg_dres = nullptr;
    c.reg_cap = 0;
    const size_t cap = std::max<size_t>(need, 4096);
    HIPX(hipHostMalloc((void**)&c.reg_hops, cap * sizeof(BlkOp), hipHostMallocDefault));
    HIPX(hipHostMalloc((void**)&c.reg_hres, cap * 4, hipHostMallocDefault));
    HIPX(hipMalloc((void**)&c.reg_dops, cap * sizeof(BlkOp)));
    HIPX(hipMalloc((void**)&c.reg_dres, cap * 4));
    c.reg_cap = cap;
  };
  hipStream_t ctl = c.ctl;
  auto launch_ops = [&](const BlkOp* dev_ops, uint32_t n, uint32_t* dev_res) {
    const int tok = c.timer.start("blkcopy", ctl, 1);
    HIPX(launch_blkcopy(dev_ops, n, dev_res, c.max_groups_copy(), ctl));
    c.timer.stop(tok, ctl);
  };
  auto start_deferred = [&] {
    if (dv.empty() && dc.empty()) return;
    HIPX(hipEventSynchronize(c.reg_ev));  // the previous registration's COPY has read the lists
    reg_reserve(dv.size() + dc.size());
    const uint32_t nv = (uint32_t)dv.size(), nc = (uint32_t)dc.size();
    std::memcpy(c.reg_hops, dv.data(), nv * sizeof(BlkOp));
    std::memcpy(c.reg_hops + nv, dc.data(), nc * sizeof(BlkOp));
    HIPX(hipMemcpyAsync(c.reg_dops, c.reg_hops, (size_t)(nv + nc) * sizeof(BlkOp), hipMemcpyHostToDevice, ctl));
    if (nv) {
      launch_ops(c.reg_dops, nv, c.reg_dres);
      HIPX(hipMemcpyAsync(c.reg_hres, c.reg_dres, nv * 4, hipMemcpyDeviceToHost, ctl));
      HIPX(hipEventRecord(c.reg_vev, ctl));
    }
    if (nc) launch_ops(c.reg_dops + nv, nc, c.reg_dres + nv);
    HIPX(hipEventRecord(c.reg_ev, ctl));
    dc.clear();
  };
  bool counted = false;
  auto count_in = [&] {
    for (uint32_t cl : f.cls) P.cls[cl].members++;
    counted = true;
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
  };
  auto finish_deferred = [&] {
    if (!dv.empty()) {
      const double tv = now_ms();
      HIPX(hipEventSynchronize(c.reg_vev));
      c.t_verify += now_ms() - tv;
      bool all_equal = true;
      for (size_t q = 0; q < dv.size() && all_equal; q++) all_equal = c.reg_hres[q] == 0;
      if (!all_equal) {
        for (uint32_t cl : f.cls) P.cls[cl].members--;
        counted = false;
        for (uint32_t cl : f.cls) P.cls[cl].mark = mark;  // protected again while classes split off
        bool first_round = true;
        while (!dv.empty()) {
          if (!first_round) {
            const double tr = now_ms();
            const uint32_t n = (uint32_t)dv.size();
            std::memcpy(c.reg_hops, dv.data(), n * sizeof(BlkOp));
            HIPX(hipMemcpyAsync(c.reg_dops, c.reg_hops, n * sizeof(BlkOp), hipMemcpyHostToDevice, ctl));
            launch_ops(c.reg_dops, n, c.reg_dres);
            HIPX(hipMemcpyAsync(c.reg_hres, c.reg_dres, n * 4, hipMemcpyDeviceToHost, ctl));
            HIPX(hipEventRecord(c.reg_vev, ctl));
            HIPX(hipEventSynchronize(c.reg_vev));
            c.t_verify += now_ms() - tr;
          }
          first_round = false;
          std::vector<BlkOp> dv2;
          std::vector<DPend> dp2;
          for (const DPend& q : dpend) {
            if (c.reg_hres[q.op] == 0) {
              f.cls[q.gb] = q.cand;
              continue;
            }
            c.mismatches++;
            const uint32_t len = f.block_len(q.gb);
            const uint32_t nxt = next_cand(f.fps[q.gb], len, q.cand);
            if (nxt != kNone) {
              f.cls[q.gb] = nxt;
              dp2.push_back({q.gb, nxt, (uint32_t)dv2.size(), q.data});
              dv2.push_back(BlkOp{(uint64_t)q.data, ref_addr(nxt), len, 1});
            } else {
              const uint32_t cl = new_class_for(q.gb, q.data);
              dc.push_back(BlkOp{(uint64_t)q.data, (uint64_t)P.addr(P.cls[cl].slot), len, 0});
              dnew.push_back(cl);
            }
          }
          dv.swap(dv2);
          dpend.swap(dp2);
        }
        if (!dc.empty()) {
          const uint32_t n = (uint32_t)dc.size();
          std::memcpy(c.reg_hops, dc.data(), n * sizeof(BlkOp));
          HIPX(hipMemcpyAsync(c.reg_dops, c.reg_hops, n * sizeof(BlkOp), hipMemcpyHostToDevice, ctl));
          launch_ops(c.reg_dops, n, c.reg_dres);
          HIPX(hipEventRecord(c.reg_ev, ctl));
        }
        count_in();
      }
    }
    for (uint32_t cl : dnew) P.cls[cl].pending = nullptr;  // their COPYs are ordered on the control stream
  };

  try {
    std::deque<size_t> inflight;
    size_t next = 0;
    for (; next < n_pre; next++) inflight.push_back(next);
    while (next < chunks.size() || !inflight.empty()) {
      while (next < chunks.size() && !free_slots.empty()) {
        issue(chunks[next]);
        inflight.push_back(next++);
      }
      const size_t i = inflight.front();
      inflight.pop_front();
      process(chunks[i]);
      if (i < n_pre) R.held[chunks[i].slot] = 0;
      free_slots.push_back(chunks[i].slot);
    }
    start_deferred();
    count_in();  // optimistic for the deferred VERIFYs: corrected above if one fails
    finish_deferred();
  } catch (...) {
    for (hipStream_t s : c.streams) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(c.ctl);
    for (size_t i = 0; i < n_pre; i++) R.held[chunks[i].slot] = 0;  // prefetched chunks not processed yet
    if (counted)
      for (uint32_t cl : f.cls) P.cls[cl].members--;
    for (uint32_t cl : created) P.drop_class(cl);
    throw;
  }
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
        HIPX(hipEventSynchronize(R.ev[slot]));  // slot's previous copy done
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
// source is read-only and was verified equal at registration).
//
// The classes go in the order of their first block in `f`, so for the MLP
// kinds layer l's weights are complete once every class first used at or
// before layer l's last block has landed.  Every class gets its slot, and the
// block table and one op list for the whole reload go out, before any copy.
// The copies are issued in batches of at most one chunk, never across a
// layer's end, round the copy streams.  Host bytes pass through a device
// staging area of kReloadStageBlocks blocks cut into one region per batch; a
// region is taken again once the batch that last used it (in this reload or
// an earlier one) has completed, so the host waits only when a reload is
// larger than the staging area.  Pinned bytes (the host cache) reach it in
// one DMA per contiguous run; pageable source bytes first go, one parallel
// memcpy per run, to the pinned buffer of a registration ring slot (taken
// once the slot's event has completed); device sources are copied in place.
//
// Progressive (cfg.progressive, MLP kinds, some bytes over the host link):
// at each layer's end the copy streams are joined into the control stream
// and f.seg[l] is recorded there, and the call returns without waiting;
// layer l's launch waits for f.seg[l] (the kernel executor's readiness
// check, per kernel).  Otherwise the call waits for the whole reload.  Either
// way f.ready and reload_done mark its end, and its op list and the
// host-cache copies that fed it are released once it has completed.
void reload_classes(Ctx& c, Fn& f, const std::vector<uint32_t>& missing_in) {
  if (missing_in.empty()) return;
  const double t_start = now_ms();
  Pool& P = c.pool;
  settle_reloads(c, false);
  std::unordered_map<uint32_t, uint32_t> first;
  for (uint32_t b = 0; b < f.n_blocks; b++) first.emplace(f.cls[b], b);
  std::vector<uint32_t> missing = missing_in;
  const size_t n = missing.size();
  std::stable_sort(missing.begin(), missing.end(),
                   [&](uint32_t a, uint32_t b) { return first.at(a) < first.at(b); });
  const bool mlp = !is_grid(f.d.kind) && f.d.layers > 0;
  const uint32_t n_seg = mlp ? f.d.layers : 1;
  std::vector<size_t> seg_end(n_seg, n);
  if (mlp) {
    std::vector<uint32_t> firsts(n);
    for (size_t j = 0; j < n; j++) firsts[j] = first.at(missing[j]);
    seg_end = layer_segments(firsts, n_seg, (uint64_t)f.d.width * f.d.width * (f.d.kind == SAGE_MLP_F32 ? 4 : 2));
  }
  const uint32_t mark = P.new_mark();
  for (uint32_t cl : f.distinct) P.cls[cl].mark = mark;
  auto protect = [&](uint32_t cl) { return P.cls[cl].mark == mark; };
  for (size_t j = 0; j < n; j++) {
    const uint32_t slotid = P.alloc_slot(protect);
    if (slotid == kNone) {
      for (size_t r = 0; r < j; r++) P.evict(missing[r]);
      fail(SAGE_ENOMEM, "pool full during reload");
    }
    P.cls[missing[j]].slot = slotid;
    P.index_add(missing[j]);
  }
  // from here on the classes hold slots their bytes have not reached: a
  // failure takes them out again, so that no later setup reads them
  try {
    // where each class comes from: 0 device source, 1 host cache (pinned,
    // whole blocks), 2 registered pageable host source (through pinned
    // staging), 3 registered pinned host source, a whole block (by DMA like
    // the host cache; a short last block takes the staged way)
    std::vector<uint8_t> kind(n);
    std::vector<const uint8_t*> src(n);
    size_t n_host = 0, n_page = 0;
    for (size_t j = 0; j < n; j++) {
      const Class& k = P.cls[missing[j]];
      bool dev = false, pinned = false;
      if (k.hbuf != kNone) {
        kind[j] = 1;
        src[j] = P.hbufs[k.hbuf].p + (uint64_t)k.hoff * kBlock;
      } else {
        src[j] = f.block_src(first.at(missing[j]), &dev, &pinned);
        kind[j] = dev ? 0 : pinned && k.len == kBlock ? 3 : 2;
      }
      n_host += kind[j] != 0;
      n_page += kind[j] == 2;
    }
    const bool gate = c.cfg.progressive && mlp && n_host > 0;
    // batches and their staging regions
    const size_t per_batch = std::min<size_t>(std::max<size_t>(1, c.ring.chunk / kBlock), kReloadStageBlocks);
    const size_t n_regions = kReloadStageBlocks / per_batch;
    if (n_host && !c.rstage_dev) HIPX(hipMalloc((void**)&c.rstage_dev, kReloadStageBlocks * kBlock));
    Ring& R = c.ring;
    while (c.rstage_ev.size() < n_regions) {
      hipEvent_t e;
      HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c.rstage_ev.push_back(e);
    }
    struct Batch {
      size_t j0, j1;
      uint32_t seg;
      int region;  // -1: no host bytes
    };
    std::vector<Batch> batches;
    std::vector<size_t> stage_at(n, 0);
    for (uint32_t l = 0, j = 0; l < n_seg; l++) {
      while (j < seg_end[l]) {
        Batch bt{j, std::min(seg_end[l], j + per_batch), l, -1};
        size_t h = 0;
        for (size_t q = bt.j0; q < bt.j1; q++)
          if (kind[q]) {
            if (bt.region < 0) bt.region = (int)(c.rstage_next++ % n_regions);
            stage_at[q] = (size_t)bt.region * per_batch + h++;
          }
        batches.push_back(bt);
        j = (uint32_t)bt.j1;
      }
    }
    // the op list: the previous reload's upload has read the pinned buffer
    HIPX(hipEventSynchronize(c.prog_ops_ev));
    if (c.prog_hops_cap < n * sizeof(BlkOp)) {
      if (c.prog_hops) HIPX(hipHostFree(c.prog_hops));
      c.prog_hops = nullptr;
      c.prog_hops_cap = 0;
      HIPX(hipHostMalloc((void**)&c.prog_hops, n * sizeof(BlkOp), hipHostMallocDefault));
      c.prog_hops_cap = n * sizeof(BlkOp);
    }
    uint8_t* dmeta = (uint8_t*)c.cache.get(n * (sizeof(BlkOp) + 4));
    c.deferred_dev.push_back(dmeta);
    BlkOp* dops = reinterpret_cast<BlkOp*>(dmeta);
    uint32_t* dres = reinterpret_cast<uint32_t*>(dmeta + n * sizeof(BlkOp));
    BlkOp* hops = reinterpret_cast<BlkOp*>(c.prog_hops);
    for (size_t j = 0; j < n; j++) {
      const Class& k = P.cls[missing[j]];
      const uint64_t from = kind[j] ? (uint64_t)(c.rstage_dev + stage_at[j] * kBlock) : (uint64_t)src[j];
      hops[j] = BlkOp{from, (uint64_t)P.addr(k.slot), k.len, 0};
      c.h2d += k.len;
      c.reloads++;
      if (kind[j] == 1) c.host_reloads++;
    }
    // control stream: op list, block table, then the mark the copy streams start
    // behind (a freed slot may still be the target of a copy in flight there)
    HIPX(hipMemcpyAsync(dops, hops, n * sizeof(BlkOp), hipMemcpyHostToDevice, c.ctl));
    HIPX(hipEventRecord(c.prog_ops_ev, c.ctl));
    refresh_table(c, f);
    HIPX(hipEventRecord(c.ctl_ev, c.ctl));
    for (hipStream_t cs : c.streams) HIPX(hipStreamWaitEvent(cs, c.ctl_ev, 0));
    while (gate && f.seg.size() < f.d.layers) {
      hipEvent_t e;
      HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      f.seg.push_back(e);
    }
    std::vector<bool> dirty(c.streams.size(), false);
    auto join = [&] {  // the control stream waits for the copy streams used since the last join
      for (size_t k = 0; k < c.streams.size(); k++) {
        if (!dirty[k]) continue;
        HIPX(hipEventRecord(c.join_ev[k], c.streams[k]));
        HIPX(hipStreamWaitEvent(c.ctl, c.join_ev[k], 0));
        dirty[k] = false;
      }
    };
    size_t bi = 0;
    for (uint32_t l = 0; l < n_seg; l++) {
      for (; bi < batches.size() && batches[bi].seg == l; bi++) {
        const Batch& bt = batches[bi];
        const size_t si = bi % c.streams.size();
        hipStream_t s = c.streams[si];
        if (bt.region >= 0) {
          HIPX(hipEventSynchronize(c.rstage_ev[bt.region]));  // its last batch has read the region
          // pageable source runs into a ring slot's pinned buffer, one parallel memcpy each
          int hs = -1;
          size_t hn = 0;
          std::vector<const uint8_t*> pinned_at(bt.j1 - bt.j0, nullptr);
          uint8_t* cp_to = nullptr;
          const uint8_t* cp_from = nullptr;
          size_t cp_n = 0;
          for (size_t q = bt.j0; q < bt.j1; q++) {
            if (kind[q] != 2) continue;
            if (hs < 0) {
              hs = (int)(c.rhost_next++ % R.slots);
              HIPX(hipEventSynchronize(R.ev[hs]));  // the slot's last user has read its buffer
            }
            uint8_t* to = R.host[hs] + hn++ * kBlock;
            pinned_at[q - bt.j0] = to;
            if (!(cp_n && cp_n % kBlock == 0 && to == cp_to + cp_n && src[q] == cp_from + cp_n)) {
              if (cp_n) fill_parallel(c, cp_to, cp_from, cp_n);
              cp_to = to;
              cp_from = src[q];
              cp_n = 0;
            }
            cp_n += P.cls[missing[q]].len;
          }
          if (cp_n) fill_parallel(c, cp_to, cp_from, cp_n);
          // pinned bytes to the device staging, one DMA per run contiguous on both sides
          const uint8_t* run_src = nullptr;
          size_t run_at = 0, run_n = 0;
          auto flush = [&] {
            if (run_n)
              HIPX(hipMemcpyAsync(c.rstage_dev + run_at * kBlock, run_src, run_n * kBlock, hipMemcpyHostToDevice,
                                  s));
            run_n = 0;
          };
          for (size_t q = bt.j0; q < bt.j1; q++) {
            if (!kind[q]) continue;
            const uint8_t* from = kind[q] == 2 ? pinned_at[q - bt.j0] : src[q];
            if (!(run_n && from == run_src + run_n * kBlock && stage_at[q] == run_at + run_n)) {
              flush();
              run_src = from;
              run_at = stage_at[q];
            }
            run_n++;
          }
          flush();
          if (hs >= 0) HIPX(hipEventRecord(R.ev[hs], s));
        }
        const int tok = c.timer.start("blkcopy", s, 1);
        HIPX(launch_blkcopy(dops + bt.j0, (uint32_t)(bt.j1 - bt.j0), dres + bt.j0, c.max_groups_copy(), s));
        c.timer.stop(tok, s);
        if (bt.region >= 0) HIPX(hipEventRecord(c.rstage_ev[bt.region], s));
        dirty[si] = true;
      }
      if (gate) {
        join();
        HIPX(hipEventRecord(f.seg[l], c.ctl));
      }
    }
    if (gate) {
      join();
    } else {
      // the host waits for the copy streams themselves; the marks below then
      // follow only the control stream's own uploads
      for (hipStream_t cs : c.streams) HIPX(hipStreamSynchronize(cs));
    }
    HIPX(hipEventRecord(f.ready, c.ctl));
    HIPX(hipEventRecord(c.reload_done, c.ctl));
    c.reload_seq++;
    for (uint32_t cl : missing) P.cls[cl].fill = c.reload_seq;
    c.prog_fn = gate ? f.id : 0;
    for (size_t q = 0; q < n; q++)
      if (kind[q] == 1) c.deferred_host.push_back({missing[q], P.cls[missing[q]].hgen});
    if (!gate) settle_reloads(c, true);  // resident on return; the host copies go
  } catch (...) {
    for (hipStream_t cs : c.streams) (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(c.ctl);
    for (uint32_t cl : missing)
      if (P.cls[cl].slot != kNone) P.evict(cl);
    throw;
  }
  c.t_reload += now_ms() - t_start;
}

// Whether every progressive reload issued so far has completed.
static bool reloads_done(Ctx& c) {
  if (c.reload_seq_done == c.reload_seq) return true;
  const hipError_t q = hipEventQuery(c.reload_done);
  if (q == hipErrorNotReady) {
    (void)hipGetLastError();
    return false;
  }
  HIPX(q);
  c.reload_seq_done = c.reload_seq;
  return true;
}

// Layer l of a function whose blocks [l * layer_bytes, (l + 1) * layer_bytes)
// hold its weights needs every class used by a block overlapping that range.
// With the classes of a reload ordered by their first block (`first`,
// non-decreasing), the classes used by layers 0..l are exactly those whose
// first block is at most layer l's last block: a prefix of the order.
std::vector<size_t> layer_segments(const std::vector<uint32_t>& first, uint32_t layers, uint64_t layer_bytes) {
  std::vector<size_t> end(layers, first.size());
  size_t j = 0;
  for (uint32_t l = 0; l < layers; l++) {
    const uint64_t last = ((uint64_t)(l + 1) * layer_bytes - 1) / kBlock;
    while (j < first.size() && first[j] <= last) j++;
    end[l] = j;
  }
  if (layers) end[layers - 1] = first.size();
  return end;
}

void settle_reloads(Ctx& c, bool wait) {
  if (c.deferred_host.empty() && c.deferred_dev.empty()) return;
  if (wait) {
    HIPX(hipEventSynchronize(c.reload_done));
    c.reload_seq_done = c.reload_seq;
  } else if (!reloads_done(c)) {
    return;
  }
  Pool& P = c.pool;
  for (const auto& [cl, gen] : c.deferred_host) {
    const Class& k = P.cls[cl];
    if (k.alive && k.hbuf != kNone && k.hgen == gen) P.host_release(cl);
  }
  c.deferred_host.clear();
  for (void* q : c.deferred_dev) c.cache.put(q);
  c.deferred_dev.clear();
}

bool reload_landing(Ctx& c, const Fn& f) {
  if (c.prog_fn != f.id || f.seg.size() != f.d.layers) return false;
  return !reloads_done(c);
}

bool reload_feeds(Ctx& c, const Fn& f) {
  if (reloads_done(c)) return false;
  for (uint32_t cl : f.distinct)
    if (c.pool.cls[cl].fill > c.reload_seq_done) return true;
  return false;
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
