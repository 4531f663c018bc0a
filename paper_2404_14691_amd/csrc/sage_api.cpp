// The C ABI (include/sage.h): context, functions, invocations, statistics,
// kernel entry points and timing.
#include <algorithm>
#include <tuple>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <unordered_set>

#include "internal.h"

using namespace sage;

struct sage_ctx {
  Ctx c;
};

namespace {

Ctx& ctx_of(sage_ctx* p) {
  if (!p) fail(SAGE_EINVAL, "null context");
  return p->c;
}

Fn& fn_of(Ctx& c, sage_fn id) {
  auto it = c.fns.find(id);
  if (it == c.fns.end()) fail(SAGE_ENOTFOUND, "unknown function handle %llu", (unsigned long long)id);
  return *it->second;
}

// Released invocations leave the table; handles are never reused, so an id
// below the next one that is not a live function was released before.
Inv& inv_of(Ctx& c, sage_inv id) {
  auto it = c.invs.find(id);
  if (it == c.invs.end()) {
    if (id != 0 && id < c.next_id && !c.fns.count(id))
      fail(SAGE_ESTATE, "invocation %llu already released", (unsigned long long)id);
    fail(SAGE_ENOTFOUND, "unknown invocation handle %llu", (unsigned long long)id);
  }
  return *it->second;
}

bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

void check_aligned(const void* p, const char* what) {
  if ((uintptr_t)p & 15) fail(SAGE_EINVAL, "%s must be 16-byte aligned", what);
}

// Validate a function description against its read-only blobs.
void validate(const sage_fn_desc& d, const sage_blob* blobs, size_t n) {
  if (d.kind == SAGE_MLP_F32 || d.kind == SAGE_MLP_BF16) {
    const uint64_t es = d.kind == SAGE_MLP_BF16 ? 2 : 4;
    if (d.layers < 1 || !pow2(d.width) || d.width < 128 || (uint64_t)d.width * es > kBlock)
      fail(SAGE_EINVAL, "MLP needs layers >= 1 and a power-of-two width >= 128 with rows <= 64 KiB");
  } else if (d.kind == SAGE_STENCIL7_F32) {
    if (!pow2(d.nx) || (uint64_t)d.nx * 4 > kBlock || d.nx < 4 || d.ny < 3 || d.nz < 3)
      fail(SAGE_EINVAL, "stencil needs a power-of-two nx with nx*4 <= 65536 and extents >= 3");
  } else if (d.kind == SAGE_RELAX7_F32) {
    if (d.nx % 4 || d.nx < 4 || d.ny < 3 || d.nz < 3 || !std::isfinite(d.coef))
      fail(SAGE_EINVAL, "relaxation needs nx a multiple of 4, extents >= 3 and a finite coefficient");
    if (n != 0) fail(SAGE_EINVAL, "this kind has no read-only data: register it with no blobs");
    return;
  } else {
    fail(SAGE_EINVAL, "unknown function kind %u", d.kind);
  }
  if (n != 1 || !blobs) fail(SAGE_EINVAL, "this kind takes exactly one read-only blob");
  for (size_t i = 0; i < n; i++) {
    const sage_blob& b = blobs[i];
    if (b.access != SAGE_RO) fail(SAGE_EINVAL, "only read-only blobs are registered; writable data goes to fn_invoke");
    if (!b.src && b.nbytes) fail(SAGE_EINVAL, "blob %zu has no source", i);
    if (b.where == SAGE_SRC_DEVICE) check_aligned(b.src, "device blob source");
    else if (b.where != SAGE_SRC_HOST) fail(SAGE_EINVAL, "blob %zu: unknown location", i);
  }
  if (blobs[0].nbytes != ro_bytes_for(d))
    fail(SAGE_EINVAL, "blob holds %zu bytes, the kind needs %llu", blobs[0].nbytes,
         (unsigned long long)ro_bytes_for(d));
}

void free_inv_buffers(Ctx& c, Inv& v) {
  c.cache.put(v.priv);
  c.cache.put(v.priv_table);
  c.cache.put(v.ws);
  c.cache.put(v.io_in);
  c.cache.put(v.io_out);
  v.priv = v.ws = v.io_in = v.io_out = nullptr;
  v.priv_table = nullptr;
}

}  // namespace

namespace sage {

// Admission and references for one invocation (see fn_setup in sage.h).
uint64_t setup_internal(Ctx& c, uint64_t id, uint32_t batch) {
  if (batch < 1) fail(SAGE_EINVAL, "batch must be >= 1");
  HIPX(hipSetDevice(c.device));
  advance_exit(c);
  Fn& f = fn_of(c, id);
  // after the third exit stage the code object is loaded again, beside the data
  auto code = [&] { load_module(c, f.d.kind); };
  const bool need_code = f.mod && !f.mod->mod;
  auto v = std::make_unique<Inv>();
  v->id = c.next_id++;
  v->fn = &f;
  v->batch = batch;
  if (c.cfg.share) {
    Pool& P = c.pool;
    std::vector<uint32_t> missing;
    if (f.resident_epoch != P.epoch)  // something was evicted since all of f was last resident
      for (uint32_t cl : f.distinct)
        if (P.cls[cl].slot == kNone) missing.push_back(cl);
    if (!missing.empty()) {
      // admission: all missing classes need slots; evict only if enough can be freed
      const uint64_t free_slots = P.budget > P.used_ ? P.budget - P.used_ : 0;
      if (missing.size() > free_slots) {
        const uint32_t mark = P.new_mark();
        for (uint32_t cl : f.distinct) P.cls[cl].mark = mark;
        std::vector<uint32_t> victims;
        const uint64_t short_by = missing.size() - free_slots;
        for (uint32_t cl = P.lru_front(); cl != kNone && victims.size() < short_by; cl = P.cls[cl].lru_next)
          if (P.cls[cl].mark != mark) victims.push_back(cl);
        if (victims.size() < short_by)
          fail(SAGE_ENOMEM, "cannot admit: %zu blocks missing, %llu evictable", missing.size(),
               (unsigned long long)(free_slots + victims.size()));
        for (uint32_t cl : victims) P.evict(cl);
      }
      if (need_code) run_two_branches(code, [&] { reload_classes(c, f, missing); }, c.cfg.serial_setup != 0, &c.worker);
      else reload_classes(c, f, missing);
    } else if (need_code) {
      code();
    }
    refresh_table(c, f);
    f.resident_epoch = P.epoch;
    if (f.live == 0)
      for (uint32_t cl : f.distinct)
        if (P.cls[cl].active++ == 0) P.lru_remove(cl);
  } else {
    if (need_code) code();
    // private copy of the read-only data for this invocation
    const size_t bytes = (size_t)f.n_blocks * kBlock;
    v->priv = c.cache.get(bytes);
    v->priv_table = (uint64_t*)c.cache.get((size_t)f.n_blocks * 8);
    try {
      copy_private(c, f, (uint8_t*)v->priv, c.ctl);
      std::vector<uint64_t> t(f.n_blocks);
      for (uint32_t b = 0; b < f.n_blocks; b++) t[b] = (uint64_t)((uint8_t*)v->priv + (uint64_t)b * kBlock);
      if (!t.empty()) HIPX(hipMemcpyAsync(v->priv_table, t.data(), t.size() * 8, hipMemcpyHostToDevice, c.ctl));
      HIPX(hipStreamSynchronize(c.ctl));
    } catch (...) {
      free_inv_buffers(c, *v);
      throw;
    }
  }
  v->live = true;
  f.live++;
  if (f.mod && c.cfg.exit_stage_ms > 0) f.mod->last_use = now_ms();
  const uint64_t out = v->id;
  c.invs[v->id] = std::move(v);
  return out;
}

void release_internal(Ctx& c, uint64_t id) {
  Inv& v = inv_of(c, id);
  Fn& f = *v.fn;
  if (f.live <= 0) fail(SAGE_ESTATE, "reference count underflow");
  if (c.cfg.share && f.live == 1) {
    Pool& P = c.pool;
    const double now = now_ms();
    for (uint32_t cl : f.distinct) {  // increasing class order
      Class& k = P.cls[cl];
      if (k.active == 0) fail(SAGE_ESTATE, "reference count underflow");
      if (--k.active == 0) P.lru_back(cl, now);
    }
  }
  free_inv_buffers(c, v);
  v.live = false;
  f.live--;
  if (f.live == 0 && f.mod && c.cfg.exit_stage_ms > 0) f.mod->last_use = now_ms();
  c.invs.erase(id);
}

Fn& find_fn(Ctx& c, uint64_t id) { return fn_of(c, id); }
Ctx& ctx_ref(sage_ctx* p) { return ctx_of(p); }
Inv& find_inv(Ctx& c, uint64_t id) { return inv_of(c, id); }

}  // namespace sage

bool Ctx::is_pinned(const void* p, size_t n) const {
  auto it = pinned.upper_bound(const_cast<void*>(p));
  if (it == pinned.begin()) return false;
  --it;
  const uint8_t* base = (const uint8_t*)it->first;
  return (const uint8_t*)p >= base && (const uint8_t*)p + n <= base + it->second;
}

extern "C" {

void sage_config_default(sage_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->ring_slots = 8;
  cfg->chunk_bytes = 8u << 20;
  cfg->streams = 4;
  cfg->fill_threads = 4;
  cfg->inflight_groups = 4;
  cfg->share = 1;
  cfg->batch = 1;
  cfg->serial_setup = 0;
  cfg->pool_budget_bytes = 0;
  cfg->tune_cache = nullptr;
}

const char* sage_last_error(void) { return last_error().c_str(); }

sage_status sage_open(int device, const sage_config* cfg, sage_ctx** out) {
  return guard([&] {
    if (!out) fail(SAGE_EINVAL, "null output");
    *out = nullptr;
    auto h = std::make_unique<sage_ctx>();
    Ctx& c = h->c;
    c.device = device;
    if (cfg) c.cfg = *cfg;
    else sage_config_default(&c.cfg);
    if (c.cfg.ring_slots < 1 || c.cfg.chunk_bytes < kBlock || c.cfg.chunk_bytes % kBlock || c.cfg.streams < 1)
      fail(SAGE_EINVAL, "ring_slots >= 1, streams >= 1, chunk_bytes a multiple of 64 KiB");
    if (!(c.cfg.exit_stage_ms >= 0)) fail(SAGE_EINVAL, "exit_stage_ms must be >= 0");
    // environment knobs (tests and measurements), checked before anything starts
    if (const char* e = std::getenv("SAGE_TILE")) c.force_tile = e;
    if (const char* e = std::getenv("SAGE_FAULT_ALLOC_AFTER")) {
      const long long v = std::strtoll(e, nullptr, 0);
      if (v < 0) fail(SAGE_EINVAL, "SAGE_FAULT_ALLOC_AFTER must be >= 0");
      c.alloc_fault.left = v;
    }
    c.pool.fault = &c.alloc_fault;
    c.cache.fault = &c.alloc_fault;
    if (const char* e = std::getenv("SAGE_STENCIL_FUSE")) c.stencil_fuse = std::strtol(e, nullptr, 0) != 0;
    if (const char* e = std::getenv("SAGE_F32_COLS")) {
      c.f32_cols = (uint32_t)std::strtoul(e, nullptr, 0);
      if (c.f32_cols != 4 && c.f32_cols != 8) fail(SAGE_EINVAL, "SAGE_F32_COLS must be 4 or 8");
    }
    if (const char* e = std::getenv("SAGE_DEV_CHUNK_BYTES")) {
      const uint64_t v = std::strtoull(e, nullptr, 0);
      if (v < kBlock || v % kBlock) fail(SAGE_EINVAL, "SAGE_DEV_CHUNK_BYTES must be a positive multiple of 65536");
      c.dev_chunk = v;
    }
    if (const char* e = std::getenv("SAGE_TEST_FP_CONST")) {
      c.test_fp_const = true;
      c.test_fp_value = std::strtoull(e, nullptr, 0);
    }
    int ndev = 0;
    HIPX(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(SAGE_EINVAL, "device %d not present (%d devices)", device, ndev);
    HIPX(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPX(hipGetDeviceProperties(&prop, device));
    c.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    HIPX(hipStreamCreateWithFlags(&c.ctl, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&c.stage_ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c.ctl_ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c.reload_done, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c.prog_ops_ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c.reg_ev, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&c.reg_vev, hipEventDisableTiming));
    for (uint32_t i = 0; i < c.cfg.streams; i++) {
      hipStream_t s;
      HIPX(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      c.streams.push_back(s);
      hipEvent_t e;
      HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c.join_ev.push_back(e);
    }
    size_t free_b = 0, total_b = 0;
    HIPX(hipMemGetInfo(&free_b, &total_b));
    uint64_t budget = c.cfg.pool_budget_bytes ? c.cfg.pool_budget_bytes : free_b / 2;
    budget /= kBlock;
    if (budget < 1) fail(SAGE_EINVAL, "pool budget below one block");
    c.pool.init(budget, (size_t)std::min<uint64_t>(16384, budget));
    ring_init(c);
    if (c.cfg.share) HIPX(hipMalloc((void**)&c.rstage_dev, kReloadStageBlocks * kBlock));  // reload staging
    // fn_invoke_noalloc: this GPU's fixed scratch (looked up with the device
    // current) and a pinned mirror of its metadata part
    HIPX(noalloc_scratch(device, &c.na_scratch));
    HIPX(hipHostMalloc((void**)&c.na_hmeta, kNoAllocMetaBytes, hipHostMallocDefault));
    flights_init(c);
    tune_load(c);
    c.worker.start(device);
    c.copier.start(std::max<uint32_t>(1, c.cfg.fill_threads) - 1);
    *out = h.release();
  });
}

sage_status sage_close(sage_ctx* p) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    serve_destroy(c);
    c.worker.stop();
    c.copier.stop();
    {
      std::lock_guard<std::recursive_mutex> lk(c.mu);
      (void)hipSetDevice(c.device);
      (void)hipDeviceSynchronize();
      flights_destroy(c);
      for (auto& kv : c.fns) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        for (hipEvent_t e : kv.second->seg) (void)hipEventDestroy(e);
      }
      c.fns.clear();
      c.invs.clear();
      c.cache.release_all();
      c.pool.destroy();
      ring_destroy(c);
      for (auto& kv : c.modules)
        if (kv.second->mod) (void)hipModuleUnload(kv.second->mod);
      c.modules.clear();
      for (auto& kv : c.pinned) (void)hipHostFree(kv.first);
      c.pinned.clear();
      if (c.h_stage) (void)hipHostFree(c.h_stage);
      c.h_stage = nullptr;
      if (c.stage_ev) (void)hipEventDestroy(c.stage_ev);
      if (c.ctl_ev) (void)hipEventDestroy(c.ctl_ev);
      if (c.reload_done) (void)hipEventDestroy(c.reload_done);
      if (c.prog_ops_ev) (void)hipEventDestroy(c.prog_ops_ev);
      if (c.prog_hops) (void)hipHostFree(c.prog_hops);
      if (c.reg_ev) (void)hipEventDestroy(c.reg_ev);
      if (c.reg_vev) (void)hipEventDestroy(c.reg_vev);
      if (c.reg_hops) (void)hipHostFree(c.reg_hops);
      if (c.reg_hres) (void)hipHostFree(c.reg_hres);
      if (c.reg_dops) (void)hipFree(c.reg_dops);
      if (c.reg_dres) (void)hipFree(c.reg_dres);
      if (c.rstage_dev) (void)hipFree(c.rstage_dev);
      if (c.na_hmeta) (void)hipHostFree(c.na_hmeta);
      c.na_hmeta = nullptr;
      for (hipEvent_t e : c.rstage_ev) (void)hipEventDestroy(e);
      c.deferred_dev.clear();
      c.deferred_host.clear();
      for (hipEvent_t e : c.join_ev) (void)hipEventDestroy(e);
      c.timer.destroy();
      for (hipStream_t s : c.streams) (void)hipStreamDestroy(s);
      (void)hipStreamDestroy(c.ctl);
    }
    delete p;
  });
}

void* sage_host_alloc(sage_ctx* p, size_t n) {
  void* out = nullptr;
  const sage_status st = guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    HIPX(hipHostMalloc(&out, n ? n : 1, hipHostMallocDefault));
    c.pinned[out] = n;
  });
  return st == SAGE_OK ? out : nullptr;
}

void sage_host_free(sage_ctx* p, void* q) {
  (void)guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    auto it = c.pinned.find(q);
    if (it == c.pinned.end()) return;
    c.pinned.erase(it);
    HIPX(hipHostFree(q));
  });
}

// ------------------------------------------------------------- functions
// A function's record before its data is in: sources, block count, ready
// event and (sharing on) its block table from the device cache.
static std::unique_ptr<Fn> new_fn(Ctx& c, const sage_fn_desc& desc, const sage_blob* blobs, size_t n_blobs) {
  auto f = std::make_unique<Fn>();
  f->id = c.next_id++;
  f->d = desc;
  uint32_t first = 0;
  for (size_t i = 0; i < n_blobs; i++) {
    const sage_blob& b = blobs[i];
    const bool dev = b.where == SAGE_SRC_DEVICE;
    f->srcs.push_back(Src{(const uint8_t*)b.src, b.nbytes, dev, !dev && c.is_pinned(b.src, b.nbytes)});
    f->blob_first.push_back(first);
    first += (uint32_t)((b.nbytes + kBlock - 1) / kBlock);
    f->ro_bytes += b.nbytes;
  }
  f->n_blocks = first;
  HIPX(hipEventCreateWithFlags(&f->ready, hipEventDisableTiming));
  // the block table comes from the device cache (no hipMalloc/hipFree per function)
  if (c.cfg.share) {
    try {
      f->d_table = (uint64_t*)c.cache.get(std::max<size_t>(8, (size_t)f->n_blocks * 8));
    } catch (...) {
      (void)hipEventDestroy(f->ready);
      throw;
    }
  }
  return f;
}

// Release what a record that is not (or no longer) being registered holds.
static void drop_fn_shell(Ctx& c, Fn& F) {
  register_drop_prefetch(c, F);
  if (F.d_table) c.cache.put(F.d_table);
  F.d_table = nullptr;
  if (F.ready) (void)hipEventDestroy(F.ready);
  F.ready = nullptr;
}

// The two setup branches of a registration: code (module) and data (the
// blobs).  On failure the record's resources are released.  Returns the
// code branch's time.
static double register_fn(Ctx& c, Fn& F) {
  double t_code = 0;
  bool data_in = false;  // register_shared returned: the blocks are counted into their classes
  auto code = [&] {
    const double t0 = now_ms();
    F.mod = load_module(c, F.d.kind);
    t_code = now_ms() - t0;
  };
  auto data = [&] {
    if (c.cfg.share) {
      register_shared(c, F);
      data_in = true;
    }
  };
  try {
    run_two_branches(code, data, c.cfg.serial_setup != 0, &c.worker);
    if (c.cfg.share) refresh_table(c, F);
    HIPX(hipEventRecord(F.ready, c.ctl));
  } catch (...) {
    (void)hipStreamSynchronize(c.ctl);
    if (data_in) {  // the other branch failed after the data was in: take the blocks out again
      Pool& P = c.pool;
      for (uint32_t cl : F.cls) P.cls[cl].members--;
      for (uint32_t cl : F.distinct)
        if (P.cls[cl].members == 0) P.drop_class(cl);
    }
    drop_fn_shell(c, F);
    throw;
  }
  return t_code;
}

static sage_fn commit_fn(Ctx& c, std::unique_ptr<Fn> f, double t_code, double ms) {
  const sage_fn id = f->id;
  c.logical += f->ro_bytes;
  c.registrations++;
  c.t_code += t_code;
  c.t_register += ms;
  c.fns[id] = std::move(f);
  return id;
}

sage_status fn_register(sage_ctx* p, const sage_fn_desc* desc, const sage_blob* blobs, size_t n_blobs,
                        sage_fn* out) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!desc || !out) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const double t_start = now_ms();
    HIPX(hipSetDevice(c.device));
    validate(*desc, blobs, n_blobs);
    advance_exit(c);
    auto f = new_fn(c, *desc, blobs, n_blobs);
    const double t_code = register_fn(c, *f);
    *out = commit_fn(c, std::move(f), t_code, now_ms() - t_start);
  });
}

// Unregister a function with no live setups.
static void unregister_fn(Ctx& c, sage_fn id) {
  Fn& f = fn_of(c, id);
  for (size_t i = 0; i < c.flights.size(); i++) finish_flight(c, (int)i);
  // copies from f's sources or host-cache copies may still be in flight;
  // the caller may free the sources on return
  HIPX(hipEventSynchronize(f.ready));
  settle_reloads(c, true);
  Pool& P = c.pool;
  for (uint32_t cl : f.cls) P.cls[cl].members--;
  for (uint32_t cl : f.distinct)
    if (P.cls[cl].members == 0) P.drop_class(cl);
  c.logical -= f.ro_bytes;
  if (f.d_table) c.cache.put(f.d_table);
  (void)hipEventDestroy(f.ready);
  for (hipEvent_t e : f.seg) (void)hipEventDestroy(e);
  c.fns.erase(id);
}

sage_status fn_register_batch(sage_ctx* p, size_t n, const sage_fn_desc* descs, const sage_blob* const* blobs,
                              const size_t* n_blobs, sage_fn* out, double* register_ms) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (n == 0) return;
    if (!descs || !blobs || !n_blobs || !out) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    double t = now_ms();
    HIPX(hipSetDevice(c.device));
    for (size_t i = 0; i < n; i++) validate(descs[i], blobs[i], n_blobs[i]);
    advance_exit(c);
    std::vector<std::unique_ptr<Fn>> fs;
    std::vector<sage_fn> ids;
    try {
      for (size_t i = 0; i < n; i++) fs.push_back(new_fn(c, descs[i], blobs[i], n_blobs[i]));
      // each function's device-source fingerprints go out before the
      // previous function's host classification, so the two overlap
      register_prefetch(c, *fs[0]);
      for (size_t i = 0; i < n; i++) {
        if (i + 1 < n) register_prefetch(c, *fs[i + 1]);
        const double t_code = register_fn(c, *fs[i]);
        const double t1 = now_ms();
        if (register_ms) register_ms[i] = t1 - t;
        ids.push_back(commit_fn(c, std::move(fs[i]), t_code, t1 - t));
        t = t1;
      }
    } catch (...) {
      for (auto& f : fs)
        if (f) drop_fn_shell(c, *f);
      for (sage_fn id : ids) unregister_fn(c, id);  // all or nothing
      throw;
    }
    for (size_t i = 0; i < n; i++) out[i] = ids[i];
  });
}

sage_status fn_unregister(sage_ctx* p, sage_fn id) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    Fn& f = fn_of(c, id);
    const double t0 = now_ms();
    if (f.live > 0) fail(SAGE_EBUSY, "function has %d live setups", f.live);
    unregister_fn(c, id);
    c.t_unregister += now_ms() - t0;
  });
}

sage_status fn_setup(sage_ctx* p, sage_fn id, uint32_t batch, sage_inv* out) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!out) fail(SAGE_EINVAL, "null output");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const double t0 = now_ms();
    *out = setup_internal(c, id, batch);
    c.t_setup += now_ms() - t0;
  });
}

sage_status fn_setup_batch(sage_ctx* p, size_t n, const sage_fn* fns, const uint32_t* batches, sage_inv* out,
                           size_t* n_done, double* setup_ms) {
  size_t k = 0;
  const sage_status st = guard([&] {
    Ctx& c = ctx_of(p);
    if (n && (!fns || !batches || !out)) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const double t0 = now_ms();
    try {
      for (double t = t0; k < n; k++) {
        out[k] = setup_internal(c, fns[k], batches[k]);
        const double t1 = now_ms();
        if (setup_ms) setup_ms[k] = t1 - t;
        t = t1;
      }
    } catch (...) {
      c.t_setup += now_ms() - t0;
      throw;
    }
    c.t_setup += now_ms() - t0;
  });
  if (n_done) *n_done = k;
  return st;
}

sage_status fn_release_batch(sage_ctx* p, size_t n, const sage_inv* invs) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (n && !invs) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const double t0 = now_ms();
    for (size_t i = 0; i < n; i++) release_internal(c, invs[i]);
    c.t_release += now_ms() - t0;
  });
}

sage_status fn_release(sage_ctx* p, sage_inv id) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const double t0 = now_ms();
    release_internal(c, id);
    c.t_release += now_ms() - t0;
  });
}

static void run_calls(Ctx& c, const std::vector<Call>& calls, uint32_t io) {
  // partition: MLPs by (kind, width, layers); stencils by coefficient table
  using Key = std::tuple<uint32_t, uint32_t, uint32_t, const void*>;
  std::vector<std::vector<Call>> parts;
  std::vector<Key> keys;
  for (const Call& cl : calls) {
    const sage_fn_desc& d = cl.inv->fn->d;
    const Key k = is_grid(d.kind) ? Key{d.kind, 0u, 0u, (const void*)cl.inv->table()}
                                              : Key{d.kind, d.width, d.layers, nullptr};
    size_t i = 0;
    while (i < keys.size() && keys[i] != k) i++;
    if (i == keys.size()) {
      keys.push_back(k);
      parts.emplace_back();
    }
    parts[i].push_back(cl);
  }
  std::vector<int> used;
  for (auto& part : parts) {
    const int fl = is_grid(part[0].inv->fn->d.kind) ? launch_stencil_group(c, part, io)
                                                                  : launch_mlp_group(c, part, io);
    used.push_back(fl);
  }
  for (int fl : used) finish_flight(c, fl);
  c.invocations += calls.size();
}

sage_status fn_invoke(sage_ctx* p, sage_inv id, const void* in, size_t in_bytes, void* out, size_t out_bytes,
                      uint32_t io) {
  return fn_invoke_batch(p, 1, &id, &in, &in_bytes, &out, &out_bytes, io);
}

sage_status fn_invoke_batch(sage_ctx* p, size_t n, const sage_inv* ids, const void* const* in,
                            const size_t* in_bytes, void* const* out, const size_t* out_bytes, uint32_t io) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (n == 0) return;
    if (!ids || !in || !in_bytes || !out || !out_bytes) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (c.serve) fail(SAGE_ESTATE, "the serving loop owns the launch flights: use sage_submit");
    HIPX(hipSetDevice(c.device));
    std::vector<Call> calls;
    std::unordered_set<uint64_t> seen;
    for (size_t i = 0; i < n; i++) {
      Inv& v = inv_of(c, ids[i]);
      if (!seen.insert(ids[i]).second) fail(SAGE_EINVAL, "invocation %llu listed twice", (unsigned long long)ids[i]);
      const sage_fn_desc& d = v.fn->d;
      if (in_bytes[i] != in_bytes_for(d, v.batch) || out_bytes[i] != out_bytes_for(d, v.batch))
        fail(SAGE_EINVAL, "call %zu: in/out bytes %zu/%zu, expected %zu/%zu", i, in_bytes[i], out_bytes[i],
             in_bytes_for(d, v.batch), out_bytes_for(d, v.batch));
      if (!in[i] || !out[i]) fail(SAGE_EINVAL, "call %zu: null buffer", i);
      if (io & SAGE_IO_DEVICE_IN) check_aligned(in[i], "device input");
      if (io & SAGE_IO_DEVICE_OUT) check_aligned(out[i], "device output");
      calls.push_back(Call{&v, in[i], in_bytes[i], out[i], out_bytes[i]});
    }
    const double t0 = now_ms();
    run_calls(c, calls, io);
    c.t_invoke += now_ms() - t0;
  });
}

// fn_invoke for callers that cannot allocate: the body's metadata and
// activations live in the GPU's fixed scratch array instead of the flight's
// buffers, launches are eager, and the tile plan comes from timings already
// measured (no autotuning).  Calls on one GPU share that scratch.
sage_status fn_invoke_noalloc(sage_ctx* p, sage_inv id, const void* in, size_t in_bytes, void* out,
                              size_t out_bytes) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!in || !out) fail(SAGE_EINVAL, "null buffer");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (c.serve) fail(SAGE_ESTATE, "the serving loop owns the launch flights: use sage_submit");
    HIPX(hipSetDevice(c.device));
    Inv& v = inv_of(c, id);
    const sage_fn_desc& d = v.fn->d;
    if (is_grid(d.kind)) fail(SAGE_EINVAL, "fn_invoke_noalloc runs the MLP kinds only");
    if (in_bytes != in_bytes_for(d, v.batch) || out_bytes != out_bytes_for(d, v.batch))
      fail(SAGE_EINVAL, "in/out bytes %zu/%zu, expected %zu/%zu", in_bytes, out_bytes, in_bytes_for(d, v.batch),
           out_bytes_for(d, v.batch));
    check_aligned(in, "device input");
    check_aligned(out, "device output");
    const size_t act = in_elem_size(d);
    if (v.batch > kNoAllocRows || (size_t)v.batch * d.width * act > kNoAllocActBytes)
      fail(SAGE_EINVAL,
           "batch %u x width %u exceeds the fixed scratch of fn_invoke_noalloc: at most %u rows and "
           "rows x width x %zu <= %zu bytes",
           v.batch, d.width, kNoAllocRows, act, kNoAllocActBytes);
    const ExtScratch ext{c.na_scratch, c.na_hmeta, kNoAllocMetaBytes, c.na_scratch + kNoAllocMetaBytes,
                         2 * kNoAllocActBytes};
    const double t0 = now_ms();
    const std::vector<Call> calls{Call{&v, in, in_bytes, out, out_bytes}};
    const int fl = launch_mlp_group(c, calls, SAGE_IO_DEVICE_IN | SAGE_IO_DEVICE_OUT, -1, &ext);
    finish_flight(c, fl);
    c.invocations++;
    c.t_invoke += now_ms() - t0;
  });
}

// ---------------------------------------------------------- introspection
sage_status sage_get_stats(sage_ctx* p, sage_stats* out) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!out) fail(SAGE_EINVAL, "null output");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    HIPX(hipSetDevice(c.device));
    advance_exit(c);
    settle_reloads(c, false);
    std::memset(out, 0, sizeof *out);
    const Pool& P = c.pool;
    for (const Class& k : P.cls) {
      if (!k.alive) continue;
      out->classes++;
      out->unique_bytes += k.len;
      if (k.members >= 2) out->shared_bytes += (uint64_t)k.len * k.members;
      else out->private_bytes += (uint64_t)k.len * k.members;
      if (k.slot != kNone) {
        out->resident_bytes += k.len;
        out->resident_slots++;
      }
    }
    for (auto& kv : c.fns) out->refcount_sum += (uint64_t)kv.second->live * kv.second->distinct.size();
    out->logical_bytes = c.logical;
    out->budget_slots = P.budget;
    out->h2d_bytes = c.h2d;
    for (auto& kv : c.invs) out->live_setups += kv.second->live ? 1 : 0;
    out->evictions = P.evictions;
    out->reloads = c.reloads;
    out->registrations = c.registrations;
    out->invocations = c.invocations;
    out->verify_mismatches = c.mismatches;
    out->workspace_bytes = c.cache.in_use();
    out->t_register_ms = c.t_register;
    out->t_code_ms = c.t_code;
    out->t_fp_wait_ms = c.t_fp_wait;
    out->t_dedup_ms = c.t_dedup;
    out->t_verify_ms = c.t_verify;
    out->t_setup_ms = c.t_setup;
    out->t_invoke_ms = c.t_invoke;
    out->host_cached_bytes = P.host_bytes;
    out->demotions = P.demotions;
    out->host_reloads = c.host_reloads;
    out->module_unloads = c.module_unloads;
    out->t_reload_ms = c.t_reload;
    out->t_release_ms = c.t_release;
    out->t_unregister_ms = c.t_unregister;
    {
      std::lock_guard<std::mutex> mk(c.module_mu);
      out->module_loads = c.module_loads;
      out->t_module_ms = c.t_module;
    }
  });
}

sage_status sage_fn_fingerprints(sage_ctx* p, sage_fn id, uint64_t* out, size_t n) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    Fn& f = fn_of(c, id);
    if (!c.cfg.share) fail(SAGE_ESTATE, "fingerprints exist only with sharing on");
    if (n != f.n_blocks || (!out && n)) fail(SAGE_EINVAL, "need %u entries", f.n_blocks);
    std::copy(f.fps.begin(), f.fps.end(), out);
  });
}

sage_status sage_fn_block_count(sage_ctx* p, sage_fn id, size_t* out) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (!out) fail(SAGE_EINVAL, "null output");
    *out = fn_of(c, id).n_blocks;
  });
}

sage_status sage_fn_block_info(sage_ctx* p, sage_fn id, uint32_t* cls, uint32_t* slot, uint32_t* refs, size_t n) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    Fn& f = fn_of(c, id);
    if (!c.cfg.share) fail(SAGE_ESTATE, "block classes exist only with sharing on");
    if (n != f.n_blocks) fail(SAGE_EINVAL, "need %u entries", f.n_blocks);
    // references of a class = live setups of every function using it
    std::unordered_map<uint32_t, uint32_t> rc;
    for (uint32_t cl : f.distinct) rc[cl] = 0;
    for (auto& kv : c.fns) {
      const Fn& g = *kv.second;
      if (g.live <= 0) continue;
      for (uint32_t cl : g.distinct) {
        auto it = rc.find(cl);
        if (it != rc.end()) it->second += g.live;
      }
    }
    for (uint32_t b = 0; b < f.n_blocks; b++) {
      const Class& k = c.pool.cls[f.cls[b]];
      if (cls) cls[b] = f.cls[b];
      if (slot) slot[b] = k.slot;
      if (refs) refs[b] = rc[f.cls[b]];
    }
  });
}

sage_status sage_read_slot(sage_ctx* p, uint32_t slot, void* host) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (!host) fail(SAGE_EINVAL, "null output");
    bool found = false;
    for (const Class& k : c.pool.cls) found |= k.alive && k.slot == slot;
    if (!found) fail(SAGE_ENOTFOUND, "slot %u holds no class", slot);
    HIPX(hipStreamSynchronize(c.ctl));  // pool writes are ordered on the control stream
    HIPX(hipMemcpy(host, c.pool.addr(slot), kBlock, hipMemcpyDeviceToHost));
  });
}

// ---------------------------------------------------- kernel entry points
sage_status sage_fingerprint(sage_ctx* p, const void* dev, size_t nbytes, uint64_t* dev_out, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (nbytes && (!dev || !dev_out)) fail(SAGE_EINVAL, "null buffer");
    check_aligned(dev, "data");
    check_aligned(dev_out, "output");
    if ((nbytes + kBlock - 1) / kBlock > 0xFFFFFFFFull) fail(SAGE_EINVAL, "too many blocks");
    hipStream_t s = stream ? (hipStream_t)stream : c.ctl;
    const int tok = c.timer.start("fp64k", s, 1);
    HIPX(launch_fp64k(dev, nbytes, dev_out, c.max_groups_stream(), s));
    c.timer.stop(tok, s);
  });
}

sage_status sage_blkcopy(sage_ctx* p, const sage_blk_op* ops, size_t n, uint32_t* result, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (n && (!ops || !result)) fail(SAGE_EINVAL, "null buffer");
    if (n > 0xFFFFFFFFull) fail(SAGE_EINVAL, "too many operations");
    hipStream_t s = stream ? (hipStream_t)stream : c.ctl;
    const int tok = c.timer.start("blkcopy", s, 1);
    HIPX(launch_blkcopy(reinterpret_cast<const BlkOp*>(ops), (uint32_t)n, result, c.max_groups_copy(), s));
    c.timer.stop(tok, s);
  });
}

// ------------------------------------------------------------------ timing
sage_status sage_timing_enable(sage_ctx* p, int on) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    c.timer.on = on != 0;
    if (c.timer.on) c.timer.reserve(kTimerPairs);
  });
}

sage_status sage_timing_get(sage_ctx* p, const char* kernel, double* total_ms, uint64_t* launches) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!kernel || !total_ms || !launches) fail(SAGE_EINVAL, "null argument");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    c.timer.get(kernel, total_ms, launches);
  });
}

sage_status sage_mfma_ceiling(sage_ctx* p, uint32_t k, uint32_t reps, double* us_per_launch, double* shader_ghz) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!us_per_launch || !shader_ghz) fail(SAGE_EINVAL, "null argument");
    if (k == 0 || k % 32 || k > 65536 || reps == 0 || reps > 1000) fail(SAGE_EINVAL, "k %u or reps %u out of range", k, reps);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const uint32_t grid = (uint32_t)c.cus;
    hipStream_t s = c.ctl;
    float* out = nullptr;
    unsigned long long* clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Release {  // on every way out, after the stream has drained
      Ctx& c;
      hipStream_t s;
      float*& out;
      unsigned long long*& clk;
      hipEvent_t &e0, &e1;
      ~Release() {
        (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (out) c.cache.put(out);
        if (clk) c.cache.put(clk);
      }
    } release{c, s, out, clk, e0, e1};
    out = static_cast<float*>(c.cache.get((size_t)grid * 512 * sizeof(float)));
    clk = static_cast<unsigned long long*>(c.cache.get((size_t)grid * 2 * sizeof(unsigned long long)));
    HIPX(hipEventCreate(&e0));
    HIPX(hipEventCreate(&e1));
    HIPX(launch_mfma_ceiling(grid, k / 32, out, clk, s));  // warm-up
    HIPX(hipEventRecord(e0, s));
    for (uint32_t r = 0; r < reps; r++) HIPX(launch_mfma_ceiling(grid, k / 32, out, clk, s));
    HIPX(hipEventRecord(e1, s));
    HIPX(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPX(hipEventElapsedTime(&ms, e0, e1));
    std::vector<unsigned long long> h((size_t)grid * 2);
    HIPX(hipMemcpyAsync(h.data(), clk, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    std::vector<double> ghz;
    for (uint32_t g = 0; g < grid; g++)
      if (h[2 * g + 1]) ghz.push_back((double)h[2 * g] / (double)h[2 * g + 1] * 0.1);  // reference clock 100 MHz
    std::sort(ghz.begin(), ghz.end());
    *us_per_launch = (double)ms * 1e3 / reps;
    *shader_ghz = ghz.empty() ? 0.0 : ghz[ghz.size() / 2];
  });
}

sage_status sage_timing_only(sage_ctx* p, const char* kernel) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    const std::string k = kernel ? kernel : "";
    static const char* const kNames[] = {"fp64k", "blkcopy", "ggemm_bf16", "mlp_f32", "stencil7"};
    if (!k.empty() && std::find(std::begin(kNames), std::end(kNames), k) == std::end(kNames))
      fail(SAGE_EINVAL, "unknown kernel name %s", k.c_str());
    c.timer.only = k;
  });
}

sage_status sage_timing_reset(sage_ctx* p) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    c.timer.reset();
  });
}

sage_status sage_selftest_plan(uint32_t width, const uint32_t* rows, size_t n_groups, const char* const* shapes,
                               const double* wave_ms, size_t n_shapes, uint32_t cus, char* out, size_t cap) {
  return guard([&] {
    if (!rows || !out || (n_shapes && (!shapes || !wave_ms)) || !n_groups || !cus)
      fail(SAGE_EINVAL, "null argument or empty input");
    std::map<std::string, TuneEntry> tune;
    for (size_t i = 0; i < n_shapes; i++) {
      if (!shapes[i]) fail(SAGE_EINVAL, "null shape name");
      if (!tile_shape_known(shapes[i])) fail(SAGE_EINVAL, "unknown tile shape %s", shapes[i]);
      tune[tune_key_for(width, shapes[i])] = TuneEntry{shapes[i], wave_ms[i]};
    }
    const std::string s = plan_describe(tune, cus, width, std::vector<uint32_t>(rows, rows + n_groups));
    if (s.size() + 1 > cap) fail(SAGE_EINVAL, "need %zu bytes", s.size() + 1);
    std::memcpy(out, s.c_str(), s.size() + 1);
  });
}

sage_status sage_selftest_segments(const uint32_t* first, size_t n, uint32_t layers, uint64_t layer_bytes,
                                   size_t* out) {
  return guard([&] {
    if ((n && !first) || !out || !layers || !layer_bytes) fail(SAGE_EINVAL, "null argument or empty input");
    for (size_t j = 1; j < n; j++)
      if (first[j] < first[j - 1]) fail(SAGE_EINVAL, "first blocks must be non-decreasing");
    const std::vector<size_t> end = layer_segments(std::vector<uint32_t>(first, first + n), layers, layer_bytes);
    std::copy(end.begin(), end.end(), out);
  });
}

sage_status sage_tick(sage_ctx* p) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    HIPX(hipSetDevice(c.device));
    advance_exit(c);
  });
}

sage_status sage_last_launch(sage_ctx* p, char* out, size_t cap) {
  return guard([&] {
    Ctx& c = ctx_of(p);
    if (!out) fail(SAGE_EINVAL, "null output");
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (c.last_launch.empty()) fail(SAGE_ENOTFOUND, "no MLP launch yet");
    if (c.last_launch.size() + 1 > cap) fail(SAGE_EINVAL, "need %zu bytes", c.last_launch.size() + 1);
    std::memcpy(out, c.last_launch.c_str(), c.last_launch.size() + 1);
  });
}

}  // extern "C"
