// Host-side runtime of libsage: context, block pool, function and
// invocation records, staging ring, grouped launcher.  Internal only; the
// public interface is include/sage.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sage.h"
#include "layout.h"

namespace sage {

// ------------------------------------------------------------------ timing
inline double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ errors
struct Error {
  sage_status status;
  std::string msg;
};
[[noreturn]] void fail(sage_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void set_last_error(const std::string& msg);
const std::string& last_error();
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPX(call) ::sage::hip_check((call), #call, __FILE__, __LINE__)

// Kinds whose body is the grid sweep (read-only coefficient grid or none).
inline bool is_grid(uint32_t kind) { return kind == SAGE_STENCIL7_F32 || kind == SAGE_RELAX7_F32; }

// Run `body` and translate an Error / std::exception into a status.
sage_status guard(const std::function<void()>& body);

// ------------------------------------------------------------ kernels (rt)
hipError_t launch_fp64k(const void* data, uint64_t nbytes, uint64_t* out, int max_groups, hipStream_t s);
hipError_t launch_blkcopy(const BlkOp* ops, uint32_t n, uint32_t* result, int max_groups, hipStream_t s);
hipError_t launch_mfma_ceiling(uint32_t grid, uint32_t k_slices, float* out, unsigned long long* clk, hipStream_t s);

// Fixed device scratch of fn_invoke_noalloc: one array per GPU in the
// library's code object, never freed.  Layout: [metadata: kNoAllocMetaBytes]
// [activations: 2 x kNoAllocActBytes, ping-pong].  Limits: kNoAllocRows rows,
// rows x width x activation element size <= kNoAllocActBytes.
constexpr size_t kNoAllocMetaBytes = 64u << 10;
constexpr size_t kNoAllocActBytes = 4u << 20;
constexpr size_t kNoAllocScratchBytes = kNoAllocMetaBytes + 2 * kNoAllocActBytes;
constexpr uint32_t kNoAllocRows = 512;
// Device address of the current device's scratch array (looked up once per
// device; `device` must be current).
hipError_t noalloc_scratch(int device, uint8_t** out);

// Allocation-failure injection (SAGE_FAULT_ALLOC_AFTER=N): after N device
// allocations of the pool arena and the workspace cache have succeeded,
// every later one fails as if the device were out of memory.  Off (-1) by
// default.
struct AllocFault {
  int64_t left = -1;
  bool fail_now() {
    if (left < 0) return false;
    if (left == 0) return true;
    left--;
    return false;
  }
};

// --------------------------------------------------- device memory caching
// Size-binned cache of hipMalloc blocks for workspaces and private copies;
// memory returns to the bin on put() and to HIP only at close.
class DevCache {
 public:
  void* get(size_t n);
  void put(void* p);
  void release_all();
  size_t held() const { return held_; }
  size_t in_use() const { return in_use_; }
  static size_t round(size_t n);
  AllocFault* fault = nullptr;

 private:
  std::map<size_t, std::vector<void*>> free_;
  std::unordered_map<void*, size_t> live_;
  size_t held_ = 0, in_use_ = 0;
};

// ------------------------------------------------------------------ timing
class KernelTimer {
 public:
  bool on = false;
  std::string only;  // when not empty: the one name timed
  // Have n event pairs ready (created outside the timed work; a start then
  // costs two event records and no allocation).
  void reserve(size_t n);
  // Record a start event on s; returns a token for stop().
  int start(const char* name, hipStream_t s, uint32_t launches);
  void stop(int token, hipStream_t s);
  void collect();  // resolve finished pairs (events must be complete)
  void reset();
  bool get(const std::string& name, double* ms, uint64_t* n);
  void destroy();

 private:
  struct Pair {
    hipEvent_t a, b;
    std::string name;
    uint32_t launches;
    bool busy;
  };
  std::vector<Pair> pairs_;
  std::vector<int> free_;  // indices of pairs not in use
  std::map<std::string, std::pair<double, uint64_t>> acc_;
  int add_pair();
};

// ------------------------------------------------------------------- pool
constexpr uint32_t kNone = 0xFFFFFFFFu;

// A class is a set of identical blocks; while resident it owns one slot.
// References are counted per function: `active` is the number of functions
// with live setups that use the class, so a setup or release touches the
// classes only when its function's live count crosses zero.  The class's
// reference count in the paper-level sense (live setups using it) is the
// sum of the live counts of those functions.  Class storage is recycled;
// `seq` (creation order) is what orders classes.
struct Class {
  uint64_t fp = 0;
  uint64_t seq = 0;           // creation order
  uint32_t len = 0;
  uint32_t slot = kNone;
  uint32_t active = 0;        // functions with live setups using the class
  uint32_t members = 0;       // registered (fn, block) references
  uint32_t next = kNone;      // next class in its fingerprint chain
  uint32_t mark = 0;          // protection stamp of the running registration / reload
  uint32_t lru_prev = kNone, lru_next = kNone;
  bool alive = false;
  bool in_lru = false;
  bool indexed = false;
  const uint8_t* pending = nullptr;  // device bytes of its first block while its chunk is in flight
  double idle_since = 0;      // when it last became unreferenced (host ms)
  uint32_t hbuf = kNone;      // host-cache buffer holding its bytes after demotion, or kNone
  uint32_t hoff = 0;          // block index inside that buffer
  uint64_t hgen = 0;          // demotion number of its current host copy
  uint64_t fill = 0;          // number of the progressive reload that last filled its slot
};

// Pinned host buffer of the host cache: blocks demoted together.
struct HostBuf {
  uint8_t* p = nullptr;
  uint32_t blocks = 0;
  uint32_t live = 0;  // classes still holding a block of it
};

// Open-addressing map fingerprint -> first class of its chain.
class FpIndex {
 public:
  uint32_t find(uint64_t fp) const;
  void set(uint64_t fp, uint32_t head);  // insert or overwrite
  // insert unless present (one probe sequence): the value already there, or kNone
  uint32_t insert_if_absent(uint64_t fp, uint32_t head);
  // the value at fp (kNone if absent); if it is `head`, it becomes `next`,
  // or the entry goes when next is kNone (one probe sequence)
  uint32_t pop_head(uint64_t fp, uint32_t head, uint32_t next);
  void erase(uint64_t fp);
  void clear();

 private:
  void grow();
  void erase_at(size_t i);
  std::vector<uint64_t> key_;
  std::vector<uint32_t> val_;  // kNone = empty
  size_t mask_ = 0, n_ = 0;
};

class Pool {
 public:
  // host_standin: slot addresses are stand-ins that are never dereferenced
  // and no device memory is allocated (host-only self-test)
  void init(uint64_t budget_slots, size_t seg_slots, bool host_standin = false);
  void destroy();
  uint8_t* addr(uint32_t slot) const {
    return segs_[slot >> seg_shift_] + (uint64_t)(slot & (seg_slots_ - 1)) * kBlock;
  }
  // Take a free slot, growing the arena up to the budget, else evicting the
  // front unreferenced class that `protect` does not hold.  kNone if none.
  template <class Protect>
  uint32_t alloc_slot(const Protect& protect);
  void free_slot(uint32_t s) { free_.push_back(s); used_--; }
  uint32_t new_class(uint64_t fp, uint32_t len);
  void drop_class(uint32_t c);          // dead class: slot freed, index entry removed, storage recycled
  void evict(uint32_t c, bool demotion = false);  // demotion: counted as such, not as an eviction
  void index_add(uint32_t c);           // append to the end of its fingerprint chain
  void index_remove(uint32_t c);
  void lru_back(uint32_t c, double now);  // now: when it became unreferenced (host ms)
  void lru_remove(uint32_t c);
  uint32_t lru_front() const { return lru_head_; }
  uint32_t chain_head(uint64_t fp) const { return index_.find(fp); }
  uint32_t new_mark() { return ++mark_; }
  // Sort class ids by creation order (LSD radix on the sequence numbers).
  void sort_by_seq(std::vector<uint32_t>& ids) const;
  // Host cache: a new buffer for `blocks` demoted blocks (kNone if the
  // budget or the allocation fails), and dropping one class's host copy.
  uint32_t host_buffer(uint32_t blocks, uint64_t budget_bytes);
  void host_release(uint32_t c);

  std::vector<Class> cls;
  uint64_t budget = 0, used_ = 0, evictions = 0, epoch = 0, live_classes = 0;
  std::vector<HostBuf> hbufs;
  std::deque<std::pair<uint32_t, uint64_t>> host_lru;  // (class, demotion number), in demotion order
  uint64_t host_bytes = 0, demotions = 0;
  AllocFault* fault = nullptr;

 private:
  bool grow_arena();
  bool standin_ = false;
  std::vector<uint8_t*> segs_;
  size_t seg_slots_ = 16384;  // slot ids of segment k start at k * seg_slots_ (a power of two)
  uint32_t seg_shift_ = 14;
  std::vector<uint32_t> free_;
  std::vector<uint32_t> free_cls_;
  std::vector<uint32_t> free_hbufs_;
  std::multimap<uint32_t, uint8_t*> spare_host_;  // released pinned buffers by size in blocks
  uint64_t spare_bytes_ = 0;
  static constexpr uint64_t kSpareHostBytes = 1ull << 30;
  FpIndex index_;
  uint32_t lru_head_ = kNone, lru_tail_ = kNone;
  uint32_t mark_ = 0;
  uint64_t seq_ = 0;
};

template <class Protect>
uint32_t Pool::alloc_slot(const Protect& protect) {
  if (free_.empty() && used_ < budget) grow_arena();
  if (free_.empty() || used_ >= budget) {
    uint32_t victim = lru_head_;
    while (victim != kNone && protect(victim)) victim = cls[victim].lru_next;
    if (victim == kNone) return kNone;
    evict(victim);
  }
  if (free_.empty()) return kNone;
  const uint32_t s = free_.back();
  free_.pop_back();
  used_++;
  return s;
}

// --------------------------------------------------------------- modules
// A code object.  The record lives as long as the context; the loaded
// module may be unloaded by the multi-stage exit and is loaded again by the
// next setup that needs it.
struct Module {
  hipModule_t mod = nullptr;
  std::map<std::string, hipFunction_t> fn;
  std::string path;
  int key = 0;
  double last_use = 0;  // host ms of the last setup or release of one of its functions
  hipFunction_t get(const char* name);
};

// ------------------------------------------------------------- functions
struct Src {
  const uint8_t* p;
  size_t n;
  bool dev;
  bool pinned;
};

// One chunk of a registration's read-only data: staged through a ring slot
// (host sources) or fingerprinted in place (device sources).
struct RegChunk {
  uint32_t blob;
  uint64_t off, bytes;
  uint32_t first, nblk;
  int slot;
  const uint8_t* data;  // device address of the chunk's bytes
};

struct Fn {
  uint64_t id = 0;
  sage_fn_desc d{};
  std::vector<Src> srcs;
  std::vector<uint32_t> blob_first;   // first block index of each blob
  uint32_t n_blocks = 0;
  uint64_t ro_bytes = 0;
  std::vector<uint32_t> cls;          // class of each block (shared mode)
  std::vector<uint32_t> distinct;     // sorted distinct classes
  std::vector<uint64_t> fps;          // fingerprint of each block
  uint64_t* d_table = nullptr;        // device: block -> address
  std::vector<uint64_t> h_table;      // host copy of d_table
  uint64_t table_epoch = ~0ull;
  uint64_t resident_epoch = ~0ull;    // pool eviction epoch at which all classes were resident
  int live = 0;
  Module* mod = nullptr;
  hipEvent_t ready = nullptr;         // data of the function is in place
  std::vector<hipEvent_t> seg;        // progressive reload: layer l's blocks are in place
  std::vector<RegChunk> pre;          // chunks whose fingerprints went out ahead of the registration
  uint32_t block_len(uint32_t b) const;
  const uint8_t* block_src(uint32_t b, bool* dev, bool* pinned = nullptr) const;
};

struct Inv {
  uint64_t id = 0;
  Fn* fn = nullptr;
  uint32_t batch = 0;
  bool live = false;
  void* priv = nullptr;               // private RO copy (share=0)
  uint64_t* priv_table = nullptr;
  void* ws = nullptr;                 // stencil: field-sized scratch
  void* io_in = nullptr;              // staging for host inputs
  void* io_out = nullptr;             // staging for host outputs
  const uint64_t* table() const { return priv_table ? priv_table : fn->d_table; }
};

// ------------------------------------------------------------ in-flight
struct GraphKey {
  std::string kernel;
  uint32_t layers, width;
  bool operator<(const GraphKey& o) const {
    return std::tie(kernel, layers, width) < std::tie(o.kernel, o.layers, o.width);
  }
};

struct Flight {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  // device + pinned mirrors of: header, groups, input row table, output row table
  uint8_t* d_meta = nullptr;
  uint8_t* h_meta = nullptr;
  size_t meta_cap = 0;
  uint8_t* ws = nullptr;             // activations ping-pong
  size_t ws_cap = 0;
  uint8_t* d_in = nullptr;           // packed host inputs
  uint8_t* h_in = nullptr;
  size_t in_cap = 0;
  uint8_t* d_out = nullptr;          // packed outputs for host delivery
  uint8_t* h_out = nullptr;
  size_t out_cap = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  // host delivery after completion
  std::vector<std::pair<void*, std::pair<size_t, size_t>>> deliver;  // host dst, (offset, bytes)
  std::vector<int> timer_tokens;
};

// ------------------------------------------------------------ staging ring
struct Ring {
  size_t slots = 0, chunk = 0;
  std::vector<uint8_t*> host, dev;
  std::vector<uint64_t*> dfp, hfp;
  std::vector<BlkOp*> dops, hops;       // VERIFY (and synchronous) operations
  std::vector<uint32_t*> dres, hres;
  std::vector<BlkOp*> dops_c, hops_c;   // COPY operations left in flight on the control stream
  std::vector<uint32_t*> dres_c;
  std::vector<hipEvent_t> ev;           // fingerprints (then VERIFY results) of the slot's chunk
  std::vector<hipEvent_t> ev_c;         // the slot's last in-flight COPY
  std::vector<uint8_t> held;            // the slot holds a chunk fingerprinted ahead of its registration
  std::vector<size_t> cap;  // blocks the fp/op/result buffers of each slot hold
  size_t ops_cap = 0;
};

struct Serve;  // serving loop state (serve.cpp)

// -------------------------------------------------------------- autotuner
struct TuneEntry {
  std::string kernel;
  double ms;
};

// Long-lived helper thread that runs the code branch of function setup.
// One host copy (bytes from src to dst).
struct HostCopy {
  uint8_t* dst;
  const uint8_t* src;
  size_t n;
};

// Persistent host copy threads: the workers and the calling thread take the
// pieces of one job round robin, and run() returns when all are copied.  One
// job at a time (its callers hold the context's mutex).
class CopyPool {
 public:
  ~CopyPool() { stop(); }
  void start(size_t workers);
  void stop();
  void run(const std::vector<HostCopy>& pieces);

 private:
  void work();
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  const HostCopy* job_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  uint64_t gen_ = 0;
  size_t busy_ = 0;
  bool quit_ = false;
};

class Worker {
 public:
  ~Worker() { stop(); }
  void start(int device);
  void stop();
  void run(std::function<void()> task);  // queue one task
  void wait();                           // until the queued task finished; rethrows its error
 private:
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::function<void()> task_;
  bool has_ = false, done_ = true, quit_ = false;
  std::exception_ptr err_;
};

// ------------------------------------------------------------------ context
constexpr size_t kReloadStageBlocks = 4096;  // reload staging: 256 MiB, cycled by region
constexpr size_t kTimerPairs = 2048;          // event pairs made ready when kernel timing is switched on
// Registration chunk of a device-resident source (SAGE_DEV_CHUNK_BYTES
// overrides it, e.g. for tests that span several chunks).  One launch
// fingerprints a whole chunk: large chunks keep the kernel streaming at HBM
// rate instead of paying a launch and a result copy per 64 MiB.
constexpr uint64_t kDevChunkBytes = 1ull << 30;

struct Ctx {
  int device = 0;
  int cus = 256;
  sage_config cfg{};
  std::recursive_mutex mu;
  hipStream_t ctl = nullptr;                 // control stream
  std::vector<hipStream_t> streams;          // copy / fingerprint streams
  Ring ring;
  Pool pool;
  DevCache cache;
  KernelTimer timer;
  std::map<int, std::unique_ptr<Module>> modules;  // per kind
  std::mutex module_mu;
  std::map<uint64_t, std::unique_ptr<Fn>> fns;
  std::unordered_map<uint64_t, std::unique_ptr<Inv>> invs;
  std::vector<Flight> flights;
  size_t next_flight = 0;
  uint64_t next_id = 1;
  std::map<void*, size_t> pinned;            // sage_host_alloc ranges
  uint64_t* h_stage = nullptr;               // pinned staging for block-table uploads
  hipEvent_t stage_ev = nullptr;             // last upload from h_stage (on ctl)
  hipEvent_t ctl_ev = nullptr;               // marks the control stream for other streams to wait on
  // progressive reloads (cfg.progressive): the last one's function and its
  // completion (on ctl, after every copy stream joined), the copy streams'
  // join markers, pinned op list and staging (the op list's upload marked by
  // prog_ops_ev), and what is released once the last one has completed:
  // host-cache copies that fed it and its device staging
  uint64_t prog_fn = 0;
  uint64_t reload_seq = 0, reload_seq_done = 0;  // progressive reloads issued / known complete
  hipEvent_t reload_done = nullptr;
  std::vector<hipEvent_t> join_ev;
  uint8_t* prog_hops = nullptr;
  size_t prog_hops_cap = 0;
  hipEvent_t prog_ops_ev = nullptr;
  // registration-wide VERIFY / COPY op lists of device-source chunks:
  // pinned and device buffers, reg_ev marking the last upload that reads them
  BlkOp* reg_hops = nullptr;
  BlkOp* reg_dops = nullptr;
  uint32_t* reg_hres = nullptr;
  uint32_t* reg_dres = nullptr;
  size_t reg_cap = 0;
  hipEvent_t reg_ev = nullptr;   // behind the last COPY that reads the lists
  hipEvent_t reg_vev = nullptr;  // behind the last VERIFY results' copy to the host
  // reload staging: device area, one region per batch, each with the event
  // of the batch that last used it; pageable sources go through ring slots
  uint8_t* rstage_dev = nullptr;
  std::vector<hipEvent_t> rstage_ev;
  size_t rstage_next = 0, rhost_next = 0;
  std::vector<std::pair<uint32_t, uint64_t>> deferred_host;  // (class, host generation)
  std::vector<void*> deferred_dev;                           // DevCache buffers
  size_t h_stage_cap = 0;
  std::map<std::string, TuneEntry> tune;     // "width:shape" -> time of one full wave of tiles (ms)
  // counters
  uint64_t logical = 0, h2d = 0, reloads = 0, registrations = 0, invocations = 0, mismatches = 0;
  double t_register = 0, t_code = 0, t_fp_wait = 0, t_dedup = 0, t_verify = 0, t_setup = 0, t_invoke = 0;
  uint64_t host_reloads = 0, module_unloads = 0;
  double t_reload = 0, t_release = 0, t_unregister = 0;
  uint64_t module_loads = 0;                 // under module_mu
  double t_module = 0;                       // under module_mu
  // running serving loop, if any; callers outside the loop thread take a
  // reference under `mu` and keep the state alive while they wait on it
  std::shared_ptr<Serve> serve;
  Worker worker;                             // code branch of fn_register
  CopyPool copier;                           // fill_threads - 1 host copy threads
  std::string force_tile;                    // SAGE_TILE: fixed GEMM tile shape (tests)
  std::string last_launch;                   // kernels and tiles of the last MLP launch
  bool test_fp_const = false;                // force every fingerprint equal (collision test)
  uint64_t dev_chunk = kDevChunkBytes;       // registration chunk of device-resident sources
  AllocFault alloc_fault;                    // SAGE_FAULT_ALLOC_AFTER
  uint32_t f32_cols = 4;                     // output columns per workgroup of the FP32 layer (4, or 8: SAGE_F32_COLS)
  bool stencil_fuse = true;                  // sweeps in passes of two (SAGE_STENCIL_FUSE=0: one per pass)
  uint8_t* na_scratch = nullptr;             // device address of this GPU's fn_invoke_noalloc scratch
  uint8_t* na_hmeta = nullptr;               // pinned host mirror of its metadata part
  uint64_t test_fp_value = 0;

  bool is_pinned(const void* p, size_t n) const;
  int max_groups_stream() const { return cus * 8; }
  int max_groups_copy() const { return cus * 32; }
};

// ------------------------------------------------------------- components
void ring_init(Ctx& c);
void ring_destroy(Ctx& c);
void fill_parallel(Ctx& c, uint8_t* dst, const uint8_t* src, size_t n);
void copy_parallel(Ctx& c, const std::vector<HostCopy>& items);

// Two setup branches: the code branch on `w` (or a new thread when w is
// null), the data branch on the caller; serial runs code then data.
void run_two_branches(const std::function<void()>& code, const std::function<void()>& data, bool serial,
                      Worker* w = nullptr);

Module* load_module(Ctx& c, int kind);     // loads (again) if not loaded
void unload_module(Ctx& c, Module& m);
void advance_exit(Ctx& c);                 // multi-stage exit of idle data and code
void flights_drop_graphs(Ctx& c);          // finish every flight and drop its captured graphs
void register_shared(Ctx& c, Fn& f);
// Fingerprint a device-source function's chunks ahead of its registration
// (fn_register_batch: while the host classifies the previous function).
// The chunks keep their ring slots (held) until register_shared processes
// them.  false (nothing issued) unless sharing is on, every source is on
// the device and enough slots are free.
bool register_prefetch(Ctx& c, Fn& f);
// Give back the slots of a prefetch that will not be registered.
void register_drop_prefetch(Ctx& c, Fn& f);
void copy_private(Ctx& c, Fn& f, uint8_t* dst, hipStream_t s);
void reload_classes(Ctx& c, Fn& f, const std::vector<uint32_t>& missing);
void refresh_table(Ctx& c, Fn& f);
// Progressive reloads: release the host-cache copies of completed ones
// (waiting for the last one first if `wait`); whether f's own reload may
// still be landing, its layers then gated one by one.
void settle_reloads(Ctx& c, bool wait);
// per layer, how many leading classes of a reload (ordered by first block)
// hold every block of layers 0..l
std::vector<size_t> layer_segments(const std::vector<uint32_t>& first, uint32_t layers, uint64_t layer_bytes);
bool reload_landing(Ctx& c, const Fn& f);
bool reload_feeds(Ctx& c, const Fn& f);  // a progressive reload in flight fills a class of f

// grouped execution
struct Call {
  Inv* inv;
  const void* in;
  size_t in_bytes;
  void* out;
  size_t out_bytes;
};
// Caller-provided device metadata / activation buffers and their pinned
// host mirror for the metadata (fn_invoke_noalloc).
struct ExtScratch {
  uint8_t* d_meta;
  uint8_t* h_meta;
  size_t meta_cap;
  uint8_t* ws;
  size_t ws_cap;
};
// Launch a group on flight `flight` (-1: the next one, waiting if busy).
int launch_mlp_group(Ctx& c, const std::vector<Call>& calls, uint32_t io, int flight = -1,
                     const ExtScratch* ext = nullptr);
int launch_stencil_group(Ctx& c, const std::vector<Call>& calls, uint32_t io, int flight = -1);
void finish_flight(Ctx& c, int flight);
void flights_init(Ctx& c);
void flights_destroy(Ctx& c);
void tune_load(Ctx& c);
// Launch plan of a BF16 layer for groups of `rows` under full-wave times
// `tune` on `cus` CUs, as text (host logic only; for self tests).
std::string plan_describe(const std::map<std::string, TuneEntry>& tune, uint32_t cus, uint32_t W,
                          const std::vector<uint32_t>& rows);
std::string tune_key_for(uint32_t width, const std::string& shape);
bool tile_shape_known(const std::string& name);

uint64_t setup_internal(Ctx& c, uint64_t fn, uint32_t batch);
void release_internal(Ctx& c, uint64_t inv);
Fn& find_fn(Ctx& c, uint64_t id);
Inv& find_inv(Ctx& c, uint64_t id);
int free_flight(Ctx& c);  // index of an idle flight, or -1
Ctx& ctx_ref(sage_ctx* p);
void serve_destroy(Ctx& c);

size_t in_elem_size(const sage_fn_desc& d);
size_t in_bytes_for(const sage_fn_desc& d, uint32_t batch);
size_t out_bytes_for(const sage_fn_desc& d, uint32_t batch);
uint64_t ro_bytes_for(const sage_fn_desc& d);

}  // namespace sage
