// Serving loop: requests arrive at any time (sage_submit); one internal
// thread admits them (fn_setup: reload + references, evicting unreferenced
// blocks when the pool is full), packs every admitted request of one body
// shape into the next grouped launch, and keeps up to `inflight_groups`
// launches on the device while new arrivals queue for the following one
// (continuous batching).  A finished launch releases its invocations and
// records setup and end-to-end latency per request.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace sage {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t id = 0, fn = 0, inv = 0;
  uint32_t batch = 0, io = 0;
  const void* in = nullptr;
  void* out = nullptr;
  size_t in_bytes = 0, out_bytes = 0;
  Clock::time_point t_arr, t_setup, t_done;
  sage_status st = SAGE_OK;
  std::string err;
  bool done = false;
};

struct Serve {
  std::thread th;
  bool running = false, stop = false;
  std::mutex qmu;
  std::condition_variable qcv, donecv;
  std::deque<std::shared_ptr<Req>> incoming;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
  std::vector<double> setup_ms, e2e_ms;
  uint64_t completed = 0, failed = 0, launches = 0, rows = 0;
  Clock::time_point t_first, t_last;
  bool any = false;
  uint32_t max_rows = 8192;
  std::once_flag joined;  // the loop thread is joined once, whoever stops it
};

static double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// Requests whose bodies can share one launch.
static bool same_shape(Ctx& c, const Req& a, const Req& b) {
  if (a.io != b.io) return false;
  const sage_fn_desc& x = find_fn(c, a.fn).d;
  const sage_fn_desc& y = find_fn(c, b.fn).d;
  if (x.kind != y.kind) return false;
  if (is_grid(x.kind)) return a.fn == b.fn;
  return x.width == y.width && x.layers == y.layers;
}

static void finish_req(Serve& S, const std::shared_ptr<Req>& r) {
  r->t_done = Clock::now();
  r->done = true;
  if (r->st == SAGE_OK) {
    S.completed++;
    S.setup_ms.push_back(ms_between(r->t_arr, r->t_setup));
    S.e2e_ms.push_back(ms_between(r->t_arr, r->t_done));
    S.t_last = r->t_done;
  } else {
    S.failed++;
  }
}

static void serve_loop(Ctx& c, Serve& S) {
  (void)hipSetDevice(c.device);
  std::deque<std::shared_ptr<Req>> pending;
  std::vector<std::vector<std::shared_ptr<Req>>> inflight(c.flights.size());
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S.qmu);
      const bool idle = pending.empty() &&
                        std::all_of(inflight.begin(), inflight.end(), [](auto& v) { return v.empty(); });
      if (idle && S.incoming.empty()) {
        if (S.stop) break;
        S.qcv.wait_for(lk, std::chrono::milliseconds(2));
      }
      while (!S.incoming.empty()) {
        pending.push_back(std::move(S.incoming.front()));
        S.incoming.pop_front();
      }
    }
    bool progressed = false;
    std::vector<std::shared_ptr<Req>> finished;
    {
      std::lock_guard<std::recursive_mutex> lk(c.mu);
      // completions
      for (size_t f = 0; f < inflight.size(); f++) {
        if (inflight[f].empty()) continue;
        const hipError_t q = hipEventQuery(c.flights[f].done);
        if (q == hipErrorNotReady) continue;
        sage_status st = SAGE_OK;
        std::string msg;
        st = guard([&] {
          HIPX(q);
          finish_flight(c, (int)f);
        });
        if (st != SAGE_OK) msg = last_error();
        for (auto& r : inflight[f]) {
          if (st != SAGE_OK) {
            r->st = st;
            r->err = msg;
          }
          (void)guard([&] { release_internal(c, r->inv); });
          c.invocations++;
          finished.push_back(r);
        }
        inflight[f].clear();
        progressed = true;
      }
      // admission + launch while an idle flight exists
      for (;;) {
        if (pending.empty()) break;
        int fl = -1;
        for (size_t f = 0; f < inflight.size(); f++)
          if (inflight[f].empty() && !c.flights[f].busy) {
            fl = (int)f;
            break;
          }
        if (fl < 0) break;
        const bool device_idle =
            std::all_of(inflight.begin(), inflight.end(), [](auto& v) { return v.empty(); });
        std::vector<std::shared_ptr<Req>> group;
        std::vector<Call> calls;
        uint32_t rows = 0;
        const Req* key = nullptr;
        // Residency-aware order: the oldest admissible request leads the
        // launch whatever it costs; the others join only while their
        // function's read-only data is all resident, so one launch triggers
        // at most one reload and a cold function's requests wait to be
        // served together by one reload instead of each evicting the others'
        // blocks (cache replacement with the processing order adjusted,
        // section "Other Lessons Learned").
        std::unordered_map<uint64_t, bool> warm;
        uint64_t warm_epoch = c.pool.epoch;
        auto is_warm = [&](uint64_t id) {
          if (!c.cfg.share) return true;
          if (warm_epoch != c.pool.epoch) {
            warm.clear();
            warm_epoch = c.pool.epoch;
          }
          auto it = warm.find(id);
          if (it != warm.end()) return it->second;
          const Fn& f = find_fn(c, id);
          bool w = f.live > 0 || f.resident_epoch == c.pool.epoch;
          if (!w) {
            w = true;
            for (uint32_t cl : f.distinct)
              if (c.pool.cls[cl].slot == kNone) {
                w = false;
                break;
              }
          }
          warm.emplace(id, w);
          return w;
        };
        for (auto it = pending.begin(); it != pending.end();) {
          Req& r = **it;
          bool drop = false;
          if (!c.fns.count(r.fn)) {
            // unregistered while it was queued: it can never be admitted
            r.st = SAGE_ENOTFOUND;
            r.err = "function " + std::to_string(r.fn) + " was unregistered while the request was queued";
            drop = true;
          } else if (!key || (same_shape(c, *key, r) && rows + r.batch <= S.max_rows && is_warm(r.fn))) {
            const sage_status st = guard([&] { r.inv = setup_internal(c, r.fn, r.batch); });
            if (st == SAGE_OK) {
              r.t_setup = Clock::now();
              if (!key) key = &r;
              rows += r.batch;
              calls.push_back(Call{&find_inv(c, r.inv), r.in, r.in_bytes, r.out, r.out_bytes});
              group.push_back(*it);
              it = pending.erase(it);
              continue;
            }
            // admission failed: wait for releases, unless nothing can ever free memory
            if (st != SAGE_ENOMEM || (device_idle && group.empty() && it == pending.begin())) {
              r.st = st;
              r.err = last_error();
              drop = true;
            }
          }
          if (drop) {
            finished.push_back(*it);
            it = pending.erase(it);
            continue;
          }
          ++it;
        }
        if (group.empty()) break;
        const uint32_t io = group[0]->io;
        const bool stencil = is_grid(find_fn(c, group[0]->fn).d.kind);
        const sage_status st = guard([&] {
          if (stencil) launch_stencil_group(c, calls, io, fl);
          else launch_mlp_group(c, calls, io, fl);
        });
        S.launches++;
        S.rows += rows;
        if (st != SAGE_OK) {
          const std::string msg = last_error();
          for (auto& r : group) {
            r->st = st;
            r->err = msg;
            (void)guard([&] { release_internal(c, r->inv); });
            finished.push_back(r);
          }
        } else {
          inflight[fl] = std::move(group);
        }
        progressed = true;
      }
    }
    if (!finished.empty()) {
      std::lock_guard<std::mutex> lk(S.qmu);
      for (auto& r : finished) finish_req(S, r);
      S.donecv.notify_all();
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// A reference to the running loop's state, taken under the context mutex;
// it stays valid while the caller waits on it, even across a concurrent stop.
static std::shared_ptr<Serve> serve_of(Ctx& c) {
  std::lock_guard<std::recursive_mutex> lk(c.mu);
  if (!c.serve) fail(SAGE_ESTATE, "serving loop not started");
  return c.serve;
}

// Stop the loop: new submissions are refused, queued and in-flight requests
// drain, then the thread is joined.  The context keeps the loop's state until
// the join, so fn_invoke stays refused while the loop still owns the flights.
void serve_destroy(Ctx& c) {
  std::shared_ptr<Serve> sp;
  {
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    sp = c.serve;
  }
  if (!sp) return;
  {
    std::lock_guard<std::mutex> lk(sp->qmu);
    sp->stop = true;
  }
  sp->qcv.notify_all();
  std::call_once(sp->joined, [&] {
    if (sp->th.joinable()) sp->th.join();
  });
  std::lock_guard<std::recursive_mutex> lk(c.mu);
  if (c.serve == sp) c.serve.reset();
}

static double pct(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(q / 100.0 * v.size());
  if (k < 1) k = 1;
  return v[k - 1];
}

}  // namespace sage

using namespace sage;

extern "C" {

sage_status sage_serve_start(sage_ctx* p, uint32_t max_rows) {
  return guard([&] {
    Ctx& c = ctx_ref(p);
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    if (c.serve) fail(SAGE_ESTATE, "serving loop already running");
    auto sp = std::make_shared<Serve>();
    Serve* S = sp.get();
    if (max_rows) S->max_rows = max_rows;
    S->running = true;
    c.serve = sp;
    S->th = std::thread([&c, S] { serve_loop(c, *S); });
  });
}

sage_status sage_serve_stop(sage_ctx* p) {
  return guard([&] {
    Ctx& c = ctx_ref(p);
    (void)serve_of(c);  // ESTATE when not running
    serve_destroy(c);
  });
}

sage_status sage_submit(sage_ctx* p, sage_fn fn, uint32_t batch, const void* in, size_t in_bytes, void* out,
                        size_t out_bytes, uint32_t io_flags, uint64_t* req_id) {
  return guard([&] {
    Ctx& c = ctx_ref(p);
    if (!req_id || !in || !out) fail(SAGE_EINVAL, "null argument");
    auto r = std::make_shared<Req>();
    r->t_arr = Clock::now();
    std::shared_ptr<Serve> sp;
    {
      std::lock_guard<std::recursive_mutex> lk(c.mu);
      sp = serve_of(c);
      const Fn& f = find_fn(c, fn);
      if (batch < 1 || in_bytes != in_bytes_for(f.d, batch) || out_bytes != out_bytes_for(f.d, batch))
        fail(SAGE_EINVAL, "request sizes do not match the function");
      if (((io_flags & SAGE_IO_DEVICE_IN) && ((uintptr_t)in & 15)) ||
          ((io_flags & SAGE_IO_DEVICE_OUT) && ((uintptr_t)out & 15)))
        fail(SAGE_EINVAL, "device buffers must be 16-byte aligned");
      r->id = c.next_id++;
    }
    r->fn = fn;
    r->batch = batch;
    r->in = in;
    r->in_bytes = in_bytes;
    r->out = out;
    r->out_bytes = out_bytes;
    r->io = io_flags;
    Serve& S = *sp;
    {
      std::lock_guard<std::mutex> lk(S.qmu);
      if (S.stop) fail(SAGE_ESTATE, "serving loop is stopping");
      if (!S.any) {
        S.any = true;
        S.t_first = r->t_arr;
      }
      S.reqs[r->id] = r;
      S.incoming.push_back(r);
    }
    S.qcv.notify_one();
    *req_id = r->id;
  });
}

sage_status sage_wait(sage_ctx* p, uint64_t req_id, double timeout_ms, sage_req_info* info) {
  Ctx* cp = &ctx_ref(p);
  std::shared_ptr<Req> r;
  sage_status st = guard([&] {
    const std::shared_ptr<Serve> sp = serve_of(*cp);
    Serve& S = *sp;
    std::unique_lock<std::mutex> lk(S.qmu);
    auto it = S.reqs.find(req_id);
    if (it == S.reqs.end()) fail(SAGE_ENOTFOUND, "unknown request %llu", (unsigned long long)req_id);
    r = it->second;
    const auto pred = [&] { return r->done; };
    if (timeout_ms < 0) S.donecv.wait(lk, pred);
    else if (!S.donecv.wait_for(lk, std::chrono::microseconds((long long)(timeout_ms * 1000)), pred))
      fail(SAGE_EBUSY, "request %llu not finished", (unsigned long long)req_id);
    S.reqs.erase(it);
    if (info) {
      info->setup_ms = r->st == SAGE_OK ? ms_between(r->t_arr, r->t_setup) : 0.0;
      info->e2e_ms = ms_between(r->t_arr, r->t_done);
      info->status = r->st;
    }
  });
  if (st == SAGE_OK && r && r->st != SAGE_OK) {
    set_last_error(r->err);
    return r->st;
  }
  return st;
}

sage_status sage_serve_stats(sage_ctx* p, sage_serve_report* out) {
  return guard([&] {
    Ctx& c = ctx_ref(p);
    if (!out) fail(SAGE_EINVAL, "null output");
    const std::shared_ptr<Serve> sp = serve_of(c);
    Serve& S = *sp;
    std::lock_guard<std::mutex> lk(S.qmu);
    std::memset(out, 0, sizeof *out);
    out->completed = S.completed;
    out->failed = S.failed;
    out->launches = S.launches;
    out->rows = S.rows;
    out->setup_p50_ms = pct(S.setup_ms, 50);
    out->setup_p99_ms = pct(S.setup_ms, 99);
    out->e2e_p50_ms = pct(S.e2e_ms, 50);
    out->e2e_p99_ms = pct(S.e2e_ms, 99);
    const double span = S.completed ? ms_between(S.t_first, S.t_last) : 0.0;
    out->span_ms = span;
    out->throughput = span > 0 ? S.completed / (span * 1e-3) : 0.0;
  });
}

sage_status sage_serve_reset_stats(sage_ctx* p) {
  return guard([&] {
    Ctx& c = ctx_ref(p);
    const std::shared_ptr<Serve> sp = serve_of(c);
    Serve& S = *sp;
    std::lock_guard<std::mutex> lk(S.qmu);
    S.setup_ms.clear();
    S.e2e_ms.clear();
    S.completed = S.failed = S.launches = S.rows = 0;
    S.any = false;
  });
}

}  // extern "C"
