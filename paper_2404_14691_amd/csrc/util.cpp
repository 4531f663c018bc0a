// Errors, device-memory cache, event timing and the two-branch setup
// orchestrator.
#include <chrono>
#include <cstdarg>
#include <cstring>

#include "internal.h"

namespace sage {

static thread_local std::string t_last_error;

void set_last_error(const std::string& msg) { t_last_error = msg; }
const std::string& last_error() { return t_last_error; }

void fail(sage_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error{st, buf};
}

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) fail(SAGE_EHIP, "%s: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

sage_status guard(const std::function<void()>& body) {
  try {
    body();
    return SAGE_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return SAGE_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SAGE_EINVAL;
  }
}

// ------------------------------------------------------------ DevCache
size_t DevCache::round(size_t n) {
  if (n <= (1u << 20)) {
    size_t r = 4096;
    while (r < n) r <<= 1;
    return r;
  }
  const size_t mb = 1u << 20;
  return (n + mb - 1) / mb * mb;
}

void* DevCache::get(size_t n) {
  const size_t r = round(n ? n : 1);
  auto it = free_.find(r);
  void* p = nullptr;
  if (it != free_.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
  } else {
    hipError_t e = fault && fault->fail_now() ? hipErrorOutOfMemory : hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // give cached blocks back to HIP and retry once
      for (auto& kv : free_)
        for (void* q : kv.second) {
          (void)hipFree(q);
          held_ -= kv.first;
        }
      free_.clear();
      e = fault && fault->fail_now() ? hipErrorOutOfMemory : hipMalloc(&p, r);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(SAGE_ENOMEM, "device allocation of %zu bytes failed", r);
      }
    }
    held_ += r;
  }
  live_[p] = r;
  in_use_ += r;
  return p;
}

void DevCache::put(void* p) {
  if (!p) return;
  auto it = live_.find(p);
  if (it == live_.end()) return;
  free_[it->second].push_back(p);
  in_use_ -= it->second;
  live_.erase(it);
}

void DevCache::release_all() {
  for (auto& kv : free_)
    for (void* q : kv.second) (void)hipFree(q);
  for (auto& kv : live_) (void)hipFree(kv.first);
  free_.clear();
  live_.clear();
  held_ = in_use_ = 0;
}

// ---------------------------------------------------------- KernelTimer
int KernelTimer::add_pair() {
  Pair p{};
  HIPX(hipEventCreate(&p.a));
  HIPX(hipEventCreate(&p.b));
  pairs_.push_back(p);
  return (int)pairs_.size() - 1;
}

void KernelTimer::reserve(size_t n) {
  while (pairs_.size() < n) free_.push_back(add_pair());
}

int KernelTimer::start(const char* name, hipStream_t s, uint32_t launches) {
  if (!on || (!only.empty() && only != name)) return -1;
  if (free_.empty()) collect();  // pairs whose interval completed come back
  int tok;
  if (!free_.empty()) {
    tok = free_.back();
    free_.pop_back();
  } else {
    tok = add_pair();
  }
  Pair& p = pairs_[tok];
  p.busy = true;
  p.name = name;
  p.launches = launches;
  HIPX(hipEventRecord(p.a, s));
  return tok;
}

void KernelTimer::stop(int tok, hipStream_t s) {
  if (tok < 0) return;
  HIPX(hipEventRecord(pairs_[tok].b, s));
}

void KernelTimer::collect() {
  for (auto& p : pairs_) {
    if (!p.busy) continue;
    if (hipEventQuery(p.b) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    float ms = 0.f;
    HIPX(hipEventElapsedTime(&ms, p.a, p.b));
    auto& a = acc_[p.name];
    a.first += ms;
    a.second += p.launches;
    p.busy = false;
    free_.push_back((int)(&p - pairs_.data()));
  }
}

void KernelTimer::reset() {
  collect();
  acc_.clear();
}

bool KernelTimer::get(const std::string& name, double* ms, uint64_t* n) {
  collect();
  auto it = acc_.find(name);
  if (it == acc_.end()) {
    *ms = 0;
    *n = 0;
    return false;
  }
  *ms = it->second.first;
  *n = it->second.second;
  return true;
}

void KernelTimer::destroy() {
  for (auto& p : pairs_) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pairs_.clear();
  free_.clear();
}

// ------------------------------------------------------ setup branches
// Parallelized function setup: the code branch (module load, allocation)
// and the data branch run at the same time; compute starts when both are
// done.  With `serial`, code first, then data (the one-after-the-other
// baseline).  An error in either branch is rethrown after both finished.
void Worker::start(int device) {
  quit_ = false;
  th_ = std::thread([this, device] {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return has_ || quit_; });
      if (quit_) return;
      auto task = std::move(task_);
      has_ = false;
      lk.unlock();
      std::exception_ptr e;
      try {
        task();
      } catch (...) {
        e = std::current_exception();
      }
      lk.lock();
      err_ = e;
      done_ = true;
      cv_.notify_all();
    }
  });
}

void Worker::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    quit_ = true;
  }
  cv_.notify_all();
  if (th_.joinable()) th_.join();
}

void Worker::run(std::function<void()> task) {
  std::lock_guard<std::mutex> lk(mu_);
  task_ = std::move(task);
  has_ = true;
  done_ = false;
  err_ = nullptr;
  cv_.notify_all();
}

void Worker::wait() {
  std::unique_lock<std::mutex> lk(mu_);
  cv_.wait(lk, [&] { return done_; });
  if (err_) {
    auto e = err_;
    err_ = nullptr;
    std::rethrow_exception(e);
  }
}

// ------------------------------------------------------ host copy threads
void CopyPool::start(size_t workers) {
  quit_ = false;
  for (size_t i = 0; i < workers; i++)
    th_.emplace_back([this] {
      uint64_t seen = 0;
      for (;;) {
        {
          std::unique_lock<std::mutex> lk(mu_);
          cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
          if (quit_) return;
          seen = gen_;
        }
        work();
        std::lock_guard<std::mutex> lk(mu_);
        if (--busy_ == 0) done_.notify_all();
      }
    });
}

void CopyPool::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    quit_ = true;
  }
  cv_.notify_all();
  for (auto& t : th_)
    if (t.joinable()) t.join();
  th_.clear();
}

void CopyPool::work() {
  for (size_t q; (q = next_.fetch_add(1)) < n_;) std::memcpy(job_[q].dst, job_[q].src, job_[q].n);
}

void CopyPool::run(const std::vector<HostCopy>& pieces) {
  if (th_.empty() || pieces.size() < 2) {
    for (const HostCopy& p : pieces) std::memcpy(p.dst, p.src, p.n);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    job_ = pieces.data();
    n_ = pieces.size();
    next_ = 0;
    busy_ = th_.size();
    gen_++;
  }
  cv_.notify_all();
  work();
  std::unique_lock<std::mutex> lk(mu_);
  done_.wait(lk, [&] { return busy_ == 0; });
  job_ = nullptr;
  n_ = 0;
}

void run_two_branches(const std::function<void()>& code, const std::function<void()>& data, bool serial,
                      Worker* w) {
  if (serial) {
    code();
    data();
    return;
  }
  if (w) {
    w->run(code);
    std::exception_ptr data_err;
    try {
      data();
    } catch (...) {
      data_err = std::current_exception();
    }
    if (data_err) {
      try {
        w->wait();
      } catch (...) {
      }
      std::rethrow_exception(data_err);
    }
    w->wait();
    return;
  }
  std::exception_ptr code_err;
  std::thread th([&] {
    try {
      code();
    } catch (...) {
      code_err = std::current_exception();
    }
  });
  std::exception_ptr data_err;
  try {
    data();
  } catch (...) {
    data_err = std::current_exception();
  }
  th.join();
  if (data_err) std::rethrow_exception(data_err);
  if (code_err) std::rethrow_exception(code_err);
}

}  // namespace sage

using namespace sage;

extern "C" sage_status sage_selftest_setup_overlap(double load_ms, double host_ms, double copy_ms, int serial,
                                                   double* measured_ms) {
  return guard([&] {
    if (!measured_ms || load_ms < 0 || host_ms < 0 || copy_ms < 0) fail(SAGE_EINVAL, "bad arguments");
    auto sleep_ms = [](double ms) {
      std::this_thread::sleep_for(std::chrono::microseconds((long long)(ms * 1000.0)));
    };
    const auto t0 = std::chrono::steady_clock::now();
    run_two_branches([&] { sleep_ms(load_ms); },
                     [&] {
                       sleep_ms(host_ms);
                       sleep_ms(copy_ms);
                     },
                     serial != 0);
    const auto t1 = std::chrono::steady_clock::now();
    *measured_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  });
}
