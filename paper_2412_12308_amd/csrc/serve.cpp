// serve.cpp -- the request server: a scheduler thread with first-come
// first-served admission by HBM budget and free slots, iteration-level
// continuous batching over the running requests, per-request resident
// spectra, latency statistics; a HIP backend and a host backend (for testing
// the scheduler without a GPU); the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fftpde.h"
#include "context.hpp"
#include "diag.hpp"
#include "serve.hpp"
#include "solve.hpp"

using namespace fftpde;

namespace {

enum { kQueued = 0, kRunning = 1, kEnded = 2 };
constexpr int kChunk = kDiagMaxTimes;  // steps of diagnostics per iteration (one launch)
constexpr long long kHostPoolMax = 1ll << 30;
constexpr int kHostStreams = 2;

int ilog2s(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}
size_t up256(size_t x) { return (x + 255) / 256 * 256; }

struct Req {
  unsigned long long id = 0;
  fftpde_request r{};
  int state = kQueued;
  int status = FFTPDE_PENDING;
  double t_submit = 0, t_admit = -1, t_done = -1;
  long long footprint = 0;  // bytes charged while running
  // pool blocks: work (spectra, scratch) and a server-owned output
  size_t work_bytes = 0, out_bytes = 0;
  size_t work_off = Pool::kNone, out_off = Pool::kNone;
  void* F = nullptr;
  void* G = nullptr;
  double* scratch = nullptr;
  void* out = nullptr;
  int stream = 0;
  long long next_step = 1;
  bool started = false, enq_done = false;
  int fail = FFTPDE_OK;      // first error of the work issued
  std::atomic<int> abort{0}; // FFTPDE_ECANCELED / FFTPDE_ETIMEOUT once asked
  hipEvent_t done_ev = nullptr;
  hipEvent_t dep_ev = nullptr;  // recorded on the caller's stream at submission
  std::atomic<int> host_done{0}, host_rc{0};  // host backend
};

// ---------------------------------------------------------------------------
// backends
// ---------------------------------------------------------------------------
struct Backend {
  virtual ~Backend() = default;
  virtual char* pool_base() = 0;
  virtual void thread_init() {}
  virtual int depend(Req&, void* /*stream*/) { return FFTPDE_OK; }
  virtual int admit(Req&) { return FFTPDE_OK; }
  virtual int start(Req&) = 0;                          // Poisson: the whole solve
  virtual int steps(Req&, long long n0, int nt) = 0;    // diagnostics at t_n0 .. t_(n0+nt-1)
  virtual int finish(Req&) = 0;                         // u(T) into out (evolutions)
  virtual void mark(Req&) {}                            // completion marker after the work issued
  virtual int query(Req&) = 0;                          // OK, PENDING or an error
  virtual double done_time(Req&, double now) { return now; }
  virtual void retire(Req&) {}
  // Iterations are paced two deep: iteration i+1 is issued once iteration
  // i-1 has finished on every stream (ready() polls; mark() ends an iteration).
  virtual bool ready() { return true; }
  virtual void mark_iteration() {}
  virtual int copy(void* dst, const void* src, size_t bytes, void* stream) = 0;
  virtual void drain() {}
};

class HipBackend : public Backend {
 public:
  int init(int device, long long budget, int nstreams, double now) {
    device_ = device;
    if (hipSetDevice(device) != hipSuccess) return FFTPDE_EDEVICE;
    int rc = fftpde_create(&own_, device);
    if (rc != FFTPDE_OK) return rc;
    c_ = reinterpret_cast<Context*>(own_);
    hipError_t e = hipMalloc(&pool_, (size_t)budget);
    if (e != hipSuccess) {
      set_last_error("server pool", e);
      return e == hipErrorOutOfMemory ? FFTPDE_ENOMEM : FFTPDE_EDEVICE;
    }
    streams_.resize(nstreams, nullptr);
    prev_.resize(nstreams, nullptr);
    cur_.resize(nstreams, nullptr);
    for (int i = 0; i < nstreams; i++) {
      if (hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&prev_[i], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&cur_[i], hipEventDisableTiming) != hipSuccess)
        return FFTPDE_EDEVICE;
    }
    // reference event: device timestamps of completions map to the host clock
    if (hipEventCreate(&ref_) != hipSuccess || hipEventRecord(ref_, streams_[0]) != hipSuccess ||
        hipEventSynchronize(ref_) != hipSuccess)
      return FFTPDE_EDEVICE;
    t_ref_ = now;
    return FFTPDE_OK;
  }
  ~HipBackend() override {
    (void)hipSetDevice(device_);
    (void)hipDeviceSynchronize();
    for (auto e : events_) (void)hipEventDestroy(e);
    for (auto e : prev_)
      if (e) (void)hipEventDestroy(e);
    for (auto e : cur_)
      if (e) (void)hipEventDestroy(e);
    if (ref_) (void)hipEventDestroy(ref_);
    for (auto s : streams_)
      if (s) (void)hipStreamDestroy(s);
    if (pool_) (void)hipFree(pool_);
    if (own_) fftpde_destroy(own_);
  }
  void set_ref_time(double t) { t_ref_ = t; }
  char* pool_base() override { return static_cast<char*>(pool_); }
  void thread_init() override { (void)hipSetDevice(device_); }
  hipEvent_t take_event() {
    if (!events_.empty()) {
      hipEvent_t e = events_.back();
      events_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
  int depend(Req& q, void* stream) override {
    if (!stream) return FFTPDE_OK;
    q.dep_ev = take_event();
    if (!q.dep_ev) return FFTPDE_EDEVICE;
    const hipError_t e = hipEventRecord(q.dep_ev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
      set_last_error("server submit", e);
      return FFTPDE_EDEVICE;
    }
    return FFTPDE_OK;
  }
  int admit(Req& q) override {
    q.done_ev = take_event();
    return q.done_ev ? FFTPDE_OK : FFTPDE_EDEVICE;
  }
  int start(Req& q) override {
    const fftpde_request& r = q.r;
    hipStream_t s = streams_[q.stream];
    if (q.dep_ev && hipStreamWaitEvent(s, q.dep_ev, 0) != hipSuccess) return FFTPDE_EDEVICE;
    if (r.op == FFTPDE_POISSON) {
      // the spectrum between the passes goes to the request's pool block, so
      // the solve neither allocates nor escapes the budget
      SolveScratch sc;
      sc.p = q.F;
      sc.bytes = q.work_bytes;
      return run_solve(c_, r.dtype, FFTPDE_POISSON, r.in, nullptr, q.out, nullptr, r.nx, r.ny, 1, r.lx, r.ly, 0.0,
                       0.0, s, sc);
    }
    int rc = run_transform(c_, r.dtype, false, r.in, q.F, r.nx, r.ny, 1, s);
    if (rc == FFTPDE_OK && q.G) rc = run_transform(c_, r.dtype, false, r.v0, q.G, r.nx, r.ny, 1, s);
    return rc;
  }
  int steps(Req& q, long long n0, int nt) override {
    const fftpde_request& r = q.r;
    return run_diag(c_, r.dtype, r.op, q.F, q.G, r.nx, r.ny, 1, r.lx, r.ly, r.coef, n0, r.dt, nt, q.scratch,
                    r.diag + 3 * (n0 - 1), streams_[q.stream]);
  }
  int finish(Req& q) override {
    const fftpde_request& r = q.r;
    if (r.op == FFTPDE_POISSON) return FFTPDE_OK;
    return run_materialize(c_, r.dtype, r.op, q.F, q.G, q.out, nullptr, r.nx, r.ny, 1, r.lx, r.ly, r.coef,
                           (double)r.steps * r.dt, streams_[q.stream]);
  }
  void mark(Req& q) override { (void)hipEventRecord(q.done_ev, streams_[q.stream]); }
  int query(Req& q) override {
    const hipError_t e = hipEventQuery(q.done_ev);
    if (e == hipSuccess) return FFTPDE_OK;
    if (e == hipErrorNotReady) return FFTPDE_PENDING;
    set_last_error("server request", e);
    return FFTPDE_EDEVICE;
  }
  double done_time(Req& q, double now) override {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ref_, q.done_ev) != hipSuccess) return now;
    const double t = t_ref_ + ms * 1e-3;
    return t < now ? t : now;
  }
  void retire(Req& q) override {
    if (q.done_ev) events_.push_back(q.done_ev);
    if (q.dep_ev) events_.push_back(q.dep_ev);
    q.done_ev = q.dep_ev = nullptr;
  }
  // cur_: where each stream was at the end of the last iteration; prev_: at
  // the end of the one before.
  bool ready() override {
    if (!have_prev_) return true;
    for (auto e : prev_)
      if (hipEventQuery(e) == hipErrorNotReady) return false;
    return true;
  }
  void mark_iteration() override {
    std::swap(prev_, cur_);
    for (size_t i = 0; i < streams_.size(); i++) (void)hipEventRecord(cur_[i], streams_[i]);
    have_prev_ = have_cur_;
    have_cur_ = true;
  }
  void drain() override {
    for (auto s : streams_) (void)hipStreamSynchronize(s);
  }
  int copy(void* dst, const void* src, size_t bytes, void* stream) override {
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
      set_last_error("server copy", e);
      return FFTPDE_EDEVICE;
    }
    return FFTPDE_OK;
  }

 private:
  int device_ = 0;
  fftpde_ctx* own_ = nullptr;
  Context* c_ = nullptr;
  void* pool_ = nullptr;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> prev_, cur_, events_;
  bool have_prev_ = false, have_cur_ = false;
  hipEvent_t ref_ = nullptr;
  double t_ref_ = 0.0;
};

// Host backend: each "stream" is a worker thread that runs its tasks in order
// (start, steps, final field, completion marker), so the scheduler never
// blocks on the work itself -- as with device streams.
class HostBackend : public Backend {
 public:
  HostBackend(fftpde_host_exec fn, void* user, size_t bytes, int nstreams) : fn_(fn), user_(user) {
    mem_ = static_cast<char*>(std::malloc(bytes ? bytes : 1));
    for (int i = 0; i < nstreams; i++) {
      workers_.emplace_back(new Worker());
      Worker* w = workers_.back().get();
      w->th = std::thread([this, w] { run(w); });
    }
  }
  ~HostBackend() override {
    for (auto& w : workers_) {
      {
        std::lock_guard<std::mutex> lk(w->m);
        w->stop = true;
      }
      w->cv.notify_all();
      w->th.join();
    }
    std::free(mem_);
  }
  bool ok() const { return mem_ != nullptr; }
  char* pool_base() override { return mem_; }
  int start(Req& q) override { return push(q, 0, 0, 0); }
  int steps(Req& q, long long n0, int nt) override { return push(q, 1, n0, nt); }
  int finish(Req& q) override { return push(q, 2, q.r.steps, 0); }
  void mark(Req& q) override { (void)push(q, 3, 0, 0); }
  bool ready() override {
    for (auto& w : workers_)
      if (w->iter_done.load() + 1 < iter_) return false;
    return true;
  }
  void mark_iteration() override {
    iter_++;
    for (auto& w : workers_) {
      {
        std::lock_guard<std::mutex> lk(w->m);
        w->tasks.push_back({nullptr, 4, iter_, 0});
      }
      w->cv.notify_one();
    }
  }
  int query(Req& q) override {
    if (!q.host_done.load()) return FFTPDE_PENDING;
    const int rc = q.host_rc.load();
    return rc == 0 ? FFTPDE_OK : rc;
  }
  int copy(void* dst, const void* src, size_t bytes, void*) override {
    std::memcpy(dst, src, bytes);
    return FFTPDE_OK;
  }

 private:
  struct Task {
    Req* q;
    int phase;  // 0 start, 1 steps, 2 final field, 3 completion marker, 4 end of iteration n0
    long long n0;
    int nt;
  };
  struct Worker {
    std::thread th;
    std::mutex m;
    std::condition_variable cv;
    std::deque<Task> tasks;
    bool stop = false;
    std::atomic<long long> iter_done{0};
  };
  int push(Req& q, int phase, long long n0, int nt) {
    Worker* w = workers_[q.stream % workers_.size()].get();
    {
      std::lock_guard<std::mutex> lk(w->m);
      w->tasks.push_back({&q, phase, n0, nt});
    }
    w->cv.notify_one();
    return FFTPDE_OK;
  }
  void run(Worker* w) {
    while (true) {
      Task t;
      {
        std::unique_lock<std::mutex> lk(w->m);
        w->cv.wait(lk, [w] { return w->stop || !w->tasks.empty(); });
        if (w->tasks.empty()) return;  // stop requested and nothing left
        t = w->tasks.front();
        w->tasks.pop_front();
      }
      Req* q = t.q;
      if (t.phase == 4) {
        w->iter_done.store(t.n0);
      } else if (t.phase == 3) {
        q->host_done.store(1);
      } else if (q->host_rc.load() == 0) {  // a failed request runs nothing more
        const int rc = fn_(user_, q->id, &q->r, q->out, t.phase, t.n0, t.nt);
        if (rc != 0) q->host_rc.store(rc < 0 ? rc : FFTPDE_EDEVICE);
      }
    }
  }
  fftpde_host_exec fn_;
  void* user_;
  char* mem_ = nullptr;
  std::vector<std::unique_ptr<Worker>> workers_;
  long long iter_ = 0;  // iterations marked (scheduler thread only)
};

// ---------------------------------------------------------------------------
// request checks and sizes
// ---------------------------------------------------------------------------
bool side_ok(int n) { return n >= 2 && n <= 4096 && (n & (n - 1)) == 0; }

int check_request(const fftpde_request& r) {
  if (r.op != FFTPDE_POISSON && r.op != FFTPDE_DIFFUSION && r.op != FFTPDE_WAVE) return FFTPDE_EINVAL;
  if (r.dtype != FFTPDE_C64 && r.dtype != FFTPDE_C128) return FFTPDE_EINVAL;
  if (!side_ok(r.nx) || !side_ok(r.ny)) return FFTPDE_EINVAL;
  if (!(std::isfinite(r.lx) && r.lx > 0 && std::isfinite(r.ly) && r.ly > 0)) return FFTPDE_EINVAL;
  if (r.steps < 1 || r.steps > (1ll << 40)) return FFTPDE_EINVAL;
  if (!r.in) return FFTPDE_EINVAL;
  if (r.flags & ~FFTPDE_REQ_AUTORELEASE) return FFTPDE_EINVAL;
  if (std::isnan(r.deadline)) return FFTPDE_EINVAL;
  const uintptr_t al = r.dtype == FFTPDE_C64 ? 8 : 16;
  auto mis = [&](const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & (al - 1)); };
  if (mis(r.in) || mis(r.v0) || mis(r.out) || (r.diag && (reinterpret_cast<uintptr_t>(r.diag) & 7)))
    return FFTPDE_EINVAL;
  if (r.op == FFTPDE_POISSON) {
    if (r.steps != 1 || r.v0 || r.diag) return FFTPDE_EINVAL;
  } else {
    const double T = (double)r.steps * r.dt;
    if (!(std::isfinite(r.coef) && r.coef >= 0 && std::isfinite(r.dt) && std::isfinite(T))) return FFTPDE_EINVAL;
    if (r.op == FFTPDE_DIFFUSION && (r.dt < 0 || r.v0)) return FFTPDE_EINVAL;
  }
  return FFTPDE_OK;
}

// server-allocated bytes: the work block (spectra, scratch) and the output
void sizes(const fftpde_request& r, size_t* work, size_t* out, long long* footprint) {
  const size_t fb = (size_t)r.nx * r.ny * (r.dtype == FFTPDE_C64 ? 8 : 16);
  size_t w = 0;
  if (r.op == FFTPDE_POISSON) {
    w += up256(fb);                  // the spectrum between the solve's passes
  } else {
    w += up256(fb);                  // F
    if (r.v0) w += up256(fb);        // G
    if (r.diag) w += up256(diag_scratch_doubles(ilog2s(r.nx), ilog2s(r.ny), 1) * sizeof(double));
  }
  *work = w;
  *out = r.out ? 0 : up256(fb);
  long long f = (long long)fb;       // in
  if (r.v0) f += (long long)fb;
  if (r.out) f += (long long)fb;
  if (r.diag) f += 24ll * r.steps;
  *footprint = f + (long long)w + (long long)*out;
}

}  // namespace

// ---------------------------------------------------------------------------
// the server
// ---------------------------------------------------------------------------
struct fftpde_server {
  std::unique_ptr<Backend> be;
  long long budget = 0;
  int slots = 1, nstreams = 1;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_end;
  std::deque<Req*> queue;
  std::vector<Req*> running;
  std::unordered_map<unsigned long long, std::unique_ptr<Req>> reqs;
  unsigned long long next_id = 1;
  long long in_use = 0, high_water = 0;
  long long submitted = 0, rejected = 0, admitted = 0, completed = 0, failed = 0, canceled = 0, timed_out = 0;
  long long iterations = 0;
  std::vector<double> lat_ms;
  bool stop = false;
  int rr = 0;
  std::thread th;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  void place(Req* q) {
    char* base = be->pool_base();
    const fftpde_request& r = q->r;
    const size_t fb = (size_t)r.nx * r.ny * (r.dtype == FFTPDE_C64 ? 8 : 16);
    if (q->work_off != Pool::kNone) {
      char* p = base + q->work_off;
      q->F = p;
      p += up256(fb);
      if (r.v0) {
        q->G = p;
        p += up256(fb);
      }
      if (r.diag) q->scratch = reinterpret_cast<double*>(p);
    }
    q->out = r.out ? r.out : base + q->out_off;
  }

  // Ends a request: releases its budget and pool blocks (a server-owned
  // output of a successful request stays until fftpde_server_release).
  void end(Req* q, int status, double t) {
    q->status = status;
    q->state = kEnded;
    if (q->t_done < 0) q->t_done = t;
    if (q->work_off != Pool::kNone) pool.release(q->work_off);
    q->work_off = Pool::kNone;
    long long keep = 0;
    const bool autorel = (q->r.flags & FFTPDE_REQ_AUTORELEASE) != 0;
    if (q->out_off != Pool::kNone) {
      if (status == FFTPDE_OK && !autorel) {
        keep = (long long)q->out_bytes;
      } else {
        pool.release(q->out_off);
        q->out_off = Pool::kNone;
      }
    }
    if (q->t_admit >= 0) in_use -= q->footprint - keep;
    q->footprint = keep;
    if (status == FFTPDE_OK) {
      completed++;
      lat_ms.push_back((q->t_done - q->t_submit) * 1e3);
    } else if (status == FFTPDE_ECANCELED) {
      canceled++;
    } else if (status == FFTPDE_ETIMEOUT) {
      timed_out++;
    } else {
      failed++;
    }
    be->retire(*q);
    if (autorel) reqs.erase(q->id);  // q is gone after this
  }

  void loop() {
    be->thread_init();
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      const double t = now();
      for (auto it = queue.begin(); it != queue.end();) {
        Req* q = *it;
        const bool late = q->r.deadline > 0 && t > q->t_submit + q->r.deadline;
        if (late || q->abort.load()) {
          it = queue.erase(it);
          end(q, late ? FFTPDE_ETIMEOUT : FFTPDE_ECANCELED, t);
        } else {
          ++it;
        }
      }
      for (Req* q : running)
        if (q->r.deadline > 0 && t > q->t_submit + q->r.deadline && !q->abort.load()) q->abort = FFTPDE_ETIMEOUT;
      // admission: first come, first served, while slots and budget allow
      while (!queue.empty() && (int)running.size() < slots) {
        Req* q = queue.front();
        if (q->footprint > budget - in_use) break;
        size_t w = Pool::kNone, o = Pool::kNone;
        if (q->work_bytes && (w = pool.alloc(q->work_bytes)) == Pool::kNone) break;
        if (q->out_bytes && (o = pool.alloc(q->out_bytes)) == Pool::kNone) {
          if (w != Pool::kNone) pool.release(w);
          break;
        }
        queue.pop_front();
        q->work_off = w;
        q->out_off = o;
        place(q);
        q->state = kRunning;
        q->t_admit = t;
        q->stream = rr++ % nstreams;
        in_use += q->footprint;
        high_water = std::max(high_water, in_use);
        admitted++;
        if (be->admit(*q) != FFTPDE_OK) {
          end(q, FFTPDE_EDEVICE, t);
          continue;
        }
        running.push_back(q);
      }
      if (running.empty()) {
        cv_end.notify_all();
        if (stop && queue.empty()) break;
        cv_work.wait_for(lk, std::chrono::milliseconds(queue.empty() ? 50 : 1));
        continue;
      }
      // one iteration -- the next piece of work of every running request --
      // once the iteration before the last has finished on the device
      bool issued = false;
      if (be->ready()) {
        const std::vector<Req*> run = running;
        lk.unlock();
        for (Req* q : run) {
          if (q->enq_done) continue;
          const fftpde_request& r = q->r;
          int rc = FFTPDE_OK;
          if (q->abort.load()) {
            be->mark(*q);
            q->enq_done = true;
            continue;
          }
          if (!q->started) {
            rc = be->start(*q);
            q->started = true;
            if (!r.diag) q->next_step = r.steps + 1;
          } else if (q->next_step <= r.steps) {
            const int nt = (int)std::min<long long>(kChunk, r.steps - q->next_step + 1);
            rc = be->steps(*q, q->next_step, nt);
            q->next_step += nt;
          }
          if (rc == FFTPDE_OK && q->next_step > r.steps) {
            rc = be->finish(*q);
            be->mark(*q);
            q->enq_done = true;
          }
          if (rc != FFTPDE_OK) {
            q->fail = rc;
            if (!q->enq_done) {
              be->mark(*q);
              q->enq_done = true;
            }
          }
          issued = true;
        }
        if (issued) be->mark_iteration();
        lk.lock();
        if (issued) iterations++;
      }
      const double t2 = now();
      for (auto it = running.begin(); it != running.end();) {
        Req* q = *it;
        if (!q->enq_done) {
          ++it;
          continue;
        }
        const int st = be->query(*q);
        if (st == FFTPDE_PENDING) {
          ++it;
          continue;
        }
        const int ab = q->abort.load();
        const int final_status = ab ? ab : (q->fail != FFTPDE_OK ? q->fail : st);
        q->t_done = be->done_time(*q, t2);
        it = running.erase(it);
        end(q, final_status, t2);
      }
      cv_end.notify_all();
      // nothing could be issued: poll again shortly (the device is busy, or
      // every running request only waits for its completion)
      if (!issued) cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }

  void fill(const Req* q, fftpde_result* res) const {
    if (!res) return;
    res->status = q->state == kEnded ? q->status : FFTPDE_PENDING;
    res->state = q->state;
    res->t_submit = q->t_submit;
    res->t_admit = q->t_admit;
    res->t_done = q->t_done;
    res->out = q->state == kQueued ? q->r.out : q->out;
    res->footprint = q->footprint;
  }
};

namespace {

int start_server(fftpde_server* s, fftpde_server** out) {
  try {
    s->th = std::thread([s] { s->loop(); });
  } catch (...) {
    delete s;
    return FFTPDE_ENOMEM;
  }
  *out = s;
  return FFTPDE_OK;
}

}  // namespace

extern "C" {

int fftpde_server_create(fftpde_ctx* ctx, long long hbm_budget, int max_slots, int nstreams,
                         fftpde_server** server) {
  if (server) *server = nullptr;
  if (!ctx || !server || hbm_budget < 4096 || max_slots < 1 || nstreams < 1 || nstreams > 8) return FFTPDE_EINVAL;
  const int device = reinterpret_cast<Context*>(ctx)->device;
  auto* s = new (std::nothrow) fftpde_server();
  if (!s) return FFTPDE_ENOMEM;
  auto* be = new (std::nothrow) HipBackend();
  if (!be) {
    delete s;
    return FFTPDE_ENOMEM;
  }
  s->be.reset(be);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  const int rc = be->init(device, hbm_budget, nstreams, 0.0);
  be->set_ref_time(s->now());  // the reference event has just completed
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc != FFTPDE_OK) {
    delete s;
    return rc;
  }
  s->budget = hbm_budget;
  s->slots = max_slots;
  s->nstreams = nstreams;
  s->pool.reset((size_t)hbm_budget);
  return start_server(s, server);
}

int fftpde_server_create_host(long long hbm_budget, int max_slots, fftpde_host_exec exec, void* user,
                              fftpde_server** server) {
  if (server) *server = nullptr;
  if (!server || !exec || hbm_budget < 4096 || hbm_budget > kHostPoolMax || max_slots < 1) return FFTPDE_EINVAL;
  auto* s = new (std::nothrow) fftpde_server();
  if (!s) return FFTPDE_ENOMEM;
  auto* be = new (std::nothrow) HostBackend(exec, user, (size_t)hbm_budget, kHostStreams);
  if (!be || !be->ok()) {
    delete be;
    delete s;
    return FFTPDE_ENOMEM;
  }
  s->be.reset(be);
  s->budget = hbm_budget;
  s->slots = max_slots;
  s->nstreams = kHostStreams;
  s->pool.reset((size_t)hbm_budget);
  return start_server(s, server);
}

int fftpde_server_submit(fftpde_server* s, const fftpde_request* req, unsigned long long* id) {
  if (!s || !req || !id) return FFTPDE_EINVAL;
  *id = 0;
  if (check_request(*req) != FFTPDE_OK) return FFTPDE_EINVAL;
  auto q = std::unique_ptr<Req>(new (std::nothrow) Req());
  if (!q) return FFTPDE_ENOMEM;
  q->r = *req;
  sizes(q->r, &q->work_bytes, &q->out_bytes, &q->footprint);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return FFTPDE_EINVAL;
  s->submitted++;
  // larger than the whole budget (or than the pool can ever hold): never admitted
  if (q->footprint > s->budget || q->work_bytes > s->pool.size() || q->out_bytes > s->pool.size() ||
      q->work_bytes + q->out_bytes > s->pool.size()) {
    s->rejected++;
    return FFTPDE_EBUDGET;
  }
  if (req->stream && s->be->depend(*q, req->stream) != FFTPDE_OK) {
    s->be->retire(*q);
    return FFTPDE_EDEVICE;
  }
  q->id = s->next_id++;
  q->t_submit = s->now();
  *id = q->id;
  s->queue.push_back(q.get());
  s->reqs[q->id] = std::move(q);
  s->cv_work.notify_one();
  return FFTPDE_OK;
}

int fftpde_server_poll(fftpde_server* s, unsigned long long id, fftpde_result* res) {
  if (!s) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return FFTPDE_ENOTFOUND;
  s->fill(it->second.get(), res);
  return it->second->state == kEnded ? it->second->status : FFTPDE_PENDING;
}

int fftpde_server_wait(fftpde_server* s, unsigned long long id, double timeout, fftpde_result* res) {
  if (!s || std::isnan(timeout)) return FFTPDE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ended = [&] {
    auto it = s->reqs.find(id);
    return it == s->reqs.end() || it->second->state == kEnded;
  };
  if (timeout < 0) {
    s->cv_end.wait(lk, ended);
  } else {
    s->cv_end.wait_for(lk, std::chrono::duration<double>(std::min(timeout, 1e6)), ended);
  }
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return FFTPDE_ENOTFOUND;
  s->fill(it->second.get(), res);
  return it->second->state == kEnded ? it->second->status : FFTPDE_PENDING;
}

int fftpde_server_cancel(fftpde_server* s, unsigned long long id) {
  if (!s) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return FFTPDE_ENOTFOUND;
  Req* q = it->second.get();
  if (q->state == kEnded) return FFTPDE_OK;
  int expected = 0;
  q->abort.compare_exchange_strong(expected, FFTPDE_ECANCELED);
  if (q->state == kQueued) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), q));
    s->end(q, FFTPDE_ECANCELED, s->now());
    s->cv_end.notify_all();
  }
  s->cv_work.notify_one();
  return FFTPDE_OK;
}

int fftpde_server_release(fftpde_server* s, unsigned long long id) {
  if (!s) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return FFTPDE_ENOTFOUND;
  Req* q = it->second.get();
  if (q->state != kEnded) return FFTPDE_EINVAL;
  if (q->out_off != Pool::kNone) {
    s->pool.release(q->out_off);
    s->in_use -= q->footprint;
  }
  s->reqs.erase(it);
  s->cv_work.notify_one();  // memory may have freed up for the queue
  return FFTPDE_OK;
}

int fftpde_server_copy_out(fftpde_server* s, unsigned long long id, void* dst, fftpde_stream stream) {
  if (!s || !dst) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return FFTPDE_ENOTFOUND;
  const Req* q = it->second.get();
  if (q->state != kEnded || q->status != FFTPDE_OK) return FFTPDE_EINVAL;
  const size_t bytes = (size_t)q->r.nx * q->r.ny * (q->r.dtype == FFTPDE_C64 ? 8 : 16);
  return s->be->copy(dst, q->out, bytes, stream);
}

int fftpde_server_stats(fftpde_server* s, int reset, fftpde_stats* st) {
  if (!s || !st) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->rejected = s->rejected;
  st->admitted = s->admitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->canceled = s->canceled;
  st->timed_out = s->timed_out;
  st->queued = (long long)s->queue.size();
  st->running = (long long)s->running.size();
  st->hbm_budget = s->budget;
  st->hbm_in_use = s->in_use;
  st->hbm_high_water = s->high_water;
  st->iterations = s->iterations;
  std::vector<double> v = s->lat_ms;
  st->latency_count = (long long)v.size();
  st->p50_ms = st->p99_ms = st->mean_ms = st->max_ms = 0.0;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    // nearest rank: the smallest value with at least p of the sample at or below it
    auto rank = [&](double p) {
      size_t k = (size_t)std::ceil(p * (double)v.size());
      return v[k == 0 ? 0 : k - 1];
    };
    st->p50_ms = rank(0.50);
    st->p99_ms = rank(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
    st->max_ms = v.back();
  }
  st->now = s->now();
  if (reset) {
    s->lat_ms.clear();
    s->high_water = s->in_use;
  }
  return FFTPDE_OK;
}

int fftpde_server_destroy(fftpde_server* s) {
  if (!s) return FFTPDE_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    const double t = s->now();
    while (!s->queue.empty()) {
      Req* q = s->queue.front();
      s->queue.pop_front();
      s->end(q, FFTPDE_ECANCELED, t);
    }
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  s->be->drain();
  delete s;
  return FFTPDE_OK;
}

}  // extern "C"
