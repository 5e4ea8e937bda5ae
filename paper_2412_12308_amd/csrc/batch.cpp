// batch.cpp -- planning and launching a batch of uneven solves: job checks,
// the item queue, device tables and the captured graph (reset + kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <climits>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fftpde.h"
#include "batch.hpp"
#include "context.hpp"
#include "solve.hpp"
#include "util.hpp"

using namespace fftpde;

struct fftpde_batch {
  Context* ctx = nullptr;
  int dtype = 0;
  int njobs = 0;
  long long nitems = 0;
  int grid = 0;
  double bytes = 0.0;  // algorithmic HBM bytes of one run
  void* dmem = nullptr;
  BatchArgs args{};
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the plan table (each row / column item carries its class's plan) and
  // what the queue holds
  unsigned char plan[2 * (kBatchMaxLog + 1)] = {};
  std::vector<BatchItem> items;  // host copy of the queue
  BatchItem* ditems = nullptr;
  long long tiles[2][kBatchMaxLog + 1] = {};  // row / column tiles per log2 length
  int k4_jobs = 0, k4_items = 0;
  std::vector<fftpde_job> jobs;  // as submitted (the tuner reads the outputs)
  bool in_place = false;
  std::string tune_log;  // candidates of the last fftpde_batch_tune, JSON objects
};

namespace {

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}

bool side_ok(int n) { return n >= (1 << kBatchMinLog) && n <= (1 << kBatchMaxLog) && (n & (n - 1)) == 0; }

int check_job(const fftpde_job& j, int dtype) {
  if (j.op != FFTPDE_POISSON && j.op != FFTPDE_DIFFUSION && j.op != FFTPDE_WAVE) return FFTPDE_EINVAL;
  if (!side_ok(j.nx) || !side_ok(j.ny)) return FFTPDE_EINVAL;
  if (!(std::isfinite(j.lx) && j.lx > 0 && std::isfinite(j.ly) && j.ly > 0)) return FFTPDE_EINVAL;
  if (!j.in || !j.out) return FFTPDE_EINVAL;
  const uintptr_t al = dtype == FFTPDE_C64 ? 8 : 16;
  if ((reinterpret_cast<uintptr_t>(j.in) | reinterpret_cast<uintptr_t>(j.out)) & (al - 1)) return FFTPDE_EINVAL;
  if (j.op == FFTPDE_DIFFUSION && !(std::isfinite(j.coef) && j.coef >= 0 && std::isfinite(j.t) && j.t >= 0))
    return FFTPDE_EINVAL;
  if (j.op == FFTPDE_WAVE && !(std::isfinite(j.coef) && j.coef >= 0 && std::isfinite(j.t))) return FFTPDE_EINVAL;
  return FFTPDE_OK;
}

struct Range {
  uintptr_t lo, hi;
  int job;
};

// Outputs must be disjoint from every other job's input and output; a job may
// work in place (in == out) but not on partly overlapping in and out.
int check_overlap(const fftpde_job* jobs, int n, size_t elem) {
  std::vector<Range> outs(n), ins(n);
  for (int i = 0; i < n; i++) {
    const size_t b = elem * (size_t)jobs[i].nx * (size_t)jobs[i].ny;
    const uintptr_t o = reinterpret_cast<uintptr_t>(jobs[i].out), p = reinterpret_cast<uintptr_t>(jobs[i].in);
    outs[i] = {o, o + b, i};
    ins[i] = {p, p + b, i};
  }
  std::sort(outs.begin(), outs.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
  for (int i = 1; i < n; i++)
    if (outs[i].lo < outs[i - 1].hi) return FFTPDE_EINVAL;
  for (const Range& r : ins) {
    // first output ending after r.lo; outputs are disjoint, so sorted by end too
    auto it = std::upper_bound(outs.begin(), outs.end(), r.lo, [](uintptr_t v, const Range& o) { return v < o.hi; });
    for (; it != outs.end() && it->lo < r.hi; ++it)
      if (!(it->job == r.job && it->lo == r.lo)) return FFTPDE_EINVAL;
  }
  return FFTPDE_OK;
}

void destroy_batch(fftpde_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dmem) (void)hipFree(b->dmem);
  delete b;
}

hipError_t enqueue(fftpde_batch* b, hipStream_t s) {
  hipError_t e = batch_reset(b->args.ctl, b->args.done, b->njobs, s);
  if (e == hipSuccess) e = batch_launch(b->dtype == FFTPDE_C128, b->args, b->grid, s);
  return e;
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

int fftpde_batch_create(fftpde_ctx* ctx, const fftpde_job* jobs, int njobs, int dtype, fftpde_batch** out) {
  if (out) *out = nullptr;
  if (!ctx || !jobs || !out || njobs < 1 || njobs > (1 << 20)) return FFTPDE_EINVAL;
  if (dtype != FFTPDE_C64 && dtype != FFTPDE_C128) return FFTPDE_EINVAL;
  for (int i = 0; i < njobs; i++)
    if (check_job(jobs[i], dtype) != FFTPDE_OK) return FFTPDE_EINVAL;
  const size_t elem = dtype == FFTPDE_C64 ? 8 : 16;
  if (check_overlap(jobs, njobs, elem) != FFTPDE_OK) return FFTPDE_EINVAL;

  Context* c = reinterpret_cast<Context*>(ctx);
  const int fp64 = dtype == FFTPDE_C128;
  const int logtile = batch_log_tile(fp64);

  // job descriptors, and the queue: largest jobs first within each step;
  // jobs that fit one tile go to single-pass items of up to kTile / P jobs
  // of one shape and operator (one HBM read and one write per field)
  auto* b = new fftpde_batch();
  std::vector<BatchJobDesc> desc(njobs);
  std::vector<int> ntile[3];
  for (int s = 0; s < 3; s++) ntile[s].resize(njobs);
  std::vector<char> single(njobs, 0);
  double bytes = 0.0;
  for (int i = 0; i < njobs; i++) {
    const fftpde_job& j = jobs[i];
    const int sop = j.op == FFTPDE_POISSON ? kSymPoisson : j.op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave;
    desc[i] = {j.in, j.out, make_sym(sop, j.nx, j.ny, j.lx, j.ly, j.coef, j.t)};
    const int lx = ilog2(j.nx), ly = ilog2(j.ny);
    if (lx + ly <= logtile) {
      single[i] = 1;
      bytes += 2.0 * (double)elem * j.nx * j.ny;
      continue;
    }
    const int lines = 1 << (logtile - lx), cols = 1 << (logtile - ly);
    ntile[0][i] = ntile[2][i] = (j.ny + lines - 1) / lines;
    ntile[1][i] = (j.nx + cols - 1) / cols;
    b->tiles[0][lx] += 2ll * ntile[0][i];
    b->tiles[1][ly] += ntile[1][i];
    bytes += 6.0 * (double)elem * j.nx * j.ny;
  }
  std::vector<int> order(njobs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long long)jobs[a].nx * jobs[a].ny > (long long)jobs[b].nx * jobs[b].ny;
  });
  // single-pass groups: (lx, ly, op) in order of first appearance in `order`
  std::vector<int> k4ids;
  std::vector<BatchItem> k4items;
  {
    std::vector<std::vector<int>> groups;
    std::vector<long long> keys;
    for (int i : order) {
      if (!single[i]) continue;
      const long long key = ((long long)ilog2(jobs[i].nx) * 16 + ilog2(jobs[i].ny)) * 4 + jobs[i].op;
      size_t g = 0;
      while (g < keys.size() && keys[g] != key) g++;
      if (g == keys.size()) {
        keys.push_back(key);
        groups.emplace_back();
      }
      groups[g].push_back(i);
    }
    for (auto& grp : groups) {
      const int per = 1 << (logtile - ilog2(jobs[grp[0]].nx) - ilog2(jobs[grp[0]].ny));
      for (size_t k = 0; k < grp.size(); k += per) {
        const int n = (int)std::min<size_t>(per, grp.size() - k);
        k4items.push_back({(int)k4ids.size(), 3, n, 0});
        for (int q = 0; q < n; q++) k4ids.push_back(grp[k + q]);
      }
    }
  }
  std::vector<BatchItem> items;
  for (int s = 0; s < 3; s++) {
    for (int i : order)
      for (int t = 0; t < ntile[s][i]; t++) items.push_back({i, s, t, s > 0 ? ntile[s - 1][i] : 0});
    if (s == 0) items.insert(items.end(), k4items.begin(), k4items.end());
  }

  if (items.size() > (size_t)0x7fffffff) {  // 32-bit tile counters
    delete b;
    return FFTPDE_EINVAL;
  }

  b->ctx = c;
  b->dtype = dtype;
  b->njobs = njobs;
  b->nitems = (long long)items.size();
  b->bytes = bytes;
  b->k4_jobs = (int)k4ids.size();
  b->k4_items = (int)k4items.size();
  b->jobs.assign(jobs, jobs + njobs);
  for (int i = 0; i < njobs; i++)
    if (jobs[i].in == jobs[i].out) b->in_place = true;
  const int occ = batch_occupancy(fp64);
  b->grid = std::max(1, occ) * std::max(1, c->num_cus);
  if (b->grid > b->nitems) b->grid = (int)b->nitems;

  // one device allocation: control word, counters, jobs, items, single-pass
  // job lists
  const size_t o_ctl = 0, o_done = align_up(sizeof(BatchCtl));
  const size_t o_jobs = o_done + align_up(sizeof(unsigned) * 2 * (size_t)njobs);
  const size_t o_items = o_jobs + align_up(sizeof(BatchJobDesc) * (size_t)njobs);
  const size_t o_k4 = o_items + align_up(sizeof(BatchItem) * items.size());
  const size_t total = o_k4 + align_up(sizeof(int) * std::max<size_t>(1, k4ids.size()));
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipMalloc(&b->dmem, total);
  if (e != hipSuccess) {
    set_last_error("batch allocation", e);
    destroy_batch(b);
    return e == hipErrorOutOfMemory ? FFTPDE_ENOMEM : FFTPDE_EDEVICE;
  }
  char* base = static_cast<char*>(b->dmem);
  b->args.ctl = reinterpret_cast<BatchCtl*>(base + o_ctl);
  b->args.done = reinterpret_cast<unsigned*>(base + o_done);
  b->args.jobs = reinterpret_cast<const BatchJobDesc*>(base + o_jobs);
  b->args.items = reinterpret_cast<const BatchItem*>(base + o_items);
  b->args.nitems = b->nitems;
  b->args.njobs = njobs;
  for (int s = 0; s < 2; s++) {
    long long n = 0;
    for (int i = 0; i < njobs; i++) n += ntile[s][i];
    b->args.step_items[s] = (unsigned)n;
  }
  b->args.tw = fp64 ? static_cast<const void*>(c->tw64) : static_cast<const void*>(c->tw32);
  for (int alt = 0; alt < 2; alt++)
    for (int l = 0; l <= kBatchMaxLog; l++)
      for (int r = 0; r < 2; r++)
        b->args.stw[alt][l][r] = l >= 1 ? c->stage_tw_at[l][batch_maxlr_dt(fp64, alt)][r] : 0;
  b->ditems = reinterpret_cast<BatchItem*>(base + o_items);
  b->args.k4jobs = reinterpret_cast<const int*>(base + o_k4);
  e = hipMemcpy(base + o_jobs, desc.data(), sizeof(BatchJobDesc) * desc.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + o_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !k4ids.empty())
    e = hipMemcpy(base + o_k4, k4ids.data(), sizeof(int) * k4ids.size(), hipMemcpyHostToDevice);

  // capture reset + kernel once; every run replays the graph
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = enqueue(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    set_last_error("batch plan", e);
    destroy_batch(b);
    return FFTPDE_EDEVICE;
  }
  b->items = std::move(items);
  *out = b;
  return FFTPDE_OK;
}

int fftpde_batch_run(fftpde_batch* b, int use_graph, fftpde_stream stream) {
  if (!b) return FFTPDE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* name = b->dtype == FFTPDE_C64 ? "batch_float" : "batch_double";
  hipError_t e = timed_launch(b->ctx, name, b->bytes, s, [&] {
    return use_graph ? hipGraphLaunch(b->exec, s) : enqueue(b, s);
  });
  if (e != hipSuccess) {
    set_last_error(name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

int fftpde_batch_status(fftpde_batch* b, fftpde_stream stream) {
  if (!b) return FFTPDE_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, &b->args.ctl->error, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_last_error("batch status", e);
    return FFTPDE_EDEVICE;
  }
  return flag ? FFTPDE_ETIMEOUT : FFTPDE_OK;
}

int fftpde_batch_info(const fftpde_batch* b, long long* items, int* grid, double* bytes) {
  if (!b) return FFTPDE_EINVAL;
  if (items) *items = b->nitems;
  if (grid) *grid = b->grid;
  if (bytes) *bytes = b->bytes;
  return FFTPDE_OK;
}

int fftpde_batch_plan(fftpde_batch* b, int kind, int logn, int plan) {
  if (!b || kind < 0 || kind > 1 || logn < kBatchMinLog || logn > kBatchMaxLog || plan < 0 || plan > 1 ||
      (plan == 1 && b->dtype != FFTPDE_C64))
    return FFTPDE_EINVAL;
  const int idx = kind * (kBatchMaxLog + 1) + logn;
  b->plan[idx] = (unsigned char)plan;
  for (BatchItem& it : b->items) {
    const int step = it.step & 3;
    if (step == 3) continue;
    const fftpde_job& j = b->jobs[it.job];
    if ((kind == 0 && step != 1 && ilog2(j.nx) == logn) || (kind == 1 && step == 1 && ilog2(j.ny) == logn))
      it.step = step | (plan ? kBatchAltPlan : 0);
  }
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != b->ctx->device) (void)hipSetDevice(b->ctx->device);
  // a synchronous copy; the caller ensures that no run is in flight
  const hipError_t e = hipMemcpy(b->ditems, b->items.data(), sizeof(BatchItem) * b->items.size(),
                                 hipMemcpyHostToDevice);
  if (prev >= 0 && prev != b->ctx->device) (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    set_last_error("batch plan", e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

int fftpde_batch_tune(fftpde_batch* b, int reps, fftpde_stream stream) {
  if (!b || b->in_place) return FFTPDE_EINVAL;
  if (reps < 1) reps = 10;
  Context* c = b->ctx;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != c->device) (void)hipSetDevice(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dt = b->dtype;
  const size_t elem = dt == FFTPDE_C64 ? 8 : 16;
  std::vector<size_t> off(b->njobs + 1, 0);
  for (int i = 0; i < b->njobs; i++) off[i + 1] = off[i] + (size_t)b->jobs[i].nx * b->jobs[i].ny;
  char* ref = nullptr;
  double* acc = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = FFTPDE_OK;
  auto done = [&](int code) {
    if (ref) (void)hipFree(ref);
    if (acc) (void)hipFree(acc);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
    return code;
  };
  if (hipMalloc(&ref, off[b->njobs] * elem) != hipSuccess ||
      hipMalloc(&acc, 2 * sizeof(double) * (size_t)b->njobs) != hipSuccess)
    return done(FFTPDE_ENOMEM);
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return done(FFTPDE_EDEVICE);
  auto dev = [&](hipError_t e) {
    if (e != hipSuccess) set_last_error("batch tune", e);
    return e == hipSuccess;
  };
  // the current plan's outputs are the reference
  if (!dev(hipGraphLaunch(b->exec, s))) return done(FFTPDE_EDEVICE);
  for (int i = 0; i < b->njobs; i++)
    if (!dev(hipMemcpyAsync(ref + off[i] * elem, b->jobs[i].out, (off[i + 1] - off[i]) * elem,
                            hipMemcpyDeviceToDevice, s)))
      return done(FFTPDE_EDEVICE);
  // fastest of three timings of `reps` replays each, then the worst job's
  // relative L2 distance from the reference
  auto measure = [&](double* us, double* err) -> int {
    double best = 1e30;
    for (int g = 0; g < 3; g++) {
      if (!dev(hipGraphLaunch(b->exec, s)) || !dev(hipEventRecord(e0, s))) return FFTPDE_EDEVICE;
      for (int r = 0; r < reps; r++)
        if (!dev(hipGraphLaunch(b->exec, s))) return FFTPDE_EDEVICE;
      float ms = 0.f;
      if (!dev(hipEventRecord(e1, s)) || !dev(hipEventSynchronize(e1)) || !dev(hipEventElapsedTime(&ms, e0, e1)))
        return FFTPDE_EDEVICE;
      best = std::min(best, 1e3 * ms / reps);
    }
    *us = best;
    if (!dev(zero_doubles(acc, 2ll * b->njobs, s))) return FFTPDE_EDEVICE;
    for (int i = 0; i < b->njobs; i++)
      if (!dev(diff_norms(b->jobs[i].out, ref + off[i] * elem, (long long)(off[i + 1] - off[i]), dt, acc + 2 * i, s)))
        return FFTPDE_EDEVICE;
    std::vector<double> h(2 * (size_t)b->njobs);
    if (!dev(hipMemcpyAsync(h.data(), acc, h.size() * sizeof(double), hipMemcpyDeviceToHost, s)) ||
        !dev(hipStreamSynchronize(s)))
      return FFTPDE_EDEVICE;
    int status = FFTPDE_OK;
    if (!dev(hipMemcpy(&status, &b->args.ctl->error, sizeof(int), hipMemcpyDeviceToHost))) return FFTPDE_EDEVICE;
    if (status) return FFTPDE_ETIMEOUT;
    double worst = 0.0;
    for (int i = 0; i < b->njobs; i++)
      worst = std::max(worst, h[2 * i + 1] > 0 ? std::sqrt(h[2 * i] / h[2 * i + 1]) : std::sqrt(h[2 * i]));
    *err = worst;
    return FFTPDE_OK;
  };
  int maxlog = 1;
  for (const fftpde_job& j : b->jobs) maxlog = std::max(maxlog, std::max(ilog2(j.nx), ilog2(j.ny)));
  // the two plans differ by rounding only
  const double tol = dt == FFTPDE_C64 ? 2.0 * 2e-6 * maxlog : 1e-12;
  // about 100 ms of replays before the first timing: the first tens of
  // milliseconds after the GPU idles run up to 15 % slower (clocks settling),
  // which would make the starting plan look slow against every flip
  {
    float spent = 0.f;
    for (int i = 0; i < 16 && spent < 100.f; i++) {
      if (!dev(hipEventRecord(e0, s))) return done(FFTPDE_EDEVICE);
      for (int r = 0; r < 8; r++)
        if (!dev(hipGraphLaunch(b->exec, s))) return done(FFTPDE_EDEVICE);
      float ms = 0.f;
      if (!dev(hipEventRecord(e1, s)) || !dev(hipEventSynchronize(e1)) || !dev(hipEventElapsedTime(&ms, e0, e1)))
        return done(FFTPDE_EDEVICE);
      spent += ms;
    }
  }
  double cur_us = 0, err = 0;
  rc = measure(&cur_us, &err);
  if (rc != FFTPDE_OK) return done(rc);
  b->tune_log.clear();
  auto note = [&](const char* kind, int logn, int plan, double us, double e, bool ok, bool kept) {
    char line[200];
    std::snprintf(line, sizeof(line),
                  "%s{\"kind\": \"%s\", \"logn\": %d, \"plan\": %d, \"us\": %.2f, \"err\": %.3e, \"ok\": %d, "
                  "\"kept\": %d}",
                  b->tune_log.empty() ? "" : ", ", kind, logn, plan, us, e, ok ? 1 : 0, kept ? 1 : 0);
    b->tune_log += line;
  };
  note("start", 0, -1, cur_us, err, true, true);  // the plan table as it was
  // classes by tile count, largest first; each flipped once, kept if faster
  std::vector<std::pair<long long, int>> cls;  // (FP64 has one plan)
  for (int kind = 0; kind < 2 && dt == FFTPDE_C64; kind++)
    for (int l = kBatchMinLog; l <= kBatchMaxLog; l++)
      if (b->tiles[kind][l] > 0) cls.push_back({b->tiles[kind][l], kind * (kBatchMaxLog + 1) + l});
  std::stable_sort(cls.begin(), cls.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  for (const auto& cl : cls) {
    const int kind = cl.second / (kBatchMaxLog + 1), l = cl.second % (kBatchMaxLog + 1);
    const int was = b->plan[cl.second];
    if ((rc = fftpde_batch_plan(b, kind, l, was ^ 1)) != FFTPDE_OK) return done(rc);
    double us = 0, e = 0;
    rc = measure(&us, &e);
    if (rc != FFTPDE_OK) {
      (void)fftpde_batch_plan(b, kind, l, was);
      return done(rc);
    }
    const bool ok = e <= tol, keep = ok && us < cur_us;
    note(kind ? "col" : "row", l, was ^ 1, us, e, ok, keep);
    if (keep) {
      cur_us = us;
    } else if ((rc = fftpde_batch_plan(b, kind, l, was)) != FFTPDE_OK) {
      return done(rc);
    }
  }
  return done(FFTPDE_OK);
}

int fftpde_batch_describe(const fftpde_batch* b, char* buf, size_t cap, size_t* need) {
  if (!b) return FFTPDE_EINVAL;
  char head[320];
  std::snprintf(head, sizeof(head),
                "{\"dtype\": %d, \"jobs\": %d, \"items\": %lld, \"grid\": %d, \"bytes\": %.0f, "
                "\"single_pass\": {\"jobs\": %d, \"items\": %d}, \"classes\": [",
                b->dtype, b->njobs, b->nitems, b->grid, b->bytes, b->k4_jobs, b->k4_items);
  std::string out = head;
  bool first = true;
  for (int kind = 0; kind < 2; kind++)
    for (int l = kBatchMinLog; l <= kBatchMaxLog; l++) {
      if (b->tiles[kind][l] == 0) continue;
      const int plan = b->plan[kind * (kBatchMaxLog + 1) + l];
      char line[160];
      std::snprintf(line, sizeof(line), "%s{\"kind\": \"%s\", \"logn\": %d, \"tiles\": %lld, \"plan\": %d, "
                    "\"max_radix\": %d}",
                    first ? "" : ", ", kind ? "col" : "row", l, b->tiles[kind][l], plan,
                    1 << batch_maxlr_dt(b->dtype == FFTPDE_C128, plan));
      out += line;
      first = false;
    }
  out += "], \"tune\": [" + b->tune_log + "]}";
  if (need) *need = out.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
    if (n < out.size()) return FFTPDE_EINVAL;
  }
  return FFTPDE_OK;
}

int fftpde_batch_destroy(fftpde_batch* b) {
  if (!b) return FFTPDE_OK;
  (void)hipSetDevice(b->ctx->device);
  destroy_batch(b);
  return FFTPDE_OK;
}

}  // extern "C"
