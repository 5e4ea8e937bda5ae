// batch.cpp -- planning and launching a batch of uneven solves: job checks,
// the item queue, device tables and the captured graph (reset + kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <climits>
#include <numeric>
#include <vector>

#include "../../include/fftpde.h"
#include "batch.hpp"
#include "context.hpp"
#include "solve.hpp"

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

  // job descriptors, and the queue: largest jobs first within each step
  std::vector<BatchJobDesc> desc(njobs);
  std::vector<int> ntile[3];
  for (int s = 0; s < 3; s++) ntile[s].resize(njobs);
  double bytes = 0.0;
  for (int i = 0; i < njobs; i++) {
    const fftpde_job& j = jobs[i];
    const int sop = j.op == FFTPDE_POISSON ? kSymPoisson : j.op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave;
    desc[i] = {j.in, j.out, make_sym(sop, j.nx, j.ny, j.lx, j.ly, j.coef, j.t)};
    const int lx = ilog2(j.nx), ly = ilog2(j.ny);
    const int lines = 1 << (logtile - lx), cols = 1 << (logtile - ly);
    ntile[0][i] = ntile[2][i] = (j.ny + lines - 1) / lines;
    ntile[1][i] = (j.nx + cols - 1) / cols;
    bytes += 6.0 * (double)elem * j.nx * j.ny;
  }
  std::vector<int> order(njobs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long long)jobs[a].nx * jobs[a].ny > (long long)jobs[b].nx * jobs[b].ny;
  });
  std::vector<BatchItem> items;
  for (int s = 0; s < 3; s++)
    for (int i : order)
      for (int t = 0; t < ntile[s][i]; t++) items.push_back({i, s, t, s > 0 ? ntile[s - 1][i] : 0});

  if (items.size() > (size_t)0x7fffffff) return FFTPDE_EINVAL;  // 32-bit tile counters

  auto* b = new fftpde_batch();
  b->ctx = c;
  b->dtype = dtype;
  b->njobs = njobs;
  b->nitems = (long long)items.size();
  b->bytes = bytes;
  const int occ = batch_occupancy(fp64);
  b->grid = std::max(1, occ) * std::max(1, c->num_cus);
  if (b->grid > b->nitems) b->grid = (int)b->nitems;

  // one device allocation: control word, counters, jobs, items
  const size_t o_ctl = 0, o_done = align_up(sizeof(BatchCtl));
  const size_t o_jobs = o_done + align_up(sizeof(unsigned) * 2 * (size_t)njobs);
  const size_t o_items = o_jobs + align_up(sizeof(BatchJobDesc) * (size_t)njobs);
  const size_t total = o_items + align_up(sizeof(BatchItem) * items.size());
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
  for (int l = 0; l <= kBatchMaxLog; l++)
    for (int r = 0; r < 2; r++) b->args.stw[l][r] = l >= 1 ? c->stage_tw_at[l][3][r] : 0;
  e = hipMemcpy(base + o_jobs, desc.data(), sizeof(BatchJobDesc) * desc.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + o_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);

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

int fftpde_batch_destroy(fftpde_batch* b) {
  if (!b) return FFTPDE_OK;
  (void)hipSetDevice(b->ctx->device);
  destroy_batch(b);
  return FFTPDE_OK;
}

}  // extern "C"
