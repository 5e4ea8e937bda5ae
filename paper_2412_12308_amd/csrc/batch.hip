// batch.hip -- the persistent batch kernel: queue, per-job dependencies and
// the row / column tiles for every side 16..4096 (one workgroup of 512).
#include "batch.hpp"

namespace fftpde {
namespace {

// Row tile: LINES rows of length 2^LOGN, forward (or inverse by conjugation).
template <typename T, int LOGN>
__device__ __forceinline__ void row_tile(const cx<T>* __restrict__ in, cx<T>* out, int nrows, int tile,
                                         bool inverse, const cx<T>* __restrict__ tw, const BatchArgs& a, cx<T>* lds,
                                         int tid) {
  constexpr int E = BatchCfg<T>::E;
  constexpr int N = 1 << LOGN;
  constexpr int LINES = BatchCfg<T>::kTile / N;
  using Map = RowMap<LOGN, LINES, plan_pad(LOGN, 3, false)>;
  using Eng = Engine<T, LOGN, E, kBatchTH, 3, false, Map, false>;
  static_assert(Map::kLdsElems <= BatchCfg<T>::kLdsElems, "row tile exceeds the batch LDS buffer");
  const T sgn = inverse ? T(-1) : T(1);
  const int row0 = tile * LINES;
  cx<T> x[E];
  // rows past the field reread the last row and are never stored
  Eng::for_each_input(tid, [&](int i, int line, int n) {
    const int row = min(row0 + line, nrows - 1);
    const cx<T> v = in[((long long)row << LOGN) + n];
    x[i] = {v.re, sgn * v.im};
  });
  Eng::run_stage(x, lds, tw + a.stw[LOGN][0], tid);
  Eng::for_each_output(tid, [&](int i, int line, int n) {
    const int row = row0 + line;
    if (row < nrows) out[((long long)row << LOGN) + n] = {x[i].re, sgn * x[i].im};
  });
}

// Column tile of one job: 2^LOGT columns of length 2^LOGN; forward y
// transform, the real symbol (1/(nx ny) folded in), inverse y transform.
template <typename T, int LOGN>
__device__ __forceinline__ void col_tile(cx<T>* data, int lognx, int tile, const SymParams& sym,
                                         const cx<T>* __restrict__ tw, const BatchArgs& a, cx<T>* lds, int tid) {
  constexpr int E = BatchCfg<T>::E;
  constexpr int LOGT = BatchCfg<T>::kLogTile - LOGN;
  constexpr int TT = 1 << LOGT;
  static_assert(TT << LOGN == BatchCfg<T>::kTile, "tile holds whole columns");
  static_assert(kBatchTH % TT == 0, "every thread stays on one column of the tile");
  using FMap = ColMap<LOGN, LOGT, plan_pad(LOGN, 3, false)>;
  using IMap = ColMap<LOGN, LOGT, plan_pad(LOGN, 3, true)>;
  using Fwd = Engine<T, LOGN, E, kBatchTH, 3, false, FMap, false>;
  using Inv = Engine<T, LOGN, E, kBatchTH, 3, true, IMap, false>;
  static_assert(FMap::kLdsElems <= BatchCfg<T>::kLdsElems && IMap::kLdsElems <= BatchCfg<T>::kLdsElems,
                "column tile exceeds the batch LDS buffer");
  const int ncols = 1 << lognx;
  // this thread's column; columns past the field reread the last column and
  // are never stored, so the loads carry no branches
  const int C = (tile << LOGT) + (tid & (TT - 1));
  const int Cl = min(C, ncols - 1);
  const cx<T>* src = data + Cl;
  cx<T> x[E];
  Fwd::for_each_input(tid, [&](int i, int, int n) { x[i] = src[(long long)n << lognx]; });
  Fwd::run_stage(x, lds, tw + a.stw[LOGN][0], tid);
  auto mul = [&](auto tag) {
    constexpr int OP = decltype(tag)::value;
    const Symbol<T, OP> s(sym, Cl);
    Inv::for_each_input(tid, [&](int i, int, int n) {
      const T m = s(n);
      x[i] = {x[i].re * m, -x[i].im * m};
    });
  };
  switch (sym.op) {
    case kSymPoisson: mul(std::integral_constant<int, kSymPoisson>()); break;
    case kSymDiffusion: mul(std::integral_constant<int, kSymDiffusion>()); break;
    case kSymWave: mul(std::integral_constant<int, kSymWave>()); break;
    default: mul(std::integral_constant<int, kSymScale>()); break;
  }
  Inv::run_stage(x, lds, tw + a.stw[LOGN][1], tid);
  if (C < ncols) {
    cx<T>* dst = data + C;
    Inv::for_each_output(tid, [&](int i, int, int n) { dst[(long long)n << lognx] = conjg(x[i]); });
  }
}

template <typename T, int L = kBatchMinLog>
__device__ __forceinline__ void dispatch_row(int logn, const cx<T>* in, cx<T>* out, int nrows, int tile,
                                             bool inverse, const cx<T>* tw, const BatchArgs& a, cx<T>* lds, int tid) {
  if constexpr (L <= kBatchMaxLog) {
    if (logn == L) row_tile<T, L>(in, out, nrows, tile, inverse, tw, a, lds, tid);
    else dispatch_row<T, L + 1>(logn, in, out, nrows, tile, inverse, tw, a, lds, tid);
  }
}

template <typename T, int L = kBatchMinLog>
__device__ __forceinline__ void dispatch_col(int logn, cx<T>* data, int lognx, int tile, const SymParams& sym,
                                             const cx<T>* tw, const BatchArgs& a, cx<T>* lds, int tid) {
  if constexpr (L <= kBatchMaxLog) {
    if (logn == L) col_tile<T, L>(data, lognx, tile, sym, tw, a, lds, tid);
    else dispatch_col<T, L + 1>(logn, data, lognx, tile, sym, tw, a, lds, tid);
  }
}

// about a second of polling
constexpr long kSpinLimit = 1l << 22;
// completions a workgroup may hold before it publishes them
constexpr int kMaxPending = 64;
// consecutive queue items taken by one atomic: the queue head is one counter
// that every workgroup updates, and its atomics serialize (one item per
// atomic spent about 0.65 ms of queue traffic per run of the 1024-job batch)
constexpr int kClaim = 4;

// Publication.  A finished row-forward or column tile is not announced at
// once: the workgroup notes it (job counter index) in LDS and publishes its
// notes together -- every wave drains its stores, one agent-scope release
// (an L2 write-back) covers the workgroup, then relaxed counter increments --
// before it takes an item of a later step (the only items that may wait),
// when the notes are full, and when the queue is empty.  A workgroup holding
// unpublished notes is thus always working on an item that does not wait, so
// every note is eventually published and no wait can be circular.
//
// Acquisition.  A waiting item spins on its job's counter, then one wave
// performs an agent-scope acquire (invalidating this CU's and XCD's cached
// lines) before any wave reads.  Once a workgroup has done that after the
// whole batch's previous step was published (the step counters), its later
// items of that step need neither the wait nor the invalidation.
template <typename T>
__global__ void __launch_bounds__(kBatchTH) batch_kernel(BatchArgs a) {
  __shared__ cx<T> lds[BatchCfg<T>::kLdsElems];
  __shared__ long long s_item;
  __shared__ int s_note[kMaxPending];
  __shared__ int s_flag;
  int tid = threadIdx.x;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw);
  int nnote = 0, note_step = 0;  // uniform across the workgroup
  int acquired = 0;              // bit s: step s items need no wait

  auto publish = [&]() {
    if (nnote == 0) return;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached its L2
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int k = 0; k < nnote; k++)
        __hip_atomic_fetch_add(&a.done[s_note[k]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&a.ctl->step_done[note_step], (unsigned)nnote, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    nnote = 0;
  };

  auto claim = [&]() {
    return __hip_atomic_fetch_add(&a.ctl->head, (unsigned long long)kClaim, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  };
  if (tid == 0) s_item = (long long)claim();
  __syncthreads();
  long long base = s_item;
  while (base < a.nitems) {
    // the next claim travels while this one is worked on
    unsigned long long next = 0;
    if (tid == 0) next = claim();
    const long long end = min(base + kClaim, a.nitems);
    for (long long it = base; it < end; it++) {
      // keeps per-stage addresses from being hoisted out of the item loop
      // (they would all stay live in registers across items)
      tid = opaque(tid);
      const BatchItem item = a.items[it];
      if (nnote > 0 && (item.step != note_step || nnote == kMaxPending)) publish();
      if (item.step > 0 && !((acquired >> item.step) & 1)) {
        if (tid == 0) {
          const unsigned* cnt = &a.done[2 * item.job + item.step - 1];
          long spins = 0;
          while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)item.need) {
            __builtin_amdgcn_s_sleep(8);
            if (++spins > kSpinLimit) {
              __hip_atomic_store(&a.ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
          const unsigned all = __hip_atomic_load(&a.ctl->step_done[item.step - 1], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          s_flag = all >= a.step_items[item.step - 1];
        }
        __syncthreads();
        if (s_flag) acquired |= 1 << item.step;
      }
      const BatchJobDesc& job = a.jobs[item.job];
      const int lognx = job.sym.lognx, logny = job.sym.logny;
      cx<T>* out = static_cast<cx<T>*>(job.out);
      if (item.step == 1) {
        dispatch_col<T>(logny, out, lognx, item.tile, job.sym, tw, a, lds, tid);
      } else {
        const cx<T>* src = item.step == 0 ? static_cast<const cx<T>*>(job.in) : out;
        dispatch_row<T>(lognx, src, out, 1 << logny, item.tile, item.step == 2, tw, a, lds, tid);
      }
      if (item.step < 2) {
        if (tid == 0) s_note[nnote] = 2 * item.job + item.step;
        note_step = item.step;
        nnote++;
      }
    }
    __syncthreads();  // every thread has read s_item
    if (tid == 0) s_item = (long long)next;
    __syncthreads();
    base = s_item;
  }
  publish();
}

__global__ void batch_reset_kernel(BatchCtl* ctl, unsigned* done, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctl->head = 0;
    ctl->step_done[0] = 0;
    ctl->step_done[1] = 0;
    ctl->error = 0;
  }
  if (i < n) done[i] = 0;
}

template <typename T>
int occ() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<T>, kBatchTH, 0) != hipSuccess) return 0;
  return n;
}

}  // namespace

hipError_t batch_launch(int fp64, const BatchArgs& a, int grid, hipStream_t s) {
  if (fp64) hipLaunchKernelGGL(batch_kernel<double>, dim3(grid), dim3(kBatchTH), 0, s, a);
  else hipLaunchKernelGGL(batch_kernel<float>, dim3(grid), dim3(kBatchTH), 0, s, a);
  return hipGetLastError();
}

hipError_t batch_reset(BatchCtl* ctl, unsigned* done, int njobs, hipStream_t s) {
  const int n = 2 * njobs;
  const int blocks = n / 256 + 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(blocks), dim3(256), 0, s, ctl, done, n);
  return hipGetLastError();
}

int batch_occupancy(int fp64) { return fp64 ? occ<double>() : occ<float>(); }

}  // namespace fftpde
