// batch.hip -- the batch's three step kernels (row forward, column, row
// inverse): queue claims and the row / column tiles for every side 16..4096
// (workgroups of 512).
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

// One step of the batch: every tile of that step of every job, persistent
// workgroups claiming runs of kBatchClaim items.  The steps are three launches in
// stream order, so a step reads what the previous one wrote with no waits or
// fences of its own.
template <typename T, int STEP>
__global__ void __launch_bounds__(kBatchTH) batch_step_kernel(BatchArgs a) {
  __shared__ cx<T> lds[BatchCfg<T>::kLdsElems];
  __shared__ long long s_item;
  int tid = threadIdx.x;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw);
  const long long lo = a.begin[STEP], hi = a.begin[STEP + 1];
  auto claim = [&]() {
    return lo + (long long)__hip_atomic_fetch_add(&a.ctl->head[STEP], (unsigned long long)kBatchClaim, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
  };
  if (tid == 0) s_item = claim();
  __syncthreads();
  long long base = s_item;
  while (base < hi) {
    // the next claim travels while this one is worked on
    long long next = 0;
    if (tid == 0) next = claim();
    const long long end = min(base + kBatchClaim, hi);
    for (long long it = base; it < end; it++) {
      // keeps per-stage addresses from being hoisted out of the item loop
      // (they would all stay live in registers across items)
      tid = opaque(tid);
      const BatchItem item = a.items[it];
      const BatchJobDesc& job = a.jobs[item.job];
      const int lognx = job.sym.lognx, logny = job.sym.logny;
      cx<T>* out = static_cast<cx<T>*>(job.out);
      if constexpr (STEP == 1) {
        dispatch_col<T>(logny, out, lognx, item.tile, job.sym, tw, a, lds, tid);
      } else {
        const cx<T>* src = STEP == 0 ? static_cast<const cx<T>*>(job.in) : out;
        dispatch_row<T>(lognx, src, out, 1 << logny, item.tile, STEP == 2, tw, a, lds, tid);
      }
    }
    __syncthreads();  // every thread has read s_item
    if (tid == 0) s_item = next;
    __syncthreads();
    base = s_item;
  }
}

__global__ void batch_reset_kernel(BatchCtl* ctl) {
  if (threadIdx.x == 0) {
    ctl->head[0] = 0;
    ctl->head[1] = 0;
    ctl->head[2] = 0;
    ctl->error = 0;
  }
}

template <typename T, int STEP>
int occ() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step_kernel<T, STEP>, kBatchTH, 0) != hipSuccess)
    return 0;
  return n;
}

template <typename T>
void launch_steps(const BatchArgs& a, const int grid[3], hipStream_t s) {
  hipLaunchKernelGGL((batch_step_kernel<T, 0>), dim3(grid[0]), dim3(kBatchTH), 0, s, a);
  hipLaunchKernelGGL((batch_step_kernel<T, 1>), dim3(grid[1]), dim3(kBatchTH), 0, s, a);
  hipLaunchKernelGGL((batch_step_kernel<T, 2>), dim3(grid[2]), dim3(kBatchTH), 0, s, a);
}

}  // namespace

hipError_t batch_launch(int fp64, const BatchArgs& a, const int grid[3], hipStream_t s) {
  if (fp64) launch_steps<double>(a, grid, s);
  else launch_steps<float>(a, grid, s);
  return hipGetLastError();
}

hipError_t batch_reset(BatchCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

int batch_occupancy(int fp64, int step) {
  if (fp64) return step == 0 ? occ<double, 0>() : step == 1 ? occ<double, 1>() : occ<double, 2>();
  return step == 0 ? occ<float, 0>() : step == 1 ? occ<float, 1>() : occ<float, 2>();
}

}  // namespace fftpde
