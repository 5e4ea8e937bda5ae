// batch.hip -- the persistent batch kernel: queue, per-job dependencies and
// the row / column tiles for every side 16..4096 (one workgroup of 512).
#include "batch.hpp"

namespace fftpde {
namespace {

// Row tile: LINES rows of length 2^LOGN, forward (or inverse by conjugation),
// radix plan ALT (batch_maxlr).
template <typename T, int LOGN, int ALT>
__device__ __forceinline__ void row_tile(const cx<T>* __restrict__ in, cx<T>* out, int nrows, int tile,
                                         bool inverse, const cx<T>* __restrict__ tw, const BatchArgs& a, cx<T>* lds,
                                         int tid) {
  constexpr int E = BatchCfg<T>::E;
  constexpr int N = 1 << LOGN;
  constexpr int LINES = BatchCfg<T>::kTile / N;
  constexpr int MAXLR = batch_maxlr<T>(ALT);
  using Map = RowMap<LOGN, LINES, plan_pad(LOGN, MAXLR, false)>;
  using Eng = Engine<T, LOGN, E, kBatchTH, MAXLR, false, Map, false>;
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
  Eng::run_stage(x, lds, tw + a.stw[ALT][LOGN][0], tid);
  Eng::for_each_output(tid, [&](int i, int line, int n) {
    const int row = row0 + line;
    if (row < nrows) out[((long long)row << LOGN) + n] = {x[i].re, sgn * x[i].im};
  });
}

template <typename T, int OP>
__device__ __forceinline__ void apply_symbol(cx<T>& v, const Symbol<T, OP>& s, int n) {
  const T m = s(n);
  v = {v.re * m, -v.im * m};
}

// Single-pass item: G = kTile / P jobs of one shape 2^LX x 2^LY and one
// operator, the whole solve of each in LDS and registers -- row forward,
// column forward, symbol, column inverse (by conjugation), row inverse -- as
// the one-launch small-grid kernel does for one field.  The G fields are G
// NY-row blocks of one tile of G NY rows (rows) and G NX columns (columns);
// slots past the item's njob jobs reread its last job and store nothing.
template <typename T, int LX, int LY>
__device__ __forceinline__ void k4_tile(const int* job_ids, int njob, const BatchArgs& a, const cx<T>* __restrict__ tw,
                                        cx<T>* lds, const void** ptrs, int tid) {
  constexpr int E = BatchCfg<T>::E;
  constexpr int NX = 1 << LX, NY = 1 << LY, P = NX * NY;
  constexpr int G = BatchCfg<T>::kTile / P;
  constexpr int LG = BatchCfg<T>::kLogTile - LX - LY;
  static_assert(G * P == BatchCfg<T>::kTile && G >= 1 && G <= (BatchCfg<T>::kTile >> 8), "whole fields per tile");
  static_assert(kBatchTH % (G * NX) == 0, "every thread stays on one column");
  using RMap = RowMap<LX, G * NY, plan_pad(LX, 3, false)>;
  using Row = Engine<T, LX, E, kBatchTH, 3, false, RMap, false>;
  using CFMap = ColMap<LY, LG + LX, plan_pad(LY, 3, false)>;
  using CIMap = ColMap<LY, LG + LX, plan_pad(LY, 3, true)>;
  using ColF = Engine<T, LY, E, kBatchTH, 3, false, CFMap, false>;
  using ColI = Engine<T, LY, E, kBatchTH, 3, true, CIMap, false>;
  // the fields between the passes: field g, row y, column x at
  // g FW + y FS + x (rows padded so that column reads spread over banks)
  constexpr int FS = NX + NX / 8;
  constexpr int FW = NY * FS;
  static_assert(G * FW <= BatchCfg<T>::kLdsElems && RMap::kLdsElems <= BatchCfg<T>::kLdsElems &&
                    CFMap::kLdsElems <= BatchCfg<T>::kLdsElems && CIMap::kLdsElems <= BatchCfg<T>::kLdsElems,
                "single-pass tile exceeds the batch LDS buffer");
  // the item's field pointers, once, into LDS: ptrs[g] input, ptrs[G + g]
  // output of slot g (every element's address is then an LDS read, not a
  // dependent global load of its job's descriptor)
  if (tid < G) {
    const BatchJobDesc& d = a.jobs[job_ids[min(tid, njob - 1)]];
    ptrs[tid] = d.in;
    ptrs[G + tid] = d.out;
  }
  lds_barrier();
  cx<T> x[E];
  // rows: x transforms of every row of every field
  Row::for_each_input(tid, [&](int i, int line, int n) {
    const cx<T>* in = static_cast<const cx<T>*>(ptrs[line >> LY]);
    x[i] = in[(line & (NY - 1)) * NX + n];
  });
  Row::run_stage(x, lds, tw + a.stw[0][LX][0], tid);
  Row::for_each_output(tid, [&](int i, int line, int n) { lds[(line >> LY) * FW + (line & (NY - 1)) * FS + n] = x[i]; });
  lds_barrier();
  // columns: y transforms of every column of every field; this thread's
  // column is line = tid mod (G NX): field line / NX, frequency line mod NX
  const int cline = tid & (G * NX - 1);
  const int cg = cline >> LX, cx_ = cline & (NX - 1);
  ColF::for_each_input(tid, [&](int i, int line, int n) { x[i] = lds[(line >> LX) * FW + n * FS + (line & (NX - 1))]; });
  lds_barrier();
  ColF::run_stage(x, lds, tw + a.stw[0][LY][0], tid);
  const SymParams& sym = a.jobs[job_ids[min(cg, njob - 1)]].sym;
  auto mul = [&](auto tag) {
    constexpr int OP = decltype(tag)::value;
    const Symbol<T, OP> s(sym, cx_);
    ColI::for_each_input(tid, [&](int i, int, int n) { apply_symbol(x[i], s, n); });
  };
  switch (sym.op) {
    case kSymPoisson: mul(std::integral_constant<int, kSymPoisson>()); break;
    case kSymDiffusion: mul(std::integral_constant<int, kSymDiffusion>()); break;
    case kSymWave: mul(std::integral_constant<int, kSymWave>()); break;
    default: mul(std::integral_constant<int, kSymScale>()); break;
  }
  ColI::run_stage(x, lds, tw + a.stw[0][LY][1], tid);
  ColI::for_each_output(tid, [&](int i, int line, int n) { lds[(line >> LX) * FW + n * FS + (line & (NX - 1))] = x[i]; });
  lds_barrier();
  Row::for_each_input(tid, [&](int i, int line, int n) { x[i] = lds[(line >> LY) * FW + (line & (NY - 1)) * FS + n]; });
  lds_barrier();
  Row::run_stage(x, lds, tw + a.stw[0][LX][0], tid);
  Row::for_each_output(tid, [&](int i, int line, int n) {
    const int g = line >> LY;
    if (g < njob) {
      cx<T>* out = static_cast<cx<T>*>(const_cast<void*>(ptrs[G + g]));
      out[(line & (NY - 1)) * NX + n] = conjg(x[i]);
    }
  });
  lds_barrier();  // the LDS buffer is free for the workgroup's next item
}

// Column tile of one job: 2^LOGT columns of length 2^LOGN; forward y
// transform, the real symbol (1/(nx ny) folded in), inverse y transform;
// radix plan ALT.
template <typename T, int LOGN, int ALT>
__device__ __forceinline__ void col_tile(cx<T>* data, int lognx, int tile, const SymParams& sym,
                                         const cx<T>* __restrict__ tw, const BatchArgs& a, cx<T>* lds, int tid) {
  constexpr int E = BatchCfg<T>::E;
  constexpr int LOGT = BatchCfg<T>::kLogTile - LOGN;
  constexpr int TT = 1 << LOGT;
  constexpr int MAXLR = batch_maxlr<T>(ALT);
  static_assert(TT << LOGN == BatchCfg<T>::kTile, "tile holds whole columns");
  static_assert(kBatchTH % TT == 0, "every thread stays on one column of the tile");
  using FMap = ColMap<LOGN, LOGT, plan_pad(LOGN, MAXLR, false)>;
  using IMap = ColMap<LOGN, LOGT, plan_pad(LOGN, MAXLR, true)>;
  using Fwd = Engine<T, LOGN, E, kBatchTH, MAXLR, false, FMap, false>;
  using Inv = Engine<T, LOGN, E, kBatchTH, MAXLR, true, IMap, false>;
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
  Fwd::run_stage(x, lds, tw + a.stw[ALT][LOGN][0], tid);
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
  Inv::run_stage(x, lds, tw + a.stw[ALT][LOGN][1], tid);
  if (C < ncols) {
    cx<T>* dst = data + C;
    Inv::for_each_output(tid, [&](int i, int, int n) { dst[(long long)n << lognx] = conjg(x[i]); });
  }
}

template <typename T, int L = kBatchMinLog>
__device__ __forceinline__ void dispatch_row(int logn, int alt, const cx<T>* in, cx<T>* out, int nrows, int tile,
                                             bool inverse, const cx<T>* tw, const BatchArgs& a, cx<T>* lds, int tid) {
  if constexpr (L <= kBatchMaxLog) {
    if (logn == L) {
      if constexpr (batch_has_alt<T>()) {
        if (alt) {
          row_tile<T, L, 1>(in, out, nrows, tile, inverse, tw, a, lds, tid);
          return;
        }
      }
      row_tile<T, L, 0>(in, out, nrows, tile, inverse, tw, a, lds, tid);
    } else {
      dispatch_row<T, L + 1>(logn, alt, in, out, nrows, tile, inverse, tw, a, lds, tid);
    }
  }
}

template <typename T, int L = kBatchMinLog>
__device__ __forceinline__ void dispatch_col(int logn, int alt, cx<T>* data, int lognx, int tile,
                                             const SymParams& sym, const cx<T>* tw, const BatchArgs& a, cx<T>* lds,
                                             int tid) {
  if constexpr (L <= kBatchMaxLog) {
    if (logn == L) {
      if constexpr (batch_has_alt<T>()) {
        if (alt) {
          col_tile<T, L, 1>(data, lognx, tile, sym, tw, a, lds, tid);
          return;
        }
      }
      col_tile<T, L, 0>(data, lognx, tile, sym, tw, a, lds, tid);
    } else {
      dispatch_col<T, L + 1>(logn, alt, data, lognx, tile, sym, tw, a, lds, tid);
    }
  }
}

// single-pass items: every (lx, ly) with both sides >= 16 and P <= kTile
template <typename T, int LX = kBatchMinLog, int LY = kBatchMinLog>
__device__ __forceinline__ void dispatch_k4(int lx, int ly, const int* job_ids, int njob, const BatchArgs& a,
                                            const cx<T>* tw, cx<T>* lds, const void** ptrs, int tid) {
  constexpr int LT = BatchCfg<T>::kLogTile;
  if constexpr (LX + kBatchMinLog <= LT) {
    if constexpr (LX + LY <= LT) {
      if (lx == LX && ly == LY) k4_tile<T, LX, LY>(job_ids, njob, a, tw, lds, ptrs, tid);
      else dispatch_k4<T, LX, LY + 1>(lx, ly, job_ids, njob, a, tw, lds, ptrs, tid);
    } else {
      dispatch_k4<T, LX + 1, kBatchMinLog>(lx, ly, job_ids, njob, a, tw, lds, ptrs, tid);
    }
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
  // field pointers of a single-pass item: up to kTile / 256 jobs, in and out
  __shared__ const void* s_ptrs[2 * (BatchCfg<T>::kTile >> (2 * kBatchMinLog))];
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
      const int step = item.step & 3, alt = (item.step & kBatchAltPlan) ? 1 : 0;
      // (a single-pass item neither waits nor publishes, but notes are not
      // held across it: a run of them is long, and the step's tiles behind
      // the notes would hold up every wait of the next step meanwhile)
      if (nnote > 0 && (step != note_step || nnote == kMaxPending)) publish();
      if ((step == 1 || step == 2) && !((acquired >> step) & 1)) {
        if (tid == 0) {
          const unsigned* cnt = &a.done[2 * item.job + step - 1];
          long spins = 0;
          while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)item.need) {
            __builtin_amdgcn_s_sleep(8);
            if (++spins > kSpinLimit) {
              __hip_atomic_store(&a.ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
          const unsigned all = __hip_atomic_load(&a.ctl->step_done[step - 1], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          s_flag = all >= a.step_items[step - 1];
        }
        __syncthreads();
        if (s_flag) acquired |= 1 << step;
      }
      if (step == 3) {
        const int* ids = a.k4jobs + item.job;
        const SymParams& s0 = a.jobs[ids[0]].sym;
        dispatch_k4<T>(s0.lognx, s0.logny, ids, item.tile, a, tw, lds, s_ptrs, tid);
        continue;
      }
      const BatchJobDesc& job = a.jobs[item.job];
      const int lognx = job.sym.lognx, logny = job.sym.logny;
      cx<T>* out = static_cast<cx<T>*>(job.out);
      if (step == 1) {
        dispatch_col<T>(logny, alt, out, lognx, item.tile, job.sym, tw, a, lds, tid);
      } else {
        const cx<T>* src = step == 0 ? static_cast<const cx<T>*>(job.in) : out;
        dispatch_row<T>(lognx, alt, src, out, 1 << logny, item.tile, step == 2, tw, a, lds, tid);
      }
      if (step < 2) {
        if (tid == 0) s_note[nnote] = 2 * item.job + step;
        note_step = step;
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
