// batch.hpp -- one persistent kernel for a batch of independent solves of
// uneven power-of-two shapes (many small and medium fields at once, each with
// its own box, operator and time).
//
// Every job is three steps of tiles: row tiles of x forward transforms
// (in -> out), column tiles that run the y forward transform, multiply by the
// job's symbol and run the y inverse (out -> out), and row tiles of x inverse
// transforms (out -> out).  A job whose field fits one tile (P <= kTile) is
// instead solved in one pass: an item of its own kind holds up to
// kTile / P such jobs of one shape and operator and runs all five steps in
// LDS (one HBM read and one write per field, no dependencies).  All items sit
// in one queue: every row-forward tile, the single-pass items, every column
// tile, then every row-inverse tile, largest jobs first.  Workgroups claim a
// few consecutive items at a time with one atomic counter (the next claim
// travels while the current one is worked on) and work through them in queue
// order; an item of step s waits until its job's step s-1 tiles are all
// published (a per-job counter).  An item only ever waits on items earlier in the queue, so the
// queue drains whatever the number of resident workgroups (see the
// publication rule in batch.hip).  Each wait is still bounded and reports a
// timeout through an error flag instead of spinning forever.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fftpde {

constexpr int kBatchTH = 512;
constexpr int kBatchMinLog = 4;   // sides 16 ..
constexpr int kBatchMaxLog = 12;  // .. 4096

template <typename T>
struct BatchCfg {
  // points per tile: 8192 FP32 / 4096 FP64 (16 / 8 per thread)
  static constexpr int E = sizeof(T) == 4 ? 16 : 8;
  static constexpr int kLogTile = sizeof(T) == 4 ? 13 : 12;
  static constexpr int kTile = E * kBatchTH;
  static constexpr int kLdsElems = kTile + kTile / 8;  // the engines pad by at most 1 in 8
};

constexpr int batch_log_tile(int dtype_fp64) { return dtype_fp64 ? 12 : 13; }

struct BatchJobDesc {
  const void* in;
  void* out;
  SymParams sym;  // op, lognx, logny, wavenumber scales, 1/(nx ny)
};

struct BatchItem {
  int job;    // step 3: first entry of the item's jobs in BatchArgs::k4jobs
  int step;   // bits 0-1: 0 row forward, 1 column, 2 row inverse, 3 single
              // pass; bit 2: the tile's radix plan (kBatchAltPlan)
  int tile;   // step 3: number of jobs in the item
  int need;   // tiles of the job's previous step (0 for steps 0 and 3)
};

// Radix plans.  In FP32, row and column tiles of every log2 length run one
// of two compiled plans, chosen per (tile kind, length) class and written
// into each item (so the choice costs the kernel no extra load): 0 = stages
// of radix up to 8 (the default), 1 = up to 16.  FP64 tiles (8 points per
// thread) have plan 0 only: their one alternative, radix up to 4, was slower
// in every class, and compiling it in slowed plan 0 by 8 %.
constexpr int kBatchAltPlan = 4;
template <typename T>
constexpr bool batch_has_alt() {
  return sizeof(T) == 4;
}
template <typename T>
constexpr int batch_maxlr(int alt) {
  return alt ? 4 : 3;
}
constexpr int batch_maxlr_dt(int fp64, int alt) { return alt && !fp64 ? 4 : 3; }

struct BatchCtl {
  unsigned long long head;  // next item
  unsigned step_done[2];    // published tiles of steps 0 and 1, whole batch
  int error;                // 1: a dependency wait timed out
  int pad;
};

struct BatchArgs {
  const BatchJobDesc* jobs;
  const BatchItem* items;
  long long nitems;
  BatchCtl* ctl;
  unsigned* done;  // per job: [row-forward tiles done, column tiles done]
  int njobs;
  unsigned step_items[2];  // tiles of steps 0 and 1, whole batch
  const void* tw;
  // entry offsets from tw of the stage tables (Engine::stw_off):
  // stw[plan][log2 length][0 forward, 1 reversed]
  int stw[2][kBatchMaxLog + 1][2];
  const int* k4jobs;  // job indices of the single-pass items, item by item
};

hipError_t batch_launch(int fp64, const BatchArgs& a, int grid, hipStream_t s);
// Clears the queue head, the error flag and the per-job counters (a kernel,
// so the reset may be captured in a graph).
hipError_t batch_reset(BatchCtl* ctl, unsigned* done, int njobs, hipStream_t s);
int batch_occupancy(int fp64);

}  // namespace fftpde
