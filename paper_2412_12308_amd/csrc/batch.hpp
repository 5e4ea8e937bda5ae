// batch.hpp -- one persistent kernel for a batch of independent solves of
// uneven power-of-two shapes (many small and medium fields at once, each with
// its own box, operator and time).
//
// Every job is three steps of tiles: row tiles of x forward transforms
// (in -> out), column tiles that run the y forward transform, multiply by the
// job's symbol and run the y inverse (out -> out), and row tiles of x inverse
// transforms (out -> out).  Each step is one launch of a persistent kernel
// over that step's tiles of every job (largest jobs first); the three
// launches run in stream order, so a step sees everything the previous one
// wrote without any waits.  Workgroups claim a few consecutive tiles at a
// time from the step's queue counter (the next claim travels while the
// current one is worked on).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fftpde {

constexpr int kBatchTH = 512;
constexpr int kBatchMinLog = 4;   // sides 16 ..
constexpr int kBatchMaxLog = 12;  // .. 4096
// consecutive queue items taken by one atomic: a step's queue head is one
// counter that all its workgroups update, and those atomics serialize (one
// item per atomic spent about 0.65 ms of queue traffic per run of a
// 1024-job batch)
constexpr int kBatchClaim = 4;

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
  int job;
  int tile;
};

struct BatchCtl {
  unsigned long long head[3];  // next item of each step (relative to its range)
  int error;                   // always 0 (no step waits); read by fftpde_batch_status
  int pad;
};

struct BatchArgs {
  const BatchJobDesc* jobs;
  const BatchItem* items;
  long long begin[4];  // items of step s: [begin[s], begin[s + 1])
  BatchCtl* ctl;
  int njobs;
  const void* tw;
  // entry offsets from tw of the stage tables (Engine::stw_off) of the
  // radix-8 plans: stw[log2 length][0 forward, 1 reversed]
  int stw[kBatchMaxLog + 1][2];
};

// the three step launches, grid[s] persistent workgroups each
hipError_t batch_launch(int fp64, const BatchArgs& a, const int grid[3], hipStream_t s);
// Clears the queue heads and the error word (a kernel, so the reset may be
// captured in a graph).
hipError_t batch_reset(BatchCtl* ctl, hipStream_t s);
int batch_occupancy(int fp64, int step);

}  // namespace fftpde
