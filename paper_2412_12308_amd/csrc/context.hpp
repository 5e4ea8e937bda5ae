// context.hpp -- state behind an fftpde_ctx handle: the device, the twiddle
// tables, the per-shape kernel choices and a reusable workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "small.hpp"

namespace fftpde {

// index of a (dtype, pass kind, log2 length, fields per pass) plan slot
constexpr int plan_key(int dtype, int kind, int logn, int nf) {
  return ((dtype * 2 + kind) * 13 + logn) * 3 + (nf - 1);
}
constexpr int kPlanSlots = 2 * 2 * 13 * 3;

struct Context {
  int device = 0;
  cx<float>* tw32 = nullptr;   // exp(-2 pi i e/4096), FP64-generated, rounded once
  cx<double>* tw64 = nullptr;  // the same in FP64
  // Behind the 4096 entries of both tables: the stage tables of every plan
  // (log2 length 1..12, max log-radix 1..kStageMaxLr, forward / reversed),
  // entry offsets stage_tw_at[logn][maxlr][rev] (Engine::stw_off).
  static constexpr int kStageMaxLr = 5;
  int stage_tw_at[13][kStageMaxLr + 1][2] = {};
  template <typename T>
  const cx<T>* stage_tw(int logn, int maxlr, bool rev) const {
    if (logn < 1 || logn > 12 || maxlr < 1 || maxlr > kStageMaxLr) return nullptr;
    const int o = stage_tw_at[logn][maxlr][rev ? 1 : 0];
    if constexpr (sizeof(T) == 4) return tw32 + o;
    else return tw64 + o;
  }
  // Scratch fields for solves that need one, one per stream so that calls on
  // different streams never share it (grown on demand, freed at destroy).
  struct Work {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::unordered_map<void*, Work> work;
  // Kernel choice per plan slot; null = the first compiled variant of that length.
  const RowVariant* row_choice[kPlanSlots] = {};
  const ColVariant* col_choice[kPlanSlots] = {};

  // Optional per-kernel timing: a HIP event pair around every launch.
  struct TimedLaunch {
    const char* name;
    double bytes;  // algorithmic HBM bytes of the launch
    hipEvent_t start, stop;
  };
  bool profiling = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t take_event();

  int num_cus = 0;
  std::unordered_map<const void*, int> occupancy;  // variant -> resident workgroups per CU
  // Workgroup cap for a persistent (prefetching) launch: all resident at once.
  long long max_blocks(const void* variant, OccFn occ);

  // Single-pass small-grid kernels: used whenever one is compiled for the
  // shape, unless switched off (fftpde_plan_small).
  bool use_small = true;
  const SmallVariant* small_variant(int dtype, int lognx, int logny) const;

  // Solves keep their spectrum between the passes in column blocks of
  // tiled_bytes per row (at least the column plan's tile) x ny rows; 0:
  // row-major in the output field.  Set with fftpde_plan_tiled.  1024 bytes
  // measured best at 2048^2 (FP32 and FP64): wide enough for full-line row
  // writes, narrow enough that the column tiles of a block stay close.
  int tiled_bytes = 1024;
  // Batches of 3-pass solves run in chunks of about chunk_bytes of field
  // data, all three passes per chunk, so that the spectrum a pass writes is
  // still in the 256 MiB Infinity Cache when the next pass reads it (0: the
  // whole batch at once).  Set with fftpde_plan_chunk.
  long long chunk_bytes = 256ll << 20;
  // per-shape block size and chunk size chosen by the autotuner (key: tiled_key)
  std::unordered_map<int, int> tiled_for;
  std::unordered_map<int, long long> chunk_for;
  long long chunk_bytes_for(int dtype, int lognx, int logny) const {
    auto it = chunk_for.find(tiled_key(dtype, lognx, logny));
    return it == chunk_for.end() ? chunk_bytes : it->second;
  }
  static int tiled_key(int dtype, int lognx, int logny) { return (dtype * 16 + lognx) * 16 + logny; }
  int tiled_bytes_for(int dtype, int lognx, int logny) const {
    auto it = tiled_for.find(tiled_key(dtype, lognx, logny));
    return it == tiled_for.end() ? tiled_bytes : it->second;
  }

  // Twiddle tables of the mixed-radix path, exp(-2 pi i e/n) for e < n, per
  // line length n (made on first use; one allocation, f64 at its start).
  struct MrTables {
    cx<double>* f64;
    cx<float>* f32;
  };
  std::unordered_map<int, MrTables> mr_tw;

  const RowVariant* row_variant(int dtype, int logn) const;
  const ColVariant* col_variant(int dtype, int logn, int nf) const;
  int workspace(size_t bytes, hipStream_t s, void** p);
};

void set_last_error(const char* what, hipError_t e);

}  // namespace fftpde
