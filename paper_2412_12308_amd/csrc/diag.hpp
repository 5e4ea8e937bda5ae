// diag.hpp -- mean and energy of an evolving solution from its spectra.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "fft_engine.hpp"

namespace fftpde {

template <typename T>
struct DiagArgs {
  const cx<T>* F;  // spectra of u0, batch fields
  const cx<T>* G;  // spectra of v0 (wave), or null
  int kind;        // 0 diffusion, 1 wave
  int lognx, logny;
  double kxs, kys;  // 2 pi / lx, 2 pi / ly
  double coef;      // kappa or c
  long long n0;     // times t_j = (n0 + j) * dt, j < nt (each one FP64 product)
  double dt;
  int nt;           // 1 .. kDiagMaxTimes
  double dxdy;      // (lx / nx) * (ly / ny)
};

// Times one launch evaluates (one read of the spectra for all of them).
constexpr int kDiagMaxTimes = 16;

// Doubles of scratch the reduction needs (for up to kDiagMaxTimes times);
// launches sharing a scratch must be ordered (one stream).
size_t diag_scratch_doubles(int lognx, int logny, int batch);

// out[3 (j batch + f) + {0, 1, 2}] = mean (re, im) and energy of field f at t_j.
template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, int batch, double* scratch, double* out, hipStream_t s);

}  // namespace fftpde
