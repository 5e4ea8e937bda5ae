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
  double t;
  double dxdy;      // (lx / nx) * (ly / ny)
};

// Doubles of scratch the reduction needs.
size_t diag_scratch_doubles(int lognx, int logny, int batch);

// out[3 f + {0, 1, 2}] = mean (re, im) and energy of field f.
template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, int batch, double* scratch, double* out, hipStream_t s);

}  // namespace fftpde
