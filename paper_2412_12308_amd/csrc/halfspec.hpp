// halfspec.hpp -- conversions between the spectrum of a pair of real fields
// (transformed as one complex field) and the two half spectra
// [ny][nx/2 + 1] of the fields (fft2d_r2c / fft2d_c2r).  Any sides: the
// spectra come from the power-of-two or the mixed-radix passes.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace fftpde {

template <typename T>
struct HalfArgs {
  cx<T>* spec;       // npairs complex [ny][nx] spectra (read by untangle, written by tangle)
  cx<T>* half;       // nreal half spectra [ny][nx/2 + 1] (written by untangle, read by tangle)
  int nx, ny;
  long long npairs;  // pairs in this launch
  long long nreal;   // real fields in this launch (2 npairs, or one less)
  // Layout of spec: t < 0 row-major; else blocks of 2^t columns x ny rows,
  // element (y, x) at block (x >> t), offset y 2^t + (x mod 2^t) within it
  // (the column passes' tiled layout), ny = 2^logny.
  int t = -1;
  int logny = 0;
};

template <typename T>
hipError_t launch_untangle(const HalfArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_tangle(const HalfArgs<T>& a, hipStream_t s);

}  // namespace fftpde
