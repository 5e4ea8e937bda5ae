// halfrow.hpp -- half spectra of real fields through half-length complex
// row transforms.
//
// A real row x of even length N read as the complex row z[m] = x[2m] +
// i x[2m + 1] of length M = N/2 has the M-point spectrum Z = E + i O, with
// E, O the spectra of the even and odd samples.  Both are Hermitian (the
// samples are real, Sec. II.B), so with Zm[k] = conj(Z[(M - k) mod M])
//   E[k] = (Z[k] + Zm[k]) / 2,   O[k] = -i (Z[k] - Zm[k]) / 2,
// and the row's N-point spectrum for k = 0..M is the even/odd combination of
// Sec. II.C, X[k] = E[k] + w^k O[k], w = exp(-2 pi i / N).  X[0] and X[M]
// are real; they travel packed as X[0] + i X[M] in column 0, so every row
// stays M complex values and the column pass is the complex one over M
// columns.  The packed column transforms to P = Y0 + i YM, where Y0 and YM
// (the spectra of two real columns) are Hermitian in the row index b:
//   Y0[b] = (P[b] + conj P[-b]) / 2,   YM[b] = -i (P[b] - conj P[-b]) / 2.
// The inverse runs the same steps backwards: columns of the half spectrum
// (column 0 packed with the Hermitian parts of columns 0 and M), then per
// row E[k] = (X[k] + conj X[M - k]) / 2, O[k] = w^-k (X[k] - conj X[M - k]) / 2,
// Z = E + i O and the M-point inverse transform, whose real and imaginary
// parts are the even and odd samples of the real row.
//
// Two passes, each one read and one write: real fields (b P) -> M x ny
// complex work field (b P) -> half spectra, and back.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace fftpde {

template <typename T>
struct HalfRowArgs {
  const T* rin;         // r2c: real fields [fields][ny][nx]
  T* rout;              // c2r: real fields
  cx<T>* work;          // [fields][M x ny], blocks of 2^lt columns x ny rows
  const cx<T>* hin;     // c2r: half spectra [fields][ny][M + 1]
  cx<T>* hout;          // r2c: half spectra
  const cx<T>* tw;      // exp(-2 pi i e / 4096), e < 4096
  const cx<T>* stw;     // stage table of the column plan (column passes)
  long long fields;
  int lognx, logny, lt;
  T scale;              // c2r row pass: 1 / (M ny)
};

// Shapes with compiled half-row kernels: nx in [16, 4096], ny in [16, 4096],
// and a column tile (halfrow_col_logt columns) no wider than M = nx / 2.
bool halfrow_supported(int fp64, int lognx, int logny);
// log2 of the column tile width for ny = 2^logny
int halfrow_col_logt(int fp64, int logny);
// radix plan of the column passes (maximum log-radix)
int halfrow_col_maxlr(int fp64);

template <typename T>
hipError_t launch_r2c_rows(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_r2c_cols(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_c2r_cols(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_c2r_rows(const HalfRowArgs<T>& a, hipStream_t s);

}  // namespace fftpde
