// halfrow.hpp -- half spectra of real fields in two passes, columns first.
//
// A real field x[ny][nx] read as complex points is z[y][a] = x[y][2a] +
// i x[y][2a + 1], a < M = nx/2: a complex field of M columns.  Its column
// transforms Zc[b][a] (b the row frequency) hold the column spectra of the
// even and odd columns of x, Ge + i Go; both are Hermitian in b (the columns
// are real, Sec. II.B), so with the mirrored row -b
//   Ge[b] = (Zc[b] + conj Zc[-b]) / 2,   Go[b] = -i (Zc[b] - conj Zc[-b]) / 2.
// The row transform over x of row b then splits into the M-point transforms
// of its even and odd samples (Sec. II.C): with Zr[b] the M-point transform of
// Zc[b][.] and E[k], O[k] those of Ge[b], Go[b],
//   E[k] = (Zr[b][k] + conj Zr[-b][-k]) / 2,   O[k] = -i (Zr[b][k] - conj Zr[-b][-k]) / 2,
//   X[b][k] = E[k mod M] + w^k O[k mod M],  k = 0..M,  w = exp(-2 pi i / nx).
// So r2c is a column pass over the complex view (-> work field) and a row
// pass over row pairs (b, -b): M-point transforms of both rows, the
// combination above, and whole half-spectrum rows [ny][M + 1] written out.
// c2r runs the same steps backwards: per row pair, from the Hermitian
// extension X~ of the half spectrum (columns 0 and M replaced by their
// Hermitian parts, X~[b][k + M] = conj X~[-b][M - k]),
//   E[k] = (X~[b][k] + X~[b][k + M]) / 2,   O[k] = w^-k (X~[b][k] - X~[b][k + M]) / 2,
//   Zr[b][k] = E[k] + i O[k],
// M-point inverse transforms into the work field, then the inverse column
// pass writes the complex view of the real field.
//
// Each pass reads and writes once: real field (b P) <-> work field of M x ny
// complex points (b P) <-> half spectra.
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
  T scale;              // c2r column pass: 1 / (M ny)
};

// Shapes with compiled half-row kernels: nx in [16, 4096], ny in [16, 4096],
// and a column tile (halfrow_col_logt columns) no wider than M = nx / 2.
bool halfrow_supported(int fp64, int lognx, int logny);
// log2 of the column tile width for ny = 2^logny
int halfrow_col_logt(int fp64, int logny);
// radix plan of the column passes (maximum log-radix)
int halfrow_col_maxlr(int fp64);

// r2c: launch_r2c_cols (real fields -> work), then launch_r2c_rows (work ->
// half spectra).  c2r: launch_c2r_rows (half spectra -> work), then
// launch_c2r_cols (work -> real fields).
template <typename T>
hipError_t launch_r2c_cols(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_r2c_rows(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_c2r_rows(const HalfRowArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_c2r_cols(const HalfRowArgs<T>& a, hipStream_t s);

}  // namespace fftpde
