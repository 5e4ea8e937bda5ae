// rpass.hpp -- row and column passes for sides n = R 2^m, R = 1, 3, 5 or 7:
// one radix-R step in registers around the power-of-two register engine.
//
// With n = R P (P = 2^m), input index j = P j1 + j2 and output index
// k = k1 + R k2 (j1, k1 < R; j2, k2 < P), the DFT sum of Eq. (DFT) factors
// (the R-way split of the sum that Sec. II.C makes two-way):
//   X[k1 + R k2] = sum_j2 w_P^(j2 k2) [ w_n^(j2 k1) sum_j1 x[P j1 + j2] w_R^(j1 k1) ]
// so each thread takes, for every position j2 the engine gives it, the R
// points x[P j1 + j2], forms their R-point DFT, multiplies by w_n^(j2 k1),
// and then runs the P-point engine R times (lines k1) without any exchange
// between the two steps.  The outputs of line k1 at k2 are X[k1 + R k2].
// The fused column pass of a solve applies the symbol there and runs the
// decimation-in-frequency mirror of the same factorisation on the
// conjugated spectrum: P-point engines over k2 per line k1, the twiddles
// w_n^(k1 j2), R-point DFTs over k1, out at P j1 + j2 -- the positions the
// loads came from -- so the tile never leaves registers and LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "mixed.hpp"

namespace fftpde {

// n = R 2^lp with R in {1, 3, 5, 7} (FP64: {1, 3}, the registers of R
// engine tiles) and 2^lp in the compiled range for the pass (rows: lp
// 5..11, columns: lp 5..12), n <= 4096; false otherwise.
bool rp_split(int n, bool col, bool fp64, int* r, int* lp);
// The fused column pass of a solve keeps R engine tiles in registers through
// the evaluation of the symbol.  For R >= 5 (FP32) and R = 3 (FP64) its
// engine takes 4 points per thread in radix-4 stages (half the tile), which
// fits the registers without spills; otherwise 8 points, radix-8 stages.
constexpr bool rp_col_small(bool fp64, int r, bool solve) { return solve && (fp64 ? r >= 3 : r >= 5); }
constexpr int rp_col_maxlr(bool fp64, int r, bool solve) { return rp_col_small(fp64, r, solve) ? 2 : 3; }
constexpr bool rp_solve_radix(bool fp64, int r) { return fp64 ? r <= 3 : r <= 7; }
// A pass of `mode` (kMr*) over lines of length n that these kernels take.
bool rp_pass_ok(int mode, int n, bool fp64);

template <typename T>
struct RpArgs {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* twn;   // exp(-2 pi i e / n), e < n: the radix-R step's twiddles
  const cx<T>* tw;    // exp(-2 pi i e / 4096): the row engine's
  const cx<T>* stwf;  // column engine's stage tables, forward plan (rp_col_maxlr)
  const cx<T>* stwr;  // and reversed plan (the solve's inverse)
  int nx, ny;
  long long fields;
  int mode;           // kMrRowFwd, kMrRowInv, kMrColFwd, kMrColInv, kMrColSolve
  T scale;            // kMrRowInv
  MrSym sym;          // kMrColSolve
};

// Launches the pass of a.mode (the line length is nx for rows, ny for
// columns); hipErrorInvalidValue if rp_split rejects it.
template <typename T>
hipError_t rp_launch(const RpArgs<T>& a, hipStream_t s);

}  // namespace fftpde
