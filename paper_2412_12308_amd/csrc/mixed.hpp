// mixed.hpp -- 2D transforms and solves on sides that are not powers of two:
// any side in [2, 4096] whose prime factors are 2, 3, 5 and 7.
//
// Sec. II.D builds the method on N = 2^m; the mixed-radix path is the same
// row-column scheme with Stockham stages of radix 2, 3, 4, 5, 7 and 8 (a
// stage of radix R fuses the R-way split of the DFT sum, Eq. (DFT), the way
// a radix-2 stage is the even/odd split of Sec. II.C).  Three passes, as on
// the power-of-two path: x rows forward, then per tile of adjacent columns
// the y forward transform, the pointwise symbol and the y inverse (the
// spectrum never goes back to HBM between them), then x rows inverse.
//
// A workgroup loads one tile (whole lines, at most 4096 points per field)
// into LDS, runs every stage there -- each thread takes its butterflies'
// inputs into registers, the workgroup synchronises, the outputs go back to
// the same buffer -- and writes the tile out.  Twiddles are the N-th roots
// of unity of the line length, generated in FP64 on the host and rounded
// once (one table per length, cached in the context).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fftpde {

constexpr int kMrTH = 1024;         // threads per workgroup (4 points each at 4096)
constexpr int kMrMaxSide = 4096;
constexpr int kMrTilePts = 4096;    // points per field and tile
constexpr int kMrMaxColLines = 64;  // columns per column tile
constexpr int kMrLds = kMrTilePts + kMrMaxColLines;  // column tiles pad each line by one
constexpr int kMrMaxStages = 12;

// Sides the mixed-radix path takes: 2..4096, 7-smooth.
__host__ __device__ constexpr bool mr_side_ok(int n) {
  if (n < 2 || n > kMrMaxSide) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  while (n % 7 == 0) n /= 7;
  return n == 1;
}

// Radix sequence of a length: 8s first, then a 4 or a 2 for the rest of the
// power of two, then 7s, 5s and 3s.
struct MrPlan {
  int n = 0;
  int nst = 0;
  int radix[kMrMaxStages] = {};
};

inline MrPlan mr_plan(int n) {
  MrPlan p;
  p.n = n;
  int m = n;
  auto take = [&](int r) {
    while (m % r == 0 && p.nst < kMrMaxStages) {
      p.radix[p.nst++] = r;
      m /= r;
    }
  };
  take(8);
  take(4);
  take(2);
  take(7);
  take(5);
  take(3);
  if (m != 1) p.nst = 0;  // not 7-smooth: no plan
  return p;
}

// Pass modes.
enum : int {
  kMrRowFwd = 0,   // rows: forward transform
  kMrRowInv = 1,   // rows: inverse (exp(+) sum) times scale
  kMrColFwd = 2,   // columns: forward transform
  kMrColInv = 3,   // columns: inverse (exp(+) sum), unscaled
  kMrColSolve = 4  // columns: forward, symbol (1/(nx ny) folded in), inverse
};

// Pointwise symbols of the solves on signed frequency indices a' (x), b' (y).
struct MrSym {
  int op = kSymScale;  // kSymPoisson / kSymDiffusion / kSymWave / kSymScale
  double kxs = 0, kys = 0;  // 2 pi / lx, 2 pi / ly
  double kt = 0;            // diffusion: kappa t
  double hx = 0, hy = 0;    // wave: 2 c t / lx, 2 c t / ly (w t / pi = |(hx a', hy b')|)
  double c = 0, t = 0;      // wave: speed and time
  double scale = 1;         // 1 / (nx ny)
};

template <typename T>
struct MrArgs {
  const cx<T>* in0;
  const cx<T>* in1;  // second field (the wave's initial velocity); null: zero
  cx<T>* out0;
  cx<T>* out1;       // second output (the wave's velocity); null: not written
  const cx<T>* tw;   // tw[e] = exp(-2 pi i e / n), e < n, n the line length
  MrPlan plan;
  int nx, ny;
  long long fields;
  int lines;  // lines per tile
  int ls;     // LDS distance between lines
  int mode;
  T scale;    // kMrRowInv
  MrSym sym;  // kMrColSolve
};

template <typename T>
hipError_t mr_launch(const MrArgs<T>& a, int nf, hipStream_t s);
// workgroups of a launch
template <typename T>
long long mr_tiles(const MrArgs<T>& a);

}  // namespace fftpde
