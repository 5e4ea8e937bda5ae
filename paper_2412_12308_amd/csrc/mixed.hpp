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
// Persistent workgroups walk the tiles (whole lines, up to mr_cap points per
// field).  A tile is loaded into LDS, every stage runs there -- each thread
// takes its butterflies' inputs into registers, the workgroup synchronises,
// the outputs go back to the same buffer -- and the tile is written out.
// Twiddles are the n-th roots of unity of the line length, generated in FP64
// on the host and rounded once (one table per length, cached in the
// context), copied into LDS by each workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fftpde {

// Threads per workgroup, both dtypes; FP32 one-field row passes use the
// smaller variant below (on column passes it ran 30 % slower: a column tile
// of half the points holds half the adjacent columns).
constexpr int mr_threads(bool /*fp64*/) { return 1024; }
constexpr int kMrMaxSide = 4096;
constexpr int kMrMaxColLines = 64;  // columns per column tile
constexpr int kMrMaxStages = 12;

// Points per field and tile: 8192 FP32 (4096 per field with a second
// field), 4096 FP64 (the longest line).  With the padding of column tiles
// and the twiddle table of the line length in LDS (not for FP64 with two
// fields): at most 133 KB of LDS.  Measured at 1000^2..2000^2: FP32 tiles
// of 8192 points beat 4096 (with the next tile staged in registers) and
// 12288 (register spills); the table in LDS beats reading it from L1/L2.
constexpr int mr_cap(bool fp64, int nf) { return fp64 ? 4096 : 8192 / nf; }
// FP32 one-field row passes: 512-thread workgroups on 4096-point tiles, two
// per CU, so that one workgroup's loads overlap the other's stages (1536^2
// rows, 8 fields: 118 us against 127 with the 1024-thread variant).
constexpr int kMrRowTH = 512;
constexpr int kMrRowCap = 4096;
constexpr bool mr_row_small(bool fp64, int nf, bool col) { return !fp64 && nf == 1 && !col; }
constexpr bool mr_tw_in_lds(bool fp64, int nf) { return !(fp64 && nf == 2); }

// Sides the mixed-radix path takes: 2..4096, 7-smooth.
__host__ __device__ constexpr bool mr_side_ok(int n) {
  if (n < 2 || n > kMrMaxSide) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  while (n % 7 == 0) n /= 7;
  return n == 1;
}

// Exact x / d for 0 <= x < 2^16 and 1 <= d < 2^16 by one multiply:
// floor(x M / 2^32) with M = floor(2^32 / d) + 1 (the error x (M - 2^32/d)
// / 2^32 < 2^-16 < 1/d never crosses an integer).
struct MrDiv {
  unsigned long long m = 0;
  MrDiv() = default;
  explicit MrDiv(int d) : m((1ull << 32) / (unsigned long long)d + 1) {}
  __device__ __forceinline__ int operator()(int x) const {
    return (int)(((unsigned long long)(unsigned)x * m) >> 32);
  }
};

// Radix sequence of a length: 8s first, then a 4 or a 2 for the rest of the
// power of two, then 7s, 5s and 3s.
struct MrPlan {
  int n = 0;
  int nst = 0;
  int radix[kMrMaxStages] = {};
  MrDiv by_m[kMrMaxStages];   // n / radix[s]: butterflies per line
  MrDiv by_ns[kMrMaxStages];  // product of the radices before stage s
  MrDiv by_n;
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
  int ns = 1;
  for (int s = 0; s < p.nst; s++) {
    p.by_m[s] = MrDiv(n / p.radix[s]);
    p.by_ns[s] = MrDiv(ns);
    ns *= p.radix[s];
  }
  p.by_n = MrDiv(n);
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
  MrDiv by_lines;
  int ls;     // LDS distance between lines
  long long tiles;
  int mode;
  T scale;    // kMrRowInv
  MrSym sym;  // kMrColSolve
  // Real fields in pairs (rows only): with rin the forward row pass reads
  // pair field p as real fields 2p + i (2p + 1) of rin (the odd last one
  // paired with zero); with rout the inverse row pass writes the real and
  // imaginary parts to them.  nreal real fields; by_ny splits a pair-field
  // row index into (pair, row).
  const T* rin;
  T* rout;
  long long nreal;
  MrDiv by_ny;
};

// grid: persistent workgroups (at most a.tiles); small: the row variant of
// mr_row_small
template <typename T>
hipError_t mr_launch(const MrArgs<T>& a, int nf, bool small, int grid, hipStream_t s);
// resident workgroups per CU of the kernel for (T, nf, small)
template <typename T>
int mr_occupancy(int nf, bool small);

}  // namespace fftpde
