// kernels.hpp -- row-pass and column-pass kernels of the 2D FFT and of the
// fused spectral solves, and the variant tables the host plans from.
//
// A 2D transform is the x-direction (row) transforms for every fixed y,
// then the y-direction (column) transforms for every fixed x frequency
// (Sec. II.D).  A solve is
//     row pass (forward)  ->  column pass [forward, symbol, inverse]  ->  row pass (inverse)
// so the spectrum never leaves registers between the forward column
// transform, the pointwise symbol and the inverse column transform: three
// HBM round trips in all.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace fftpde {

// Column-pass modes.
enum ColMode : int {
  kColForward = 0,     // y-transform forward
  kColInverse = 1,     // y-transform inverse (conjugation identity), times `scale`
  kColFwdMulInv = 2,   // forward, times symbol (with 1/(nx ny) folded in), inverse
  kColMulInv = 3,      // input is already a spectrum: symbol, then inverse
};

// Spectral operators applied between the transforms.
enum SymOp : int {
  kSymScale = 0,      // multiply by `scale` only
  kSymPoisson = 1,    // -1/|k|^2, k = 0 -> 0           (Eq. (SolutionPoisson))
  kSymDiffusion = 2,  // exp(-kappa |k|^2 t)           (Eq. (solCalorFourier))
  kSymWave = 3,       // cos(w t); with a velocity field the full propagator
};

struct SymParams {
  int op;
  int lognx, logny;
  double kxs, kys;  // 2 pi / lx, 2 pi / ly
  double kt;        // diffusion: kappa * t
  double hx, hy;    // wave: 2 c t / lx, 2 c t / ly, so w t / pi = sqrt((hx a')^2 + (hy b')^2)
  double c, t;      // wave: speed and time (for sin(w t)/w and w)
  double scale;     // 1 / (nx ny) for modes that end with the inverse
};

template <typename T>
struct RowArgs {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* tw;
  long long nrows;  // ny * batch
  int inverse;      // 0: forward; 1: inverse (conjugate in and out), times scale
  T scale;
};

template <typename T>
struct ColArgs {
  const cx<T>* in0;   // field (or spectrum) u0
  const cx<T>* in1;   // second field (wave velocity), may be null => 0
  cx<T>* out0;
  cx<T>* out1;        // second output (wave velocity), may be null
  const cx<T>* tw;
  long long ncols;    // nx * batch
  int lognx;
  int mode;           // ColMode
  SymParams sym;
};

// signed frequency index a' of slot a on a 2^logn axis
__device__ __forceinline__ int signed_index(int a, int logn) {
  return a < (1 << (logn - 1)) ? a : a - (1 << logn);
}

// Real symbol M(a, b) for the single-field solves (scale folded in).
template <typename T>
__device__ __forceinline__ T symbol_real(const SymParams& p, int a, int b);

template <>
__device__ __forceinline__ float symbol_real<float>(const SymParams& p, int a, int b) {
  const int ai = signed_index(a, p.lognx), bi = signed_index(b, p.logny);
  switch (p.op) {
    case kSymPoisson: {
      if (ai == 0 && bi == 0) return 0.0f;
      const float kx = float(p.kxs) * float(ai), ky = float(p.kys) * float(bi);
      return -float(p.scale) / (kx * kx + ky * ky);
    }
    case kSymDiffusion: {
      const double kx = p.kxs * ai, ky = p.kys * bi;
      const double arg = p.kt * (kx * kx + ky * ky);  // FP64 exponent
      return float(p.scale) * expf(-float(arg));
    }
    case kSymWave: {
      const double hx = p.hx * ai, hy = p.hy * bi;
      double h = sqrt(hx * hx + hy * hy);  // w t / pi in FP64
      h -= 2.0 * rint(0.5 * h);           // exact reduction to [-1, 1]
      return float(p.scale) * cospif(float(h));
    }
    default:
      return float(p.scale);
  }
}

template <>
__device__ __forceinline__ double symbol_real<double>(const SymParams& p, int a, int b) {
  const int ai = signed_index(a, p.lognx), bi = signed_index(b, p.logny);
  switch (p.op) {
    case kSymPoisson: {
      if (ai == 0 && bi == 0) return 0.0;
      const double kx = p.kxs * ai, ky = p.kys * bi;
      return -p.scale / (kx * kx + ky * ky);
    }
    case kSymDiffusion: {
      const double kx = p.kxs * ai, ky = p.kys * bi;
      return p.scale * exp(-p.kt * (kx * kx + ky * ky));
    }
    case kSymWave: {
      const double hx = p.hx * ai, hy = p.hy * bi;
      return p.scale * cospi(sqrt(hx * hx + hy * hy));
    }
    default:
      return p.scale;
  }
}

// Wave propagator coefficients at mode (a, b): cw = cos(w t), sw = sin(w t),
// sow = sin(w t)/w (t at w = 0), w = c |k|; all but the final rounding in FP64.
template <typename T>
__device__ __forceinline__ void wave_coeffs(const SymParams& p, int a, int b, T& cw, T& sw, T& sow,
                                            T& w_out) {
  const int ai = signed_index(a, p.lognx), bi = signed_index(b, p.logny);
  const double hx = p.hx * ai, hy = p.hy * bi;
  const double kx = p.kxs * ai, ky = p.kys * bi;
  const double w = p.c * sqrt(kx * kx + ky * ky);
  // w t / pi; hx, hy carry t squared away, so restore its sign (sin is odd)
  double h = sqrt(hx * hx + hy * hy);
  if (p.t < 0) h = -h;
  if constexpr (sizeof(T) == 4) {
    h -= 2.0 * rint(0.5 * h);
    float s, c;
    sincospif(float(h), &s, &c);
    cw = c;
    sw = s;
    sow = w == 0.0 ? T(p.t) : T(double(s) / w);
  } else {
    double s, c;
    sincospi(h, &s, &c);
    cw = c;
    sw = s;
    sow = w == 0.0 ? p.t : s / w;
  }
  w_out = T(w);
}

// ---------------------------------------------------------------------------
// Row pass: LINES = E*TH/N rows per workgroup, x contiguous.
// ---------------------------------------------------------------------------
template <typename T, int LOGN, int E, int TH, int MAXLR>
__global__ void __launch_bounds__(TH) row_kernel(RowArgs<T> a) {
  constexpr int N = 1 << LOGN;
  constexpr int LINES = E * TH / N;
  static_assert(LINES >= 1 && LINES * N == E * TH, "tile must hold whole rows");
  using Map = RowMap<LOGN, LINES>;
  using Eng = Engine<T, LOGN, E, TH, MAXLR, false, Map>;
  __shared__ cx<T> lds[Eng::NST > 1 ? Map::kLdsElems : 1];

  const int tid = threadIdx.x;
  const long long row0 = (long long)blockIdx.x * LINES;
  const T sgn = a.inverse ? T(-1) : T(1);
  cx<T> x[E];
  Eng::for_each_input(tid, [&](int i, int line, int n) {
    const long long row = row0 + line;
    cx<T> v = {T(0), T(0)};
    if (row < a.nrows) v = a.in[row * N + n];
    x[i] = {v.re, sgn * v.im};
  });
  Eng::run(x, lds, a.tw, tid);
  const T sr = a.scale, si = sgn * a.scale;
  Eng::for_each_output(tid, [&](int i, int line, int n) {
    const long long row = row0 + line;
    if (row < a.nrows) a.out[row * N + n] = {x[i].re * sr, x[i].im * si};
  });
}

// ---------------------------------------------------------------------------
// Column pass: a tile of T = 2^LOGT adjacent columns of one field; columns
// are numbered C = field * nx + x over the whole batch.
// NF = 2 carries a second field (the wave's velocity) through the pass.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  // Workgroups go round-robin over the 8 XCDs; give each XCD a contiguous
  // range of tiles so that neighbouring tiles (which share 128-byte lines)
  // meet in the same L2.
  const int per = nblocks >> 3;
  if ((nblocks & 7) != 0 || per == 0) return bid;
  return (bid & 7) * per + (bid >> 3);
}

template <typename T, int LOGN, int LOGT, int E, int TH, int MAXLR, int NF>
__global__ void __launch_bounds__(TH) col_kernel(ColArgs<T> a) {
  constexpr int N = 1 << LOGN;
  constexpr int TT = 1 << LOGT;
  static_assert(N * TT == E * TH, "tile must hold whole columns");
  using Map = ColMap<LOGN, LOGT>;
  using Fwd = Engine<T, LOGN, E, TH, MAXLR, false, Map>;
  using Inv = Engine<T, LOGN, E, TH, MAXLR, true, Map>;
  __shared__ cx<T> lds[Fwd::NST > 1 ? Map::kLdsElems : 1];

  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const long long col0 = (long long)tile * TT;
  const int lognx = a.lognx;
  const long long nx = 1ll << lognx;
  const long long fmask = nx - 1;
  // address of element n of tile line `line`, or -1 when the column is padding
  auto addr = [&](int line, int n) -> long long {
    const long long C = col0 + line;
    if (C >= a.ncols) return -1;
    const long long f = C >> lognx, cxi = C & fmask;
    return (f << (lognx + LOGN)) + ((long long)n << lognx) + cxi;
  };
  auto colx = [&](int line) -> int { return int((col0 + line) & fmask); };

  cx<T> x[E];
  cx<T> y[NF == 2 ? E : 1];
  const int mode = a.mode;

  if (mode == kColMulInv) {
    // spectrum in: load at the inverse engine's first-stage positions
    Inv::for_each_input(tid, [&](int i, int line, int n) {
      const long long p = addr(line, n);
      x[i] = p >= 0 ? a.in0[p] : cx<T>{T(0), T(0)};
      if constexpr (NF == 2) y[i] = (p >= 0 && a.in1) ? a.in1[p] : cx<T>{T(0), T(0)};
    });
  } else {
    const T sgn = mode == kColInverse ? T(-1) : T(1);
    Fwd::for_each_input(tid, [&](int i, int line, int n) {
      const long long p = addr(line, n);
      cx<T> v = p >= 0 ? a.in0[p] : cx<T>{T(0), T(0)};
      x[i] = {v.re, sgn * v.im};
      if constexpr (NF == 2) y[i] = (p >= 0 && a.in1) ? a.in1[p] : cx<T>{T(0), T(0)};
    });
    Fwd::run(x, lds, a.tw, tid);
    if constexpr (NF == 2) {
      if (a.in1) Fwd::run(y, lds, a.tw, tid);
    }
    if (mode == kColForward || mode == kColInverse) {
      const T s = mode == kColInverse ? T(a.sym.scale) : T(1);
      Fwd::for_each_output(tid, [&](int i, int line, int n) {
        const long long p = addr(line, n);
        if (p >= 0) a.out0[p] = {x[i].re * s, sgn * x[i].im * s};
      });
      return;
    }
  }

  // Pointwise symbol at (a = column x index, b = n), then conjugate for the
  // inverse (conjugation identity).  The forward engine's last radix is the
  // inverse engine's first, so the positions line up register by register.
  if constexpr (NF == 1) {
    Inv::for_each_input(tid, [&](int i, int line, int n) {
      const T m = symbol_real<T>(a.sym, colx(line), n);
      x[i] = {x[i].re * m, -x[i].im * m};
    });
  } else {
    const bool want_v = a.out1 != nullptr;
    const T sc = T(a.sym.scale);
    Inv::for_each_input(tid, [&](int i, int line, int n) {
      T cw, sw, sow, w;
      wave_coeffs<T>(a.sym, colx(line), n, cw, sw, sow, w);
      const cx<T> F = x[i], G = y[i];
      const cx<T> U = {cw * F.re + sow * G.re, cw * F.im + sow * G.im};
      x[i] = {U.re * sc, -U.im * sc};
      if (want_v) {
        const T ws = -w * sw;
        const cx<T> V = {ws * F.re + cw * G.re, ws * F.im + cw * G.im};
        y[i] = {V.re * sc, -V.im * sc};
      }
    });
  }
  Inv::run(x, lds, a.tw, tid);
  Inv::for_each_output(tid, [&](int i, int line, int n) {
    const long long p = addr(line, n);
    if (p >= 0) a.out0[p] = conjg(x[i]);
  });
  if constexpr (NF == 2) {
    if (a.out1) {
      Inv::run(y, lds, a.tw, tid);
      Inv::for_each_output(tid, [&](int i, int line, int n) {
        const long long p = addr(line, n);
        if (p >= 0) a.out1[p] = conjg(y[i]);
      });
    }
  }
}

// ---------------------------------------------------------------------------
// Variant tables (one entry per compiled kernel configuration).
// ---------------------------------------------------------------------------
using LaunchFn = hipError_t (*)(const void* args, long long units, hipStream_t stream);

struct RowVariant {
  LaunchFn launch;
  int logn, e, th, maxlr, lines;
  int lds_bytes;
  const char* name;
};

struct ColVariant {
  LaunchFn launch;
  int logn, logt, e, th, maxlr, nf;
  int lds_bytes;
  const char* name;
};

template <typename T, int LOGN, int E, int TH, int MAXLR>
hipError_t launch_row(const void* args, long long nrows, hipStream_t s) {
  constexpr int LINES = E * TH / (1 << LOGN);
  const long long grid = (nrows + LINES - 1) / LINES;
  if (grid <= 0 || grid > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL((row_kernel<T, LOGN, E, TH, MAXLR>), dim3((unsigned)grid), dim3(TH), 0, s,
                     *static_cast<const RowArgs<T>*>(args));
  return hipGetLastError();
}

template <typename T, int LOGN, int LOGT, int E, int TH, int MAXLR, int NF>
hipError_t launch_col(const void* args, long long ncols, hipStream_t s) {
  const long long grid = (ncols + (1 << LOGT) - 1) >> LOGT;
  if (grid <= 0 || grid > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL((col_kernel<T, LOGN, LOGT, E, TH, MAXLR, NF>), dim3((unsigned)grid), dim3(TH),
                     0, s, *static_cast<const ColArgs<T>*>(args));
  return hipGetLastError();
}

template <int LOGN, int MAXLR>
constexpr int lds_elems_row(int lines) {
  return plan_nstages(LOGN, MAXLR) > 1 ? lines * ((1 << LOGN) + ((1 << LOGN) >> 3)) : 1;
}
template <int LOGN, int MAXLR>
constexpr int lds_elems_col(int logt) {
  return plan_nstages(LOGN, MAXLR) > 1 ? (((1 << LOGN) + ((1 << LOGN) >> 3)) << logt) : 1;
}

#define FFTPDE_ROW_VARIANT(T, LOGN, E, TH, MAXLR)                                              \
  {&::fftpde::launch_row<T, LOGN, E, TH, MAXLR>, LOGN, E, TH, MAXLR, (E) * (TH) >> (LOGN),     \
   int(::fftpde::lds_elems_row<LOGN, MAXLR>((E) * (TH) >> (LOGN)) * sizeof(::fftpde::cx<T>)), \
   "row_" #T "_n" #LOGN "_e" #E "_th" #TH "_r" #MAXLR}

#define FFTPDE_COL_VARIANT(T, LOGN, LOGT, E, TH, MAXLR, NF)                                       \
  {&::fftpde::launch_col<T, LOGN, LOGT, E, TH, MAXLR, NF>, LOGN, LOGT, E, TH, MAXLR, NF,          \
   int(::fftpde::lds_elems_col<LOGN, MAXLR>(LOGT) * sizeof(::fftpde::cx<T>)),                     \
   "col_" #T "_n" #LOGN "_t" #LOGT "_e" #E "_th" #TH "_r" #MAXLR "_f" #NF}

// Tables defined in the per-dtype translation units.
const RowVariant* row_variants_f32(int* count);
const RowVariant* row_variants_f64(int* count);
const ColVariant* col_variants_f32_nf1(int* count);
const ColVariant* col_variants_f32_nf2(int* count);
const ColVariant* col_variants_f64_nf1(int* count);
const ColVariant* col_variants_f64_nf2(int* count);

}  // namespace fftpde
