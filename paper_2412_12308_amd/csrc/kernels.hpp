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

#include <type_traits>

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
  kSymDiffSource = 4, // diffusion with a source constant in time (three-field pass)
  kSymWaveSource = 5, // wave with a source constant in time (three-field pass)
};

// Where the passes read their twiddles (see Engine::TwSrc).  kTwStageGrp:
// stage tables, each value loaded by one lane of the tile's columns and
// moved to the others across lanes (column tiles of 2 or 4 columns).
enum TwMode : int { kTwGlobal = 0, kTwRegs = 1, kTwLds = 2, kTwStage = 3, kTwStageGrp = 4 };

struct SymParams {
  int op;
  int lognx, logny;
  double kxs, kys;  // 2 pi / lx, 2 pi / ly
  double kt;        // diffusion: kappa * t
  double hx, hy;    // wave: 2 c t / lx, 2 c t / ly, so w t / pi = sqrt((hx a')^2 + (hy b')^2)
  double c, t;      // wave: speed and time (for sin(w t)/w and w); diffusion with a source: kappa and time
  double scale;     // 1 / (nx ny) for modes that end with the inverse
  // 3D solves (the pass along z, whose columns are the nx*ny points of a z
  // plane): lx3 = log2 nx > 0 splits the column index a into x = a mod nx and
  // y = a / nx; ky3s = 2 pi / ly and hy3 = 2 c t / ly scale y, while kxs, hx
  // scale x and kys, hy scale z.  lx3 = 0: 2D.
  int lx3;
  double ky3s, hy3;
  // wave, FP32 fields: every nonzero (w t / pi)^2 of the grid lies in
  // [1e-30, 1e36], so the phase may take the FP32-seeded square root without
  // a range check per coefficient (set by the host from the extreme
  // wavenumbers; 0 = check each coefficient)
  int phase_fast;
};

// A load of streamed data read once: the non-temporal hint keeps it from
// displacing cached lines (twiddles, neighbouring tiles).  Measured on the
// 2048-point row passes: 5 % faster in FP32 and FP64.
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  return {__builtin_nontemporal_load(&p->re), __builtin_nontemporal_load(&p->im)};
}

template <typename T>
struct RowArgs {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* tw;
  long long nrows;  // ny * batch
  int inverse;      // 0: forward; 1: inverse (conjugate in and out), times scale
  T scale;
  // Layouts of in and out: a field is stored in blocks of 2^t columns x ny
  // rows, element (y, x) at block (x >> t), offset y * 2^t + (x & (2^t - 1))
  // within it; t = log2 of the row length is the plain row-major layout.
  int logny;
  int in_t, out_t;
  // Real fields in pairs (row kernels compiled with RIO = 1: real input,
  // RIO = 2: real output; the other side is complex as usual): row r of the
  // pass is row y = r mod ny of real fields 2p and 2p + 1 (p = r / ny),
  // row-major points of type T, taken as the real and imaginary parts of one
  // complex row.  nreal fields exist: field 2p + 1 >= nreal reads as zero and
  // is not written.
  long long nreal;
};

template <typename T>
struct ColArgs {
  const cx<T>* in0;   // field (or spectrum) u0
  const cx<T>* in1;   // second field (wave velocity), may be null => 0
  const cx<T>* in2;   // third field (NF = 3: the source)
  cx<T>* out0;
  cx<T>* out1;        // second output (wave velocity), may be null
  const cx<T>* tw;
  long long ncols;    // nx * batch
  int lognx;
  int mode;           // ColMode
  SymParams sym;
  int layout_t;       // fields stored in blocks of 2^layout_t >= 2^LOGT columns (see RowArgs); -1 row-major
  // Stage tables (Engine::stw_off) of the forward and the inverse engine's
  // plans, for TWM = kTwStage.
  const cx<T>* twf;
  const cx<T>* twi;
};

// a type carried as a value (to pass an engine type to a generic lambda)
template <class E>
struct EngTag {
  using type = E;
};

// signed frequency index a' of slot a on a 2^logn axis
__device__ __forceinline__ int signed_index(int a, int logn) {
  return a < (1 << (logn - 1)) ? a : a - (1 << logn);
}

// ---------------------------------------------------------------------------
// Spectral symbols.  A column tile holds one x frequency a per line, so each
// evaluator is built once per column (terms in k_x) and then called for each
// y frequency b.  The multipliers include the inverse's 1/(nx ny).
// ---------------------------------------------------------------------------

// sqrt of a non-negative FP64 value to about 1e-14 relative: an FP32 square
// root refined by one Newton step in FP64 (the error squares), cheaper than
// the correctly rounded FP64 root and ample for an FP32 result.  Values that
// the FP32 seed cannot represent (positive below 1e-30, e.g. a wave speed
// near zero, or above 1e36) take the FP64 root; 0 and negatives give 0.
__device__ __forceinline__ double sqrt_fp64_from_fp32(double v) {
  if (!(v >= 1e-30 && v <= 1e36)) return v > 0.0 ? sqrt(v) : 0.0;
  const float s0 = __builtin_amdgcn_sqrtf(float(v));
  const double d = double(s0);
  const double r = fma(-d, d, v);
  return fma(r, double(0.5f * __builtin_amdgcn_rcpf(s0)), d);
}

// cos(pi r) for |r| <= 1/2 in FP32: the Taylor series of cos about 0 in
// u = r^2, terms (-1)^k pi^(2k) / (2k)! u^k for k <= 6, evaluated by Horner's
// rule.  The first omitted term is below (pi/2)^14 / 14! < 7e-9, under FP32
// rounding of values near 1.
constexpr double cospi_taylor(int k) {
  double c = 1.0;
  for (int i = 1; i <= 2 * k; i++) c *= 3.14159265358979323846264338327950288 / i;
  return (k & 1) ? -c : c;
}
__device__ __forceinline__ float cospi_half(float r) {
  const float u = r * r;
  float p = float(cospi_taylor(6));
  p = fmaf(p, u, float(cospi_taylor(5)));
  p = fmaf(p, u, float(cospi_taylor(4)));
  p = fmaf(p, u, float(cospi_taylor(3)));
  p = fmaf(p, u, float(cospi_taylor(2)));
  p = fmaf(p, u, float(cospi_taylor(1)));
  return fmaf(p, u, 1.0f);
}

template <typename T, int OP>
struct Symbol;

// -1/|k|^2, k = 0 -> 0 (Eq. (SolutionPoisson) with the mean dropped, Eq. (Poisson2))
template <typename T>
struct Symbol<T, kSymPoisson> {
  T kx2, kys, nscale;
  bool a0;
  int logny;
  __device__ __forceinline__ Symbol(const SymParams& p, int a) {
    if (p.lx3 > 0) {
      const int xi = signed_index(a & ((1 << p.lx3) - 1), p.lx3), yi = signed_index(a >> p.lx3, p.lognx - p.lx3);
      const T kx = T(p.kxs) * T(xi), ky = T(p.ky3s) * T(yi);
      kx2 = kx * kx + ky * ky;
      a0 = xi == 0 && yi == 0;
    } else {
      const int ai = signed_index(a, p.lognx);
      const T kx = T(p.kxs) * T(ai);
      kx2 = kx * kx;
      a0 = ai == 0;
    }
    kys = T(p.kys);
    nscale = -T(p.scale);
    logny = p.logny;
  }
  __device__ __forceinline__ T operator()(int b) const {
    const int bi = signed_index(b, logny);
    const T ky = kys * T(bi);
    const T k2 = kx2 + ky * ky;
    T m;
    if constexpr (sizeof(T) == 4) m = nscale * __builtin_amdgcn_rcpf(k2);
    else m = nscale / k2;
    return (a0 && bi == 0) ? T(0) : m;
  }
  // at b' = j + dd (see Symbol<T, kSymWave>::split)
  __device__ __forceinline__ bool split_ok() const { return true; }
  __device__ __forceinline__ T split(int j, int dd) const { return (*this)(0, j + dd); }
  __device__ __forceinline__ T operator()(int, int bi) const {
    const T ky = kys * T(bi);
    const T k2 = kx2 + ky * ky;
    T m;
    if constexpr (sizeof(T) == 4) m = nscale * __builtin_amdgcn_rcpf(k2);
    else m = nscale / k2;
    return (a0 && bi == 0) ? T(0) : m;
  }
};

// exp(-kappa |k|^2 t) (Eq. (solCalorFourier)); exponent formed in FP64
template <typename T>
struct Symbol<T, kSymDiffusion> {
  double ex, kt, kys;
  T scale;
  int logny;
  __device__ __forceinline__ Symbol(const SymParams& p, int a) {
    kt = p.kt;
    if (p.lx3 > 0) {
      const double kx = p.kxs * signed_index(a & ((1 << p.lx3) - 1), p.lx3);
      const double ky = p.ky3s * signed_index(a >> p.lx3, p.lognx - p.lx3);
      ex = kt * fma(kx, kx, ky * ky);
    } else {
      const double kx = p.kxs * signed_index(a, p.lognx);
      ex = kt * kx * kx;
    }
    kys = p.kys;
    scale = T(p.scale);
    logny = p.logny;
  }
  __device__ __forceinline__ T operator()(int b) const {
    const double ky = kys * signed_index(b, logny);
    const double arg = fma(kt * ky, ky, ex);
    if constexpr (sizeof(T) == 4) return scale * expf(-float(arg));
    else return scale * exp(-arg);
  }
  // at b' = j + dd (see Symbol<T, kSymWave>::split)
  __device__ __forceinline__ bool split_ok() const { return true; }
  __device__ __forceinline__ T split(int j, int dd) const {
    const double ky = fma(kys, double(dd), kys * double(j));
    const double arg = fma(kt * ky, ky, ex);
    if constexpr (sizeof(T) == 4) return scale * expf(-float(arg));
    else return scale * exp(-arg);
  }
};

// sqrt of v in [1e-30, 1e36] (or 0) to about 1e-14 relative: an FP32
// reciprocal square root y of v, then one Newton step in FP64 on s = v y,
// s + (y/2)(v - s^2) (the error squares).  The FP32 operand is kept at
// 1e-30 or above, so v = 0 gives y finite and s = 0 exactly.
__device__ __forceinline__ double sqrt_fp64_ranged(double v) {
  const float y = __builtin_amdgcn_rsqf(fmaxf(float(v), 1e-30f));
  const double yd = double(y);
  const double s = v * yd;
  return fma(0.5 * yd, fma(-s, s, v), s);
}

// cos(pi r) for |r| <= 1/2 in FP64: the same series through u^11; the first
// omitted term is below (pi/2)^24 / 24! < 1e-19.
__device__ __forceinline__ double cospi_half_fp64(double r) {
  const double u = r * r;
  double p = cospi_taylor(11);
  p = fma(p, u, cospi_taylor(10));
  p = fma(p, u, cospi_taylor(9));
  p = fma(p, u, cospi_taylor(8));
  p = fma(p, u, cospi_taylor(7));
  p = fma(p, u, cospi_taylor(6));
  p = fma(p, u, cospi_taylor(5));
  p = fma(p, u, cospi_taylor(4));
  p = fma(p, u, cospi_taylor(3));
  p = fma(p, u, cospi_taylor(2));
  p = fma(p, u, cospi_taylor(1));
  return fma(p, u, 1.0);
}

// sqrt of v in [1e-30, 1e36] (or 0) to FP64 rounding: sqrt_fp64_ranged's
// step taken twice (the second leaves an error near 1e-21 before rounding).
__device__ __forceinline__ double sqrt_fp64_ranged2(double v) {
  const float y = __builtin_amdgcn_rsqf(fmaxf(float(v), 1e-30f));
  const double hy = 0.5 * double(y);
  double s = v * double(y);
  s = fma(hy, fma(-s, s, v), s);
  return fma(hy, fma(-s, s, v), s);
}

// cos(pi h) for FP64 h >= 0 in FP32: h is reduced exactly to r in [-1, 1]
// (h minus an even integer), then to f = r - m in [-1/2, 1/2] with m in
// {-1, 0, 1}; cos(pi r) = (-1)^m cos(pi f).
__device__ __forceinline__ float cospi_reduced(double h) {
  const double r = fma(-2.0, rint(0.5 * h), h);
  const double m = rint(r);
  const float c = cospi_half(float(r - m));
  return m != 0.0 ? -c : c;
}
// the same in FP64
__device__ __forceinline__ double cospi_reduced_fp64(double h) {
  const double r = fma(-2.0, rint(0.5 * h), h);
  const double m = rint(r);
  const double c = cospi_half_fp64(r - m);
  return m != 0.0 ? -c : c;
}

// cos(c |k| t), the wave propagator with zero initial velocity
// (Eq. (OmegaNonZero), (OmegaZero)); phase in FP64 half-turns, reduced in FP64
template <typename T>
struct Symbol<T, kSymWave> {
  double hx2, hy;
  T scale;
  int logny;
  bool fast;
  __device__ __forceinline__ Symbol(const SymParams& p, int a) {
    fast = p.phase_fast != 0;
    if (p.lx3 > 0) {
      const double hx = p.hx * signed_index(a & ((1 << p.lx3) - 1), p.lx3);
      const double hyy = p.hy3 * signed_index(a >> p.lx3, p.lognx - p.lx3);
      hx2 = fma(hx, hx, hyy * hyy);
    } else {
      const double hx = p.hx * signed_index(a, p.lognx);
      hx2 = hx * hx;
    }
    hy = p.hy;
    scale = T(p.scale);
    logny = p.logny;
  }
  __device__ __forceinline__ T operator()(int b) const {
    const double hyb = hy * signed_index(b, logny);
    const double h2 = fma(hyb, hyb, hx2);
    if constexpr (sizeof(T) == 4) {
      double h = sqrt_fp64_from_fp32(h2);  // w t / pi
      h = fma(-2.0, rint(0.5 * h), h);     // exact reduction to [-1, 1]
      // cos(pi h) = (-1)^m cos(pi (h - m)), m = rint(h) in {-1, 0, 1}; h - m
      // is exact and lies in [-1/2, 1/2]
      const double m = rint(h);
      const float c = cospi_half(float(h - m));
      return (m != 0.0 ? -scale : scale) * c;
    } else {
      return scale * cospi(sqrt(h2));
    }
  }
  // The same at the signed index b' = j + dd (j >= 0; dd a compile-time
  // offset of the caller's unrolled loop, so hy j is formed once per j), only
  // where `fast` holds (split_ok): the square root starts from an FP32 seed.
  __device__ __forceinline__ bool split_ok() const { return fast; }
  __device__ __forceinline__ T split(int j, int dd) const {
    const double hyb = fma(hy, double(dd), hy * double(j));
    const double h2 = fma(hyb, hyb, hx2);
    if constexpr (sizeof(T) == 4) return scale * cospi_reduced(sqrt_fp64_ranged(h2));
    else return scale * cospi_reduced_fp64(sqrt_fp64_ranged2(h2));
  }
};

template <typename T>
struct Symbol<T, kSymScale> {
  T scale;
  __device__ __forceinline__ Symbol(const SymParams& p, int) : scale(T(p.scale)) {}
  __device__ __forceinline__ T operator()(int) const { return scale; }
  __device__ __forceinline__ bool split_ok() const { return true; }
  __device__ __forceinline__ T split(int, int) const { return scale; }
};

// Wave propagator with an initial velocity: cw = cos(w t), sw = sin(w t),
// sow = sin(w t)/w (t at w = 0), w = c |k|.  FP64: all but the final
// rounding in FP64.  FP32: the phase w t formed and reduced in FP64, then
// FP32 sin/cos; w and sin(w t)/w, which only scale FP32 values, in FP32.
template <typename T>
struct WaveCoeffs {
  double hx2, hy, kx2, kys, c, t;
  int logny;
  __device__ __forceinline__ WaveCoeffs(const SymParams& p, int a) {
    const int ai = signed_index(a, p.lognx);
    const double hx = p.hx * ai, kx = p.kxs * ai;
    hx2 = hx * hx;
    kx2 = kx * kx;
    hy = p.hy;
    kys = p.kys;
    c = p.c;
    t = p.t;
    logny = p.logny;
  }
  __device__ __forceinline__ void operator()(int b, T& cw, T& sw, T& sow, T& w_out) const {
    const int bi = signed_index(b, logny);
    const double hyb = hy * bi, ky = kys * bi;
    if constexpr (sizeof(T) == 4) {
      // the phase w t / pi in FP64 (square root from an FP32 seed and one
      // FP64 correction), reduced exactly; w itself only scales FP32 values,
      // so it and sin(w t)/w are formed in FP32
      double h = sqrt_fp64_from_fp32(fma(hyb, hyb, hx2));
      if (t < 0) h = -h;  // hx, hy carry t squared away; sin is odd
      h = fma(-2.0, rint(0.5 * h), h);
      float s, cc;
      sincospif(float(h), &s, &cc);
      const float w = float(c) * __builtin_amdgcn_sqrtf(float(fma(ky, ky, kx2)));
      cw = cc;
      sw = s;
      // below 1e-18, sin(w t)/w = t to far better than FP32 (and 1/w would overflow)
      sow = w > 1e-18f ? s * __builtin_amdgcn_rcpf(w) : T(t);
      w_out = w;
    } else {
      const double w = c * sqrt(fma(ky, ky, kx2));
      // w t / pi; hx, hy carry t squared away, so restore its sign (sin is odd)
      double h = sqrt(fma(hyb, hyb, hx2));
      if (t < 0) h = -h;
      double s, cc;
      sincospi(h, &s, &cc);
      cw = cc;
      sw = s;
      sow = w == 0.0 ? t : s / w;
      w_out = w;
    }
  }
};

// Sources constant in time, per coefficient (the forced decay and the
// forced oscillator of Sec. III.B and III.C, with the oscillator's constant
// particular solution s^/w^2):
//   diffusion  U = e F + m S,  e = exp(-q t), m = (1 - e)/q (t at q = 0), q = kappa|k|^2
//   wave       U = cos(w t) F + sin(w t)/w G + p S,  V = -w sin(w t) F + cos(w t) G + sin(w t)/w S,
//              p = (1 - cos(w t))/w^2 = 2 sin^2(w t/2)/w^2 (t^2/2 at w = 0)
// The half-angle form and expm1 keep p and m accurate where w t or q t is
// small.  Arguments (q t and the phase w t) are formed in FP64; with FP32
// fields, w and the ratios that only scale FP32 values are FP32.
template <typename T>
struct SourceCoeffs {
  int op, logny;
  double kx2, kys, hx2, hy, c, t;
  __device__ __forceinline__ SourceCoeffs(const SymParams& p, int a) {
    const int ai = signed_index(a, p.lognx);
    const double kx = p.kxs * ai, hx = p.hx * ai;
    op = p.op;
    logny = p.logny;
    kx2 = kx * kx;
    kys = p.kys;
    hx2 = hx * hx;
    hy = p.hy;
    c = p.c;
    t = p.t;
  }
  // (uf, ug, us): U's weights of F, G, S; (vf, vg, vs): V's
  __device__ __forceinline__ void operator()(int b, T& uf, T& ug, T& us, T& vf, T& vg, T& vs) const {
    const int bi = signed_index(b, logny);
    const double ky = kys * bi;
    const double k2 = fma(ky, ky, kx2);
    if (op == kSymDiffSource) {
      const double q = c * k2;  // c carries kappa
      const double em1 = expm1(-q * t);
      uf = T(1.0 + em1);
      us = q > 0.0 ? T(-em1 / q) : T(t);
      ug = vf = vg = vs = T(0);
      return;
    }
    const double hyb = hy * bi;
    if constexpr (sizeof(T) == 4) {
      // the phase in FP64 (square root from an FP32 seed and one FP64
      // correction) reduced exactly to [-1, 1]; w, which only scales FP32
      // values, in FP32
      double h = sqrt_fp64_from_fp32(fma(hyb, hyb, hx2));  // |w t| / pi
      if (t < 0) h = -h;
      h = fma(-2.0, rint(0.5 * h), h);
      float s1, c1;
      sincospif(float(h), &s1, &c1);
      const float hs = sinpif(float(0.5 * h));  // sin(w t/2) up to sign
      const float w = float(c) * __builtin_amdgcn_sqrtf(float(k2));
      // below 1e-18 the w -> 0 limits hold to far better than FP32
      const bool live = w > 1e-18f;
      const float rw = live ? __builtin_amdgcn_rcpf(w) : 0.0f;
      const float sow = live ? s1 * rw : float(t);
      const float hw = hs * rw;
      uf = c1;
      ug = sow;
      us = live ? 2.0f * hw * hw : float(0.5 * t * t);
      vf = -w * s1;
      vg = c1;
      vs = sow;
    } else {
      const double w = c * sqrt(k2);
      double h = sqrt(fma(hyb, hyb, hx2));  // |w t| / pi
      if (t < 0) h = -h;
      double cw, sw;
      sincospi(h, &sw, &cw);
      const double hs = sinpi(0.5 * h);
      const double sow = w == 0.0 ? t : sw / w;
      uf = cw;
      ug = sow;
      us = w == 0.0 ? 0.5 * t * t : 2.0 * hs * hs / (w * w);
      vf = -w * sw;
      vg = cw;
      vs = sow;
    }
  }
};

// ---------------------------------------------------------------------------
// Row pass: LINES = E*TH/N rows per tile, x contiguous.  Workgroups walk
// tiles persistently; with PF the next tile's rows are loaded into registers
// while the current tile is transformed, so HBM reads continue through the
// LDS exchanges.
// ---------------------------------------------------------------------------
// 16-byte (or narrower, for rows shorter than that) vectors of real points.
template <typename T, int VEC>
struct RealVec {
  typedef T type __attribute__((ext_vector_type(VEC)));
};

// RIO = 0: complex rows in and out.  RIO = 1: the input is real fields in
// pairs (RowArgs::real_in), RIO = 2: the output is (RowArgs::real_out).  Real
// rows move as whole 16-byte vectors, staged through the LDS buffer between
// their row-major order and the engine's first-stage (or last-stage) order.
template <typename T, int LOGN, int E, int TH, int MAXLR, bool PF, int TWM, int RIO>
__global__ void __launch_bounds__(TH) row_kernel(RowArgs<T> a) {
  constexpr int N = 1 << LOGN;
  constexpr int LINES = E * TH / N;
  static_assert(LINES >= 1 && LINES * N == E * TH, "tile must hold whole rows");
  static_assert(TWM == kTwGlobal || TWM == kTwRegs, "row pass twiddles: global table or registers");
  using Map = RowMap<LOGN, LINES, plan_pad(LOGN, MAXLR, false)>;
  using Eng = Engine<T, LOGN, E, TH, MAXLR, false, Map, false>;
  // real rows are staged through LDS even when the transform needs no exchange
  constexpr int kLds = (RIO != 0 && Map::kLdsElems > Eng::kLdsWords) ? Map::kLdsElems : Eng::kLdsWords;
  __shared__ typename Eng::Word lds[kLds];

  int tid = threadIdx.x;
  const long long ntiles = (a.nrows + LINES - 1) / LINES;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  const int logny = a.logny;
  const long long ymask = (1ll << logny) - 1;
  // element offset of (row, n) in a layout of 2^t-column blocks (t = LOGN: row-major)
  auto offset = [&](long long row, int n, int t) -> long long {
    const long long f = row >> logny, yy = row & ymask;
    return (f << (logny + LOGN)) + ((long long)(n >> t) << (logny + t)) + (yy << t) + (n & ((1 << t) - 1));
  };
  // raw loads; the inverse's conjugation is applied when the tile is consumed
  // so that a prefetch never waits for its own data
  auto load = [&](long long tile, cx<T>(&dst)[E]) {
    const long long row0 = tile * LINES;
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      // clamped, unconditional loads (padding rows reread the last row and are
      // never stored) keep the loads free of branches
      const long long row = min(row0 + line, a.nrows - 1);
      dst[i] = load_stream(&a.in[offset(row, n, a.in_t)]);
    });
  };

  // Real pairs: pass row r is row y = r mod ny of real fields 2p and 2p + 1
  // (p = r / ny); each thread moves KV vectors of VEC points per field.
  constexpr int VEC = (16 / (int)sizeof(T)) < N ? 16 / (int)sizeof(T) : N;
  using RV = typename RealVec<T, VEC>::type;
  constexpr int VROW = N / VEC;
  constexpr int KV = LINES * VROW / TH;
  static_assert(RIO == 0 || (KV >= 1 && KV * TH == LINES * VROW), "real rows: whole vectors per thread");
  const long long field_pts = 1ll << (logny + LOGN);
  auto real_row = [&](long long row) -> long long {
    const long long p = row >> logny, yy = row & ymask;
    return (((2 * p) << logny) + yy) << LOGN;
  };
  auto has_second = [&](long long row) { return 2 * (row >> logny) + 1 < a.nreal; };
  RV rv[RIO == 1 ? 2 * KV : 1];
  // loads of a tile's real rows (padding rows reread the last row); a missing
  // second field reads the first field's row and is replaced by zeros
  auto rload = [&](long long tile) {
    const T* in = reinterpret_cast<const T*>(a.in);
#pragma unroll
    for (int k = 0; k < KV; k++) {
      const int f = tid + TH * k, line = f / VROW, n0 = (f % VROW) * VEC;
      const long long row = min(tile * LINES + line, a.nrows - 1);
      const bool two = has_second(row);
      const T* re = in + real_row(row) + n0;
      const RV u = __builtin_nontemporal_load(reinterpret_cast<const RV*>(re));
      const RV v = __builtin_nontemporal_load(reinterpret_cast<const RV*>(two ? re + field_pts : re));
      rv[k] = u;
      rv[KV + k] = two ? v : RV(T(0));
    }
  };
  // the loaded real rows into the engine's input order
  auto rstage_in = [&](cx<T>(&dst)[E]) {
#pragma unroll
    for (int k = 0; k < KV; k++) {
      const int f = tid + TH * k, line = f / VROW, n0 = (f % VROW) * VEC;
#pragma unroll
      for (int j = 0; j < VEC; j++) lds[Map::lds(line, n0 + j)] = cx<T>{rv[k][j], rv[KV + k][j]};
    }
    lds_barrier();
    Eng::for_each_input(tid, [&](int i, int line, int n) { dst[i] = lds[Map::lds(line, n)]; });
    lds_barrier();
  };
  // the last stage's outputs back to real rows: real parts to field 2p,
  // imaginary parts to field 2p + 1
  auto rstore = [&](long long tile, const cx<T>(&src)[E], T sr, T si) {
    Eng::for_each_output(tid, [&](int i, int line, int n) { lds[Map::lds(line, n)] = src[i]; });
    lds_barrier();
    T* out = reinterpret_cast<T*>(a.out);
#pragma unroll
    for (int k = 0; k < KV; k++) {
      const int f = tid + TH * k, line = f / VROW, n0 = (f % VROW) * VEC;
      const long long row = tile * LINES + line;
      RV u, v;
#pragma unroll
      for (int j = 0; j < VEC; j++) {
        const cx<T> w = lds[Map::lds(line, n0 + j)];
        u[j] = w.re * sr;
        v[j] = w.im * si;
      }
      if (row < a.nrows) {
        T* re = out + real_row(row) + n0;
        *reinterpret_cast<RV*>(re) = u;
        if (has_second(row)) *reinterpret_cast<RV*>(re + field_pts) = v;
      }
    }
    lds_barrier();
  };

  cx<T> wall[TWM == kTwRegs ? Eng::kTwRegs : 1];
  if constexpr (TWM == kTwRegs) Eng::load_all_tw(wall, a.tw, tid);
  const T sgn = a.inverse ? T(-1) : T(1);
  const T sr = a.scale, si = sgn * a.scale;
  cx<T> x[E];
  cx<T> nxt[(PF && RIO != 1) ? E : 1];
  long long tile = walk.first;
  if constexpr (RIO == 1) rload(tile);
  else load(tile, x);
  while (true) {
    tid = opaque(tid);
    const long long nt = walk.next(tile);
    const bool more = nt >= 0;
    if constexpr (RIO == 1) {
      rstage_in(x);
      // the vector registers are free again: the next tile's rows go there
      if constexpr (PF) {
        if (more) rload(nt);
      }
    } else if constexpr (PF) {
      // FP32: the next tile's loads at raised wave priority, ahead of the
      // other resident workgroups' arithmetic (2048 rows: 94.3 -> 93.0 us per
      // 8-field chunk)
      if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(3);
      if (more) load(nt, nxt);
      if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
    }
#pragma unroll
    for (int i = 0; i < E; i++) x[i].im *= sgn;
    if constexpr (TWM == kTwRegs) Eng::run_regs(x, lds, wall, tid);
    else Eng::run(x, lds, a.tw, tid);
    const long long row0 = tile * LINES;
    if constexpr (RIO == 2) {
      rstore(tile, x, sr, si);
    } else {
      Eng::for_each_output(tid, [&](int i, int line, int n) {
        const long long row = row0 + line;
        if (row < a.nrows) a.out[offset(row, n, a.out_t)] = {x[i].re * sr, x[i].im * si};
      });
    }
    if (!more) break;
    if constexpr (RIO == 1) {
      if constexpr (!PF) rload(nt);
    } else if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < E; i++) x[i] = nxt[i];
    } else {
      load(nt, x);
    }
    tile = nt;
  }
}

// ---------------------------------------------------------------------------
// Column pass: a tile of T = 2^LOGT adjacent columns of one field; columns
// are numbered C = field * nx + x over the whole batch.  NF = 2 carries a
// second field (the wave's velocity) through the pass; NF = 3 a third (a
// source constant in time).  SPLIT exchanges the
// real and imaginary parts through LDS one after the other (half the LDS, so
// two workgroups fit per CU at the large sizes); PF prefetches the next tile;
// FUSED compiles the [forward, symbol, inverse] mode alone.
// ---------------------------------------------------------------------------
// XW: the two exchanges around the radix-8 stage stay inside each wavefront
// (ColMapWave: 2048-point FP32 columns, tiles of 4, 16 points per thread on
// 512 threads, the fused one-field pass).
template <typename T, int LOGN, int LOGT, int E, int TH, int MAXLR, int NF, bool SPLIT, bool PF, int TWM, bool FUSED,
          bool XW = false>
__global__ void __launch_bounds__(TH) col_kernel(ColArgs<T> a) {
  constexpr int N = 1 << LOGN;
  constexpr int TT = 1 << LOGT;
  static_assert(N * TT == E * TH, "tile must hold whole columns");
  static_assert(TWM == kTwGlobal || TWM == kTwLds || TWM == kTwStage || TWM == kTwStageGrp,
                "column pass twiddles: global table, LDS or stage tables");
  // When TH is a multiple of T every thread stays on one column of the tile.
  constexpr bool kOneCol = (TH % TT) == 0;
  // kTwStageGrp: the T consecutive lanes of a butterfly index share twiddles
  static_assert(TWM != kTwStageGrp || (kOneCol && (TT == 2 || TT == 4)), "shared twiddles: tiles of 2 or 4 columns");
  constexpr int kTwg = TWM == kTwStageGrp ? TT : 1;
  // The symbols are even in the signed row index b'.  Where the inverse's
  // first stage gives each thread two butterflies, the fused one-field pass
  // pairs them as mirrors (ColMapMirror), so that each thread evaluates the
  // symbol once for rows b' and -b' (R0 + 1 evaluations for 2 R0 values).
  constexpr int kLr0 = plan_lr(LOGN, MAXLR, 0, true);
  constexpr int kR0 = 1 << kLr0;
  static_assert(!XW || (sizeof(T) == 4 && LOGN == 11 && LOGT == 2 && E == 16 && TH == 512 && MAXLR == 4 && NF == 1 &&
                        FUSED),
                "in-wave exchanges: the fused 2048-point FP32 pass on 4-column tiles");
  constexpr bool kMirror = !XW && FUSED && NF == 1 && kOneCol && LOGN >= 3 && E == 2 * kR0;
  constexpr int kMlm = kMirror ? LOGN - kLr0 : -1;
  using FMap0 = typename std::conditional<kMirror, ColMapMirror<LOGN, LOGT, plan_pad(LOGN, MAXLR, false), kMlm>,
                                          ColMap<LOGN, LOGT, plan_pad(LOGN, MAXLR, false)>>::type;
  using IMap0 = typename std::conditional<kMirror, ColMapMirror<LOGN, LOGT, plan_pad(LOGN, MAXLR, true), kMlm>,
                                          ColMap<LOGN, LOGT, plan_pad(LOGN, MAXLR, true)>>::type;
  using FMap = typename std::conditional<XW, ColMapWave<plan_pad(LOGN, MAXLR, false), false>, FMap0>::type;
  using IMap = typename std::conditional<XW, ColMapWave<plan_pad(LOGN, MAXLR, true), true>, IMap0>::type;
  using Fwd = Engine<T, LOGN, E, TH, MAXLR, false, FMap, SPLIT, kTwg>;
  using Inv = Engine<T, LOGN, E, TH, MAXLR, true, IMap, SPLIT, kTwg>;
  constexpr int kLdsWords = Fwd::kLdsWords > Inv::kLdsWords ? Fwd::kLdsWords : Inv::kLdsWords;
  __shared__ typename Fwd::Word lds[kLdsWords];
  __shared__ cx<T> twl[TWM == kTwLds ? N : 1];

  int tid = threadIdx.x;
  const long long ntiles = (a.ncols + TT - 1) >> LOGT;
  // One tile at a time: neighbouring tiles (which share 64-byte chunks when
  // tiles are narrower) run concurrently on the same XCD, so their reads of a
  // shared chunk meet in L2.  (Walking narrow tiles in pairs per workgroup
  // merges the writes but reads the second half after its line has left L2:
  // measured 1.8x the algorithmic traffic against 1.2x for this order.)
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  const int lognx = a.lognx;
  const long long fmask = (1ll << lognx) - 1;
  // FUSED: the solves' pass [forward, symbol, inverse] only; the other modes'
  // code is left out, which frees registers (one more resident wave per SIMD).
  const int mode = FUSED ? int(kColFwdMulInv) : a.mode;
  const bool spec_in = mode == kColMulInv;
  const T sgn = mode == kColInverse ? T(-1) : T(1);
  const bool has_in1 = a.in1 != nullptr;

  // Row stride 2^ts: nx for row-major fields, the block width for fields
  // stored in column blocks (a block holds whole tiles).
  const int ts = a.layout_t >= 0 ? a.layout_t : lognx;
  const long long tmask = (1ll << ts) - 1;
  // Element offset of (column C, row 0) of the batch; row n adds n << ts.
  auto col_base = [&](long long C) -> long long {
    const long long xa = C & fmask;
    return ((C >> lognx) << (lognx + LOGN)) + ((xa >> ts) << (LOGN + ts)) + (xa & tmask);
  };
  // When nx >= T every tile lies in one block of one field: its column c at
  // row n is element base + (n << ts) + c, with base wave-uniform.  Each
  // access is then a uniform row part d << ts (d a compile-time multiple of
  // N/R) on a scalar base plus one 32-bit per-thread byte offset that is
  // formed once per butterfly, instead of a 64-bit address per element.
  const bool whole = kOneCol && lognx >= LOGT;
  auto at_row = [&](auto* base, unsigned off, int d) {
    using P = decltype(base);
    using B = typename std::conditional<std::is_const<typename std::remove_pointer<P>::type>::value, const char,
                                        char>::type;
    return reinterpret_cast<P>(reinterpret_cast<B*>(base + ((long long)d << ts)) + off);
  };
  auto row_off = [&](int j, int line) -> unsigned {
    return (((unsigned)j << ts) + (unsigned)line) * (unsigned)sizeof(cx<T>);
  };
  // Loads are clamped to the last column (padding columns are reread and never
  // stored), so loads carry no branches and prefetches stay in flight.
  auto load = [&](long long tile, cx<T>(&dx)[E], cx<T>(&dy)[NF >= 2 ? E : 1], cx<T>(&dz)[NF == 3 ? E : 1]) {
    const long long col0 = tile << LOGT;
    if (whole) {
      const long long cb = col_base(col0);
      const cx<T>* b0 = a.in0 + cb;
      const cx<T>* b1 = has_in1 ? a.in1 + cb : a.in0;
      const cx<T>* b2 = NF == 3 ? a.in2 + cb : a.in0;
      auto g = [&](int i, int line, int j, int d) {
        const unsigned off = row_off(j, line);
        dx[i] = *at_row(b0, off, d);
        if constexpr (NF >= 2) dy[i] = has_in1 ? *at_row(b1, off, d) : cx<T>{T(0), T(0)};
        if constexpr (NF == 3) dz[i] = *at_row(b2, off, d);
      };
      if (spec_in) Inv::for_each_input_split(tid, g);
      else Fwd::for_each_input_split(tid, g);
      return;
    }
    long long cb = 0;
    if constexpr (kOneCol) cb = col_base(min(col0 + (tid & (TT - 1)), a.ncols - 1));
    auto f = [&](int i, int line, int n) {
      long long p;
      if constexpr (kOneCol) p = cb + ((long long)n << ts);
      else p = col_base(min(col0 + line, a.ncols - 1)) + ((long long)n << ts);
      dx[i] = a.in0[p];
      if constexpr (NF >= 2) dy[i] = has_in1 ? a.in1[p] : cx<T>{T(0), T(0)};
      if constexpr (NF == 3) dz[i] = a.in2[p];
    };
    if (spec_in) Inv::for_each_input(tid, f);
    else Fwd::for_each_input(tid, f);
  };
  // Stores of engine Eng's last-stage outputs, skipping padding columns.
  auto emit = [&](auto eng_tag, long long col0, cx<T>* out, auto&& value) {
    using Eng = typename decltype(eng_tag)::type;
    if (whole) {
      cx<T>* b = out + col_base(col0);
      Eng::for_each_output_split(tid, [&](int i, int line, int j, int d) { *at_row(b, row_off(j, line), d) = value(i); });
    } else if constexpr (kOneCol) {
      const long long C = col0 + (tid & (TT - 1));
      if (C >= a.ncols) return;
      cx<T>* o = out + col_base(C);
      Eng::for_each_output(tid, [&](int i, int, int n) { o[(long long)n << ts] = value(i); });
    } else {
      Eng::for_each_output(tid, [&](int i, int line, int n) {
        const long long C = col0 + line;
        if (C < a.ncols) out[col_base(C) + ((long long)n << ts)] = value(i);
      });
    }
  };
  auto store = [&](long long col0, cx<T>* out, auto&& value) { emit(EngTag<Inv>(), col0, out, value); };

  if constexpr (TWM == kTwLds) {
    Fwd::load_lds_table(twl, a.tw, tid);
    lds_barrier();
  }
  auto fwd = [&](cx<T>(&v)[E], int t) {
    if constexpr (TWM == kTwLds) Fwd::run_lds(v, lds, twl, t);
    else if constexpr (TWM == kTwStage || TWM == kTwStageGrp) Fwd::run_stage(v, lds, a.twf, t);
    else Fwd::run(v, lds, a.tw, t);
  };
  auto inv = [&](cx<T>(&v)[E], int t) {
    if constexpr (TWM == kTwLds) Inv::run_lds(v, lds, twl, t);
    else if constexpr (TWM == kTwStage || TWM == kTwStageGrp) Inv::run_stage(v, lds, a.twi, t);
    else Inv::run(v, lds, a.tw, t);
  };
  // Multiply by a real symbol and conjugate (for the inverse by conjugation).
  auto apply_real = [&](auto sym_tag, long long col0, cx<T>(&v)[E]) {
    constexpr int OP = decltype(sym_tag)::value;
    if constexpr (kOneCol) {
      const Symbol<T, OP> sym(a.sym, int((col0 + (tid & (TT - 1))) & fmask));
      // (the kernels for all modes keep the general form: the split one's
      // registers would cost them a resident workgroup)
      if constexpr (XW) {
        if (sym.split_ok()) {
          // register 8 q + t holds row j_q + 256 t, j_q = 16 (h + 8 q) + k
          // (ColMapWave layout 2).  In waves 1-7 the row of register 8 + t
          // is the mirror of the row of register 7 - t of lane l ^ 60 (the
          // other residue, h -> 7 - h), so each lane evaluates its 8 rows
          // of q = 0 and reads the other 8 values from that lane; wave 0
          // (residues 0 and 8, which pair differently) evaluates all 16.
          auto sdd = [](int d) { return d >= (N >> 1) ? d - N : d; };
          const int k = FMap::residue(tid), h = (tid >> 3) & 7;
          const int j0 = 16 * h + k;
          T m0[8], m1[8];
#pragma unroll
          for (int t = 0; t < 8; t++) m0[t] = sym.split(j0, sdd(256 * t));
          if (__builtin_amdgcn_readfirstlane(tid >> 6) == 0) {
#pragma unroll
            for (int t = 0; t < 8; t++) m1[t] = sym.split(j0 + 128, sdd(256 * t));
          } else {
            const int src = ((tid & 63) ^ 60) << 2;
#pragma unroll
            for (int t = 0; t < 8; t++)
              m1[t] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(m0[7 - t])));
          }
#pragma unroll
          for (int t = 0; t < 8; t++) {
            v[t] = {v[t].re * m0[t], -v[t].im * m0[t]};
            v[8 + t] = {v[8 + t].re * m1[t], -v[8 + t].im * m1[t]};
          }
        } else {
          Inv::for_each_input(tid, [&](int i, int, int n) {
            const T m = sym(n);
            v[i] = {v[i].re * m, -v[i].im * m};
          });
        }
      } else if (kMirror && sym.split_ok()) {
        // register q R0 + t holds row j_q + t M (M = N / R0) of this
        // thread's column, j_1 the mirror of j_0 (ColMapMirror).  Slot e of
        // the R0 + 1 evaluations: rows j0 + e M; on the thread with j0 = 0,
        // rows e M for e <= R0/2 and then M/2 + (e - R0/2 - 1) M.
        constexpr int M = N / kR0, H = M / 2;
        auto sdd = [](int d) { return d >= (N >> 1) ? d - N : d; };
        const int j0 = tid >> LOGT;
        const bool sp = j0 == 0;
        T m[kR0 + 1];
#pragma unroll
        for (int e = 0; e <= kR0; e++) {
          if (e <= kR0 / 2) {
            m[e] = sym.split(j0, sdd(e * M));
          } else {
            const int es = e - kR0 / 2 - 1;
            m[e] = sym.split(sp ? H : j0, sp ? sdd(es * M) : sdd((e < kR0 ? e : 0) * M));
          }
        }
#pragma unroll
        for (int t = 0; t < kR0; t++) {
          const T m0 = (t <= kR0 / 2) ? m[t] : (sp ? m[kR0 - t] : m[t]);
          const int tt = kR0 - 1 - t;
          const T m1 = sp ? m[kR0 / 2 + 1 + (t < tt ? t : tt)] : m[tt];
          v[t] = {v[t].re * m0, -v[t].im * m0};
          v[kR0 + t] = {v[kR0 + t].re * m1, -v[kR0 + t].im * m1};
        }
      } else if (FUSED && sym.split_ok()) {
        // position n = j + d of the inverse's first stage, d = t N/R a
        // compile-time multiple of N/R: its signed index is j + d, or
        // j + d - N once d reaches N/2 (N/2 is a multiple of N/R and j < N/R)
        Inv::for_each_input_split(tid, [&](int i, int, int j, int d) {
          const T m = sym.split(j, d >= (N >> 1) ? d - N : d);
          v[i] = {v[i].re * m, -v[i].im * m};
        });
      } else {
        Inv::for_each_input(tid, [&](int i, int, int n) {
          const T m = sym(n);
          v[i] = {v[i].re * m, -v[i].im * m};
        });
      }
    } else {
      Inv::for_each_input(tid, [&](int i, int line, int n) {
        const Symbol<T, OP> sym(a.sym, int((col0 + line) & fmask));
        const T m = sym(n);
        v[i] = {v[i].re * m, -v[i].im * m};
      });
    }
  };

  cx<T> x[E];
  cx<T> y[NF >= 2 ? E : 1];
  cx<T> z[NF == 3 ? E : 1];
  cx<T> nx_[PF ? E : 1];
  cx<T> ny_[(PF && NF >= 2) ? E : 1];
  cx<T> nz_[(PF && NF == 3) ? E : 1];
  long long tile = walk.first;
  // FP32 with the LDS root table: the tile's loads are issued at raised wave
  // priority, so a workgroup that has just started gets its HBM requests out
  // ahead of the other resident workgroup's arithmetic (2048-point fused
  // pass: 131 -> 124 us per 8-field chunk; the FP64 pass, whose twiddles are
  // global loads, measured 141 -> 146 and keeps the default priority).
  constexpr bool kLoadPrio = sizeof(T) == 4 && TWM == kTwLds;
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(3);
  load(tile, x, y, z);
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(0);
  while (true) {
    tid = opaque(tid);
    const long long nt = walk.next(tile);
    const bool more = nt >= 0;
    if constexpr (PF) {
      if (more) load(nt, nx_, ny_, nz_);
    }
#pragma unroll
    for (int i = 0; i < E; i++) x[i].im *= sgn;
    const long long col0 = tile << LOGT;
    if (mode == kColForward || mode == kColInverse) {
      // a plain column transform (forward, or inverse by conjugation)
      fwd(x, tid);
      const T sc = mode == kColInverse ? T(a.sym.scale) : T(1);
      const T si = sgn * sc;
      emit(EngTag<Fwd>(), col0, a.out0, [&](int i) { return cx<T>{x[i].re * sc, x[i].im * si}; });
    } else {
      if (!spec_in) {
        fwd(x, tid);
        if constexpr (NF >= 2) {
          if (has_in1) fwd(y, tid);
        }
        if constexpr (NF == 3) fwd(z, tid);
      }
      // Pointwise symbol at (a = column x index, b = n).  The forward
      // engine's last radix is the inverse engine's first, so positions line
      // up register by register.
      if constexpr (NF == 1) {
        switch (a.sym.op) {
          case kSymPoisson: apply_real(std::integral_constant<int, kSymPoisson>(), col0, x); break;
          case kSymDiffusion: apply_real(std::integral_constant<int, kSymDiffusion>(), col0, x); break;
          case kSymWave: apply_real(std::integral_constant<int, kSymWave>(), col0, x); break;
          default: apply_real(std::integral_constant<int, kSymScale>(), col0, x); break;
        }
      } else if constexpr (NF == 3) {
        const bool want_v = a.out1 != nullptr;
        const T sc = T(a.sym.scale);
        Inv::for_each_input(tid, [&](int i, int line, int n) {
          const SourceCoeffs<T> k(a.sym, int((col0 + line) & fmask));
          T uf, ug, us, vf, vg, vs;
          k(n, uf, ug, us, vf, vg, vs);
          const cx<T> F = x[i], G = y[i], S = z[i];
          const cx<T> U = {uf * F.re + ug * G.re + us * S.re, uf * F.im + ug * G.im + us * S.im};
          x[i] = {U.re * sc, -U.im * sc};
          if (want_v) {
            const cx<T> V = {vf * F.re + vg * G.re + vs * S.re, vf * F.im + vg * G.im + vs * S.im};
            y[i] = {V.re * sc, -V.im * sc};
          }
        });
      } else {
        const bool want_v = a.out1 != nullptr;
        const T sc = T(a.sym.scale);
        Inv::for_each_input(tid, [&](int i, int line, int n) {
          const WaveCoeffs<T> wc(a.sym, int((col0 + line) & fmask));
          T cw, sw, sow, w;
          wc(n, cw, sw, sow, w);
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
      inv(x, tid);
      store(col0, a.out0, [&](int i) { return conjg(x[i]); });
      if constexpr (NF >= 2) {
        if (a.out1) {
          inv(y, tid);
          store(col0, a.out1, [&](int i) { return conjg(y[i]); });
        }
      }
    }
    if (!more) break;
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < E; i++) x[i] = nx_[i];
      if constexpr (NF >= 2) {
#pragma unroll
        for (int i = 0; i < E; i++) y[i] = ny_[i];
      }
      if constexpr (NF == 3) {
#pragma unroll
        for (int i = 0; i < E; i++) z[i] = nz_[i];
      }
    } else {
      load(nt, x, y, z);
    }
    tile = nt;
  }
}

// ---------------------------------------------------------------------------
// Variant tables (one entry per compiled kernel configuration).
// ---------------------------------------------------------------------------
// Launch over `units` rows or columns with at most `max_blocks` workgroups.
using LaunchFn = hipError_t (*)(const void* args, long long units, long long max_blocks, hipStream_t stream);
// Resident workgroups per CU for this kernel (0 on error).
using OccFn = int (*)();

struct RowVariant {
  LaunchFn launch;
  OccFn occupancy;
  // the same configuration with real-pair input (forward) / output (inverse)
  LaunchFn launch_rin;
  OccFn occupancy_rin;
  LaunchFn launch_rout;
  OccFn occupancy_rout;
  int logn, e, th, maxlr, lines, pf, twm;
  int lds_bytes;
  const char* name;
};

struct ColVariant {
  LaunchFn launch;
  OccFn occupancy;
  LaunchFn launch_fused;  // the same configuration compiled for kColFwdMulInv only
  OccFn occupancy_fused;
  int logn, logt, e, th, maxlr, nf, split, pf, twm;
  int lds_bytes;
  const char* name;
};

template <typename T, int LOGN, int E, int TH, int MAXLR, bool PF, int TWM, int RIO>
hipError_t launch_row(const void* args, long long nrows, long long max_blocks, hipStream_t s) {
  constexpr int LINES = E * TH / (1 << LOGN);
  long long grid = (nrows + LINES - 1) / LINES;
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid <= 0 || grid > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL((row_kernel<T, LOGN, E, TH, MAXLR, PF, TWM, RIO>), dim3((unsigned)grid), dim3(TH), 0, s,
                     *static_cast<const RowArgs<T>*>(args));
  return hipGetLastError();
}

template <typename T, int LOGN, int E, int TH, int MAXLR, bool PF, int TWM, int RIO>
int occ_row() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, row_kernel<T, LOGN, E, TH, MAXLR, PF, TWM, RIO>, TH, 0) !=
      hipSuccess)
    return 0;
  return n;
}

template <typename T, int LOGN, int LOGT, int E, int TH, int MAXLR, int NF, bool SPLIT, bool PF, int TWM, bool FUSED,
          bool XW = false>
hipError_t launch_col(const void* args, long long ncols, long long max_blocks, hipStream_t s) {
  long long grid = (ncols + (1 << LOGT) - 1) >> LOGT;
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid <= 0 || grid > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL((col_kernel<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, FUSED, XW>), dim3((unsigned)grid),
                     dim3(TH), 0, s, *static_cast<const ColArgs<T>*>(args));
  return hipGetLastError();
}

template <typename T, int LOGN, int LOGT, int E, int TH, int MAXLR, int NF, bool SPLIT, bool PF, int TWM, bool FUSED,
          bool XW = false>
int occ_col() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, col_kernel<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, FUSED, XW>, TH, 0) != hipSuccess)
    return 0;
  return n;
}

template <int LOGN, int MAXLR>
constexpr int lds_elems_row(int lines) {
  return plan_nstages(LOGN, MAXLR) > 1 ? lines * ((1 << LOGN) + ((1 << LOGN) >> plan_pad(LOGN, MAXLR, false))) : 1;
}
template <int LOGN, int MAXLR>
constexpr int lds_elems_col(int logt) {
  constexpr int lp = plan_pad(LOGN, MAXLR, false) < plan_pad(LOGN, MAXLR, true) ? plan_pad(LOGN, MAXLR, false)
                                                                                 : plan_pad(LOGN, MAXLR, true);
  return plan_nstages(LOGN, MAXLR) > 1 ? (((1 << LOGN) + ((1 << LOGN) >> lp)) << logt) : 1;
}

#define FFTPDE_ROW_VARIANT(T, LOGN, E, TH, MAXLR, PF, TWM)                                     \
  {&::fftpde::launch_row<T, LOGN, E, TH, MAXLR, PF, TWM, 0>,                                   \
   &::fftpde::occ_row<T, LOGN, E, TH, MAXLR, PF, TWM, 0>,                                      \
   &::fftpde::launch_row<T, LOGN, E, TH, MAXLR, PF, TWM, 1>,                                   \
   &::fftpde::occ_row<T, LOGN, E, TH, MAXLR, PF, TWM, 1>,                                      \
   &::fftpde::launch_row<T, LOGN, E, TH, MAXLR, PF, TWM, 2>,                                   \
   &::fftpde::occ_row<T, LOGN, E, TH, MAXLR, PF, TWM, 2>,                                      \
   LOGN, E, TH, MAXLR, (E) * (TH) >> (LOGN), PF, TWM,                                          \
   int(::fftpde::lds_elems_row<LOGN, MAXLR>((E) * (TH) >> (LOGN)) * sizeof(::fftpde::cx<T>)), \
   "row_" #T "_n" #LOGN "_e" #E "_th" #TH "_r" #MAXLR "_pf" #PF "_tw" #TWM}

#define FFTPDE_COL_VARIANT(T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM)                           \
  {&::fftpde::launch_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, false>,                     \
   &::fftpde::occ_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, false>,                        \
   &::fftpde::launch_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, true>,                      \
   &::fftpde::occ_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, true>,                         \
   LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM,                                                      \
   int(::fftpde::lds_elems_col<LOGN, MAXLR>(LOGT) * ((SPLIT) ? sizeof(T) : sizeof(::fftpde::cx<T>)) + \
       ((TWM) == 2 ? (1 << (LOGN)) * sizeof(::fftpde::cx<T>) : 0)),                                  \
   "col_" #T "_n" #LOGN "_t" #LOGT "_e" #E "_th" #TH "_r" #MAXLR "_f" #NF "_s" #SPLIT "_pf" #PF "_tw" #TWM}

// The same configuration with its fused pass on in-wave exchanges around the
// radix-8 stage (col_kernel XW, ColMapWave); its other modes run the plain
// kernel.
#define FFTPDE_COL_VARIANT_XW(T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM)                        \
  {&::fftpde::launch_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, false>,                     \
   &::fftpde::occ_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, false>,                        \
   &::fftpde::launch_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, true, true>,                \
   &::fftpde::occ_col<T, LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM, true, true>,                   \
   LOGN, LOGT, E, TH, MAXLR, NF, SPLIT, PF, TWM,                                                      \
   int(::fftpde::lds_elems_col<LOGN, MAXLR>(LOGT) * ((SPLIT) ? sizeof(T) : sizeof(::fftpde::cx<T>)) + \
       ((TWM) == 2 ? (1 << (LOGN)) * sizeof(::fftpde::cx<T>) : 0)),                                  \
   "col_" #T "_n" #LOGN "_t" #LOGT "_e" #E "_th" #TH "_r" #MAXLR "_f" #NF "_s" #SPLIT "_pf" #PF "_tw" #TWM "_xw"}

// Tables defined in the per-dtype translation units.
const RowVariant* row_variants_f32(int* count);
const RowVariant* row_variants_f64(int* count);
const ColVariant* col_variants_f32_nf1(int* count);
const ColVariant* col_variants_f32_nf2(int* count);
const ColVariant* col_variants_f64_nf1(int* count);
const ColVariant* col_variants_f64_nf2(int* count);
const ColVariant* col_variants_f32_nf3(int* count);
const ColVariant* col_variants_f64_nf3(int* count);

}  // namespace fftpde
