// fft_engine.hpp -- register/LDS Stockham FFT engine for gfx950 (CDNA4).
//
// A workgroup transforms a tile of independent lines (rows or columns of a
// field) of length N = 2^LOGN.  Each of its TH threads keeps E complex
// values in registers.  A stage of radix R performs N/R radix-R
// butterflies per line; thread `tid` owns butterflies g = tid + TH*q for
// q = 0 .. E/R-1.  Between stages the values move through LDS; the first
// stage reads straight from HBM and the last stage writes straight to HBM,
// both with consecutive lanes on consecutive addresses.
//
// Stage formulation (Stockham autosort, decimation in time), for a stage of
// radix R after sub-transforms of length Ns have been formed:
//   butterfly j (0 <= j < N/R), k = j mod Ns:
//     v_t = x[j + t N/R] * w_{Ns R}^{t k},  t = 0..R-1
//     v   = DFT_R(v)
//     y[(j - k) R + k + t Ns] = v_t
// Ns runs 1, R0, R0 R1, ... so the output of the last stage is in natural
// order.  This is the same transform as the paper's recursive radix-2
// split (Sec. II.C): a stage of radix R merges R interleaved sub-sequences
// with the twiddles w_N^k, and R = 2 is exactly Eq. (FFTpairodd) and
// Eq. (FFTpairodd_2); higher radices fuse several of those levels in
// registers.
//
// Twiddles come from one table of w^e = exp(-2 pi i e / 4096) generated in
// FP64 on the host and rounded once; a sub-transform of length L reads
// entry (t k) * 4096 / L.
//
// Inverse transforms reuse the forward engine through the conjugation
// identity of the iDFT (Sec. II.B): iDFT(P) = DFT(P*)* / N.
#pragma once

#include <hip/hip_runtime.h>

namespace fftpde {

constexpr int kTwLog = 12;  // twiddle table: 2^12 entries, the largest side

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> w) {
  return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) {
  return {a.re, -a.im};
}
// a * (-i)
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return {a.im, -a.re};
}
// a * w for a constant w = (c, s)
template <typename T>
__device__ __forceinline__ cx<T> mulc(cx<T> a, T c, T s) {
  return {a.re * c - a.im * s, a.re * s + a.im * c};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers, forward sign exp(-2 pi i n k / R), natural order.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
  cx<T> a2 = v[1] + v[3], a3 = mul_mi(v[1] - v[3]);
  v[0] = a0 + a2;
  v[2] = a0 - a2;
  v[1] = a1 + a3;
  v[3] = a1 - a3;
}

// 1/sqrt(2), cos(pi/8), sin(pi/8)
#define FFTPDE_R2 0.70710678118654752440084436210484903928
#define FFTPDE_C8 0.92387953251128675612818318939678828682
#define FFTPDE_S8 0.38268343236508977172845998403039886676

// Radix-8 as one radix-2 split (decimation in frequency) and two radix-4s:
// a_m = v_m + v_{m+4}, b_m = (v_m - v_{m+4}) w_8^m, X_{2p} = DFT4(a)_p,
// X_{2p+1} = DFT4(b)_p.
template <typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = T(FFTPDE_R2);
  cx<T> a[4], b[4];
#pragma unroll
  for (int m = 0; m < 4; m++) {
    a[m] = v[m] + v[m + 4];
    b[m] = v[m] - v[m + 4];
  }
  // w_8^1 = h(1 - i), w_8^2 = -i, w_8^3 = h(-1 - i)
  b[1] = {h * (b[1].re + b[1].im), h * (b[1].im - b[1].re)};
  b[2] = mul_mi(b[2]);
  b[3] = {h * (b[3].im - b[3].re), -h * (b[3].re + b[3].im)};
  dft4(a);
  dft4(b);
#pragma unroll
  for (int p = 0; p < 4; p++) {
    v[2 * p] = a[p];
    v[2 * p + 1] = b[p];
  }
}

// Radix-16 as 4 x 4: n = n1 + 4 n2, k = 4 k1 + k2:
// X[4 k1 + k2] = sum_n1 w_4^{n1 k1} w_16^{n1 k2} (sum_n2 v[n1 + 4 n2] w_4^{n2 k2}).
template <typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  const T h = T(FFTPDE_R2), c = T(FFTPDE_C8), s = T(FFTPDE_S8);
  cx<T> y[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; n1++) {
    cx<T> t4[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
    dft4(t4);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++) y[n1][k2] = t4[k2];
  }
  // twiddles w_16^{n1 k2}; exponents 1,2,3 (n1=1), 2,4,6 (n1=2), 3,6,9 (n1=3)
  y[1][1] = mulc(y[1][1], c, -s);
  y[1][2] = mulc(y[1][2], h, -h);
  y[1][3] = mulc(y[1][3], s, -c);
  y[2][1] = mulc(y[2][1], h, -h);
  y[2][2] = mul_mi(y[2][2]);
  y[2][3] = mulc(y[2][3], -h, -h);
  y[3][1] = mulc(y[3][1], s, -c);
  y[3][2] = mulc(y[3][2], -h, -h);
  y[3][3] = mulc(y[3][3], -c, s);
#pragma unroll
  for (int k2 = 0; k2 < 4; k2++) {
    cx<T> t4[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
    dft4(t4);
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) v[4 * k1 + k2] = t4[k1];
  }
}

template <int R, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 16) dft16(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans: LOGN split into ceil(LOGN/MAXLR) stages as evenly as
// possible, larger radices first.  REV = true walks the same list backwards,
// so a forward pass and an inverse pass can meet in registers (the forward's
// last radix is the inverse's first).
// ---------------------------------------------------------------------------
constexpr int plan_nstages(int logn, int maxlr) { return logn <= 0 ? 0 : (logn + maxlr - 1) / maxlr; }

constexpr int plan_lr_fwd(int logn, int maxlr, int s) {
  // stages 0..ns-1; the first (logn mod ns) stages get one extra bit
  return logn / plan_nstages(logn, maxlr) + (s < logn % plan_nstages(logn, maxlr) ? 1 : 0);
}

constexpr int plan_lr(int logn, int maxlr, int s, bool rev) {
  return rev ? plan_lr_fwd(logn, maxlr, plan_nstages(logn, maxlr) - 1 - s)
             : plan_lr_fwd(logn, maxlr, s);
}

// log2 of Ns before stage s (sum of the previous log-radices)
constexpr int plan_lns(int logn, int maxlr, int s, bool rev) {
  int acc = 0;
  for (int i = 0; i < s; i++) acc += plan_lr(logn, maxlr, i, rev);
  return acc;
}

constexpr int plan_max_lr(int logn, int maxlr) {
  return plan_lr_fwd(logn, maxlr, 0);
}

// ---------------------------------------------------------------------------
// Line maps: how a butterfly index g splits into (line, j) and where element
// n of a line lives in LDS.
// ---------------------------------------------------------------------------

// Rows: j fastest, so consecutive lanes walk along a row.  One padding
// element every 8 spreads the stride-R writes of the early stages over banks.
template <int LOGN, int LINES>
struct RowMap {
  static constexpr int N = 1 << LOGN;
  static constexpr int kStride = N + (N >> 3);
  static constexpr int kLdsElems = LINES * kStride;
  __device__ __forceinline__ static void split(int g, int lm, int& line, int& j) {
    j = g & ((1 << lm) - 1);
    line = g >> lm;
  }
  __device__ __forceinline__ static int lds(int line, int n) { return line * kStride + n + (n >> 3); }
};

// Columns: the T lines of a tile fastest, so a wavefront covers T adjacent
// columns of 64/T consecutive rows (T * element size bytes per row segment).
template <int LOGN, int LOGT>
struct ColMap {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = 1 << LOGT;
  static constexpr int kLdsElems = (N + (N >> 3)) * T;
  __device__ __forceinline__ static void split(int g, int lm, int& line, int& j) {
    line = g & (T - 1);
    j = g >> LOGT;
    (void)lm;
  }
  __device__ __forceinline__ static int lds(int line, int n) { return (n + (n >> 3)) * T + line; }
};

// ---------------------------------------------------------------------------
// The engine.  x[q R + t] holds element (line(g), j(g) + t N/R) of the
// current stage's input, g = tid + TH q.
// ---------------------------------------------------------------------------
template <typename T, int LOGN, int E, int TH, int MAXLR, bool REV, class Map>
struct Engine {
  static constexpr int N = 1 << LOGN;
  static constexpr int NST = plan_nstages(LOGN, MAXLR);
  static_assert(NST >= 1, "length must be at least 2");
  static_assert((E & (E - 1)) == 0 && E >= (1 << plan_max_lr(LOGN, MAXLR)),
                "elements per thread must be a multiple of every radix");

  template <int S>
  static constexpr int lr() { return plan_lr(LOGN, MAXLR, S, REV); }
  template <int S>
  static constexpr int lns() { return plan_lns(LOGN, MAXLR, S, REV); }

  // Visit the (line, n) positions of stage S's inputs (S = 0) or of the last
  // stage's outputs (S = NST - 1, as the "input" positions of that radix):
  // f(register index, line, n).
  template <int S, class F>
  __device__ __forceinline__ static void for_each(int tid, F&& f) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int M = N >> LR;
#pragma unroll
    for (int q = 0; q < E / R; q++) {
      int line, j;
      Map::split(tid + TH * q, LOGN - LR, line, j);
#pragma unroll
      for (int t = 0; t < R; t++) f(q * R + t, line, j + t * M);
    }
  }
  template <class F>
  __device__ __forceinline__ static void for_each_input(int tid, F&& f) {
    for_each<0>(tid, f);
  }
  template <class F>
  __device__ __forceinline__ static void for_each_output(int tid, F&& f) {
    for_each<NST - 1>(tid, f);
  }

  template <int S = 0>
  __device__ __forceinline__ static void run(cx<T> (&x)[E], cx<T>* lds, const cx<T>* __restrict__ tw,
                                             int tid) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int LNS = lns<S>();
    constexpr int NS = 1 << LNS;
    constexpr int M = N >> LR;
#pragma unroll
    for (int q = 0; q < E / R; q++) {
      cx<T>* v = &x[q * R];
      if constexpr (NS > 1) {
        int line, j;
        Map::split(tid + TH * q, LOGN - LR, line, j);
        const int k = j & (NS - 1);
#pragma unroll
        for (int t = 1; t < R; t++) v[t] = cmul(v[t], tw[(t * k) << (kTwLog - LNS - LR)]);
      }
      dft<R>(v);
    }
    if constexpr (S + 1 < NST) {
#pragma unroll
      for (int q = 0; q < E / R; q++) {
        int line, j;
        Map::split(tid + TH * q, LOGN - LR, line, j);
        const int k = j & (NS - 1);
        const int o = ((j - k) << LR) + k;
#pragma unroll
        for (int t = 0; t < R; t++) lds[Map::lds(line, o + t * NS)] = x[q * R + t];
      }
      __syncthreads();
      for_each<S + 1>(tid, [&](int i, int line, int n) { x[i] = lds[Map::lds(line, n)]; });
      __syncthreads();
      run<S + 1>(x, lds, tw, tid);
    }
    (void)M;
  }
};

}  // namespace fftpde
