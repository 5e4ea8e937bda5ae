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

#include <type_traits>

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

// Workgroup barrier that orders LDS only: outstanding global loads (the next
// tile's prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Returns v unchanged but opaque to the optimiser.  Used on the thread index
// once per tile so that per-element addresses are recomputed inside the
// persistent tile loop instead of being hoisted out of it and held in
// registers for the whole kernel.  (An empty asm with a register operand:
// no instruction is emitted and no memory is touched.)
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
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
// n of a line lives in LDS.  Element n is stored at padded position
// n + floor(n / P), P = 2^LP, which spreads the strided accesses of the
// exchanges over the LDS banks.  The engine picks P so that within every
// butterfly the R positions it writes or reads are one base plus a
// compile-time stride, which the LDS instructions take as an immediate.
// ---------------------------------------------------------------------------

// Rows: j fastest, so consecutive lanes walk along a row.
template <int LOGN, int LINES, int LP>
struct RowMap {
  static constexpr int kLP = LP;
  static constexpr int N = 1 << LOGN;
  static constexpr int kUnit = 1;  // LDS words between lines' neighbours in n
  static constexpr int kStride = N + (N >> LP);
  static constexpr int kLdsElems = LINES * kStride;
  __device__ __forceinline__ static void split(int g, int lm, int& line, int& j) {
    j = g & ((1 << lm) - 1);
    line = g >> lm;
  }
  // butterfly slot q of thread tid (g = tid + TH q) at stage S
  template <int TH, int S = 0>
  __device__ __forceinline__ static void split_q(int tid, int q, int lm, int& line, int& j) {
    split(tid + TH * q, lm, line, j);
  }
  __device__ __forceinline__ static int lds(int line, int n) { return line * kStride + n + (n >> LP); }
  // every exchange goes through LDS
  template <int S>
  static constexpr bool in_wave() { return false; }
};

// Columns: the T lines of a tile fastest, so a wavefront covers T adjacent
// columns of 64/T consecutive rows (T * element size bytes per row segment).
template <int LOGN, int LOGT, int LP>
struct ColMap {
  static constexpr int kLP = LP;
  static constexpr int N = 1 << LOGN;
  static constexpr int T = 1 << LOGT;
  static constexpr int kUnit = T;
  static constexpr int kLdsElems = (N + (N >> LP)) * T;
  __device__ __forceinline__ static void split(int g, int lm, int& line, int& j) {
    line = g & (T - 1);
    j = g >> LOGT;
    (void)lm;
  }
  template <int TH, int S = 0>
  __device__ __forceinline__ static void split_q(int tid, int q, int lm, int& line, int& j) {
    split(tid + TH * q, lm, line, j);
  }
  __device__ __forceinline__ static int lds(int line, int n) { return (n + (n >> LP)) * T + line; }
  template <int S>
  static constexpr bool in_wave() { return false; }
};

// Columns with mirror-paired butterflies: at the stages with 2^MLM
// butterflies per line (two per thread), a thread's second butterfly is the
// mirror of its first, j1 = M - j0 (M = 2^MLM), or M/2 where j0 = 0.  Its
// positions j + t M (t < R = N/M) then hold the rows n and N - n (signed
// indices b' and -b') together: (j0, t) and (j1, R - 1 - t), and for the
// thread with j0 = 0, (0, t) with (0, R - t) and (M/2, t) with (M/2, R - 1 - t).
// Any bijection of butterflies onto threads is a valid Stockham stage, so
// the pairing only changes which thread does which butterfly.
template <int LOGN, int LOGT, int LP, int MLM>
struct ColMapMirror : ColMap<LOGN, LOGT, LP> {
  template <int TH, int S = 0>
  __device__ __forceinline__ static void split_q(int tid, int q, int lm, int& line, int& j) {
    constexpr int T = 1 << LOGT;
    line = tid & (T - 1);
    j = (tid >> LOGT) + (TH >> LOGT) * q;
    if (lm == MLM && q == 1) {
      static_assert((TH >> LOGT) == (1 << (MLM - 1)) || MLM < 0, "two butterflies per thread at the mirrored stage");
      constexpr int h = TH >> LOGT;
      const int j0 = tid >> LOGT;
      j = j0 == 0 ? h : 2 * h - j0;
    }
  }
};

// Columns of N = 2048 in tiles of 4 (lane bits 0-1), 16 points per thread on
// 512 threads, radix plan 16 16 8 (forward) and 8 16 16 (reversed), with the
// exchange between the two stages that meet the radix-8 stage kept inside
// each wavefront.  For the Stockham exchange into a stage of radix R2 with
// Ns' = N / R2, butterfly j' reads the outputs of butterflies t Ns + (j' mod
// Ns), t < R2, of the stage before (Ns its sub-length): a wavefront that owns
// every butterfly of a set of residues mod Ns on both sides owns the whole
// exchange.  Wave w takes the residues {w, 16 - w} mod 16 ({0, 8} for w = 0),
// lane bit 2 choosing one of the two (kbit), lane bits 3-5 a 3-bit index h:
//   layout 1, radix 16 of sub-length 16:   j = 16 h + k
//   layout 2, radix 8 of sub-length 256:   j = 16 (h + 8 q) + k   (q the slot)
//   layout 3, radix 16 of sub-length 8:    j = 8 k + h
// Forward: stage 0 as ColMap (the loads), layout 1, in-wave exchange,
// layout 2.  Reversed: layout 2 (the same registers), in-wave exchange,
// layout 3, then ColMap (the stores).  In both in-wave exchanges the value in
// register 8 q + b of the lane with index h goes to register 8 q + h of the
// lane with index b (b, h < 8): a transpose of lane bits 3-5 with register
// bits 0-2, done as three swaps of one lane bit with one register bit.
// The other exchanges go through LDS as in ColMap.
template <int LP, bool REV>
struct ColMapWave : ColMap<11, 2, LP> {
  using Base = ColMap<11, 2, LP>;
  static constexpr int layout(int s) { return REV ? (s == 0 ? 2 : s == 1 ? 3 : 0) : (s == 0 ? 0 : s == 1 ? 1 : 2); }
  template <int S>
  static constexpr bool in_wave() { return REV ? S == 0 : S == 1; }
  // the residue mod 16 this lane's butterflies share
  __device__ __forceinline__ static int residue(int tid) {
    const int w = tid >> 6, kb = (tid >> 2) & 1;
    return kb ? (w ? 16 - w : 8) : w;
  }
  template <int TH, int S = 0>
  __device__ __forceinline__ static void split_q(int tid, int q, int lm, int& line, int& j) {
    static_assert(TH == 512, "512 threads: 8 wavefronts, one per residue pair");
    constexpr int L = layout(S);
    if constexpr (L == 0) {
      Base::template split_q<TH>(tid, q, lm, line, j);
    } else {
      line = tid & 3;
      const int k = residue(tid), h = (tid >> 3) & 7;
      if constexpr (L == 1) j = 16 * h + k;
      else if constexpr (L == 2) j = 16 * (h + 8 * q) + k;
      else j = 8 * k + h;
    }
  }
  // Swap lane bit LB with register bit RB over the 32-bit words of x:
  // afterwards the lane with lane bit 0 holds its own register with RB = 0
  // and its partner's register with RB = 0 in place of RB = 1; the lane with
  // lane bit 1 its partner's RB = 1 register in place of RB = 0.
  template <int LB, int RB, typename T, int E>
  __device__ __forceinline__ static void swap_bits(cx<T> (&x)[E], int tid) {
    static_assert(sizeof(T) == 4, "FP32 words");
    const bool hi = (tid >> LB) & 1;
#pragma unroll
    for (int r = 0; r < E; r++) {
      if ((r >> RB) & 1) continue;
      float* a = &x[r].re;
      float* b = &x[r | (1 << RB)].re;
#pragma unroll
      for (int c = 0; c < 2; c++) {
        if constexpr (LB == 5) {
          // v_permlane32_swap: the upper 32 lanes of a with the lower 32 of b
          const auto v = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[c]), __float_as_uint(b[c]), false, false);
          a[c] = __uint_as_float(v[0]);
          b[c] = __uint_as_float(v[1]);
        } else if constexpr (LB == 4) {
          // v_permlane16_swap: the odd rows of a with the even rows of b
          const auto v = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[c]), __float_as_uint(b[c]), false, false);
          a[c] = __uint_as_float(v[0]);
          b[c] = __uint_as_float(v[1]);
        } else {
          static_assert(LB == 3, "lane bits 3, 4, 5");
          // DPP row_ror:8 reads lane l ^ 8 within each row of 16
          const float send = hi ? a[c] : b[c];
          const float got = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x128, 0xf, 0xf, false));
          a[c] = hi ? got : a[c];
          b[c] = hi ? b[c] : got;
        }
      }
    }
  }
  template <int S, typename T, int E>
  __device__ __forceinline__ static void wave_exchange(cx<T> (&x)[E], int tid) {
    static_assert(E == 16, "16 points per thread");
    swap_bits<3, 0>(x, tid);
    swap_bits<4, 1>(x, tid);
    swap_bits<5, 2>(x, tid);
  }
};

// Affine padding: with P = 2^lp, stage s's writes (groups of R outputs at
// stride Ns starting at a multiple of R*Ns plus k < Ns) and the next stage's
// reads (R inputs at stride N/R) must each stay affine in t: either the stride
// is a multiple of P, or the whole group lies inside one P-aligned block.
constexpr bool plan_affine(int logn, int maxlr, bool rev, int lp) {
  const int ns = plan_nstages(logn, maxlr);
  for (int s = 0; s + 1 < ns; s++) {
    const int lr = plan_lr(logn, maxlr, s, rev), lns = plan_lns(logn, maxlr, s, rev);
    const bool w_ok = lns >= lp || lns + lr <= lp;
    const int lr2 = plan_lr(logn, maxlr, s + 1, rev);
    const bool r_ok = logn - lr2 >= lp;
    if (!w_ok || !r_ok) return false;
  }
  return true;
}
// the padding granularity used by an engine: the finest affine P among 2^3..2^6
// (finer padding spreads more), else P = 2^5 with per-element addressing
constexpr int plan_pad(int logn, int maxlr, bool rev) {
  for (int lp = 3; lp <= 6; lp++)
    if (plan_affine(logn, maxlr, rev, lp)) return lp;
  return 5;
}

// ---------------------------------------------------------------------------
// The engine.  x[q R + t] holds element (line(g), j(g) + t N/R) of the
// current stage's input, g = tid + TH q.
// ---------------------------------------------------------------------------
// Moves value v from lane src of its group of G consecutive lanes (G = 2 or
// 4) to every lane of the group: a DPP quad permutation, one move per 32-bit
// word.  src must fold to a constant.
template <int G>
__device__ __forceinline__ int group_bcast_word(int v, int src) {
  static_assert(G == 2 || G == 4, "groups of 2 or 4 lanes");
  if constexpr (G == 4) {
    switch (src) {
      case 0: return __builtin_amdgcn_update_dpp(0, v, 0x00, 0xf, 0xf, false);
      case 1: return __builtin_amdgcn_update_dpp(0, v, 0x55, 0xf, 0xf, false);
      case 2: return __builtin_amdgcn_update_dpp(0, v, 0xaa, 0xf, 0xf, false);
      default: return __builtin_amdgcn_update_dpp(0, v, 0xff, 0xf, 0xf, false);
    }
  } else {
    // quad_perm [s, s, 2 + s, 2 + s]
    return src == 0 ? __builtin_amdgcn_update_dpp(0, v, 0xa0, 0xf, 0xf, false)
                    : __builtin_amdgcn_update_dpp(0, v, 0xf5, 0xf, 0xf, false);
  }
}
template <int G, typename T>
__device__ __forceinline__ cx<T> group_bcast(cx<T> v, int src) {
  if constexpr (sizeof(T) == 4) {
    return {__int_as_float(group_bcast_word<G>(__float_as_int(v.re), src)),
            __int_as_float(group_bcast_word<G>(__float_as_int(v.im), src))};
  } else {
    auto d = [&](double x) {
      const long long b = __double_as_longlong(x);
      const int lo = group_bcast_word<G>(int(b & 0xffffffffll), src);
      const int hi = group_bcast_word<G>(int(b >> 32), src);
      return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    };
    return {d(v.re), d(v.im)};
  }
}

// TWG: lanes l with equal l / TWG hold butterflies of the same index (the
// columns of a column tile) and share their twiddles (TwSrc::stage only).
template <typename T, int LOGN, int E, int TH, int MAXLR, bool REV, class Map, bool SPLIT = false, int TWG = 1>
struct Engine {
  static constexpr int N = 1 << LOGN;
  static constexpr int NST = plan_nstages(LOGN, MAXLR);
  static_assert(NST >= 1, "length must be at least 2");
  static_assert((E & (E - 1)) == 0 && E >= (1 << plan_max_lr(LOGN, MAXLR)),
                "elements per thread must be a multiple of every radix");
  // LDS words per exchange buffer: complex values, or (SPLIT) one real
  // component at a time, which halves the buffer at twice the barriers.
  using Word = typename std::conditional<SPLIT, T, cx<T>>::type;
  static constexpr int kLdsWords = NST > 1 ? Map::kLdsElems : 1;

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
      Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
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
  // The same positions with n split as j + d: f(register index, line, j, d),
  // where d = t N/R is a compile-time constant of the unrolled visit and j
  // does not depend on t (so an address built from j is formed once per
  // butterfly and d goes into a wave-uniform part).
  template <int S, class F>
  __device__ __forceinline__ static void for_each_split(int tid, F&& f) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int M = N >> LR;
#pragma unroll
    for (int q = 0; q < E / R; q++) {
      int line, j;
      Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
#pragma unroll
      for (int t = 0; t < R; t++) f(q * R + t, line, j, t * M);
    }
  }
  template <class F>
  __device__ __forceinline__ static void for_each_input_split(int tid, F&& f) {
    for_each_split<0>(tid, f);
  }
  template <class F>
  __device__ __forceinline__ static void for_each_output_split(int tid, F&& f) {
    for_each_split<NST - 1>(tid, f);
  }

  // Stage S's outputs go to LDS; stage S+1's inputs come back.  When the map's
  // padding is affine for this plan, each butterfly's R positions are one
  // base plus a compile-time stride (an immediate LDS offset).
  template <int S>
  __device__ __forceinline__ static void exchange(cx<T> (&x)[E], Word* lds, int tid) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int LNS = lns<S>();
    constexpr int NS = 1 << LNS;
    constexpr int LR2 = lr<S + 1>();
    constexpr int R2 = 1 << LR2;
    constexpr int M2 = N >> LR2;
    constexpr int LP = Map::kLP;
    constexpr bool kAffine = plan_affine(LOGN, MAXLR, REV, LP);
    // padded distance of a step d within a group (d multiple of P, or the
    // group inside one P-block)
    constexpr int wstep = (LNS >= LP ? NS + (NS >> LP) : NS) * Map::kUnit;
    constexpr int rstep = (M2 + (M2 >> LP)) * Map::kUnit;
    auto put = [&](auto get) {
#pragma unroll
      for (int q = 0; q < E / R; q++) {
        int line, j;
        Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
        const int k = j & (NS - 1);
        const int o = ((j - k) << LR) + k;
        if constexpr (kAffine) {
          Word* b = lds + Map::lds(line, o);
#pragma unroll
          for (int t = 0; t < R; t++) b[t * wstep] = get(x[q * R + t]);
        } else {
#pragma unroll
          for (int t = 0; t < R; t++) lds[Map::lds(line, o + t * NS)] = get(x[q * R + t]);
        }
      }
    };
    auto take = [&](auto set) {
#pragma unroll
      for (int q = 0; q < E / R2; q++) {
        int line, j;
        Map::template split_q<TH, S + 1>(tid, q, LOGN - LR2, line, j);
        if constexpr (kAffine) {
          const Word* b = lds + Map::lds(line, j);
#pragma unroll
          for (int t = 0; t < R2; t++) set(x[q * R2 + t], b[t * rstep]);
        } else {
#pragma unroll
          for (int t = 0; t < R2; t++) set(x[q * R2 + t], lds[Map::lds(line, j + t * M2)]);
        }
      }
    };
    if constexpr (SPLIT) {
      put([](const cx<T>& v) { return v.re; });
      lds_barrier();
      take([](cx<T>& v, T w) { v.re = w; });
      lds_barrier();
      put([](const cx<T>& v) { return v.im; });
      lds_barrier();
      take([](cx<T>& v, T w) { v.im = w; });
      lds_barrier();
    } else {
      put([](const cx<T>& v) { return v; });
      lds_barrier();
      take([](cx<T>& v, const cx<T>& w) { v = w; });
      lds_barrier();
    }
  }

  // The exchange after stage S: across the lanes of each wavefront where the
  // map keeps it inside them, else through LDS.
  template <int S>
  __device__ __forceinline__ static void xchg(cx<T> (&x)[E], Word* lds, int tid) {
    if constexpr (Map::template in_wave<S>()) Map::template wave_exchange<S>(x, tid);
    else exchange<S>(x, lds, tid);
  }

  // Twiddles of stage S for this thread: w_{Ns R}^{t k}, t = 1..R-1, per butterfly.
  template <int S>
  static constexpr int twn() {
    return lns<S>() > 0 ? (E >> lr<S>()) * ((1 << lr<S>()) - 1) : 0;
  }
  // offset of stage S's twiddles in the all-stage register set
  template <int S>
  static constexpr int twoff() {
    if constexpr (S == 0) return 0;
    else return twoff<S - 1>() + twn<S - 1>();
  }
  static constexpr int kTwAll = twoff<NST - 1>() + twn<NST - 1>();
  static constexpr int kTwRegs = kTwAll > 0 ? kTwAll : 1;

  // Where a stage finds its twiddles:
  //   TwSrc::global  the global table, requested one stage ahead so the load
  //                  latency hides behind the previous LDS exchange;
  //   TwSrc::regs    all stages' twiddles held in registers (they do not
  //                  depend on the tile, so a persistent workgroup loads them
  //                  once);
  //   TwSrc::lds     a workgroup copy of w_N^e, e < N, in LDS;
  //   TwSrc::stage   per-stage tables in global memory (see stage_tw_off),
  //                  requested one stage ahead like the global table; with
  //                  TWG > 1, each of the TWG lanes that share a butterfly
  //                  index loads every TWG-th twiddle and the values reach
  //                  the other lanes by cross-lane moves (DPP).
  enum class TwSrc { global, regs, lds, stage };

  // Stage tables: one table per engine plan holding, for every stage S >= 1,
  // the values w_{Ns R}^{t k} at entry stw_off<S>() + (t - 1) Ns + k
  // (t = 1 .. R-1, k < Ns): t-major, so for a fixed t the lanes of a wave,
  // which hold consecutive k, read consecutive entries (one or two cache
  // lines per load instead of a gather over the 4096-entry table).  The
  // values are the 4096-entry table's entries (t k) 4096 / (Ns R), so results
  // are bit-identical to the global table's.
  template <int S>
  static constexpr int stw_off() {
    if constexpr (S <= 1) return 0;
    else return stw_off<S - 1>() + (((1 << lr<S - 1>()) - 1) << lns<S - 1>());
  }

  template <int S, class W>
  __device__ __forceinline__ static void load_tw_stage(W& w, int off, const cx<T>* __restrict__ tws, int tid) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int LNS = lns<S>();
    constexpr int NS = 1 << LNS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 0; q < E / R; q++) {
        int line, j;
        Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
        const cx<T>* b = tws + stw_off<S>() + (j & (NS - 1));
        if constexpr (TWG > 1) {
          // lane c of a group loads t = TWG u + c + 1 (the group's last lane
          // repeats t = R - 1 where R - 1 is not a multiple of TWG)
          const int c = tid & (TWG - 1);
#pragma unroll
          for (int u = 0; u < (R - 1 + TWG - 1) / TWG; u++) {
            const int t = min(TWG * u + c + 1, R - 1);
            w[off + q * (R - 1) + u] = b[(t - 1) * NS];
          }
        } else {
#pragma unroll
          for (int t = 1; t < R; t++) w[off + q * (R - 1) + t - 1] = b[(t - 1) * NS];
        }
      }
    }
  }

  template <int S, class W>
  __device__ __forceinline__ static void load_tw(W& w, int off, const cx<T>* __restrict__ tw, int tid) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int LNS = lns<S>();
    constexpr int NS = 1 << LNS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 0; q < E / R; q++) {
        int line, j;
        Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
        const int k = j & (NS - 1);
#pragma unroll
        for (int t = 1; t < R; t++) w[off + q * (R - 1) + t - 1] = tw[(t * k) << (kTwLog - LNS - LR)];
      }
    }
  }

  // All stages' twiddles into registers (for TwSrc::regs).
  template <int S = 1>
  __device__ __forceinline__ static void load_all_tw(cx<T> (&w)[kTwRegs], const cx<T>* __restrict__ tw, int tid) {
    if constexpr (S < NST) {
      load_tw<S>(w, twoff<S>(), tw, tid);
      load_all_tw<S + 1>(w, tw, tid);
    }
  }

  // The N-point roots w_N^e for e < N into LDS (for TwSrc::lds); the caller
  // synchronises before use.
  __device__ __forceinline__ static void load_lds_table(cx<T>* twl, const cx<T>* __restrict__ tw, int tid) {
    for (int e = tid; e < N; e += TH) twl[e] = tw[e << (kTwLog - LOGN)];
  }

  // Stage S on registers; `w` is the twiddle set (registers) and `off` where
  // stage S's twiddles start in it.
  template <int S, TwSrc SRC, class W>
  __device__ __forceinline__ static void stage(cx<T> (&x)[E], Word* lds, const cx<T>* __restrict__ tw,
                                               const cx<T>* twl, int tid, W& w) {
    constexpr int LR = lr<S>();
    constexpr int R = 1 << LR;
    constexpr int LNS = lns<S>();
    constexpr int NS = 1 << LNS;
    constexpr int off = SRC == TwSrc::regs ? twoff<S>() : 0;
#pragma unroll
    for (int q = 0; q < E / R; q++) {
      cx<T>* v = &x[q * R];
      if constexpr (NS > 1) {
        if constexpr (SRC == TwSrc::lds) {
          int line, j;
          Map::template split_q<TH, S>(tid, q, LOGN - LR, line, j);
          const int k = j & (NS - 1);
#pragma unroll
          for (int t = 1; t < R; t++) v[t] = cmul(v[t], twl[(t * k) << (LOGN - LNS - LR)]);
        } else if constexpr (SRC == TwSrc::stage && TWG > 1) {
#pragma unroll
          for (int t = 1; t < R; t++)
            v[t] = cmul(v[t], group_bcast<TWG>(w[off + q * (R - 1) + (t - 1) / TWG], (t - 1) % TWG));
        } else {
#pragma unroll
          for (int t = 1; t < R; t++) v[t] = cmul(v[t], w[off + q * (R - 1) + t - 1]);
        }
      }
      dft<R>(v);
    }
    if constexpr (S + 1 < NST) {
      if constexpr (SRC == TwSrc::global || SRC == TwSrc::stage) {
        cx<T> wn[twn<S + 1>() > 0 ? twn<S + 1>() : 1];
        if constexpr (SRC == TwSrc::stage) load_tw_stage<S + 1>(wn, 0, tw, tid);
        else load_tw<S + 1>(wn, 0, tw, tid);
        xchg<S>(x, lds, tid);
        stage<S + 1, SRC>(x, lds, tw, twl, tid, wn);
      } else {
        xchg<S>(x, lds, tid);
        stage<S + 1, SRC>(x, lds, tw, twl, tid, w);
      }
    }
  }

  // Global-table twiddles.
  __device__ __forceinline__ static void run(cx<T> (&x)[E], Word* lds, const cx<T>* __restrict__ tw, int tid) {
    cx<T> w0[1];
    stage<0, TwSrc::global>(x, lds, tw, nullptr, tid, w0);
  }
  // Register twiddles from load_all_tw.
  __device__ __forceinline__ static void run_regs(cx<T> (&x)[E], Word* lds, const cx<T> (&w)[kTwRegs], int tid) {
    stage<0, TwSrc::regs>(x, lds, nullptr, nullptr, tid, w);
  }
  // Stage-table twiddles (tws: this plan's table, see stw_off).
  __device__ __forceinline__ static void run_stage(cx<T> (&x)[E], Word* lds, const cx<T>* __restrict__ tws, int tid) {
    cx<T> w0[1];
    stage<0, TwSrc::stage>(x, lds, tws, nullptr, tid, w0);
  }
  // LDS table twiddles from load_lds_table.
  __device__ __forceinline__ static void run_lds(cx<T> (&x)[E], Word* lds, const cx<T>* twl, int tid) {
    cx<T> w0[1];
    stage<0, TwSrc::lds>(x, lds, nullptr, twl, tid, w0);
  }
};

// Persistent tile schedule.  Tiles are taken in groups of GROUP consecutive
// tiles, processed back to back by one workgroup (column tiles narrower than
// 64 bytes come in pairs, so both halves of each 64-byte chunk are written
// by the same workgroup while the first half is still in L2).  Workgroup b of
// G walks groups b0, b0 + step, ...; when G is a multiple of the 8 XCDs
// (workgroups are dealt to XCDs round robin), each XCD gets one contiguous
// range of groups, so neighbouring tiles meet in the same L2.
template <int GROUP>
struct TileWalk {
  long long ntiles, end, step;
  long long first = -1;
  __device__ __forceinline__ explicit TileWalk(long long nt) : ntiles(nt) {
    const long long ngroups = (nt + GROUP - 1) / GROUP;
    const int G = gridDim.x, b = blockIdx.x;
    long long g0;
    if ((G & 7) == 0 && ngroups >= G) {
      const int x = b & 7, per = G >> 3;
      const long long lo = ngroups * x / 8, hi = ngroups * (x + 1) / 8;
      g0 = lo + (b >> 3);
      end = hi;
      step = per;
    } else {
      g0 = b;
      end = ngroups;
      step = G;
    }
    if (g0 < end) first = g0 * GROUP;
  }
  // the tile after `tile` in this workgroup's walk, or -1
  __device__ __forceinline__ long long next(long long tile) const {
    if (GROUP > 1 && (tile % GROUP) + 1 < GROUP && tile + 1 < ntiles) return tile + 1;
    const long long g = tile / GROUP + step;
    return g < end ? g * GROUP : -1;
  }
};

// Entries of the stage table of the (logn, maxlr, rev) plan (host and
// device), and the value of each entry as an exponent of w = exp(-2 pi i/4096):
// entry i of the table is w^stage_tw_exponent(logn, maxlr, rev, i).
constexpr int stage_tw_entries(int logn, int maxlr, bool rev) {
  int n = 0;
  for (int s = 1; s < plan_nstages(logn, maxlr); s++)
    n += ((1 << plan_lr(logn, maxlr, s, rev)) - 1) << plan_lns(logn, maxlr, s, rev);
  return n;
}
inline int stage_tw_exponent(int logn, int maxlr, bool rev, int i) {
  for (int s = 1; s < plan_nstages(logn, maxlr); s++) {
    const int lr = plan_lr(logn, maxlr, s, rev), lns = plan_lns(logn, maxlr, s, rev);
    const int size = ((1 << lr) - 1) << lns;
    if (i < size) {
      const int t = 1 + (i >> lns), k = i & ((1 << lns) - 1);
      return (t * k) << (kTwLog - lns - lr);
    }
    i -= size;
  }
  return -1;
}

}  // namespace fftpde
