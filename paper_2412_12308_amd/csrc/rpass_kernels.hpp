// rpass_kernels.hpp -- the kernels of rpass.hpp, included by one translation
// unit per dtype.
#pragma once

#include "mixed_dev.hpp"
#include "rpass.hpp"

namespace fftpde {
namespace rp {

constexpr int kE = 8;
constexpr int kRowTH = 256;
constexpr int kColTH = 512;
constexpr int kMaxLr = 3;

// cos and sin of 2 pi q / R, q = 1..(R-1)/2, from the n-point table (n = R P)
template <int R, typename T>
struct OddRoots {
  static constexpr int H = R > 1 ? (R - 1) / 2 : 1;
  T cs[H], sn[H];
  __device__ __forceinline__ OddRoots(const cx<T>* twn, int P) {
#pragma unroll
    for (int q = 1; q <= (R - 1) / 2; q++) {
      const cx<T> w = twn[q * P];  // exp(-2 pi i q / R)
      cs[q - 1] = w.re;
      sn[q - 1] = -w.im;
    }
  }
};

// The radix-R step of the factorisation, in place on v[0..R): DFT over j1,
// then times w_n^(j2 k1) (decimation in time); or, with DIF, times
// w_n^(k1 j2) first and the DFT after.
template <int R, bool DIF, typename T>
__device__ __forceinline__ void radix_step(cx<T>* v, const OddRoots<R, T>& rt, const cx<T>* twn, int j2) {
  if constexpr (R > 1) {
    if constexpr (DIF) {
#pragma unroll
      for (int k = 1; k < R; k++) v[k] = cmul(v[k], twn[k * j2]);
      dft_odd<R>(v, rt.cs, rt.sn);
    } else {
      dft_odd<R>(v, rt.cs, rt.sn);
#pragma unroll
      for (int k = 1; k < R; k++) v[k] = cmul(v[k], twn[k * j2]);
    }
  }
}

// Rows of length n = R P: persistent workgroups over tiles of L rows.
// Forward (kMrRowFwd) or the inverse through conjugation times scale
// (kMrRowInv); in and out may be the same field.
template <typename T, int R, int LP>
__global__ void __launch_bounds__(kRowTH) rows_kernel(RpArgs<T> a) {
  constexpr int P = 1 << LP, N = R * P;
  constexpr int L = kE * kRowTH / P;
  static_assert(L >= 1 && L * P == kE * kRowTH, "tile must hold whole rows");
  using Map = RowMap<LP, L, plan_pad(LP, kMaxLr, false)>;
  using Eng = Engine<T, LP, kE, kRowTH, kMaxLr, false, Map, false>;
  __shared__ typename Eng::Word lds[Eng::kLdsWords];
  int tid = threadIdx.x;
  const long long nrows = (long long)a.ny * a.fields;
  const long long ntiles = (nrows + L - 1) / L;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  cx<T> wall[Eng::kTwRegs];
  Eng::load_all_tw(wall, a.tw, tid);
  const OddRoots<R, T> rt(a.twn, P);
  const bool inv = a.mode == kMrRowInv;
  const T sgn = inv ? T(-1) : T(1);
  const T sr = inv ? a.scale : T(1), si = sgn * sr;
  for (long long tile = walk.first; tile >= 0; tile = walk.next(tile)) {
    tid = opaque(tid);
    const long long row0 = tile * L;
    cx<T> x[R][kE];
    // FP32: the tile's loads (and the radix-R step on them) at raised wave
    // priority, ahead of the other resident workgroups' transforms (1536,
    // 2560, 3584 rows: 2-7 % faster)
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(3);
    // rows past the last reread it and are never stored
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      const cx<T>* src = a.in + min(row0 + line, nrows - 1) * N + n;
      cx<T> v[R];
#pragma unroll
      for (int j = 0; j < R; j++) {
        v[j] = src[j * P];
        v[j].im *= sgn;
      }
      radix_step<R, false>(v, rt, a.twn, n);
#pragma unroll
      for (int k = 0; k < R; k++) x[k][i] = v[k];
    });
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int k = 0; k < R; k++) Eng::run_regs(x[k], lds, wall, tid);
    Eng::for_each_output(tid, [&](int i, int line, int k2) {
      const long long row = row0 + line;
      if (row < nrows) {
        cx<T>* dst = a.out + row * N + R * k2;
#pragma unroll
        for (int k = 0; k < R; k++) dst[k] = {x[k][i].re * sr, x[k][i].im * si};
      }
    });
  }
}

// One workgroup per tile of TT adjacent columns of length n = R P of one
// field (row-major fields, row stride nx).  kMrColFwd / kMrColInv
// (unscaled), or SOLVE: forward, the symbol (1/(nx ny) folded in), inverse.
// Workgroups are dealt to the 8 XCDs round robin; tile = (b mod 8) G/8 +
// b/8 gives each XCD a contiguous range of tiles, so adjacent column tiles,
// which share the cache lines of their row pieces, meet in one L2.
// Column tile shape: E points per thread per engine tile, radix up to
// 2^MAXLR, TH threads, TT = E TH / P columns.  The solves with R > 1 and the
// FP64 passes with R > 1 keep R engine tiles (and the symbol) in registers:
// 140-250 VGPRs, two or three waves per SIMD, so a 512-thread workgroup
// (two waves per SIMD) runs alone on its CU with nothing to overlap its
// loads.  They take 256 threads (two or three workgroups per CU) where the
// tile's row pieces stay at least 16 bytes wide (solves: faster even on
// 16-byte pieces) or 128 bytes wide (plain FP64 transforms, which measured
// slower on 64-byte pieces than on one workgroup per CU with 128-byte
// pieces).
template <typename T, int R, int LP, bool SOLVE>
struct ColShape {
  static constexpr bool kSmall = rp_col_small(sizeof(T) == 8, R, SOLVE);
  static constexpr int E = kSmall ? 4 : 8;
  static constexpr int MAXLR = rp_col_maxlr(sizeof(T) == 8, R, SOLVE);
  static constexpr int kLogE = kSmall ? 2 : 3;
  static constexpr bool kHeavy = R > 1 && (SOLVE || sizeof(T) == 8);
  // bytes of a row piece with 256 threads: 2^(log2(E 256) - LP) columns
  static constexpr int kPiece256 = kLogE + 8 >= LP ? (1 << (kLogE + 8 - LP)) * int(2 * sizeof(T)) : 0;
  static constexpr int TH = kHeavy && kPiece256 >= (SOLVE ? 16 : 128) ? 256 : kColTH;
  static constexpr int LOGPTS = kLogE + (TH == 256 ? 8 : 9);  // log2(E TH)
};

template <typename T, int R, int LP, bool SOLVE>
__global__ void __launch_bounds__((ColShape<T, R, LP, SOLVE>::TH)) cols_kernel(RpArgs<T> a) {
  using S = ColShape<T, R, LP, SOLVE>;
  constexpr int kE = S::E, kMaxLr = S::MAXLR, TH = S::TH;
  constexpr int P = 1 << LP, N = R * P;
  constexpr int LOGT = S::LOGPTS - LP;  // E TH = TT P
  constexpr int TT = 1 << LOGT;
  static_assert(TH % TT == 0, "every thread stays on one column of the tile");
  using FMap = ColMap<LP, LOGT, plan_pad(LP, kMaxLr, false)>;
  using IMap = ColMap<LP, LOGT, plan_pad(LP, kMaxLr, true)>;
  using Fwd = Engine<T, LP, kE, TH, kMaxLr, false, FMap, false>;
  using Inv = Engine<T, LP, kE, TH, kMaxLr, true, IMap, false>;
  constexpr int kLds = Fwd::kLdsWords > Inv::kLdsWords ? Fwd::kLdsWords : Inv::kLdsWords;
  __shared__ cx<T> lds[kLds];
  const int tid = threadIdx.x;
  const long long b = blockIdx.x, g = gridDim.x;
  const long long tile = (g & 7) == 0 ? (b & 7) * (g >> 3) + (b >> 3) : b;
  const int nx = a.nx;
  const int tpf = (nx + TT - 1) >> LOGT;  // tiles per field
  const long long f = tile / tpf;
  const int c = (int)(tile - f * tpf) * TT + (tid & (TT - 1));
  const int cl = min(c, nx - 1);  // columns past the field reread the last one
  const cx<T>* src = a.in + f * (long long)nx * N + cl;
  cx<T>* dst = a.out + f * (long long)nx * N + c;
  const OddRoots<R, T> rt(a.twn, P);
  const T sgn = (!SOLVE && a.mode == kMrColInv) ? T(-1) : T(1);
  // the solve's symbol at the positions (a', b' = k1 + R k2) the inverse
  // engine takes, evaluated before the loads land (it needs no data)
  T msym[SOLVE ? R : 1][kE];
  if constexpr (SOLVE) {
    const int ai = mr_sidx(cl, nx);
    Inv::for_each_input(tid, [&](int i, int, int k2) {
#pragma unroll
      for (int k = 0; k < R; k++) msym[k][i] = mr_symbol<T>(a.sym, ai, mr_sidx(k + R * k2, N));
    });
  }
  cx<T> x[R][kE];
  // FP32 transforms (not the solves, which measured 2-7 % slower with it):
  // the loads at raised wave priority (3072 columns: 201 -> 170 us)
  constexpr bool kLoadPrio = sizeof(T) == 4 && !SOLVE;
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(3);
  Fwd::for_each_input(tid, [&](int i, int, int n) {
    cx<T> v[R];
#pragma unroll
    for (int j = 0; j < R; j++) {
      v[j] = src[(long long)(j * P + n) * nx];
      v[j].im *= sgn;
    }
    radix_step<R, false>(v, rt, a.twn, n);
#pragma unroll
    for (int k = 0; k < R; k++) x[k][i] = v[k];
  });
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(0);
#pragma unroll
  for (int k = 0; k < R; k++) Fwd::run_stage(x[k], lds, a.stwf, tid);
  if constexpr (!SOLVE) {
    if (c < nx) {
      Fwd::for_each_output(tid, [&](int i, int, int k2) {
#pragma unroll
        for (int k = 0; k < R; k++) dst[(long long)(k + R * k2) * nx] = {x[k][i].re, sgn * x[k][i].im};
      });
    }
  } else {
    // the symbol, then the conjugate for the inverse
#pragma unroll
    for (int k = 0; k < R; k++) {
#pragma unroll
      for (int i = 0; i < kE; i++) x[k][i] = {x[k][i].re * msym[k][i], -x[k][i].im * msym[k][i]};
    }
#pragma unroll
    for (int k = 0; k < R; k++) Inv::run_stage(x[k], lds, a.stwr, tid);
    if (c < nx) {
      Inv::for_each_output(tid, [&](int i, int, int j2) {
        cx<T> v[R];
#pragma unroll
        for (int k = 0; k < R; k++) v[k] = x[k][i];
        radix_step<R, true>(v, rt, a.twn, j2);
#pragma unroll
        for (int j = 0; j < R; j++) dst[(long long)(j * P + j2) * nx] = conjg(v[j]);
      });
    }
  }
}

// ---- launches ---------------------------------------------------------------

template <typename T>
using Launch = hipError_t (*)(const RpArgs<T>&, hipStream_t);

template <typename T, int R, int LP>
int row_slots() {
  int dev = 0, cus = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, rows_kernel<T, R, LP>, kRowTH, 0) != hipSuccess)
    return 0;
  return (n > 0 ? n : 1) * cus;
}

template <typename T, int R, int LP>
hipError_t launch_rows(const RpArgs<T>& a, hipStream_t s) {
  static const int slots = row_slots<T, R, LP>();  // thread-safe one-time query
  if (slots <= 0) return hipErrorInvalidValue;
  constexpr int L = kE * kRowTH >> LP;
  const long long ntiles = ((long long)a.ny * a.fields + L - 1) / L;
  const long long grid = ntiles < slots ? ntiles : slots;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((rows_kernel<T, R, LP>), dim3((unsigned)grid), dim3(kRowTH), 0, s, a);
  return hipGetLastError();
}

template <typename T, int R, int LP>
hipError_t launch_cols(const RpArgs<T>& a, hipStream_t s) {
  const bool solve = a.mode == kMrColSolve;
  using SS = ColShape<T, R, LP, true>;
  using SF = ColShape<T, R, LP, false>;
  const int tt = 1 << ((solve ? SS::LOGPTS : SF::LOGPTS) - LP);
  const long long grid = a.fields * (long long)((a.nx + tt - 1) / tt);
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffll) return hipErrorInvalidValue;
  if (solve) {
    if constexpr (rp_solve_radix(sizeof(T) == 8, R))
      hipLaunchKernelGGL((cols_kernel<T, R, LP, true>), dim3((unsigned)grid), dim3(SS::TH), 0, s, a);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((cols_kernel<T, R, LP, false>), dim3((unsigned)grid), dim3(SF::TH), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, int R, int LP, int HI>
Launch<T> pick_rows(int lp) {
  if constexpr (LP > HI) return nullptr;
  else return lp == LP ? &launch_rows<T, R, LP> : pick_rows<T, R, LP + 1, HI>(lp);
}
template <typename T, int R, int LP, int HI>
Launch<T> pick_cols(int lp) {
  if constexpr (LP > HI) return nullptr;
  else return lp == LP ? &launch_cols<T, R, LP> : pick_cols<T, R, LP + 1, HI>(lp);
}

// the compiled (R, lp) ranges; rp_split admits exactly these
template <typename T>
hipError_t dispatch(const RpArgs<T>& a, hipStream_t s) {
  const bool col = a.mode >= kMrColFwd;
  int r = 0, lp = 0;
  if (!rp_split(col ? a.ny : a.nx, col, sizeof(T) == 8, &r, &lp)) return hipErrorInvalidValue;
  Launch<T> l = nullptr;
  switch (r) {
    case 1: l = col ? pick_cols<T, 1, 5, 12>(lp) : pick_rows<T, 1, 5, 11>(lp); break;
    case 3: l = col ? pick_cols<T, 3, 5, 10>(lp) : pick_rows<T, 3, 5, 10>(lp); break;
    case 5:
      if constexpr (sizeof(T) == 4) l = col ? pick_cols<T, 5, 5, 9>(lp) : pick_rows<T, 5, 5, 9>(lp);
      break;
    case 7:
      if constexpr (sizeof(T) == 4) l = col ? pick_cols<T, 7, 5, 9>(lp) : pick_rows<T, 7, 5, 9>(lp);
      break;
    default: break;
  }
  return l ? l(a, s) : hipErrorInvalidValue;
}

}  // namespace rp
}  // namespace fftpde
