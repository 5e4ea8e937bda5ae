// halfrow.hip -- the half-row passes of fft2d_r2c / fft2d_c2r (see
// halfrow.hpp for the algebra).  Row passes: persistent workgroups over
// tiles of whole rows, the M-point transform in registers and LDS, the
// even/odd split (or join) through one more LDS round trip for the mirrored
// index.  Column passes: one workgroup per tile of adjacent columns of one
// field, stage-table twiddles; the tile holding column 0 unpacks (or packs)
// columns 0 and M.
#include <array>
#include <utility>

#include "halfrow.hpp"
#include "kernels.hpp"

namespace fftpde {
namespace {

constexpr int kRowE = 8;
constexpr int kRowTH = 256;
constexpr int kRowMaxLr = 3;
constexpr int kRowMinLm = 3;   // nx >= 16
constexpr int kRowMaxLm = 11;  // nx <= 4096
constexpr int kColTH = 512;
constexpr int kColMinLog = 4;
constexpr int kColMaxLog = 12;

template <typename T>
struct ColCfg {
  static constexpr int E = sizeof(T) == 4 ? 16 : 8;
  static constexpr int MAXLR = sizeof(T) == 4 ? 4 : 3;
  static constexpr int kLogTile = sizeof(T) == 4 ? 13 : 12;  // points per tile
};

// offset of element (row, n) of the work field: rows r = f ny + y, blocks of
// 2^lt columns x ny rows
template <int LM>
__device__ __forceinline__ long long work_at(long long row, int n, int logny, int lt) {
  const long long f = row >> logny, y = row & ((1ll << logny) - 1);
  return (f << (logny + LM)) + ((long long)(n >> lt) << (logny + lt)) + (y << lt) + (n & ((1 << lt) - 1));
}

template <typename T, int LM>
struct RowCfg {
  static constexpr int M = 1 << LM;
  static constexpr int LINES = kRowE * kRowTH / M;
  using Map = RowMap<LM, LINES, plan_pad(LM, kRowMaxLr, false)>;
  using Eng = Engine<T, LM, kRowE, kRowTH, kRowMaxLr, false, Map, false>;
  static constexpr int kLds = Map::kLdsElems > Eng::kLdsWords ? Map::kLdsElems : Eng::kLdsWords;
  static_assert(LINES >= 1 && LINES * M == kRowE * kRowTH, "tile must hold whole rows");
};

// Real rows -> M-point transforms -> X[0..M] (X[0] + i X[M] in column 0) into
// the work field.
template <typename T, int LM>
__global__ void __launch_bounds__(kRowTH) r2c_rows_kernel(HalfRowArgs<T> a) {
  using C = RowCfg<T, LM>;
  using Map = typename C::Map;
  using Eng = typename C::Eng;
  constexpr int M = C::M, LINES = C::LINES;
  __shared__ cx<T> lds[C::kLds];
  int tid = threadIdx.x;
  const long long nrows = a.fields << a.logny;
  const long long ntiles = (nrows + LINES - 1) / LINES;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  cx<T> wall[Eng::kTwRegs];
  Eng::load_all_tw(wall, a.tw, tid);
  const cx<T>* in = reinterpret_cast<const cx<T>*>(a.rin);  // row r: M complex points from r M
  const int sh = kTwLog - a.lognx;                          // w^n = tw[n << sh], w = exp(-2 pi i / nx)
  const T h = T(0.5);
  for (long long tile = walk.first; tile >= 0; tile = walk.next(tile)) {
    tid = opaque(tid);
    const long long row0 = tile * LINES;
    cx<T> x[kRowE];
    // rows past the last reread it and are never stored
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      const long long row = min(row0 + line, nrows - 1);
      x[i] = load_stream(&in[(row << LM) + n]);
    });
    Eng::run_regs(x, lds, wall, tid);
    Eng::for_each_output(tid, [&](int i, int line, int n) { lds[Map::lds(line, n)] = x[i]; });
    lds_barrier();
    Eng::for_each_output(tid, [&](int i, int line, int n) {
      const cx<T> z = x[i];
      cx<T> X;
      if (n == 0) {
        // E[0] = Re Z[0], O[0] = Im Z[0]: X[0] = E + O, X[M] = E - O
        X = {z.re + z.im, z.re - z.im};
      } else {
        const cx<T> zm = lds[Map::lds(line, M - n)];
        const cx<T> e = {h * (z.re + zm.re), h * (z.im - zm.im)};  // (Z + conj Zm) / 2
        const cx<T> o = {h * (z.im + zm.im), h * (zm.re - z.re)};  // -i (Z - conj Zm) / 2
        X = e + cmul(o, a.tw[n << sh]);
      }
      const long long row = row0 + line;
      if (row < nrows) a.work[work_at<LM>(row, n, a.logny, a.lt)] = X;
    });
    lds_barrier();  // the LDS is free for the next tile
  }
}

// Work field (X[0..M], column 0 packed) -> Z = E + i O -> M-point inverse
// transforms -> real rows, times a.scale.
template <typename T, int LM>
__global__ void __launch_bounds__(kRowTH) c2r_rows_kernel(HalfRowArgs<T> a) {
  using C = RowCfg<T, LM>;
  using Map = typename C::Map;
  using Eng = typename C::Eng;
  constexpr int M = C::M, LINES = C::LINES;
  __shared__ cx<T> lds[C::kLds];
  int tid = threadIdx.x;
  const long long nrows = a.fields << a.logny;
  const long long ntiles = (nrows + LINES - 1) / LINES;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  cx<T> wall[Eng::kTwRegs];
  Eng::load_all_tw(wall, a.tw, tid);
  cx<T>* out = reinterpret_cast<cx<T>*>(a.rout);
  const int sh = kTwLog - a.lognx;
  const T h = T(0.5);
  for (long long tile = walk.first; tile >= 0; tile = walk.next(tile)) {
    tid = opaque(tid);
    const long long row0 = tile * LINES;
    cx<T> x[kRowE];
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      const long long row = min(row0 + line, nrows - 1);
      x[i] = a.work[work_at<LM>(row, n, a.logny, a.lt)];
    });
    Eng::for_each_input(tid, [&](int i, int line, int n) { lds[Map::lds(line, n)] = x[i]; });
    lds_barrier();
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      const cx<T> v = x[i];
      cx<T> z;
      if (n == 0) {
        // v = X[0] + i X[M]: E[0] = (X[0] + X[M]) / 2, O[0] = (X[0] - X[M]) / 2, both real
        z = {h * (v.re + v.im), h * (v.re - v.im)};
      } else {
        const cx<T> vm = lds[Map::lds(line, M - n)];
        const cx<T> e = {h * (v.re + vm.re), h * (v.im - vm.im)};  // (X + conj Xm) / 2
        const cx<T> d = {h * (v.re - vm.re), h * (v.im + vm.im)};  // (X - conj Xm) / 2
        const cx<T> o = cmul(d, conjg(a.tw[n << sh]));             // times w^-n
        z = {e.re - o.im, e.im + o.re};                             // E + i O
      }
      x[i] = conjg(z);  // the inverse by conjugation
    });
    lds_barrier();
    Eng::run_regs(x, lds, wall, tid);
    Eng::for_each_output(tid, [&](int i, int line, int n) {
      const long long row = row0 + line;
      if (row < nrows) out[(row << LM) + n] = {x[i].re * a.scale, -x[i].im * a.scale};
    });
  }
}

// One workgroup per column tile.  Workgroups are dealt to the 8 XCDs round
// robin; tile = (b mod 8) G/8 + b/8 gives each XCD a contiguous range of
// tiles, so the tiles that share 128-byte lines (adjacent columns) meet in
// the same L2.
__device__ __forceinline__ long long xcd_tile() {
  const long long b = blockIdx.x, g = gridDim.x;
  return (g & 7) == 0 ? (b & 7) * (g >> 3) + (b >> 3) : b;
}

template <typename T, int LOGN>
struct ColTileCfg {
  static constexpr int E = ColCfg<T>::E;
  static constexpr int MAXLR = ColCfg<T>::MAXLR;
  static constexpr int N = 1 << LOGN;
  static constexpr int LOGT = ColCfg<T>::kLogTile - LOGN;
  static constexpr int TT = 1 << LOGT;
  static_assert(kColTH % TT == 0, "every thread stays on one column of the tile");
  using Map = ColMap<LOGN, LOGT, plan_pad(LOGN, MAXLR, false)>;
  using Eng = Engine<T, LOGN, E, kColTH, MAXLR, false, Map, false>;
  static constexpr int kLds = Map::kLdsElems > Eng::kLdsWords ? Map::kLdsElems : Eng::kLdsWords;
};

// Work field -> forward column transforms -> half spectra [ny][M + 1];
// column 0 (P = Y0 + i YM) unpacks into columns 0 and M.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kColTH) r2c_cols_kernel(HalfRowArgs<T> a) {
  using C = ColTileCfg<T, LOGN>;
  using Map = typename C::Map;
  using Eng = typename C::Eng;
  constexpr int N = C::N, TT = C::TT, LOGT = C::LOGT;
  __shared__ cx<T> lds[C::kLds];
  const int tid = threadIdx.x;
  const int LM = a.lognx - 1, M = 1 << LM, H = M + 1;
  const long long per = M >> LOGT;  // tiles per field
  const long long tile = xcd_tile();
  const long long f = tile / per;
  const int x0 = (int)(tile - f * per) << LOGT;
  const int col = tid & (TT - 1), x = x0 + col;
  const int lt = a.lt;
  const cx<T>* src = a.work + (f << (LOGN + LM)) + ((long long)(x >> lt) << (LOGN + lt)) + (x & ((1 << lt) - 1));
  cx<T> v[C::E];
  Eng::for_each_input(tid, [&](int i, int, int n) { v[i] = src[(long long)n << lt]; });
  Eng::run_stage(v, lds, a.stw, tid);
  cx<T>* dst = a.hout + f * (long long)N * H;
  if (x0 == 0) {
    Eng::for_each_output(tid, [&](int i, int line, int n) { lds[Map::lds(line, n)] = v[i]; });
    lds_barrier();
  }
  const T h = T(0.5);
  Eng::for_each_output(tid, [&](int i, int, int n) {
    if (x == 0) {
      const cx<T> p = v[i], pm = lds[Map::lds(0, (N - n) & (N - 1))];
      dst[(long long)n * H] = {h * (p.re + pm.re), h * (p.im - pm.im)};      // (P + conj Pm) / 2
      dst[(long long)n * H + M] = {h * (p.im + pm.im), h * (pm.re - p.re)};  // -i (P - conj Pm) / 2
    } else {
      dst[(long long)n * H + x] = v[i];
    }
  });
}

// Half spectra -> inverse column transforms -> work field; column 0 carries
// the Hermitian parts of columns 0 and M packed as H0 + i HM.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kColTH) c2r_cols_kernel(HalfRowArgs<T> a) {
  using C = ColTileCfg<T, LOGN>;
  using Eng = typename C::Eng;
  constexpr int N = C::N, TT = C::TT, LOGT = C::LOGT;
  __shared__ cx<T> lds[C::kLds];
  const int tid = threadIdx.x;
  const int LM = a.lognx - 1, M = 1 << LM, H = M + 1;
  const long long per = M >> LOGT;
  const long long tile = xcd_tile();
  const long long f = tile / per;
  const int x0 = (int)(tile - f * per) << LOGT;
  const int col = tid & (TT - 1), x = x0 + col;
  const int lt = a.lt;
  const cx<T>* src = a.hin + f * (long long)N * H;
  const T h = T(0.5);
  cx<T> v[C::E];
  Eng::for_each_input(tid, [&](int i, int, int n) {
    cx<T> w;
    if (x == 0) {
      const int nm = (N - n) & (N - 1);
      const cx<T> a0 = src[(long long)n * H], b0 = src[(long long)nm * H];
      const cx<T> aM = src[(long long)n * H + M], bM = src[(long long)nm * H + M];
      const cx<T> h0 = {h * (a0.re + b0.re), h * (a0.im - b0.im)};
      const cx<T> hM = {h * (aM.re + bM.re), h * (aM.im - bM.im)};
      w = {h0.re - hM.im, h0.im + hM.re};  // H0 + i HM
    } else {
      w = src[(long long)n * H + x];
    }
    v[i] = conjg(w);
  });
  Eng::run_stage(v, lds, a.stw, tid);
  cx<T>* dst = a.work + (f << (LOGN + LM)) + ((long long)(x >> lt) << (LOGN + lt)) + (x & ((1 << lt) - 1));
  Eng::for_each_output(tid, [&](int i, int, int n) { dst[(long long)n << lt] = conjg(v[i]); });
}

// ---- launch tables --------------------------------------------------------

template <typename T>
using Launch = hipError_t (*)(const HalfRowArgs<T>&, hipStream_t);

// persistent row passes: as many workgroups as fit, at most one per tile
template <typename T, int LM, bool FWD>
int row_slots() {
  int dev = 0, cus = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const hipError_t e = FWD ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, r2c_rows_kernel<T, LM>, kRowTH, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, c2r_rows_kernel<T, LM>, kRowTH, 0);
  return e == hipSuccess ? std::max(1, n) * cus : 0;
}

template <typename T, int LM, bool FWD>
hipError_t launch_rows(const HalfRowArgs<T>& a, hipStream_t s) {
  static const int slots = row_slots<T, LM, FWD>();  // thread-safe one-time query
  if (slots <= 0) return hipErrorInvalidValue;
  constexpr int LINES = RowCfg<T, LM>::LINES;
  const long long ntiles = ((a.fields << a.logny) + LINES - 1) / LINES;
  const long long grid = std::min<long long>(ntiles, slots);
  if (grid <= 0) return hipSuccess;
  if constexpr (FWD) hipLaunchKernelGGL((r2c_rows_kernel<T, LM>), dim3((unsigned)grid), dim3(kRowTH), 0, s, a);
  else hipLaunchKernelGGL((c2r_rows_kernel<T, LM>), dim3((unsigned)grid), dim3(kRowTH), 0, s, a);
  return hipGetLastError();
}

template <typename T, int LOGN, bool FWD>
hipError_t launch_cols(const HalfRowArgs<T>& a, hipStream_t s) {
  const long long per = (1ll << (a.lognx - 1)) >> ColTileCfg<T, LOGN>::LOGT;
  const long long grid = a.fields * per;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffll) return hipErrorInvalidValue;
  if constexpr (FWD) hipLaunchKernelGGL((r2c_cols_kernel<T, LOGN>), dim3((unsigned)grid), dim3(kColTH), 0, s, a);
  else hipLaunchKernelGGL((c2r_cols_kernel<T, LOGN>), dim3((unsigned)grid), dim3(kColTH), 0, s, a);
  return hipGetLastError();
}

template <typename T, bool FWD, int... L>
constexpr std::array<Launch<T>, sizeof...(L)> row_table(std::integer_sequence<int, L...>) {
  return {&launch_rows<T, L + kRowMinLm, FWD>...};
}
template <typename T, bool FWD, int... L>
constexpr std::array<Launch<T>, sizeof...(L)> col_table(std::integer_sequence<int, L...>) {
  return {&launch_cols<T, L + kColMinLog, FWD>...};
}

template <typename T, bool FWD>
const Launch<T>* rows_for(int lm) {
  static constexpr auto tab = row_table<T, FWD>(std::make_integer_sequence<int, kRowMaxLm - kRowMinLm + 1>());
  return lm >= kRowMinLm && lm <= kRowMaxLm ? &tab[lm - kRowMinLm] : nullptr;
}
template <typename T, bool FWD>
const Launch<T>* cols_for(int logn) {
  static constexpr auto tab = col_table<T, FWD>(std::make_integer_sequence<int, kColMaxLog - kColMinLog + 1>());
  return logn >= kColMinLog && logn <= kColMaxLog ? &tab[logn - kColMinLog] : nullptr;
}

template <typename T, bool FWD, bool ROWS>
hipError_t run(const HalfRowArgs<T>& a, hipStream_t s) {
  if (!halfrow_supported(sizeof(T) == 8, a.lognx, a.logny)) return hipErrorInvalidValue;
  const Launch<T>* l = ROWS ? rows_for<T, FWD>(a.lognx - 1) : cols_for<T, FWD>(a.logny);
  return l ? (*l)(a, s) : hipErrorInvalidValue;
}

}  // namespace

int halfrow_col_logt(int fp64, int logny) { return (fp64 ? 12 : 13) - logny; }
int halfrow_col_maxlr(int fp64) { return fp64 ? 3 : 4; }

bool halfrow_supported(int fp64, int lognx, int logny) {
  const int lm = lognx - 1;
  return lm >= kRowMinLm && lm <= kRowMaxLm && logny >= kColMinLog && logny <= kColMaxLog &&
         halfrow_col_logt(fp64, logny) <= lm;
}

template <typename T>
hipError_t launch_r2c_rows(const HalfRowArgs<T>& a, hipStream_t s) {
  return run<T, true, true>(a, s);
}
template <typename T>
hipError_t launch_r2c_cols(const HalfRowArgs<T>& a, hipStream_t s) {
  return run<T, true, false>(a, s);
}
template <typename T>
hipError_t launch_c2r_cols(const HalfRowArgs<T>& a, hipStream_t s) {
  return run<T, false, false>(a, s);
}
template <typename T>
hipError_t launch_c2r_rows(const HalfRowArgs<T>& a, hipStream_t s) {
  return run<T, false, true>(a, s);
}

template hipError_t launch_r2c_rows<float>(const HalfRowArgs<float>&, hipStream_t);
template hipError_t launch_r2c_rows<double>(const HalfRowArgs<double>&, hipStream_t);
template hipError_t launch_r2c_cols<float>(const HalfRowArgs<float>&, hipStream_t);
template hipError_t launch_r2c_cols<double>(const HalfRowArgs<double>&, hipStream_t);
template hipError_t launch_c2r_cols<float>(const HalfRowArgs<float>&, hipStream_t);
template hipError_t launch_c2r_cols<double>(const HalfRowArgs<double>&, hipStream_t);
template hipError_t launch_c2r_rows<float>(const HalfRowArgs<float>&, hipStream_t);
template hipError_t launch_c2r_rows<double>(const HalfRowArgs<double>&, hipStream_t);

}  // namespace fftpde
