// halfrow.hip -- the passes of fft2d_r2c / fft2d_c2r on real fields (see
// halfrow.hpp for the algebra).  Column passes: one workgroup per tile of
// adjacent columns of the complex view of one field, stage-table twiddles.
// Row passes: persistent workgroups over tiles of row pairs (b, -b), the
// M-point transforms in registers and LDS, the even/odd combination through
// one more LDS round trip for the mirrored row and index.
#include <array>
#include <utility>

#include "halfrow.hpp"
#include "kernels.hpp"

namespace fftpde {
namespace {

constexpr int kRowE = 8;
constexpr int kRowTH = 512;
constexpr int kRowMaxLr = 3;
constexpr int kRowMinLm = 3;   // nx >= 16
constexpr int kRowMaxLm = 11;  // nx <= 4096
constexpr int kColTH = 1024;
constexpr int kColMinLog = 4;
constexpr int kColMaxLog = 12;

template <typename T>
struct ColCfg {
  static constexpr int E = sizeof(T) == 4 ? 16 : 8;
  static constexpr int MAXLR = sizeof(T) == 4 ? 4 : 3;
  static constexpr int kLogTile = sizeof(T) == 4 ? 14 : 13;  // points per tile
};

// offset of element (row, n) of the work field: rows r = f ny + y, blocks of
// 2^lt columns x ny rows
template <int LM>
__device__ __forceinline__ long long work_at(long long row, int n, int logny, int lt) {
  const long long f = row >> logny, y = row & ((1ll << logny) - 1);
  return (f << (logny + LM)) + ((long long)(n >> lt) << (logny + lt)) + (y << lt) + (n & ((1 << lt) - 1));
}

// Row passes: tiles of LINES rows = LINES / 2 row pairs (b, -b); pair p of a
// field is rows (p, ny - p) for p > 0, and pair 0 is rows 0 and ny/2, each
// its own mirror.
template <typename T, int LM>
struct RowCfg {
  static constexpr int M = 1 << LM;
  static constexpr int LINES = kRowE * kRowTH / M;
  static constexpr int PAIRS = LINES / 2;
  using Map = RowMap<LM, LINES, plan_pad(LM, kRowMaxLr, false)>;
  using Eng = Engine<T, LM, kRowE, kRowTH, kRowMaxLr, false, Map, false>;
  static constexpr int kLds = Map::kLdsElems > Eng::kLdsWords ? Map::kLdsElems : Eng::kLdsWords;
  static_assert(PAIRS >= 1 && LINES * M == kRowE * kRowTH, "tile must hold whole row pairs");
};

struct PairLine {
  long long row;  // f ny + b
  int mirror;     // the line holding row -b (the line itself for b = 0, ny/2)
  bool live;      // a pair of the launch (padding lines reread the last pair)
};

template <int LINES>
__device__ __forceinline__ PairLine pair_line(long long tile, int line, long long npairs, int logny) {
  constexpr int PAIRS = LINES / 2;
  const long long q0 = tile * PAIRS + (line >> 1);
  const long long q = min(q0, npairs - 1);
  const int half = 1 << (logny - 1);
  const long long f = q >> (logny - 1);
  const int p = (int)(q & (half - 1));
  const int b = (line & 1) == 0 ? p : (p == 0 ? half : 2 * half - p);
  return {(f << logny) + b, p == 0 ? line : (line ^ 1), q0 < npairs};
}

// r2c, second pass: work field rows (Zc) -> M-point transforms of row pairs
// -> half-spectrum rows X[b][0..M].
template <typename T, int LM>
__global__ void __launch_bounds__(kRowTH) r2c_rows_kernel(HalfRowArgs<T> a) {
  using C = RowCfg<T, LM>;
  using Map = typename C::Map;
  using Eng = typename C::Eng;
  constexpr int M = C::M, LINES = C::LINES, PAIRS = C::PAIRS;
  __shared__ cx<T> lds[C::kLds];
  int tid = threadIdx.x;
  const long long npairs = a.fields << (a.logny - 1);
  const long long ntiles = (npairs + PAIRS - 1) / PAIRS;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  cx<T> wall[Eng::kTwRegs];
  Eng::load_all_tw(wall, a.tw, tid);
  const int sh = kTwLog - a.lognx;  // w^k = tw[k << sh], w = exp(-2 pi i / nx)
  // FP32: w^k at this thread's output positions k, which no tile changes,
  // loaded once, so no tile waits on them after its transform (FP64 loads
  // them per tile: held in registers they would cost a resident wave)
  constexpr bool kHold = sizeof(T) == 4;
  cx<T> wk[kHold ? kRowE : 1];
  if constexpr (kHold) Eng::for_each_output(tid, [&](int i, int, int k) { wk[i] = a.tw[k << sh]; });
  auto w_at = [&](int i, int k) -> cx<T> {
    if constexpr (kHold) return wk[i];
    else return a.tw[k << sh];
  };
  const T h = T(0.5);
  for (long long tile = walk.first; tile >= 0; tile = walk.next(tile)) {
    tid = opaque(tid);
    cx<T> x[kRowE];
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      x[i] = a.work[work_at<LM>(pair_line<LINES>(tile, line, npairs, a.logny).row, n, a.logny, a.lt)];
    });
    Eng::run_regs(x, lds, wall, tid);
    Eng::for_each_output(tid, [&](int i, int line, int n) { lds[Map::lds(line, n)] = x[i]; });
    lds_barrier();
    Eng::for_each_output(tid, [&](int i, int line, int k) {
      const PairLine pl = pair_line<LINES>(tile, line, npairs, a.logny);
      const cx<T> z = x[i];
      const cx<T> zm = lds[Map::lds(pl.mirror, (M - k) & (M - 1))];  // Zr[-b][-k]
      const cx<T> e = {h * (z.re + zm.re), h * (z.im - zm.im)};      // (Zr + conj Zr-) / 2
      const cx<T> o = {h * (z.im + zm.im), h * (zm.re - z.re)};      // -i (Zr - conj Zr-) / 2
      if (pl.live) {
        cx<T>* out = a.hout + pl.row * (M + 1);
        out[k] = e + cmul(o, w_at(i, k));
        if (k == 0) out[M] = e - o;  // w^M = -1
      }
    });
    lds_barrier();  // the LDS is free for the next tile
  }
}

// c2r, first pass: half-spectrum rows of each pair -> Zr = E + i O (the
// Hermitian extension) -> M-point inverse transforms -> work field rows.
template <typename T, int LM>
__global__ void __launch_bounds__(kRowTH) c2r_rows_kernel(HalfRowArgs<T> a) {
  using C = RowCfg<T, LM>;
  using Map = typename C::Map;
  using Eng = typename C::Eng;
  constexpr int M = C::M, LINES = C::LINES, PAIRS = C::PAIRS;
  __shared__ cx<T> lds[C::kLds];
  __shared__ cx<T> last[LINES];  // column M of each line's row
  int tid = threadIdx.x;
  const long long npairs = a.fields << (a.logny - 1);
  const long long ntiles = (npairs + PAIRS - 1) / PAIRS;
  const TileWalk<1> walk(ntiles);
  if (walk.first < 0) return;
  cx<T> wall[Eng::kTwRegs];
  Eng::load_all_tw(wall, a.tw, tid);
  const int sh = kTwLog - a.lognx;
  // FP32: w^-k at this thread's input positions k, loaded once (no tile
  // changes them; FP64 loads them per tile, as in the r2c rows)
  constexpr bool kHold = sizeof(T) == 4;
  cx<T> wk[kHold ? kRowE : 1];
  if constexpr (kHold) Eng::for_each_input(tid, [&](int i, int, int k) { wk[i] = conjg(a.tw[k << sh]); });
  auto wc_at = [&](int i, int k) -> cx<T> {
    if constexpr (kHold) return wk[i];
    else return conjg(a.tw[k << sh]);
  };
  const T h = T(0.5);
  for (long long tile = walk.first; tile >= 0; tile = walk.next(tile)) {
    tid = opaque(tid);
    cx<T> x[kRowE];
    // FP32: the tile's loads at raised wave priority, ahead of the other
    // resident workgroup's transform (2048: 70.4 -> 68-69 us per 8 fields)
    if constexpr (kHold) __builtin_amdgcn_s_setprio(3);
    Eng::for_each_input(tid, [&](int i, int line, int n) {
      const cx<T>* in = a.hin + pair_line<LINES>(tile, line, npairs, a.logny).row * (M + 1);
      x[i] = in[n];
      lds[Map::lds(line, n)] = x[i];
      if (n == 0) last[line] = in[M];
    });
    if constexpr (kHold) __builtin_amdgcn_s_setprio(0);
    lds_barrier();
    Eng::for_each_input(tid, [&](int i, int line, int k) {
      const PairLine pl = pair_line<LINES>(tile, line, npairs, a.logny);
      cx<T> e, o;
      if (k == 0) {
        // the Hermitian parts of columns 0 and M: H = (X[b] + conj X[-b]) / 2
        const cx<T> x0 = x[i], x0m = lds[Map::lds(pl.mirror, 0)];
        const cx<T> xM = last[line], xMm = last[pl.mirror];
        const cx<T> h0 = {h * (x0.re + x0m.re), h * (x0.im - x0m.im)};
        const cx<T> hM = {h * (xM.re + xMm.re), h * (xM.im - xMm.im)};
        e = {h * (h0.re + hM.re), h * (h0.im + hM.im)};
        o = {h * (h0.re - hM.re), h * (h0.im - hM.im)};
      } else {
        const cx<T> v = x[i];
        const cx<T> vm = lds[Map::lds(pl.mirror, M - k)];  // X~[b][k + M] = conj X[-b][M - k]
        e = {h * (v.re + vm.re), h * (v.im - vm.im)};
        o = cmul(cx<T>{h * (v.re - vm.re), h * (v.im + vm.im)}, wc_at(i, k));  // times w^-k
      }
      x[i] = {e.re - o.im, -(e.im + o.re)};  // conj(E + i O): the inverse by conjugation
    });
    lds_barrier();
    Eng::run_regs(x, lds, wall, tid);
    Eng::for_each_output(tid, [&](int i, int line, int n) {
      const PairLine pl = pair_line<LINES>(tile, line, npairs, a.logny);
      if (pl.live) a.work[work_at<LM>(pl.row, n, a.logny, a.lt)] = conjg(x[i]);
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
  static constexpr int kLds = Eng::kLdsWords;
};

// Column tile addresses: field f, first column x0, this thread's column x
struct ColTile {
  long long f;
  int x;
};

template <int LOGT>
__device__ __forceinline__ ColTile col_tile(int lm) {
  const long long per = (1ll << lm) >> LOGT;  // tiles per field
  const long long tile = xcd_tile();
  const long long f = tile / per;
  return {f, ((int)(tile - f * per) << LOGT) + (int)(threadIdx.x & ((1 << LOGT) - 1))};
}

// r2c, first pass: the complex view z[y][a] of the real fields -> forward
// column transforms -> work field.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kColTH) r2c_cols_kernel(HalfRowArgs<T> a) {
  using C = ColTileCfg<T, LOGN>;
  using Eng = typename C::Eng;
  __shared__ cx<T> lds[C::kLds];
  const int tid = threadIdx.x;
  const int lm = a.lognx - 1, lt = a.lt;
  const ColTile t = col_tile<C::LOGT>(lm);
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.rin) + (t.f << (LOGN + lm)) + t.x;
  cx<T> v[C::E];
  Eng::for_each_input(tid, [&](int i, int, int n) { v[i] = load_stream(&src[(long long)n << lm]); });
  Eng::run_stage(v, lds, a.stw, tid);
  cx<T>* dst = a.work + (t.f << (LOGN + lm)) + ((long long)(t.x >> lt) << (LOGN + lt)) + (t.x & ((1 << lt) - 1));
  Eng::for_each_output(tid, [&](int i, int, int n) { dst[(long long)n << lt] = v[i]; });
}

// c2r, second pass: work field -> inverse column transforms (by
// conjugation), times 1 / (M ny) -> the complex view of the real fields.
template <typename T, int LOGN>
__global__ void __launch_bounds__(kColTH) c2r_cols_kernel(HalfRowArgs<T> a) {
  using C = ColTileCfg<T, LOGN>;
  using Eng = typename C::Eng;
  __shared__ cx<T> lds[C::kLds];
  const int tid = threadIdx.x;
  const int lm = a.lognx - 1, lt = a.lt;
  const ColTile t = col_tile<C::LOGT>(lm);
  const cx<T>* src = a.work + (t.f << (LOGN + lm)) + ((long long)(t.x >> lt) << (LOGN + lt)) + (t.x & ((1 << lt) - 1));
  cx<T> v[C::E];
  Eng::for_each_input(tid, [&](int i, int, int n) { v[i] = conjg(src[(long long)n << lt]); });
  Eng::run_stage(v, lds, a.stw, tid);
  cx<T>* dst = reinterpret_cast<cx<T>*>(a.rout) + (t.f << (LOGN + lm)) + t.x;
  const T sc = a.scale;
  Eng::for_each_output(tid, [&](int i, int, int n) { dst[(long long)n << lm] = {v[i].re * sc, -v[i].im * sc}; });
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
  constexpr int PAIRS = RowCfg<T, LM>::PAIRS;
  const long long ntiles = ((a.fields << (a.logny - 1)) + PAIRS - 1) / PAIRS;
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

int halfrow_col_logt(int fp64, int logny) { return (fp64 ? 13 : 14) - logny; }
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
