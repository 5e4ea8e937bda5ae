// mixed.hip -- the mixed-radix (2, 3, 4, 5, 7, 8) line transforms on LDS
// tiles, and the column pass with the solve's symbol between the forward
// and the inverse transform.
#include "mixed.hpp"
#include "mixed_dev.hpp"

namespace fftpde {
namespace {

// LDS position of tile element i: one pad word every 32 elements spreads
// the strided accesses of the early stages over the banks (a bank model of
// the stages at 1000, 1536 and 2000 points: 4.4-4.9 passes per wavefront
// access without the pad, 2.3-2.7 with it; 2 is conflict free).
__device__ __forceinline__ int mr_pad(int i) { return i + (i >> 5); }
constexpr int mr_padded(int n) { return n + (n >> 5) + 1; }

// One Stockham stage of radix R on nl lines of length n (line l at
// element l ls of the tile) after sub-transforms of length ns:
//   butterfly j (0 <= j < n/R), k = j mod ns:
//     v_t = x[j + t n/R] w_{ns R}^{t k},  v = DFT_R(v),  y[(j - k) R + k + t ns] = v_t
// Every thread takes its butterflies' inputs into registers, the workgroup
// synchronises, and the outputs overwrite the same buffer.
template <typename T, int R, int CAP, int TH>
__device__ __forceinline__ void mr_stage(cx<T>* buf, int nl, int n, int ls, int ns, MrDiv by_m, MrDiv by_ns,
                                         const cx<T>* __restrict__ tw, int tid) {
  constexpr int MAXB = (CAP / R + TH - 1) / TH;  // butterflies per thread
  constexpr int H = (R & 1) ? (R - 1) / 2 : 1;
  const int m = n / R;
  const int nb = nl * m;
  const int tstep = n / (ns * R);  // w_{ns R} = w_n^{tstep}
  T cs[H], sn[H];
  if constexpr (R & 1) {
#pragma unroll
    for (int q = 1; q <= H; q++) {
      const cx<T> w = tw[q * m];  // exp(-2 pi i q / R)
      cs[q - 1] = w.re;
      sn[q - 1] = -w.im;
    }
  }
  cx<T> v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; i++) {
    const int b = tid + i * TH;
    if (b < nb) {
      const int line = by_m(b), j = b - line * m, k = j - by_ns(j) * ns;
      const int src = line * ls + j;
#pragma unroll
      for (int t = 0; t < R; t++) v[i][t] = buf[mr_pad(src + t * m)];
      if (ns > 1) {
#pragma unroll
        for (int t = 1; t < R; t++) v[i][t] = cmul(v[i][t], tw[t * k * tstep]);
      }
      if constexpr (R & 1) dft_odd<R>(v[i], cs, sn);
      else dft<R>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; i++) {
    const int b = tid + i * TH;
    if (b < nb) {
      const int line = by_m(b), j = b - line * m, k = j - by_ns(j) * ns;
      const int dst = line * ls + (j - k) * R + k;
#pragma unroll
      for (int t = 0; t < R; t++) buf[mr_pad(dst + t * ns)] = v[i][t];
    }
  }
  __syncthreads();
}

// Forward transform of nl lines in LDS (at most CAP points), natural order
// in and out.
template <typename T, int CAP, int TH>
__device__ void mr_fft(cx<T>* buf, int nl, const MrPlan& p, int ls, const cx<T>* __restrict__ tw, int tid) {
  int ns = 1;
  for (int s = 0; s < p.nst; s++) {
    const int r = p.radix[s];
    const MrDiv bm = p.by_m[s], bn = p.by_ns[s];
    switch (r) {
      case 2: mr_stage<T, 2, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
      case 3: mr_stage<T, 3, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
      case 4: mr_stage<T, 4, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
      case 5: mr_stage<T, 5, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
      case 7: mr_stage<T, 7, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
      default: mr_stage<T, 8, CAP, TH>(buf, nl, p.n, ls, ns, bm, bn, tw, tid); break;
    }
    ns *= r;
  }
}

// The wave propagator with an initial velocity at (a', b'):
//   U = cos(w t) F + sin(w t)/w G,  V = -w sin(w t) F + cos(w t) G,  w = c |k|
// (t in place of sin(w t)/w at w = 0), times 1/(nx ny).
struct MrWave {
  double cw, sow, wsw;
  __device__ __forceinline__ MrWave(const MrSym& s, int ai, int bi) {
    const double kx = s.kxs * ai, ky = s.kys * bi;
    const double w = s.c * sqrt(fma(kx, kx, ky * ky));
    const double hx = s.hx * ai, hy = s.hy * bi;
    double h = sqrt(fma(hx, hx, hy * hy));  // |w t| / pi
    if (s.t < 0) h = -h;                      // sin is odd in t
    double sn, cs;
    sincospi(h, &sn, &cs);
    cw = s.scale * cs;
    sow = s.scale * (w == 0.0 ? s.t : sn / w);
    wsw = s.scale * w * sn;
  }
};

template <typename T, int NF, bool SMALL>
__global__ void __launch_bounds__(SMALL ? kMrRowTH : mr_threads(sizeof(T) == 8)) mr_kernel(MrArgs<T> a) {
  constexpr int TH = SMALL ? kMrRowTH : mr_threads(sizeof(T) == 8);
  constexpr int CAP = SMALL ? kMrRowCap : mr_cap(sizeof(T) == 8, NF);
  // per field: column tiles pad each line by one, then the bank pad
  constexpr int LDSF = mr_padded(CAP + kMrMaxColLines);
  constexpr bool TWL = mr_tw_in_lds(sizeof(T) == 8, NF);
  __shared__ cx<T> lds[NF * LDSF];
  __shared__ cx<T> twl[TWL ? kMrMaxSide : 1];
  const int tid = threadIdx.x;
  const int n = a.plan.n;
  const bool col = a.mode >= kMrColFwd;
  const cx<T>* tw = a.tw;
  if constexpr (TWL) {
    for (int e = tid; e < n; e += TH) twl[e] = a.tw[e];  // read after the first barrier
    tw = twl;
  }
  // Tile t: nl lines; rows start at element `base`, columns at c0 of their
  // field.  Element idx of a tile: its line, position and global offset.
  // Columns walk the tile's columns fastest (a wavefront reads whole row
  // segments) over the full tile width; positions past the last column of a
  // ragged tile are skipped.
  struct Tile {
    long long base, row0;
    int nl, c0, span;
  };
  auto tile_at = [&](long long t) {
    Tile g;
    if (!col) {
      const long long nrows = (long long)a.ny * a.fields;
      const long long row0 = t * a.lines;
      g.nl = (int)min((long long)a.lines, nrows - row0);
      g.base = row0 * n;
      g.row0 = row0;
      g.c0 = 0;
      g.span = g.nl * n;
    } else {
      const int tpf = (a.nx + a.lines - 1) / a.lines;
      const long long f = t / tpf;
      g.c0 = (int)(t - f * tpf) * a.lines;
      g.nl = min(a.lines, a.nx - g.c0);
      g.base = f * (long long)a.nx * a.ny + g.c0;
      g.row0 = 0;
      g.span = a.lines * n;
    }
    return g;
  };
  auto where = [&](const Tile& g, int idx, int& line, int& j) -> long long {
    if (!col) {
      line = a.plan.by_n(idx);
      j = idx - line * n;
      return g.base + idx;
    }
    j = a.by_lines(idx);
    line = idx - j * a.lines;
    return g.base + (long long)j * a.nx + line;
  };
  // Real fields in pairs: row `line` of tile g is row r of pair field p,
  // i.e. row r of real fields 2p and 2p + 1; returns the offset r nx + j in
  // a real field and sets p.  (row0 mod ny) + line stays below 2^16.
  const long long pts = (long long)a.nx * a.ny;
  auto real_at = [&](const Tile& g, int line, int j, long long& p) -> long long {
    const long long p0 = g.row0 / a.ny;
    const int rr = (int)(g.row0 - p0 * a.ny) + line;
    const int dp = a.by_ny(rr);
    p = p0 + dp;
    return (long long)(rr - dp * a.ny) * a.nx + j;
  };
  const bool conj_in = a.mode == kMrRowInv || a.mode == kMrColInv;
  const bool has2 = NF == 2 && a.in1 != nullptr;
  const bool out2 = NF == 2 && a.out1 != nullptr;
  constexpr int PT = (CAP + TH - 1) / TH;  // points per thread of a full tile
  // Round k of the walk covers tiles [k G, (k + 1) G).  Workgroups are
  // dispatched to the 8 XCDs in turn (blockIdx mod 8), so a round hands each
  // XCD G/8 consecutive tiles: adjacent column tiles, which share the cache
  // lines of their row pieces, then meet in one L2.
  const int G = gridDim.x;
  const long long lane = (G % 8 == 0) ? (long long)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  long long t = lane;
  if (t >= a.tiles) return;
  while (true) {
    const Tile g = tile_at(t);
    // every load of the tile is issued before the first value lands in LDS
#pragma unroll
    for (int fi = 0; fi < NF; fi++) {
      const cx<T>* in = fi == 0 ? a.in0 : a.in1;
      if (fi == 1 && !has2) continue;
      cx<T>* buf = lds + fi * LDSF;
      if (NF == 1 && a.rin != nullptr) {  // forward rows of real fields in pairs
        for (int idx = tid; idx < g.span; idx += TH) {
          int line, j;
          (void)where(g, idx, line, j);
          if (line >= g.nl) continue;
          long long p;
          const long long e = real_at(g, line, j, p);
          const T re = a.rin[2 * p * pts + e];
          const T im = 2 * p + 1 < a.nreal ? a.rin[(2 * p + 1) * pts + e] : T(0);
          buf[mr_pad(line * a.ls + j)] = {re, im};
        }
      } else if constexpr (sizeof(T) == 4) {
        cx<T> v[PT];
#pragma unroll
        for (int i = 0; i < PT; i++) {
          const int idx = tid + i * TH;
          int line, j;
          const long long off = where(g, idx, line, j);
          if (idx < g.span && line < g.nl) v[i] = in[off];
        }
#pragma unroll
        for (int i = 0; i < PT; i++) {
          const int idx = tid + i * TH;
          int line, j;
          (void)where(g, idx, line, j);
          if (idx < g.span && line < g.nl) {
            if (conj_in) v[i].im = -v[i].im;
            buf[mr_pad(line * a.ls + j)] = v[i];
          }
        }
      } else {  // FP64: no registers to spare for a whole tile
        for (int idx = tid; idx < g.span; idx += TH) {
          int line, j;
          const long long off = where(g, idx, line, j);
          if (line >= g.nl) continue;
          cx<T> v = in[off];
          if (conj_in) v.im = -v.im;
          buf[mr_pad(line * a.ls + j)] = v;
        }
      }
    }
    __syncthreads();
    const int nl = g.nl, c0 = g.c0;
    mr_fft<T, CAP, TH>(lds, nl, a.plan, a.ls, tw, tid);
    if (has2) mr_fft<T, CAP, TH>(lds + LDSF, nl, a.plan, a.ls, tw, tid);
    if (a.mode == kMrColSolve) {
      // the symbol, then the inverse through the conjugation identity of
      // the iDFT (Sec. II.B): the values are conjugated here and on the way out
      const int cnt = nl * n;
      for (int idx = tid; idx < cnt; idx += TH) {
        const int line = a.plan.by_n(idx), j = idx - line * n;
        const int ai = mr_sidx(c0 + line, a.nx), bi = mr_sidx(j, a.ny);
        cx<T>* p0 = lds + mr_pad(line * a.ls + j);
        if constexpr (NF == 1) {
          const T m = mr_symbol<T>(a.sym, ai, bi);
          *p0 = {p0->re * m, -p0->im * m};
        } else {
          const MrWave w(a.sym, ai, bi);
          cx<T>* p1 = p0 + LDSF;
          const cx<T> F = *p0;
          const cx<T> G = has2 ? *p1 : cx<T>{T(0), T(0)};
          const T cw = T(w.cw), sow = T(w.sow), wsw = T(w.wsw);
          *p0 = {cw * F.re + sow * G.re, -(cw * F.im + sow * G.im)};
          if (out2) *p1 = {cw * G.re - wsw * F.re, -(cw * G.im - wsw * F.im)};
        }
      }
      __syncthreads();
      mr_fft<T, CAP, TH>(lds, nl, a.plan, a.ls, tw, tid);
      if (out2) mr_fft<T, CAP, TH>(lds + LDSF, nl, a.plan, a.ls, tw, tid);
    }
    const bool conj_out = a.mode == kMrRowInv || a.mode == kMrColInv || a.mode == kMrColSolve;
    const T sc = a.mode == kMrRowInv ? a.scale : T(1);
#pragma unroll
    for (int fi = 0; fi < NF; fi++) {
      cx<T>* out = fi == 0 ? a.out0 : a.out1;
      if (fi == 1 && !out2) continue;
      const cx<T>* buf = lds + fi * LDSF;
      if (NF == 1 && a.rout != nullptr) {  // inverse rows back to real fields in pairs
        for (int idx = tid; idx < g.span; idx += TH) {
          int line, j;
          (void)where(g, idx, line, j);
          if (line >= nl) continue;
          long long p;
          const long long e = real_at(g, line, j, p);
          const cx<T> v = buf[mr_pad(line * a.ls + j)];
          a.rout[2 * p * pts + e] = v.re * sc;
          if (2 * p + 1 < a.nreal) a.rout[(2 * p + 1) * pts + e] = -v.im * sc;
        }
        continue;
      }
      for (int idx = tid; idx < g.span; idx += TH) {
        int line, j;
        const long long off = where(g, idx, line, j);
        if (line >= nl) continue;
        const cx<T> v = buf[mr_pad(line * a.ls + j)];
        out[off] = conj_out ? cx<T>{v.re * sc, -v.im * sc} : v;
      }
    }
    t += G;
    if (t >= a.tiles) break;
    __syncthreads();  // every thread is done with LDS before the next tile lands
  }
}

template <typename T, int NF, bool SMALL>
int occupancy_of() {
  int n = 0;
  const int th = SMALL ? kMrRowTH : mr_threads(sizeof(T) == 8);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mr_kernel<T, NF, SMALL>, th, 0) != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

}  // namespace

template <typename T>
int mr_occupancy(int nf, bool small) {
  static const int o1 = occupancy_of<T, 1, false>(), o2 = occupancy_of<T, 2, false>();
  static const int os = sizeof(T) == 4 ? occupancy_of<T, 1, true>() : 1;
  if (small) return os;
  return nf == 2 ? o2 : o1;
}

template <typename T>
hipError_t mr_launch(const MrArgs<T>& a, int nf, bool small, int grid, hipStream_t s) {
  if (a.tiles < 1 || grid < 1 || grid > a.tiles) return hipErrorInvalidValue;
  if (small && !mr_row_small(sizeof(T) == 8, nf, a.mode >= kMrColFwd)) return hipErrorInvalidValue;
  const unsigned th = mr_threads(sizeof(T) == 8);
  if (small) {
    if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL((mr_kernel<T, 1, true>), dim3((unsigned)grid), dim3(kMrRowTH), 0, s, a);
  } else if (nf == 2) {
    hipLaunchKernelGGL((mr_kernel<T, 2, false>), dim3((unsigned)grid), dim3(th), 0, s, a);
  } else {
    hipLaunchKernelGGL((mr_kernel<T, 1, false>), dim3((unsigned)grid), dim3(th), 0, s, a);
  }
  return hipGetLastError();
}

template int mr_occupancy<float>(int, bool);
template int mr_occupancy<double>(int, bool);
template hipError_t mr_launch<float>(const MrArgs<float>&, int, bool, int, hipStream_t);
template hipError_t mr_launch<double>(const MrArgs<double>&, int, bool, int, hipStream_t);

}  // namespace fftpde
