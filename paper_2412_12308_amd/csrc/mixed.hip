// mixed.hip -- the mixed-radix (2, 3, 4, 5, 7, 8) line transforms on LDS
// tiles, and the column pass with the solve's symbol between the forward
// and the inverse transform.
#include "mixed.hpp"

namespace fftpde {
namespace {

// Odd radix R = 3, 5, 7, forward sign, natural order.  With the symmetric
// pairs a_m = v_m + v_{R-m} and b_m = v_m - v_{R-m} (m = 1..H, H = (R-1)/2),
// the DFT sum splits into a cosine and a sine sum:
//   X_k     = v_0 + sum_m a_m cos(2 pi m k / R) - i sum_m b_m sin(2 pi m k / R)
//   X_{R-k} = v_0 + sum_m a_m cos(2 pi m k / R) + i sum_m b_m sin(2 pi m k / R)
// for k = 1..H, and X_0 = v_0 + sum_m a_m.  cs[q-1], sn[q-1] are cos and sin
// of 2 pi q / R for q = 1..H; the other angles fold onto them.
template <int R, typename T>
__device__ __forceinline__ void dft_odd(cx<T>* v, const T* cs, const T* sn) {
  constexpr int H = (R - 1) / 2;
  cx<T> a[H], b[H];
  cx<T> x0 = v[0];
  cx<T> sum = v[0];
#pragma unroll
  for (int m = 1; m <= H; m++) {
    a[m - 1] = v[m] + v[R - m];
    b[m - 1] = v[m] - v[R - m];
    sum = sum + a[m - 1];
  }
#pragma unroll
  for (int k = 1; k <= H; k++) {
    cx<T> A = x0, B = {T(0), T(0)};
#pragma unroll
    for (int m = 1; m <= H; m++) {
      const int q = (m * k) % R;
      const T c = q <= H ? cs[q - 1] : cs[R - q - 1];
      const T s = q <= H ? sn[q - 1] : -sn[R - q - 1];
      A = {A.re + a[m - 1].re * c, A.im + a[m - 1].im * c};
      B = {B.re + b[m - 1].re * s, B.im + b[m - 1].im * s};
    }
    // A - i B and A + i B
    v[k] = {A.re + B.im, A.im - B.re};
    v[R - k] = {A.re - B.im, A.im + B.re};
  }
  v[0] = sum;
}

// One Stockham stage of radix R on nl lines of length n (line l at
// buf + l ls) after sub-transforms of length ns:
//   butterfly j (0 <= j < n/R), k = j mod ns:
//     v_t = x[j + t n/R] w_{ns R}^{t k},  v = DFT_R(v),  y[(j - k) R + k + t ns] = v_t
// Every thread takes its butterflies' inputs into registers, the workgroup
// synchronises, and the outputs overwrite the same buffer.
template <typename T, int R>
__device__ __forceinline__ void mr_stage(cx<T>* buf, int nl, int n, int ls, int ns, const cx<T>* __restrict__ tw,
                                         int tid) {
  constexpr int MAXB = (kMrTilePts / R + kMrTH - 1) / kMrTH;  // butterflies per thread
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
    const int b = tid + i * kMrTH;
    if (b < nb) {
      const int line = b / m, j = b - line * m, k = j % ns;
      const cx<T>* src = buf + line * ls + j;
#pragma unroll
      for (int t = 0; t < R; t++) v[i][t] = src[t * m];
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
    const int b = tid + i * kMrTH;
    if (b < nb) {
      const int line = b / m, j = b - line * m, k = j % ns;
      cx<T>* dst = buf + line * ls + (j - k) * R + k;
#pragma unroll
      for (int t = 0; t < R; t++) dst[t * ns] = v[i][t];
    }
  }
  __syncthreads();
}

// Forward transform of nl lines in LDS, natural order in and out.
template <typename T>
__device__ void mr_fft(cx<T>* buf, int nl, const MrPlan& p, int ls, const cx<T>* __restrict__ tw, int tid) {
  int ns = 1;
  for (int s = 0; s < p.nst; s++) {
    const int r = p.radix[s];
    switch (r) {
      case 2: mr_stage<T, 2>(buf, nl, p.n, ls, ns, tw, tid); break;
      case 3: mr_stage<T, 3>(buf, nl, p.n, ls, ns, tw, tid); break;
      case 4: mr_stage<T, 4>(buf, nl, p.n, ls, ns, tw, tid); break;
      case 5: mr_stage<T, 5>(buf, nl, p.n, ls, ns, tw, tid); break;
      case 7: mr_stage<T, 7>(buf, nl, p.n, ls, ns, tw, tid); break;
      default: mr_stage<T, 8>(buf, nl, p.n, ls, ns, tw, tid); break;
    }
    ns *= r;
  }
}

// signed frequency index: a for 2a < n, a - n otherwise
__device__ __forceinline__ int mr_sidx(int a, int n) { return 2 * a < n ? a : a - n; }

// The real symbol of a one-field solve at signed indices (a', b'), 1/(nx ny)
// included; arguments and the transcendental in FP64, rounded once.
//   Poisson   -1/|k|^2, 0 at k = 0 (Eq. (SolutionPoisson), mean dropped)
//   diffusion exp(-kappa |k|^2 t) (Eq. (solCalorFourier))
//   wave      cos(c |k| t), zero initial velocity (Eq. (OmegaNonZero))
template <typename T>
__device__ __forceinline__ T mr_symbol(const MrSym& s, int ai, int bi) {
  switch (s.op) {
    case kSymPoisson: {
      if (ai == 0 && bi == 0) return T(0);
      const double kx = s.kxs * ai, ky = s.kys * bi;
      return T(-s.scale / fma(kx, kx, ky * ky));
    }
    case kSymDiffusion: {
      const double kx = s.kxs * ai, ky = s.kys * bi;
      return T(s.scale * exp(-s.kt * fma(kx, kx, ky * ky)));
    }
    case kSymWave: {
      const double hx = s.hx * ai, hy = s.hy * bi;
      return T(s.scale * cospi(sqrt(fma(hx, hx, hy * hy))));
    }
    default: return T(s.scale);
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

template <typename T, int NF>
__global__ void __launch_bounds__(kMrTH) mr_kernel(MrArgs<T> a) {
  __shared__ cx<T> lds[NF * kMrLds];
  const int tid = threadIdx.x;
  const int n = a.plan.n;
  const bool col = a.mode >= kMrColFwd;
  // this tile: nl lines; rows start at element `base`, columns at c0 of field f
  long long base = 0;
  int nl, c0 = 0;
  if (!col) {
    const long long nrows = (long long)a.ny * a.fields;
    const long long row0 = (long long)blockIdx.x * a.lines;
    nl = (int)min((long long)a.lines, nrows - row0);
    base = row0 * n;
  } else {
    const int tpf = (a.nx + a.lines - 1) / a.lines;
    const long long f = blockIdx.x / tpf;
    c0 = (int)(blockIdx.x - f * tpf) * a.lines;
    nl = min(a.lines, a.nx - c0);
    base = f * (long long)a.nx * a.ny + c0;
  }
  const int cnt = nl * n;
  // element idx of the tile: its line, position, global offset; columns walk
  // the tile's columns fastest so that a wavefront reads whole row segments
  auto where = [&](int idx, int& line, int& j) -> long long {
    if (!col) {
      line = idx / n;
      j = idx - line * n;
      return base + idx;
    }
    j = idx / nl;
    line = idx - j * nl;
    return base + (long long)j * a.nx + line;
  };
  const bool conj_in = a.mode == kMrRowInv || a.mode == kMrColInv;
  const bool has2 = NF == 2 && a.in1 != nullptr;
#pragma unroll
  for (int fi = 0; fi < NF; fi++) {
    const cx<T>* in = fi == 0 ? a.in0 : a.in1;
    if (fi == 1 && !has2) continue;
    cx<T>* buf = lds + fi * kMrLds;
    for (int idx = tid; idx < cnt; idx += kMrTH) {
      int line, j;
      const long long g = where(idx, line, j);
      cx<T> v = in[g];
      if (conj_in) v.im = -v.im;
      buf[line * a.ls + j] = v;
    }
  }
  __syncthreads();
  mr_fft(lds, nl, a.plan, a.ls, a.tw, tid);
  if (has2) mr_fft(lds + kMrLds, nl, a.plan, a.ls, a.tw, tid);
  const bool out2 = NF == 2 && a.out1 != nullptr;
  if (a.mode == kMrColSolve) {
    // the symbol, then the inverse through the conjugation identity of the
    // iDFT (Sec. II.B): the values are conjugated here and on the way out
    for (int idx = tid; idx < cnt; idx += kMrTH) {
      const int line = idx / n, j = idx - line * n;
      const int ai = mr_sidx(c0 + line, a.nx), bi = mr_sidx(j, a.ny);
      cx<T>* p0 = lds + line * a.ls + j;
      if constexpr (NF == 1) {
        const T m = mr_symbol<T>(a.sym, ai, bi);
        *p0 = {p0->re * m, -p0->im * m};
      } else {
        const MrWave w(a.sym, ai, bi);
        cx<T>* p1 = p0 + kMrLds;
        const cx<T> F = *p0;
        const cx<T> G = has2 ? *p1 : cx<T>{T(0), T(0)};
        const T cw = T(w.cw), sow = T(w.sow), wsw = T(w.wsw);
        *p0 = {cw * F.re + sow * G.re, -(cw * F.im + sow * G.im)};
        if (out2) *p1 = {cw * G.re - wsw * F.re, -(cw * G.im - wsw * F.im)};
      }
    }
    __syncthreads();
    mr_fft(lds, nl, a.plan, a.ls, a.tw, tid);
    if (out2) mr_fft(lds + kMrLds, nl, a.plan, a.ls, a.tw, tid);
  }
  const bool conj_out = a.mode == kMrRowInv || a.mode == kMrColInv || a.mode == kMrColSolve;
  const T sc = a.mode == kMrRowInv ? a.scale : T(1);
#pragma unroll
  for (int fi = 0; fi < NF; fi++) {
    cx<T>* out = fi == 0 ? a.out0 : a.out1;
    if (fi == 1 && !out2) continue;
    const cx<T>* buf = lds + fi * kMrLds;
    for (int idx = tid; idx < cnt; idx += kMrTH) {
      int line, j;
      const long long g = where(idx, line, j);
      const cx<T> v = buf[line * a.ls + j];
      out[g] = conj_out ? cx<T>{v.re * sc, -v.im * sc} : v;
    }
  }
}

}  // namespace

template <typename T>
long long mr_tiles(const MrArgs<T>& a) {
  if (a.mode >= kMrColFwd) return a.fields * (long long)((a.nx + a.lines - 1) / a.lines);
  const long long nrows = (long long)a.ny * a.fields;
  return (nrows + a.lines - 1) / a.lines;
}

template <typename T>
hipError_t mr_launch(const MrArgs<T>& a, int nf, hipStream_t s) {
  const long long tiles = mr_tiles(a);
  if (tiles < 1 || tiles > 0x7fffffffll) return hipErrorInvalidValue;
  if (nf == 2) hipLaunchKernelGGL((mr_kernel<T, 2>), dim3((unsigned)tiles), dim3(kMrTH), 0, s, a);
  else hipLaunchKernelGGL((mr_kernel<T, 1>), dim3((unsigned)tiles), dim3(kMrTH), 0, s, a);
  return hipGetLastError();
}

template long long mr_tiles<float>(const MrArgs<float>&);
template long long mr_tiles<double>(const MrArgs<double>&);
template hipError_t mr_launch<float>(const MrArgs<float>&, int, hipStream_t);
template hipError_t mr_launch<double>(const MrArgs<double>&, int, hipStream_t);

}  // namespace fftpde
