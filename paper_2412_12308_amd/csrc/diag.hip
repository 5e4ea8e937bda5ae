// diag.hip -- diagnostics of an evolving solution read straight from its
// resident spectra: the domain mean (the k = 0 coefficient over nx*ny) and
// the energy by Parseval's identity (a consequence of W^-1 = W^dagger / N,
// Sec. II.B), accumulated in FP64 with a fixed reduction order.
//
//   diffusion:  mean = F_0 / P,  energy = integral |u|^2
//                             = (dx dy / P) sum_k |F_k|^2 exp(-2 kappa |k|^2 t)
//   wave:       mean = (F_0 + G_0 t) / P,
//               energy = 1/2 integral (|u_t|^2 + c^2 |grad u|^2)
//                      = (dx dy / (2P)) sum_k (|V_k|^2 + c^2 |k|^2 |U_k|^2),
//               U, V the spectra of u(t), u_t(t) (Sec. III.C closed forms).
#include "diag.hpp"

#include "fft_engine.hpp"

namespace fftpde {
namespace {

constexpr int kDiagThreads = 1024;

__device__ __forceinline__ int sidx(int a, int logn) { return a < (1 << (logn - 1)) ? a : a - (1 << logn); }

// sum over the 64 lanes of a wave, xor butterfly (the same order in every lane)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-block partial sums for nt <= NT times t_j = (n0 + j) dt.  Each
// element's propagator is evaluated directly at t_0 and advanced to t_j by an
// FP64 rotation through w dt (wave) or a product with exp(-2 kappa |k|^2 dt)
// (diffusion): two transcendental evaluations per element per launch, one
// rounding per further time.  partial[(field * nt + j) * nblocks + block].
// A second kernel sums the partials; the kernel boundary makes them visible
// (no fences, no atomics, a fixed order).
template <typename T, int NT>
__global__ void __launch_bounds__(kDiagThreads) diag_partial(DiagArgs<T> a, double* partial) {
  const int field = blockIdx.y;
  const int nb = gridDim.x;
  const long long P = 1ll << (a.lognx + a.logny);
  const cx<T>* F = a.F + field * P;
  const cx<T>* G = a.G ? a.G + field * P : nullptr;
  const int nt = a.nt;
  const double t0 = double(a.n0) * a.dt;
  double acc[NT];
#pragma unroll
  for (int j = 0; j < NT; j++) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)kDiagThreads + threadIdx.x; i < P; i += (long long)nb * kDiagThreads) {
    const int ai = sidx(int(i & ((1ll << a.lognx) - 1)), a.lognx);
    const int bi = sidx(int(i >> a.lognx), a.logny);
    const double kx = a.kxs * ai, ky = a.kys * bi;
    const double k2 = kx * kx + ky * ky;
    const double fr = double(F[i].re), fi = double(F[i].im);
    if (a.kind == 0) {
      const double f2 = fr * fr + fi * fi;
      double e = exp(-2.0 * a.coef * k2 * t0);
      const double ed = NT > 1 ? exp(-2.0 * a.coef * k2 * a.dt) : 1.0;
#pragma unroll
      for (int j = 0; j < NT; j++) {
        if (j < nt) acc[j] += f2 * e;
        e *= ed;
      }
    } else {
      const double w = a.coef * sqrt(k2);
      double s, c, sd = 0.0, cd = 1.0;
      sincos(w * t0, &s, &c);
      if (NT > 1) sincos(w * a.dt, &sd, &cd);
      if (!G) {
        // v0 = 0: U = F cos, V = -w F sin, so |V|^2 + w^2 |U|^2 = w^2 |F|^2 (cos^2 + sin^2)
        const double e = w * w * (fr * fr + fi * fi);
#pragma unroll
        for (int j = 0; j < NT; j++) {
          if (j < nt) acc[j] += e * (c * c + s * s);
          const double c2 = c * cd - s * sd;
          s = s * cd + c * sd;
          c = c2;
        }
      } else if (w == 0.0) {
        // U = F + G t, V = G: the energy density is |G|^2 at every time
        const double gr = double(G[i].re), gi = double(G[i].im);
#pragma unroll
        for (int j = 0; j < NT; j++)
          if (j < nt) acc[j] += gr * gr + gi * gi;
      } else {
        const double gr = double(G[i].re), gi = double(G[i].im);
        const double iw = 1.0 / w;
#pragma unroll
        for (int j = 0; j < NT; j++) {
          if (j < nt) {
            const double ur = fr * c + gr * s * iw, ui = fi * c + gi * s * iw;
            const double vr = -w * fr * s + gr * c, vi = -w * fi * s + gi * c;
            acc[j] += vr * vr + vi * vi + w * w * (ur * ur + ui * ui);
          }
          const double c2 = c * cd - s * sd;
          s = s * cd + c * sd;
          c = c2;
        }
      }
    }
  }
  // Block sums in a fixed order: an xor butterfly within each wave, then the
  // waves' values in wave order.
  constexpr int kWaves = kDiagThreads / 64;
  __shared__ double sh[NT * kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NT; j++) {
    if (j < nt) {
      const double v = wave_sum(acc[j]);
      if (lane == 0) sh[j * kWaves + wave] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nt) {
    double v = 0.0;
    for (int w = 0; w < kWaves; w++) v += sh[threadIdx.x * kWaves + w];
    partial[(field * nt + threadIdx.x) * nb + blockIdx.x] = v;
  }
}

// One block per field: the partials of every time summed in block order
// (thread k takes blocks k, k + kDiagThreads, ...; then the xor butterfly and
// the waves in order), the mean from the k = 0 mode.
template <typename T, int NT>
__global__ void __launch_bounds__(kDiagThreads) diag_final(DiagArgs<T> a, const double* partial, int nb, int batch,
                                                           double* out) {
  constexpr int kWaves = kDiagThreads / 64;
  __shared__ double sh[NT * kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int f = blockIdx.x;
  const int nt = a.nt;
  const long long P = 1ll << (a.lognx + a.logny);
  // all loads first (independent), then the reductions
  double e[NT];
#pragma unroll
  for (int j = 0; j < NT; j++) e[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kDiagThreads) {
#pragma unroll
    for (int j = 0; j < NT; j++)
      if (j < nt) e[j] += partial[(f * nt + j) * nb + b];
  }
#pragma unroll
  for (int j = 0; j < NT; j++) {
    if (j < nt) {
      const double v = wave_sum(e[j]);
      if (lane == 0) sh[j * kWaves + wave] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nt) {
    const int j = threadIdx.x;
    double en = 0.0;
    for (int w = 0; w < kWaves; w++) en += sh[j * kWaves + w];
    const double t = double(a.n0 + j) * a.dt;
    const cx<T> F0 = a.F[f * P];
    double mr = double(F0.re), mi = double(F0.im);
    if (a.kind == 1 && a.G) {
      const cx<T> G0 = a.G[f * P];
      mr += double(G0.re) * t;
      mi += double(G0.im) * t;
    }
    const double scale = a.dxdy / double(P);
    double* o = out + 3 * ((long long)j * batch + f);
    o[0] = mr / double(P);
    o[1] = mi / double(P);
    o[2] = (a.kind == 0 ? 1.0 : 0.5) * scale * en;
  }
}

int diag_blocks(long long P) {
  long long b = (P + kDiagThreads * 4 - 1) / (kDiagThreads * 4);
  return int(b < 1 ? 1 : (b > 256 ? 256 : b));
}

}  // namespace

size_t diag_scratch_doubles(int lognx, int logny, int batch) {
  return size_t(diag_blocks(1ll << (lognx + logny))) * batch * kDiagMaxTimes;
}

template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, int batch, double* scratch, double* out, hipStream_t s) {
  if (a.nt < 1 || a.nt > kDiagMaxTimes || batch < 1 || batch > 65535) return hipErrorInvalidValue;
  const int nb = diag_blocks(1ll << (a.lognx + a.logny));
  if (a.nt == 1) {
    hipLaunchKernelGGL((diag_partial<T, 1>), dim3(nb, batch), dim3(kDiagThreads), 0, s, a, scratch);
    hipLaunchKernelGGL((diag_final<T, 1>), dim3(batch), dim3(kDiagThreads), 0, s, a, scratch, nb, batch, out);
  } else {
    hipLaunchKernelGGL((diag_partial<T, kDiagMaxTimes>), dim3(nb, batch), dim3(kDiagThreads), 0, s, a, scratch);
    hipLaunchKernelGGL((diag_final<T, kDiagMaxTimes>), dim3(batch), dim3(kDiagThreads), 0, s, a, scratch, nb, batch,
                       out);
  }
  return hipGetLastError();
}

template hipError_t launch_diag<float>(const DiagArgs<float>&, int, double*, double*, hipStream_t);
template hipError_t launch_diag<double>(const DiagArgs<double>&, int, double*, double*, hipStream_t);

}  // namespace fftpde
