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

constexpr int kDiagThreads = 256;

__device__ __forceinline__ int sidx(int a, int logn) { return a < (1 << (logn - 1)) ? a : a - (1 << logn); }

// per-field partial sums: block (bx, field) writes one double per time
template <typename T, int NT>
__global__ void __launch_bounds__(kDiagThreads) diag_partial(DiagArgs<T> a, double* partial) {
  const int field = blockIdx.y;
  const long long P = 1ll << (a.lognx + a.logny);
  const cx<T>* F = a.F + field * P;
  const cx<T>* G = a.G ? a.G + field * P : nullptr;
  double acc[NT];
#pragma unroll
  for (int j = 0; j < NT; j++) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)kDiagThreads + threadIdx.x; i < P; i += (long long)gridDim.x * kDiagThreads) {
    const int ai = sidx(int(i & ((1ll << a.lognx) - 1)), a.lognx);
    const int bi = sidx(int(i >> a.lognx), a.logny);
    const double kx = a.kxs * ai, ky = a.kys * bi;
    const double k2 = kx * kx + ky * ky;
    const double fr = double(F[i].re), fi = double(F[i].im);
    const double gr = G ? double(G[i].re) : 0.0, gi = G ? double(G[i].im) : 0.0;
    const double w = a.coef * sqrt(k2);
#pragma unroll
    for (int j = 0; j < NT; j++) {
      if (j < a.nt) {
        const double t = double(a.n0 + j) * a.dt;
        if (a.kind == 0) {
          acc[j] += (fr * fr + fi * fi) * exp(-2.0 * a.coef * k2 * t);
        } else {
          double s, c;
          sincos(w * t, &s, &c);
          double ur, ui, vr, vi;
          if (w == 0.0) {
            ur = fr + gr * t;
            ui = fi + gi * t;
            vr = gr;
            vi = gi;
          } else {
            ur = fr * c + gr * s / w;
            ui = fi * c + gi * s / w;
            vr = -w * fr * s + gr * c;
            vi = -w * fi * s + gi * c;
          }
          acc[j] += vr * vr + vi * vi + w * w * (ur * ur + ui * ui);
        }
      }
    }
  }
  __shared__ double sh[kDiagThreads];
  for (int j = 0; j < a.nt && j < NT; j++) {
    sh[threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(field * a.nt + j) * gridDim.x + blockIdx.x] = sh[0];
    __syncthreads();
  }
}

// one thread per (field, time): ordered sum of the partials, mean from the
// k = 0 mode
template <typename T>
__global__ void diag_final(DiagArgs<T> a, const double* partial, int nblocks, int batch, double* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= batch * a.nt) return;
  const int field = idx / a.nt, j = idx % a.nt;
  const double t = double(a.n0 + j) * a.dt;
  double e = 0.0;
  for (int b = 0; b < nblocks; b++) e += partial[(field * a.nt + j) * nblocks + b];
  const long long P = 1ll << (a.lognx + a.logny);
  const cx<T> F0 = a.F[field * P];
  double mr = double(F0.re), mi = double(F0.im);
  if (a.kind == 1 && a.G) {
    const cx<T> G0 = a.G[field * P];
    mr += double(G0.re) * t;
    mi += double(G0.im) * t;
  }
  const double scale = a.dxdy / double(P);
  double* o = out + 3 * ((long long)j * batch + field);
  o[0] = mr / double(P);
  o[1] = mi / double(P);
  o[2] = (a.kind == 0 ? 1.0 : 0.5) * scale * e;
}

int diag_blocks(long long P) {
  long long b = (P + kDiagThreads * 8 - 1) / (kDiagThreads * 8);
  return int(b < 1 ? 1 : (b > 256 ? 256 : b));
}

}  // namespace

size_t diag_scratch_doubles(int lognx, int logny, int batch) {
  return size_t(diag_blocks(1ll << (lognx + logny))) * batch * kDiagMaxTimes;
}

template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, int batch, double* scratch, double* out, hipStream_t s) {
  if (a.nt < 1 || a.nt > kDiagMaxTimes) return hipErrorInvalidValue;
  const int nb = diag_blocks(1ll << (a.lognx + a.logny));
  if (a.nt == 1) hipLaunchKernelGGL((diag_partial<T, 1>), dim3(nb, batch), dim3(kDiagThreads), 0, s, a, scratch);
  else hipLaunchKernelGGL((diag_partial<T, kDiagMaxTimes>), dim3(nb, batch), dim3(kDiagThreads), 0, s, a, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = batch * a.nt;
  hipLaunchKernelGGL(diag_final<T>, dim3((n + 63) / 64), dim3(64), 0, s, a, scratch, nb, batch, out);
  return hipGetLastError();
}

template hipError_t launch_diag<float>(const DiagArgs<float>&, int, double*, double*, hipStream_t);
template hipError_t launch_diag<double>(const DiagArgs<double>&, int, double*, double*, hipStream_t);

}  // namespace fftpde
