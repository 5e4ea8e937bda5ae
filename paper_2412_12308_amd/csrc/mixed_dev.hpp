// mixed_dev.hpp -- device helpers of the mixed-radix passes: odd-radix
// butterflies, signed frequency indices and the solves' symbols.
#pragma once

#include <hip/hip_runtime.h>

#include "mixed.hpp"

namespace fftpde {

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
      if constexpr (sizeof(T) == 4) {
        const float kx = float(s.kxs) * float(ai), ky = float(s.kys) * float(bi);
        return -float(s.scale) * __builtin_amdgcn_rcpf(fmaf(kx, kx, ky * ky));
      } else {
        const double kx = s.kxs * ai, ky = s.kys * bi;
        return -s.scale / fma(kx, kx, ky * ky);
      }
    }
    case kSymDiffusion: {
      const double kx = s.kxs * ai, ky = s.kys * bi;
      const double arg = s.kt * fma(kx, kx, ky * ky);
      if constexpr (sizeof(T) == 4) return float(s.scale) * expf(-float(arg));
      else return s.scale * exp(-arg);
    }
    case kSymWave: {
      const double hx = s.hx * ai, hy = s.hy * bi;
      const double h2 = fma(hx, hx, hy * hy);
      if constexpr (sizeof(T) == 4) {
        // w t / pi, reduced exactly to [-1, 1] in FP64, then cos(pi h) =
        // (-1)^m cos(pi (h - m)) with m = rint(h) and h - m in [-1/2, 1/2]
        double h = sqrt_fp64_from_fp32(h2);
        h = fma(-2.0, rint(0.5 * h), h);
        const double m = rint(h);
        const float c = cospi_half(float(h - m));
        return (m != 0.0 ? -float(s.scale) : float(s.scale)) * c;
      } else {
        return s.scale * cospi(sqrt(h2));
      }
    }
    default: return T(s.scale);
  }
}

}  // namespace fftpde
