// halfspec.hip -- half spectra of real fields from the spectrum of a pair
// and back.
//
// Two real fields x1, x2 transform as one complex field z = x1 + i x2.  With
// Z its 2D spectrum and Zm[b][a] = Z[-b][-a], the transform of real data has
// X[-b][-a] = conj(X[b][a]) (Sec. II.B), so
//   X1 = (Z + conj(Zm)) / 2,   X2 = (Z - conj(Zm)) / (2i).
// Backwards, the Hermitian extension of each half spectrum gives the full
// X1, X2 and Z = X1 + i X2 is transformed back as one complex field whose
// real and imaginary parts are x1 and x2.  Sides may be odd: index -b is
// ny - b for b > 0, and on odd nx no column but a = 0 maps to itself.
#include "halfspec.hpp"

namespace fftpde {
namespace {

constexpr int kHalfTH = 256;

// offset of spectrum element (row b, column c) within one pair's field
template <typename T>
__device__ __forceinline__ long long spec_at(const HalfArgs<T>& a, int b, int c) {
  if (a.t < 0) return (long long)b * a.nx + c;
  return ((long long)(c >> a.t) << (a.logny + a.t)) + ((long long)b << a.t) + (c & ((1 << a.t) - 1));
}

// One block per spectrum row (pair p, row b); threads over the columns.
template <typename T>
__global__ void __launch_bounds__(kHalfTH) untangle_kernel(HalfArgs<T> a) {
  const long long row = blockIdx.x;  // p * ny + b
  const long long p = row / a.ny;
  const int b = (int)(row - p * a.ny);
  const int bm = b == 0 ? 0 : a.ny - b;
  const int h = a.nx / 2 + 1;
  const cx<T>* S = a.spec + p * (long long)a.nx * a.ny;
  const bool second = 2 * p + 1 < a.nreal;
  cx<T>* o1 = a.half + (2 * p * (long long)a.ny + b) * h;
  cx<T>* o2 = o1 + (long long)a.ny * h;
  for (int c = threadIdx.x; c < h; c += kHalfTH) {
    const int cm = c == 0 ? 0 : a.nx - c;
    const cx<T> z = S[spec_at(a, b, c)];
    const cx<T> zm = S[spec_at(a, bm, cm)];
    o1[c] = {T(0.5) * (z.re + zm.re), T(0.5) * (z.im - zm.im)};
    if (second) o2[c] = {T(0.5) * (z.im + zm.im), T(0.5) * (zm.re - z.re)};
  }
}

// The Hermitian extension of half spectrum X at (b, a): columns 0 < a < nx/2
// as given, a > nx/2 from conj(X[-b][nx - a]), and the self-conjugate columns
// (a = 0, and a = nx/2 on even nx) projected to (X[b][a] + conj(X[-b][a])) / 2.
template <typename T>
__device__ __forceinline__ cx<T> hermitian_at(const cx<T>* X, int h, int nx, int b, int bm, int c) {
  if (c == 0 || 2 * c == nx) {
    const cx<T> v = X[(long long)b * h + c], w = X[(long long)bm * h + c];
    return {T(0.5) * (v.re + w.re), T(0.5) * (v.im - w.im)};
  }
  if (2 * c < nx) return X[(long long)b * h + c];
  const cx<T> v = X[(long long)bm * h + (nx - c)];
  return {v.re, -v.im};
}

template <typename T>
__global__ void __launch_bounds__(kHalfTH) tangle_kernel(HalfArgs<T> a) {
  const long long row = blockIdx.x;
  const long long p = row / a.ny;
  const int b = (int)(row - p * a.ny);
  const int bm = b == 0 ? 0 : a.ny - b;
  const int h = a.nx / 2 + 1;
  cx<T>* S = a.spec + p * (long long)a.nx * a.ny;
  const cx<T>* X1 = a.half + 2 * p * (long long)a.ny * h;
  const cx<T>* X2 = X1 + (long long)a.ny * h;
  const bool second = 2 * p + 1 < a.nreal;
  for (int c = threadIdx.x; c < a.nx; c += kHalfTH) {
    const cx<T> u = hermitian_at(X1, h, a.nx, b, bm, c);
    const cx<T> v = second ? hermitian_at(X2, h, a.nx, b, bm, c) : cx<T>{T(0), T(0)};
    S[spec_at(a, b, c)] = {u.re - v.im, u.im + v.re};  // X1 + i X2
  }
}

}  // namespace

template <typename T>
hipError_t launch_untangle(const HalfArgs<T>& a, hipStream_t s) {
  const long long rows = a.npairs * a.ny;
  if (rows < 1 || rows > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(untangle_kernel<T>, dim3((unsigned)rows), dim3(kHalfTH), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tangle(const HalfArgs<T>& a, hipStream_t s) {
  const long long rows = a.npairs * a.ny;
  if (rows < 1 || rows > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tangle_kernel<T>, dim3((unsigned)rows), dim3(kHalfTH), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_untangle<float>(const HalfArgs<float>&, hipStream_t);
template hipError_t launch_untangle<double>(const HalfArgs<double>&, hipStream_t);
template hipError_t launch_tangle<float>(const HalfArgs<float>&, hipStream_t);
template hipError_t launch_tangle<double>(const HalfArgs<double>&, hipStream_t);

}  // namespace fftpde
