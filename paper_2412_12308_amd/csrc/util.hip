// util.hip -- device utilities for the host side (see util.hpp).
#include "util.hpp"

#include "fft_engine.hpp"

namespace fftpde {
namespace {

__device__ __forceinline__ unsigned mix32(unsigned x) {
  // an integer hash (xorshift-multiply rounds)
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <typename T>
__global__ void fill_kernel(cx<T>* p, long long n, unsigned seed) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned h1 = mix32(unsigned(i) * 2u + seed * 0x9e3779b9u);
    const unsigned h2 = mix32(unsigned(i) * 2u + 1u + seed * 0x9e3779b9u);
    p[i] = {T(int(h1 >> 8) - (1 << 23)) / T(1 << 23), T(int(h2 >> 8) - (1 << 23)) / T(1 << 23)};
  }
}

template <typename T>
__global__ void diff_kernel(const cx<T>* a, const cx<T>* b, long long n, double* acc) {
  double d = 0.0, r = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double dr = double(a[i].re) - double(b[i].re), di = double(a[i].im) - double(b[i].im);
    d += dr * dr + di * di;
    r += double(b[i].re) * double(b[i].re) + double(b[i].im) * double(b[i].im);
  }
  __shared__ double sd[256], sr[256];
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sr[threadIdx.x] += sr[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], sd[0]);
    atomicAdd(&acc[1], sr[0]);
  }
}

__global__ void zero_kernel(double* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t fill_pattern(void* p, long long n, int dtype, unsigned seed, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, static_cast<cx<float>*>(p), n, seed);
  else
    hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, static_cast<cx<double>*>(p), n, seed);
  return hipGetLastError();
}

hipError_t diff_norms(const void* a, const void* b, long long n, int dtype, double* acc, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(diff_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, static_cast<const cx<float>*>(a),
                       static_cast<const cx<float>*>(b), n, acc);
  else
    hipLaunchKernelGGL(diff_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, static_cast<const cx<double>*>(a),
                       static_cast<const cx<double>*>(b), n, acc);
  return hipGetLastError();
}

hipError_t zero_doubles(double* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace fftpde
