// rk4.hip -- the wave equation with a source that depends on time, integrated
// in Fourier space by the classical fourth-order Runge-Kutta method (Sec.
// III.C: the first-order system u^' = v^, v^' = -w^2 u^ + s^(t) of the forced
// oscillators, w = c|k|).  The state spectra (U, V) stay on the device; each
// step samples the source at t + dt/2 and t + dt, transforms it with the
// library's 2D FFT and advances every coefficient in one elementwise kernel
// (the source spectrum at t is the previous step's at t + dt).
#include "rk4.hpp"

#include <cmath>

#include "solve.hpp"

#include "../../include/fftpde.h"

namespace fftpde {
namespace {

// s(t, x, y) = A exp(-d^2/sigma^2) cos(gamma t), d the periodic (minimum-image)
// distance from (x_j, y_k) = (x0 + j lx/nx, y0 + k ly/ny) to the centre
// (cx + r cos(Omega t), cy + r sin(Omega t)); evaluated in FP64.
template <typename T>
__global__ void __launch_bounds__(256) orbit_source_kernel(cx<T>* s, OrbitSource src, double t, int lognx, int logny,
                                                           double x0, double y0, double lx, double ly) {
  const long long n = 1ll << (lognx + logny);
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = int(i & ((1ll << lognx) - 1)), k = int(i >> lognx);
  const double xs = src.cx + src.radius * cos(src.omega * t);
  const double ys = src.cy + src.radius * sin(src.omega * t);
  double dx = x0 + j * (lx / (1 << lognx)) - xs;
  double dy = y0 + k * (ly / (1 << logny)) - ys;
  dx -= lx * rint(dx / lx);
  dy -= ly * rint(dy / ly);
  const double v = src.amplitude * exp(-(dx * dx + dy * dy) / (src.sigma * src.sigma)) * cos(src.gamma * t);
  s[i] = {T(v), T(0)};
}

// One RK4 step of every coefficient of `batch` fields; S1, S2, S3: the source
// spectrum at t, t + dt/2, t + dt (one field, shared by the batch).
template <typename T>
__global__ void __launch_bounds__(256) rk4_step_kernel(cx<T>* U, cx<T>* V, const cx<T>* S1, const cx<T>* S2,
                                                       const cx<T>* S3, long long batch, int lognx, int logny,
                                                       double kxs, double kys, double c, double dt) {
  const long long pts = 1ll << (lognx + logny);
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= pts * batch) return;
  const long long p = i & (pts - 1);
  const int a = int(p & ((1ll << lognx) - 1)), b = int(p >> lognx);
  const int ai = a < (1 << (lognx - 1)) ? a : a - (1 << lognx);
  const int bi = b < (1 << (logny - 1)) ? b : b - (1 << logny);
  const double kx = kxs * ai, ky = kys * bi;
  const T w2 = T(c * c * (kx * kx + ky * ky));
  const T h = T(0.5 * dt), d = T(dt), d6 = T(dt / 6.0);
  const cx<T> u = U[i], v = V[i], s1 = S1[p], s2 = S2[p], s3 = S3[p];
  // k_j = (ku_j, kv_j) = (v_j, -w^2 u_j + s(t_j)) at the stage points
  const cx<T> ku1 = v;
  const cx<T> kv1 = {-w2 * u.re + s1.re, -w2 * u.im + s1.im};
  const cx<T> u2 = {u.re + h * ku1.re, u.im + h * ku1.im}, v2 = {v.re + h * kv1.re, v.im + h * kv1.im};
  const cx<T> ku2 = v2;
  const cx<T> kv2 = {-w2 * u2.re + s2.re, -w2 * u2.im + s2.im};
  const cx<T> u3 = {u.re + h * ku2.re, u.im + h * ku2.im}, v3 = {v.re + h * kv2.re, v.im + h * kv2.im};
  const cx<T> ku3 = v3;
  const cx<T> kv3 = {-w2 * u3.re + s2.re, -w2 * u3.im + s2.im};
  const cx<T> u4 = {u.re + d * ku3.re, u.im + d * ku3.im}, v4 = {v.re + d * kv3.re, v.im + d * kv3.im};
  const cx<T> ku4 = v4;
  const cx<T> kv4 = {-w2 * u4.re + s3.re, -w2 * u4.im + s3.im};
  U[i] = {u.re + d6 * (ku1.re + T(2) * ku2.re + T(2) * ku3.re + ku4.re),
          u.im + d6 * (ku1.im + T(2) * ku2.im + T(2) * ku3.im + ku4.im)};
  V[i] = {v.re + d6 * (kv1.re + T(2) * kv2.re + T(2) * kv3.re + kv4.re),
          v.im + d6 * (kv1.im + T(2) * kv2.im + T(2) * kv3.im + kv4.im)};
}

__global__ void __launch_bounds__(256) zero_kernel(double* p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

int ilog2i(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}

template <typename T>
int rk4(Context* c, const OrbitSource& src, const void* f, const void* g, void* u, void* v, int nx, int ny,
        int batch, double x0, double y0, double lx, double ly, double cs, double t0, double dt, int steps,
        hipStream_t s) {
  const int dtype = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lgx = ilog2i(nx), lgy = ilog2i(ny);
  const long long pts = (long long)nx * ny;
  const size_t field = sizeof(cx<T>) * (size_t)pts;
  void* w = nullptr;
  int rc = c->workspace(field * (size_t)(2 * batch + 3), s, &w);
  if (rc != FFTPDE_OK) return rc;
  cx<T>* U = static_cast<cx<T>*>(w);
  cx<T>* V = U + pts * batch;
  cx<T>* S[3] = {V + pts * batch, V + pts * batch + pts, V + pts * batch + 2 * pts};
  const double kxs = 2.0 * 3.14159265358979323846264338327950288 / lx;
  const double kys = 2.0 * 3.14159265358979323846264338327950288 / ly;
  const unsigned gsrc = unsigned((pts + 255) / 256), gall = unsigned((pts * batch + 255) / 256);
  auto check = [&](const char* what, hipError_t e) {
    if (e != hipSuccess) {
      set_last_error(what, e);
      return FFTPDE_EDEVICE;
    }
    return FFTPDE_OK;
  };
  // the source spectrum at time tt into S[k]
  auto source = [&](int k, double tt) {
    hipLaunchKernelGGL(orbit_source_kernel<T>, dim3(gsrc), dim3(256), 0, s, S[k], src, tt, lgx, lgy, x0, y0, lx, ly);
    int r = check("orbit_source_kernel", hipGetLastError());
    if (r == FFTPDE_OK) r = run_transform(c, dtype, false, S[k], S[k], nx, ny, 1, s);
    return r;
  };
  rc = run_transform(c, dtype, false, f, U, nx, ny, batch, s);
  if (rc == FFTPDE_OK) {
    if (g) {
      rc = run_transform(c, dtype, false, g, V, nx, ny, batch, s);
    } else {
      // V = 0 with a kernel (no memset node if the caller captures the stream)
      const long long ndbl = (long long)(field * batch / sizeof(double));
      hipLaunchKernelGGL(zero_kernel, dim3(unsigned((ndbl + 255) / 256)), dim3(256), 0, s,
                         reinterpret_cast<double*>(V), ndbl);
      rc = check("zero_kernel", hipGetLastError());
    }
  }
  if (rc == FFTPDE_OK && steps > 0) rc = source(0, t0);
  int cur = 0;  // S[cur]: the source spectrum at the step's start time
  for (int n = 0; n < steps && rc == FFTPDE_OK; n++) {
    const double t = t0 + n * dt;
    const int mid = (cur + 1) % 3, end = (cur + 2) % 3;
    rc = source(mid, t + 0.5 * dt);
    if (rc == FFTPDE_OK) rc = source(end, t + dt);
    if (rc == FFTPDE_OK) {
      hipLaunchKernelGGL(rk4_step_kernel<T>, dim3(gall), dim3(256), 0, s, U, V, S[cur], S[mid], S[end],
                         (long long)batch, lgx, lgy, kxs, kys, cs, dt);
      rc = check("rk4_step_kernel", hipGetLastError());
    }
    cur = end;
  }
  if (rc == FFTPDE_OK) rc = run_transform(c, dtype, true, U, u, nx, ny, batch, s);
  if (rc == FFTPDE_OK && v) rc = run_transform(c, dtype, true, V, v, nx, ny, batch, s);
  return rc;
}

}  // namespace

int run_wave_rk4(Context* c, int dtype, const OrbitSource& src, const void* f, const void* g, void* u, void* v,
                 int nx, int ny, int batch, double x0, double y0, double lx, double ly, double cs, double t0,
                 double dt, int steps, hipStream_t s) {
  return dtype == FFTPDE_C64 ? rk4<float>(c, src, f, g, u, v, nx, ny, batch, x0, y0, lx, ly, cs, t0, dt, steps, s)
                             : rk4<double>(c, src, f, g, u, v, nx, ny, batch, x0, y0, lx, ly, cs, t0, dt, steps, s);
}

}  // namespace fftpde
