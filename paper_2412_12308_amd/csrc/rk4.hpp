// rk4.hpp -- the wave equation with an orbiting source, RK4 in Fourier space
// (see rk4.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "context.hpp"

namespace fftpde {

// The orbiting Gaussian source of Sec. III.C (fields as fftpde_orbit_source).
struct OrbitSource {
  double amplitude, sigma, radius, omega, gamma, cx, cy;
};

// (u, u_t) at t0 + steps dt from u(t0) = f, u_t(t0) = g (null: 0), complex
// dtypes; v may be null.  Arguments are assumed valid (checked at the ABI).
int run_wave_rk4(Context* c, int dtype, const OrbitSource& src, const void* f, const void* g, void* u, void* v,
                 int nx, int ny, int batch, double x0, double y0, double lx, double ly, double cs, double t0,
                 double dt, int steps, hipStream_t s);

}  // namespace fftpde
