// evolve.cpp -- time evolution with resident spectra (diffusion and wave).
//
// The spectral solutions are exact in time (Eq. (solCalorFourier);
// Eq. (OmegaNonZero), (OmegaZero) with s = 0), so step n is the closed form
// at the absolute time t_n = n * dt, formed as one FP64 product: no error
// accumulates over steps.  The forward spectra of u0 (and v0) are computed
// once and kept on the device; a step that writes u(t_n) runs the inverse
// column pass with the propagator applied on load (one read of each resident
// spectrum) and the inverse row pass; a diagnostics-only step reads the
// spectra once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "../../include/fftpde.h"
#include "context.hpp"
#include "diag.hpp"
#include "solve.hpp"

using namespace fftpde;

struct fftpde_evolve {
  Context* ctx = nullptr;
  int kind = 0;  // FFTPDE_DIFFUSION or FFTPDE_WAVE
  int dtype = 0;
  int nx = 0, ny = 0, batch = 0;
  double lx = 0, ly = 0, coef = 0;
  void* F = nullptr;
  void* G = nullptr;
  double* scratch = nullptr;
};

namespace {

int ilog2e(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}
bool pow2_side_e(int n) { return n >= 2 && n <= 4096 && (n & (n - 1)) == 0; }

void release(fftpde_evolve* e) {
  if (!e) return;
  if (e->F) (void)hipFree(e->F);
  if (e->G) (void)hipFree(e->G);
  if (e->scratch) (void)hipFree(e->scratch);
  delete e;
}

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int step_impl(fftpde_evolve* e, long long n, double dt, void* u, void* v, double* diag, hipStream_t s) {
  int rc = FFTPDE_OK;
  if (u)
    rc = run_materialize(e->ctx, e->dtype, e->kind, e->F, e->G, u, v, e->nx, e->ny, e->batch, e->lx, e->ly, e->coef,
                         (double)n * dt, s);
  if (rc == FFTPDE_OK && diag)
    rc = run_diag(e->ctx, e->dtype, e->kind, e->F, e->G, e->nx, e->ny, e->batch, e->lx, e->ly, e->coef, n, dt, 1,
                  e->scratch, diag, s);
  return rc;
}

}  // namespace

extern "C" {

int fftpde_evolve_create(fftpde_ctx* ctx, int kind, const void* u0, const void* v0, int nx, int ny, int batch,
                         double lx, double ly, double coef, int dtype, fftpde_stream stream, fftpde_evolve** out) {
  if (!out) return FFTPDE_EINVAL;
  *out = nullptr;
  if (!ctx || !u0 || !pow2_side_e(nx) || !pow2_side_e(ny) || batch < 1) return FFTPDE_EINVAL;
  if (dtype != FFTPDE_C64 && dtype != FFTPDE_C128) return FFTPDE_EINVAL;
  if (kind != FFTPDE_DIFFUSION && kind != FFTPDE_WAVE) return FFTPDE_EINVAL;
  if (kind == FFTPDE_DIFFUSION && v0) return FFTPDE_EINVAL;
  if (!(std::isfinite(lx) && lx > 0 && std::isfinite(ly) && ly > 0 && std::isfinite(coef) && coef >= 0))
    return FFTPDE_EINVAL;
  const uintptr_t al = dtype == FFTPDE_C64 ? 8 : 16;
  if ((reinterpret_cast<uintptr_t>(u0) & (al - 1)) || (v0 && (reinterpret_cast<uintptr_t>(v0) & (al - 1))))
    return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  DevGuard g(c->device);
  fftpde_evolve* e = new (std::nothrow) fftpde_evolve();
  if (!e) return FFTPDE_ENOMEM;
  e->ctx = c;
  e->kind = kind;
  e->dtype = dtype;
  e->nx = nx;
  e->ny = ny;
  e->batch = batch;
  e->lx = lx;
  e->ly = ly;
  e->coef = coef;
  const size_t bytes = (size_t)nx * ny * batch * (dtype == FFTPDE_C64 ? 8 : 16);
  const size_t sbytes = diag_scratch_doubles(ilog2e(nx), ilog2e(ny), batch) * sizeof(double);
  if (hipMalloc(&e->F, bytes) != hipSuccess || (v0 && hipMalloc(&e->G, bytes) != hipSuccess) ||
      hipMalloc(reinterpret_cast<void**>(&e->scratch), sbytes) != hipSuccess) {
    release(e);
    return FFTPDE_ENOMEM;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = run_transform(c, dtype, false, u0, e->F, nx, ny, batch, s);
  if (rc == FFTPDE_OK && v0) rc = run_transform(c, dtype, false, v0, e->G, nx, ny, batch, s);
  if (rc != FFTPDE_OK) {
    (void)hipStreamSynchronize(s);
    release(e);
    return rc;
  }
  *out = e;
  return FFTPDE_OK;
}

int fftpde_evolve_step(fftpde_evolve* e, long long n, double dt, void* u, void* v, double* diag,
                       fftpde_stream stream) {
  if (!e) return FFTPDE_EINVAL;
  const double t = (double)n * dt;  // absolute time, one FP64 product
  if (!std::isfinite(dt) || !std::isfinite(t)) return FFTPDE_EINVAL;
  if (e->kind == FFTPDE_DIFFUSION && (t < 0 || v)) return FFTPDE_EINVAL;
  if (v && !u) return FFTPDE_EINVAL;
  const uintptr_t al = e->dtype == FFTPDE_C64 ? 8 : 16;
  if ((u && (reinterpret_cast<uintptr_t>(u) & (al - 1))) || (v && (reinterpret_cast<uintptr_t>(v) & (al - 1))) ||
      (diag && (reinterpret_cast<uintptr_t>(diag) & 7)) || (u && v && u == v))
    return FFTPDE_EINVAL;
  DevGuard g(e->ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return step_impl(e, n, dt, u, v, diag, s);
}

int fftpde_evolve_destroy(fftpde_evolve* e) {
  if (!e) return FFTPDE_OK;
  DevGuard g(e->ctx->device);
  (void)hipDeviceSynchronize();
  release(e);
  return FFTPDE_OK;
}

}  // extern "C"
