// solve.hpp -- launch sequences shared by the C ABI, the autotuner, batches
// and the request server.  Arguments are assumed valid (checked at the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "context.hpp"
#include "kernels.hpp"

namespace fftpde {

// Launch through `fn`, bracketed by events when profiling is on.
template <class F>
hipError_t timed_launch(Context* c, const char* name, double bytes, hipStream_t s, F&& fn) {
  if (!c->profiling) return fn();
  hipEvent_t a = c->take_event(), b = c->take_event();
  if (!a || !b) return fn();
  (void)hipEventRecord(a, s);
  hipError_t e = fn();
  (void)hipEventRecord(b, s);
  c->timed.push_back({name, bytes, a, b});
  return e;
}

SymParams make_sym(int op, int nx, int ny, double lx, double ly, double coef, double t);
// SymParams::phase_fast for a wave symbol on an nx x ny grid (3D, p.lx3 > 0:
// x of 2^lx3 points, y of ny3 points along hy3, z of ny points along hy).
void set_phase_range(SymParams& p, int nx, int ny, int ny3);

// One row pass over nrows = batch * 2^logny rows of length 2^lognx (forward,
// or inverse by conjugation with `scale`).  in_t / out_t: log2 of the column
// block width of the input / output layout (see RowArgs), -1 = row-major.
// real_in / real_out: that side holds nreal real fields, read or written in
// pairs (row r of the pass = row r mod ny of fields 2p, 2p + 1, p = r / ny).
template <typename T>
int row_pass(Context* c, const void* in, void* out, int lognx, int logny, long long nrows, bool inverse,
             double scale, hipStream_t s, int in_t = -1, int out_t = -1, int real_in = 0, int real_out = 0,
             long long nreal = 0);

// One column pass over `batch` fields of 2^lognx columns of length 2^logny;
// layout_t >= 0: the fields are stored in blocks of 2^layout_t columns
// (at least the variant's tile width), -1: row-major.
template <typename T>
int col_pass(Context* c, const void* in0, const void* in1, void* out0, void* out1, int lognx, int logny,
             long long batch, int mode, const SymParams& sym, int nf, hipStream_t s, int layout_t = -1);

// fft2d_forward / fft2d_inverse.
int run_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                  hipStream_t s);

// fft2d_r2c (inverse = false: real fields -> half spectra [ny][nx/2 + 1]) and
// fft2d_c2r (inverse = true, scaled by 1/(nx ny)); dtype FFTPDE_R32 / R64.
int run_half_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                       hipStream_t s);

// Device memory a caller lends to a solve for the spectrum between its
// passes; p = null: the context's per-stream workspace (grown on demand).
struct SolveScratch {
  void* p = nullptr;
  size_t bytes = 0;
};

// A solve (op = FFTPDE_POISSON / DIFFUSION / WAVE; for the wave, in2 is the
// initial velocity and out2 the velocity output, either may be null).  With
// sc.p set, complex power-of-two solves keep their spectra in sc (batches
// run in chunks of as many fields as it holds; EINVAL if not one) and never
// allocate; other paths ignore it.
int run_solve(Context* c, int dtype, int op, const void* in, const void* in2, void* out, void* out2, int nx, int ny,
              int batch, double lx, double ly, double coef, double t, hipStream_t s, const SolveScratch& sc = SolveScratch());
// Scratch bytes per field of a chunk that run_solve needs for a complex
// power-of-two solve (v0 / v: the wave's velocity input / output given); 0
// when the spectrum stays in the output or the solve runs in one launch.
size_t solve_scratch_per_field(Context* c, int dtype, int op, int nx, int ny, bool v0, bool v);

// 3D fields [nz][ny][nx]: transforms and the three solves (no velocity).
int run_transform3d(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int nz, int batch,
                    hipStream_t s);
int run_solve3d(Context* c, int dtype, int op, const void* in, void* out, int nx, int ny, int nz, int batch, double lx,
                double ly, double lz, double coef, double t, hipStream_t s);

// A solve with a source constant in time (op = FFTPDE_DIFFUSION: f, src ->
// u; FFTPDE_WAVE: f, g (may be null), src -> u, v (may be null)); coef is
// kappa or the wave speed.  Complex dtypes, or real ones in pairs.
int run_source(Context* c, int dtype, int op, const void* f, const void* g, const void* src, void* u, void* v, int nx,
               int ny, int batch, double lx, double ly, double coef, double t, hipStream_t s);

// u(t) (and u_t(t)) of an evolving field from its resident spectra F (and G):
// the inverse column pass with the propagator at time t applied on load, then
// the inverse row pass (kind = FFTPDE_DIFFUSION or FFTPDE_WAVE).
int run_materialize(Context* c, int dtype, int kind, const void* F, const void* G, void* u, void* v, int nx, int ny,
                    int batch, double lx, double ly, double coef, double t, hipStream_t s);

// Mean and energy at t_j = (n0 + j) dt, j < nt <= 16, from the spectra (one
// read); out[3 (j batch + f) + {0, 1, 2}].  scratch: diag_scratch_doubles.
int run_diag(Context* c, int dtype, int kind, const void* F, const void* G, int nx, int ny, int batch, double lx,
             double ly, double coef, long long n0, double dt, int nt, double* scratch, double* out, hipStream_t s);

// Sides of the mixed-radix path: 7-smooth, 2..4096.  Transforms and the
// three solves (the wave with or without velocity) on complex fields whose
// sides are not both powers of two.
bool mixed_side(int n);
int run_mixed_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                        hipStream_t s);
int run_mixed_solve(Context* c, int dtype, int op, const void* in, const void* in2, void* out, void* out2, int nx,
                    int ny, int batch, double lx, double ly, double coef, double t, hipStream_t s);
// half spectra of real fields (R32 / R64) on 7-smooth sides
int run_mixed_half(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                   hipStream_t s);

}  // namespace fftpde
