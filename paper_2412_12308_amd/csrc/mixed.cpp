// mixed.cpp -- host side of the mixed-radix path: per-length twiddle tables
// (cached in the context), tile shapes, and the pass sequences of the
// transforms and solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/fftpde.h"
#include "halfspec.hpp"
#include "mixed.hpp"
#include "rpass.hpp"
#include "solve.hpp"

namespace fftpde {
namespace {

constexpr double kPiM = 3.14159265358979323846264338327950288;

// cos and sin of 2 pi e / n, 0 <= e < n: theta = (q + r/n) pi/2 with
// quadrant q = floor(4e/n) and r = 4e - q n in integers; libm on angles in
// [0, pi/4] only, so the quarter and half turns come out exact.
void cos_sin_frac(long long e, long long n, double& c, double& s) {
  const long long q = (4 * e) / n, r = 4 * e - q * n;
  double c0, s0;
  if (2 * r <= n) {
    const double a = 0.5 * kPiM * (double)r / (double)n;
    c0 = std::cos(a);
    s0 = std::sin(a);
  } else {  // phi = pi/2 - phi'
    const double a = 0.5 * kPiM * (double)(n - r) / (double)n;
    c0 = std::sin(a);
    s0 = std::cos(a);
  }
  switch (q & 3) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
  }
}

// exp(-2 pi i e / n) for e < n: FP64 entries, and the same rounded once to FP32.
template <typename T>
const cx<T>* mr_table(Context* c, int n) {
  auto it = c->mr_tw.find(n);
  if (it == c->mr_tw.end()) {
    std::vector<cx<double>> t64(n);
    std::vector<cx<float>> t32(n);
    for (int e = 0; e < n; e++) {
      double cs, sn;
      cos_sin_frac(e, n, cs, sn);
      t64[e] = {cs, -sn};
      t32[e] = {(float)cs, (float)-sn};
    }
    void* p = nullptr;
    const size_t b64 = sizeof(cx<double>) * (size_t)n, b32 = sizeof(cx<float>) * (size_t)n;
    hipError_t e = hipMalloc(&p, b64 + b32);
    if (e == hipSuccess) e = hipMemcpy(p, t64.data(), b64, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(static_cast<char*>(p) + b64, t32.data(), b32, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_last_error("mixed-radix twiddle table", e);
      if (p) (void)hipFree(p);
      return nullptr;
    }
    it = c->mr_tw.emplace(n, Context::MrTables{static_cast<cx<double>*>(p),
                                               reinterpret_cast<cx<float>*>(static_cast<char*>(p) + b64)})
             .first;
  }
  if constexpr (sizeof(T) == 4) return it->second.f32;
  else return it->second.f64;
}

// Real fields in pairs: rin (forward rows) or rout (inverse rows) with nreal
// real fields; `fields` then counts pair fields.
template <typename T>
int mr_pass(Context* c, int mode, int nf, const void* in0, const void* in1, void* out0, void* out1, int nx, int ny,
            long long fields, double scale, const MrSym& sym, hipStream_t s, const void* rin = nullptr,
            void* rout = nullptr, long long nreal = 0) {
  const bool col = mode >= kMrColFwd;
  const int n = col ? ny : nx;
  const char* name = col ? (sizeof(T) == 4 ? "mixed_col_float" : "mixed_col_double")
                         : (sizeof(T) == 4 ? "mixed_row_float" : "mixed_row_double");
  if (nf == 1 && !rin && !rout && !in1 && !out1 && rp_pass_ok(mode, n, sizeof(T) == 8)) {
    // n = R 2^m: the radix-R step around the power-of-two register engine
    int r = 0, lp = 0;
    rp_split(n, col, sizeof(T) == 8, &r, &lp);
    RpArgs<T> p{};
    p.in = static_cast<const cx<T>*>(in0);
    p.out = static_cast<cx<T>*>(out0);
    p.twn = mr_table<T>(c, n);
    if (!p.twn) return FFTPDE_EDEVICE;
    if constexpr (sizeof(T) == 4) p.tw = c->tw32;
    else p.tw = c->tw64;
    const int mlr = col ? rp_col_maxlr(sizeof(T) == 8, r, mode == kMrColSolve) : 3;
    p.stwf = c->stage_tw<T>(lp, mlr, false);
    p.stwr = c->stage_tw<T>(lp, mlr, true);
    p.nx = nx;
    p.ny = ny;
    p.fields = fields;
    p.mode = mode;
    p.scale = T(scale);
    p.sym = sym;
    const double bytes = 2.0 * sizeof(cx<T>) * (double)nx * ny * (double)fields;
    const hipError_t e = timed_launch(c, name, bytes, s, [&] { return rp_launch<T>(p, s); });
    if (e != hipSuccess) {
      set_last_error(name, e);
      return FFTPDE_EDEVICE;
    }
    return FFTPDE_OK;
  }
  MrArgs<T> a{};
  a.plan = mr_plan(n);
  if (a.plan.nst == 0) return FFTPDE_EINVAL;
  a.tw = mr_table<T>(c, n);
  if (!a.tw) return FFTPDE_EDEVICE;
  a.in0 = static_cast<const cx<T>*>(in0);
  a.in1 = static_cast<const cx<T>*>(in1);
  a.out0 = static_cast<cx<T>*>(out0);
  a.out1 = static_cast<cx<T>*>(out1);
  a.nx = nx;
  a.ny = ny;
  a.fields = fields;
  a.mode = mode;
  a.scale = T(scale);
  a.sym = sym;
  a.rin = static_cast<const T*>(rin);
  a.rout = static_cast<T*>(rout);
  a.nreal = nreal;
  a.by_ny = MrDiv(ny);
  const bool small = mr_row_small(sizeof(T) == 8, nf, col);
  const int cap = small ? kMrRowCap : mr_cap(sizeof(T) == 8, nf);
  if (col) {
    // adjacent columns, each padded by one in LDS
    a.lines = std::max(1, std::min(kMrMaxColLines, cap / (n + 1)));
    a.lines = std::min(a.lines, nx);
    a.ls = a.lines > 1 ? n + 1 : n;
    a.tiles = fields * (long long)((nx + a.lines - 1) / a.lines);
  } else {
    a.lines = std::max(1, cap / n);
    a.ls = n;
    a.tiles = ((long long)ny * fields + a.lines - 1) / a.lines;
  }
  a.by_lines = MrDiv(a.lines);
  const long long grid = std::min<long long>(a.tiles, (long long)std::max(1, c->num_cus) * mr_occupancy<T>(nf, small));
  const int nin = 1 + (in1 ? 1 : 0), nout = 1 + (out1 ? 1 : 0);
  double bytes = (double)sizeof(cx<T>) * (double)nx * ny * (double)fields * (nin + nout);
  if (rin || rout)  // one real side, one pair-field side
    bytes = (double)nx * ny * ((double)sizeof(T) * (double)nreal + (double)sizeof(cx<T>) * (double)fields);
  const hipError_t e = timed_launch(c, name, bytes, s, [&] { return mr_launch<T>(a, nf, small, (int)grid, s); });
  if (e != hipSuccess) {
    set_last_error(name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

MrSym mr_sym(int op, int nx, int ny, double lx, double ly, double coef, double t) {
  MrSym m;
  m.op = op == FFTPDE_POISSON ? kSymPoisson : op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave;
  m.kxs = 2.0 * kPiM / lx;
  m.kys = 2.0 * kPiM / ly;
  m.scale = 1.0 / ((double)nx * (double)ny);
  if (op == FFTPDE_DIFFUSION) m.kt = coef * t;
  if (op == FFTPDE_WAVE) {
    m.c = coef;
    m.t = t;
    m.hx = 2.0 * coef * t / lx;
    m.hy = 2.0 * coef * t / ly;
  }
  return m;
}

template <typename T>
int transform(Context* c, bool inverse, const void* in, void* out, int nx, int ny, int batch, hipStream_t s) {
  const MrSym none;
  if (!inverse) {
    int rc = mr_pass<T>(c, kMrRowFwd, 1, in, nullptr, out, nullptr, nx, ny, batch, 1.0, none, s);
    if (rc == FFTPDE_OK) rc = mr_pass<T>(c, kMrColFwd, 1, out, nullptr, out, nullptr, nx, ny, batch, 1.0, none, s);
    return rc;
  }
  int rc = mr_pass<T>(c, kMrColInv, 1, in, nullptr, out, nullptr, nx, ny, batch, 1.0, none, s);
  if (rc == FFTPDE_OK)
    rc = mr_pass<T>(c, kMrRowInv, 1, out, nullptr, out, nullptr, nx, ny, batch, 1.0 / ((double)nx * ny), none, s);
  return rc;
}

template <typename T>
int solve(Context* c, int op, const void* in, const void* in2, void* out, void* out2, int nx, int ny, int batch,
          double lx, double ly, double coef, double t, hipStream_t s) {
  const MrSym sym = mr_sym(op, nx, ny, lx, ly, coef, t);
  const MrSym none;
  const bool two = op == FFTPDE_WAVE && (in2 || out2);
  // the velocity's spectrum: in the velocity output, else in the workspace
  void* vb = out2;
  if (two && in2 && !out2) {
    const int rc = c->workspace(sizeof(cx<T>) * (size_t)nx * ny * (size_t)batch, s, &vb);
    if (rc != FFTPDE_OK) return rc;
  }
  int rc = mr_pass<T>(c, kMrRowFwd, 1, in, nullptr, out, nullptr, nx, ny, batch, 1.0, none, s);
  if (rc == FFTPDE_OK && two && in2) rc = mr_pass<T>(c, kMrRowFwd, 1, in2, nullptr, vb, nullptr, nx, ny, batch, 1.0, none, s);
  if (rc == FFTPDE_OK)
    rc = mr_pass<T>(c, kMrColSolve, two ? 2 : 1, out, two && in2 ? vb : nullptr, out, two ? out2 : nullptr, nx, ny,
                    batch, 1.0, sym, s);
  if (rc == FFTPDE_OK) rc = mr_pass<T>(c, kMrRowInv, 1, out, nullptr, out, nullptr, nx, ny, batch, 1.0, none, s);
  if (rc == FFTPDE_OK && two && out2)
    rc = mr_pass<T>(c, kMrRowInv, 1, out2, nullptr, out2, nullptr, nx, ny, batch, 1.0, none, s);
  return rc;
}

// Real fields (R32 / R64): pairs x1 + i x2 through the complex passes.  The
// symbols are real and even in k, so the solve of the pair is the pair of the
// solves; rows read and write the real fields directly, the pair spectra
// live in the workspace.
template <typename T>
int solve_real(Context* c, int op, const void* in, const void* in2, void* out, void* out2, int nx, int ny, int batch,
               double lx, double ly, double coef, double t, hipStream_t s) {
  const MrSym sym = mr_sym(op, nx, ny, lx, ly, coef, t);
  const MrSym none;
  const bool two = op == FFTPDE_WAVE && (in2 || out2);
  const long long npairs = (batch + 1) / 2;
  const size_t pair_bytes = sizeof(cx<T>) * (size_t)nx * ny * (size_t)npairs;
  void* w = nullptr;
  const int rcw = c->workspace(pair_bytes * (two ? 2 : 1), s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  void* mid = w;
  void* mid2 = two ? static_cast<char*>(w) + pair_bytes : nullptr;
  int rc = mr_pass<T>(c, kMrRowFwd, 1, nullptr, nullptr, mid, nullptr, nx, ny, npairs, 1.0, none, s, in, nullptr, batch);
  if (rc == FFTPDE_OK && two && in2)
    rc = mr_pass<T>(c, kMrRowFwd, 1, nullptr, nullptr, mid2, nullptr, nx, ny, npairs, 1.0, none, s, in2, nullptr, batch);
  if (rc == FFTPDE_OK)
    rc = mr_pass<T>(c, kMrColSolve, two ? 2 : 1, mid, two && in2 ? mid2 : nullptr, mid, two && out2 ? mid2 : nullptr,
                    nx, ny, npairs, 1.0, sym, s);
  if (rc == FFTPDE_OK)
    rc = mr_pass<T>(c, kMrRowInv, 1, mid, nullptr, nullptr, nullptr, nx, ny, npairs, 1.0, none, s, nullptr, out, batch);
  if (rc == FFTPDE_OK && two && out2)
    rc = mr_pass<T>(c, kMrRowInv, 1, mid2, nullptr, nullptr, nullptr, nx, ny, npairs, 1.0, none, s, nullptr, out2,
                    batch);
  return rc;
}

// Half spectra of real fields: the pairs' complex spectra in the workspace,
// split into (forward) or joined from (inverse) the half spectra.
template <typename T>
int half(Context* c, bool inverse, const void* in, void* out, int nx, int ny, int batch, hipStream_t s) {
  const MrSym none;
  const long long npairs = (batch + 1) / 2;
  const long long pts = (long long)nx * ny, hpts = (long long)(nx / 2 + 1) * ny;
  void* w = nullptr;
  const int rcw = c->workspace(sizeof(cx<T>) * (size_t)pts * (size_t)npairs, s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  HalfArgs<T> h{static_cast<cx<T>*>(w), nullptr, nx, ny, npairs, batch};
  const char* name = inverse ? (sizeof(T) == 4 ? "tangle_float" : "tangle_double")
                             : (sizeof(T) == 4 ? "untangle_float" : "untangle_double");
  const double hbytes = (double)sizeof(cx<T>) * (double)(npairs * pts + batch * hpts);
  auto split_or_join = [&]() -> int {
    const hipError_t e =
        timed_launch(c, name, hbytes, s, [&] { return inverse ? launch_tangle<T>(h, s) : launch_untangle<T>(h, s); });
    if (e != hipSuccess) {
      set_last_error(name, e);
      return FFTPDE_EDEVICE;
    }
    return FFTPDE_OK;
  };
  if (!inverse) {
    h.half = static_cast<cx<T>*>(out);
    int rc = mr_pass<T>(c, kMrRowFwd, 1, nullptr, nullptr, w, nullptr, nx, ny, npairs, 1.0, none, s, in, nullptr, batch);
    if (rc == FFTPDE_OK) rc = mr_pass<T>(c, kMrColFwd, 1, w, nullptr, w, nullptr, nx, ny, npairs, 1.0, none, s);
    if (rc == FFTPDE_OK) rc = split_or_join();
    return rc;
  }
  h.half = static_cast<cx<T>*>(const_cast<void*>(in));
  int rc = split_or_join();
  if (rc == FFTPDE_OK) rc = mr_pass<T>(c, kMrColInv, 1, w, nullptr, w, nullptr, nx, ny, npairs, 1.0, none, s);
  if (rc == FFTPDE_OK)
    rc = mr_pass<T>(c, kMrRowInv, 1, w, nullptr, nullptr, nullptr, nx, ny, npairs, 1.0 / ((double)nx * ny), none, s,
                    nullptr, out, batch);
  return rc;
}

}  // namespace

bool mixed_side(int n) { return mr_side_ok(n); }

int run_mixed_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                        hipStream_t s) {
  return dtype == FFTPDE_C64 ? transform<float>(c, inverse, in, out, nx, ny, batch, s)
                             : transform<double>(c, inverse, in, out, nx, ny, batch, s);
}

int run_mixed_solve(Context* c, int dtype, int op, const void* in, const void* in2, void* out, void* out2, int nx,
                    int ny, int batch, double lx, double ly, double coef, double t, hipStream_t s) {
  switch (dtype) {
    case FFTPDE_C64: return solve<float>(c, op, in, in2, out, out2, nx, ny, batch, lx, ly, coef, t, s);
    case FFTPDE_C128: return solve<double>(c, op, in, in2, out, out2, nx, ny, batch, lx, ly, coef, t, s);
    case FFTPDE_R32: return solve_real<float>(c, op, in, in2, out, out2, nx, ny, batch, lx, ly, coef, t, s);
    case FFTPDE_R64: return solve_real<double>(c, op, in, in2, out, out2, nx, ny, batch, lx, ly, coef, t, s);
    default: return FFTPDE_EINVAL;
  }
}

int run_mixed_half(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                   hipStream_t s) {
  return dtype == FFTPDE_R32 ? half<float>(c, inverse, in, out, nx, ny, batch, s)
                             : half<double>(c, inverse, in, out, nx, ny, batch, s);
}

}  // namespace fftpde
