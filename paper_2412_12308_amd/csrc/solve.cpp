// solve.cpp -- launch sequences of the 2D transforms and the spectral
// solves: row pass (x transforms for every y, Sec. II.D), column pass (y
// transforms, with the symbol between forward and inverse), row pass.
#include "solve.hpp"

#include "diag.hpp"
#include "halfrow.hpp"
#include "halfspec.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/fftpde.h"

namespace fftpde {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}

}  // namespace

template <typename T>
static const cx<T>* twiddles(const Context* c) {
  if constexpr (sizeof(T) == 4) return c->tw32;
  else return c->tw64;
}

template <typename T>
int row_pass(Context* c, const void* in, void* out, int lognx, int logny, long long nrows, bool inverse,
             double scale, hipStream_t s, int in_t, int out_t, int real_in, int real_out, long long nreal) {
  const RowVariant* v = c->row_variant(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, lognx);
  if (!v) return FFTPDE_EINVAL;
  RowArgs<T> a{static_cast<const cx<T>*>(in), static_cast<cx<T>*>(out), twiddles<T>(c), nrows, inverse ? 1 : 0,
               T(scale), logny, in_t < 0 ? lognx : in_t, out_t < 0 ? lognx : out_t, nreal};
  const double bytes = 2.0 * sizeof(cx<T>) * (double)nrows * (double)(1 << lognx);
  const LaunchFn launch = real_in ? v->launch_rin : real_out ? v->launch_rout : v->launch;
  const OccFn occ = real_in ? v->occupancy_rin : real_out ? v->occupancy_rout : v->occupancy;
  const long long maxb = v->pf ? c->max_blocks(reinterpret_cast<const void*>(occ), occ) : 0;
  hipError_t e = timed_launch(c, v->name, bytes, s, [&] { return launch(&a, nrows, maxb, s); });
  if (e != hipSuccess) {
    set_last_error(v->name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

template <typename T>
int col_pass(Context* c, const void* in0, const void* in1, void* out0, void* out1, int lognx, int logny,
             long long batch, int mode, const SymParams& sym, int nf, hipStream_t s, int layout_t) {
  const ColVariant* v = c->col_variant(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, logny, nf);
  if (!v) return FFTPDE_EINVAL;
  // a block holds whole tiles and never spans fields
  if (layout_t >= 0 && (layout_t < v->logt || layout_t > lognx)) return FFTPDE_EINVAL;
  ColArgs<T> a{static_cast<const cx<T>*>(in0), static_cast<const cx<T>*>(in1), nullptr, static_cast<cx<T>*>(out0),
               static_cast<cx<T>*>(out1), twiddles<T>(c), batch << lognx, lognx, mode, sym, layout_t,
               c->stage_tw<T>(logny, v->maxlr, false), c->stage_tw<T>(logny, v->maxlr, true)};
  const double field = sizeof(cx<T>) * (double)batch * (double)(1ll << (lognx + logny));
  const double bytes = field * ((in0 ? 1 : 0) + (in1 ? 1 : 0) + (out0 ? 1 : 0) + (out1 ? 1 : 0));
  // the [forward, symbol, inverse] pass runs the kernel compiled for it alone
  const bool fused = mode == kColFwdMulInv;
  const LaunchFn launch = fused ? v->launch_fused : v->launch;
  const OccFn occ = fused ? v->occupancy_fused : v->occupancy;
  const long long maxb = v->pf ? c->max_blocks(reinterpret_cast<const void*>(occ), occ) : 0;
  hipError_t e = timed_launch(c, v->name, bytes, s, [&] { return launch(&a, batch << lognx, maxb, s); });
  if (e != hipSuccess) {
    set_last_error(v->name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

SymParams make_sym(int op, int nx, int ny, double lx, double ly, double coef, double t) {
  SymParams p{};
  p.op = op;
  p.lognx = ilog2(nx);
  p.logny = ilog2(ny);
  p.kxs = 2.0 * kPi / lx;
  p.kys = 2.0 * kPi / ly;
  p.scale = 1.0 / ((double)nx * (double)ny);
  if (op == kSymDiffusion) p.kt = coef * t;
  if (op == kSymWave) {
    p.c = coef;
    p.t = t;
    p.hx = 2.0 * coef * t / lx;
    p.hy = 2.0 * coef * t / ly;
    set_phase_range(p, nx, ny, 1);
  }
  return p;
}

// SymParams::phase_fast from the extreme nonzero (w t / pi)^2 of the grid:
// the smallest is one step along an axis, the largest the corner of signed
// indices n/2 (3D: the y term along hy3 with ny3 points).
void set_phase_range(SymParams& p, int nx, int ny, int ny3) {
  double lo = 1e300, hi = 0.0;
  auto axis = [&](double h, int n) {
    if (h == 0.0 || n < 2) return;
    lo = std::min(lo, h * h);
    const double e = h * (n / 2);
    hi += e * e;
  };
  axis(p.hx, p.lx3 > 0 ? (1 << p.lx3) : nx);
  axis(p.hy, ny);
  if (p.lx3 > 0) axis(p.hy3, ny3);
  p.phase_fast = (hi == 0.0 || (lo >= 1e-30 && hi <= 1e36)) ? 1 : 0;
}

// Runs f(b0, nb, byte offset) over chunks of the batch of about
// Context::chunk_bytes of field data: every pass of one chunk before the next,
// so that what a pass writes is still in the Infinity Cache for the next.
template <typename T, class F>
int for_chunks(Context* c, int nx, int ny, int batch, F&& f, long long max_chunk = 0) {
  const size_t field = sizeof(cx<T>) * (size_t)nx * ny;
  const long long cb = c->chunk_bytes_for(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, ilog2(nx), ilog2(ny));
  long long chunk = cb > 0 ? std::max<long long>(1, cb / (long long)field) : batch;
  chunk = std::min<long long>(chunk, batch);
  if (max_chunk > 0) chunk = std::min<long long>(chunk, max_chunk);
  for (long long b0 = 0; b0 < batch; b0 += chunk) {
    const long long nb = std::min<long long>(chunk, batch - b0);
    const int rc = f(b0, nb, field * (size_t)b0);
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

template <typename T>
static const void* at(const void* p, size_t off) {
  return p ? static_cast<const char*>(p) + off : nullptr;
}
template <typename T>
static void* at(void* p, size_t off) {
  return p ? static_cast<char*>(p) + off : nullptr;
}

template <typename T>
int transform(Context* c, const void* in, void* out, int nx, int ny, int batch, bool inverse, hipStream_t s) {
  const int lx = ilog2(nx), ly = ilog2(ny);
  SymParams sym = make_sym(kSymScale, nx, ny, 1.0, 1.0, 0.0, 0.0);
  return for_chunks<T>(c, nx, ny, batch, [&](long long, long long nb, size_t off) {
    const void* ib = at<T>(in, off);
    void* ob = at<T>(out, off);
    int rc;
    if (!inverse) {
      rc = row_pass<T>(c, ib, ob, lx, ly, (long long)ny * nb, false, 1.0, s);
      if (rc == FFTPDE_OK) rc = col_pass<T>(c, ob, nullptr, ob, nullptr, lx, ly, nb, kColForward, sym, 1, s);
    } else {
      rc = col_pass<T>(c, ib, nullptr, ob, nullptr, lx, ly, nb, kColInverse, sym, 1, s);
      if (rc == FFTPDE_OK) rc = row_pass<T>(c, ob, ob, lx, ly, (long long)ny * nb, true, 1.0, s);
    }
    return rc;
  });
}

// forward rows -> fused column pass -> inverse rows, for one real symbol;
// batches run in chunks (Context::chunk_bytes), every pass of a chunk before
// the next chunk
template <typename T>
int solve_real_symbol(Context* c, const void* in, void* out, int nx, int ny, int batch, const SymParams& sym,
                      hipStream_t s, const SolveScratch& sc) {
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lx = ilog2(nx), ly = ilog2(ny);
  const size_t field = sizeof(cx<T>) * (size_t)nx * ny;
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  long long chunk = cb > 0 ? std::max<long long>(1, cb / (long long)field) : batch;
  chunk = std::min<long long>(chunk, batch);
  // Tiled intermediate in a per-stream scratch field: column blocks of
  // tiled_bytes per row (whole cache lines for the row passes; the column
  // tiles of a block share its lines), at least one column tile wide.
  const ColVariant* cv = c->col_variant(dt, ly, 1);
  const int tiled_bytes = c->tiled_bytes_for(dt, lx, ly);
  int lt = -1;
  void* w = nullptr;
  if (tiled_bytes > 0 && cv) {
    int bt = 0;  // log2 of the block width in columns
    while ((int)sizeof(cx<T>) << (bt + 1) <= tiled_bytes) bt++;
    lt = bt > cv->logt ? bt : cv->logt;
    if (lt >= lx) lt = -1;
    if (lt >= 0 && sc.p) {
      // caller-provided scratch: as many fields per chunk as it holds
      const long long fit = (long long)(sc.bytes / field);
      if (fit < 1) return FFTPDE_EINVAL;
      chunk = std::min<long long>(chunk, fit);
      w = sc.p;
    } else if (lt >= 0) {
      const int rcw = c->workspace(field * (size_t)chunk, s, &w);
      if (rcw != FFTPDE_OK) return rcw;
    }
  }
  for (long long b0 = 0; b0 < batch; b0 += chunk) {
    const long long nb = std::min<long long>(chunk, batch - b0);
    const long long nrows = (long long)ny * nb;
    const void* ib = static_cast<const char*>(in) + field * b0;
    void* ob = static_cast<char*>(out) + field * b0;
    void* mid = lt >= 0 ? w : ob;  // the spectrum between the passes
    int rc = row_pass<T>(c, ib, mid, lx, ly, nrows, false, 1.0, s, -1, lt);
    if (rc == FFTPDE_OK) rc = col_pass<T>(c, mid, nullptr, mid, nullptr, lx, ly, nb, kColFwdMulInv, sym, 1, s, lt);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, mid, ob, lx, ly, nrows, true, 1.0, s, lt, -1);
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

// The wave with an initial velocity and/or the velocity output: both
// spectra go through one two-field column pass.  Like the one-field solves,
// the spectra live in per-stream scratch in column blocks (the tiled
// intermediate), two fields per 256 MiB chunk of fields.
template <typename T>
int solve_wave_two(Context* c, const void* u0, const void* v0, void* u, void* v, int nx, int ny, int batch,
                   const SymParams& sym, hipStream_t s, const SolveScratch& sc) {
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lx = ilog2(nx), ly = ilog2(ny);
  const size_t field = sizeof(cx<T>) * (size_t)nx * ny;
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  long long chunk = std::min<long long>(cb > 0 ? std::max<long long>(1, cb / (long long)field) : batch, batch);
  const ColVariant* cv = c->col_variant(dt, ly, 2);
  if (!cv) return FFTPDE_EINVAL;
  const int tiled_bytes = c->tiled_bytes_for(dt, lx, ly);
  int lt = -1;
  if (tiled_bytes > 0) {
    int bt = 0;  // log2 of the block width in columns
    while ((int)sizeof(cx<T>) << (bt + 1) <= tiled_bytes) bt++;
    lt = bt > cv->logt ? bt : cv->logt;
    if (lt >= lx) lt = -1;
  }
  // spectra: F (then U) and G (then V); in the outputs when row-major
  void* w = nullptr;
  if (lt >= 0 || (v0 && !v)) {
    const size_t per = field * (lt >= 0 ? 2 : 1);  // scratch bytes per field of a chunk
    if (sc.p) {
      const long long fit = (long long)(sc.bytes / per);
      if (fit < 1) return FFTPDE_EINVAL;
      chunk = std::min<long long>(chunk, fit);
      w = sc.p;
    } else {
      const int rc = c->workspace(per * (size_t)chunk, s, &w);
      if (rc != FFTPDE_OK) return rc;
    }
  }
  return for_chunks<T>(c, nx, ny, batch, [&](long long, long long nb, size_t off) {
    const long long nrows = (long long)ny * nb;
    void* ub = at<T>(u, off);
    void* vb = at<T>(v, off);
    void* fs = lt >= 0 ? w : ub;
    void* gs = lt >= 0 ? static_cast<char*>(w) + field * (size_t)chunk : (v ? vb : w);
    int rc = row_pass<T>(c, at<T>(u0, off), fs, lx, ly, nrows, false, 1.0, s, -1, lt);
    if (rc == FFTPDE_OK && v0) rc = row_pass<T>(c, at<T>(v0, off), gs, lx, ly, nrows, false, 1.0, s, -1, lt);
    if (rc == FFTPDE_OK)
      rc = col_pass<T>(c, fs, v0 ? gs : nullptr, fs, v ? gs : nullptr, lx, ly, nb, kColFwdMulInv, sym, 2, s, lt);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, fs, ub, lx, ly, nrows, true, 1.0, s, lt, -1);
    if (rc == FFTPDE_OK && vb) rc = row_pass<T>(c, gs, vb, lx, ly, nrows, true, 1.0, s, lt, -1);
    return rc;
  }, chunk);
}


// One launch for the whole transform or solve when a single-pass small-grid
// kernel exists for the shape; returns -100 when there is none.
template <typename T>
int small_pass(Context* c, const void* in, void* out, int nx, int ny, int batch, int mode, const SymParams& sym,
               hipStream_t s) {
  const SmallVariant* v = c->small_variant(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, ilog2(nx), ilog2(ny));
  if (!v) return -100;
  SmallArgs<T> a{static_cast<const cx<T>*>(in), static_cast<cx<T>*>(out), twiddles<T>(c), batch, mode, sym};
  const double bytes = 2.0 * sizeof(cx<T>) * (double)nx * ny * batch;
  hipError_t e = timed_launch(c, v->name, bytes, s, [&] { return v->launch(&a, batch, 0, s); });
  if (e != hipSuccess) {
    set_last_error(v->name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

// Pairs of real fields per chunk.  For the solves and the forward half
// transform the chunk size counts the real fields and their pair spectra
// together, 2 x the spectra (at the 256 MiB default, 4 FP32 2048^2 pairs: 8
// real fields).  With chunks of pair spectra alone (8 pairs) their column
// pass ran 25 % slower than on complex fields of the same bytes, with the
// same L2 traffic and hit rate; the half chunk runs the real FP32 solves 4 %
// and the forward half transform 10 % faster.  The inverse half transform
// keeps chunks of spectra alone (`halve` false): 9 % faster there.
static long long pair_chunk(const Context* c, int dt, int lx, int ly, size_t pair_bytes, long long npairs,
                            bool halve = true) {
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  const long long per = (halve ? 2 : 1) * (long long)pair_bytes;
  const long long chunk = cb > 0 ? std::max<long long>(1, cb / per) : npairs;
  return std::min<long long>(chunk, npairs);
}

// Real fields, two per complex transform.  The three symbols are real and
// even in k, so a solve S maps real fields to real fields and is complex
// linear: S(u1 + i u2) = S(u1) + i S(u2).  Fields 2p and 2p + 1 enter the
// forward row pass as the real and imaginary parts of one complex field and
// leave the inverse row pass the same way; nothing else changes, and each
// real field moves half the bytes of a complex one.  The pair's spectra live
// in the context's per-stream scratch (tiled like solve_real_symbol's when
// there is no velocity field).
template <typename T>
int solve_real_pairs(Context* c, const void* in, const void* in2, void* out, void* out2, int nx, int ny, int batch,
                     const SymParams& sym, hipStream_t s) {
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lx = ilog2(nx), ly = ilog2(ny);
  const long long pts = (long long)nx * ny;
  const size_t pair_bytes = sizeof(cx<T>) * (size_t)pts;  // one complex field per pair
  const long long npairs = (batch + 1) / 2;
  const long long chunk = pair_chunk(c, dt, lx, ly, pair_bytes, npairs);
  const int nf = (sym.op == kSymWave && (in2 || out2)) ? 2 : 1;
  const ColVariant* cv = c->col_variant(dt, ly, nf);
  if (!cv) return FFTPDE_EINVAL;
  int lt = -1;
  const int tiled_bytes = c->tiled_bytes_for(dt, lx, ly);
  if (tiled_bytes > 0) {
    int bt = 0;
    while ((int)sizeof(cx<T>) << (bt + 1) <= tiled_bytes) bt++;
    lt = bt > cv->logt ? bt : cv->logt;
    if (lt >= lx) lt = -1;
  }
  void* w = nullptr;
  const int rcw = c->workspace(pair_bytes * (size_t)chunk * nf, s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  void* mid = w;
  void* mid2 = nf == 2 ? static_cast<char*>(w) + pair_bytes * (size_t)chunk : nullptr;
  for (long long p0 = 0; p0 < npairs; p0 += chunk) {
    const long long np = std::min<long long>(chunk, npairs - p0);
    const long long nrows = (long long)ny * np;
    const long long f0 = 2 * p0, nreal = std::min<long long>(2 * np, batch - f0);
    const size_t off = sizeof(T) * (size_t)(f0 * pts);
    int rc = row_pass<T>(c, at<T>(in, off), mid, lx, ly, nrows, false, 1.0, s, -1, lt, 1, 0, nreal);
    if (rc == FFTPDE_OK && nf == 2) {
      if (in2) rc = row_pass<T>(c, at<T>(in2, off), mid2, lx, ly, nrows, false, 1.0, s, -1, lt, 1, 0, nreal);
    }
    if (rc == FFTPDE_OK)
      rc = col_pass<T>(c, mid, nf == 2 && in2 ? mid2 : nullptr, mid, nf == 2 && out2 ? mid2 : nullptr, lx, ly, np,
                       kColFwdMulInv, sym, nf, s, lt);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, mid, at<T>(out, off), lx, ly, nrows, true, 1.0, s, lt, -1, 0, 1, nreal);
    if (rc == FFTPDE_OK && out2)
      rc = row_pass<T>(c, mid2, at<T>(out2, off), lx, ly, nrows, true, 1.0, s, lt, -1, 0, 1, nreal);
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

// ---------------------------------------------------------------------------
// 3D: x rows, then y columns of every z plane, then z columns (the field seen
// as nz rows of nx*ny columns); a solve fuses its symbol into the z pass and
// runs the y and x passes back.  Five passes, all row-major.
// ---------------------------------------------------------------------------
SymParams make_sym3d(int op, int nx, int ny, int nz, double lx, double ly, double lz, double coef, double t) {
  SymParams p = make_sym(op, nx * ny, nz, lx, lz, coef, t);
  p.lx3 = ilog2(nx);
  p.kxs = 2.0 * kPi / lx;
  p.ky3s = 2.0 * kPi / ly;
  p.kys = 2.0 * kPi / lz;
  if (op == kSymWave) {
    p.hx = 2.0 * coef * t / lx;
    p.hy3 = 2.0 * coef * t / ly;
    p.hy = 2.0 * coef * t / lz;
    set_phase_range(p, nx, nz, ny);
  }
  p.scale = 1.0 / ((double)nx * (double)ny * (double)nz);
  return p;
}

template <typename T>
int pass3d(Context* c, const void* in, void* out, int nx, int ny, int nz, int batch, const SymParams* sym, bool inverse,
           hipStream_t s) {
  const int lx = ilog2(nx), ly = ilog2(ny), lz = ilog2(nz);
  const long long pts = (long long)nx * ny * nz;
  const size_t field = sizeof(cx<T>) * (size_t)pts;
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  long long chunk = cb > 0 ? std::max<long long>(1, cb / (long long)field) : batch;
  chunk = std::min<long long>(chunk, batch);
  SymParams unit = make_sym(kSymScale, nx, ny, 1.0, 1.0, 0.0, 0.0);  // plain transforms, scale 1
  unit.scale = 1.0;
  for (long long b0 = 0; b0 < batch; b0 += chunk) {
    const long long nb = std::min<long long>(chunk, batch - b0);
    const void* ib = static_cast<const char*>(in) + field * b0;
    void* ob = static_cast<char*>(out) + field * b0;
    const long long rows = (long long)ny * nz * nb;
    int rc = FFTPDE_OK;
    if (!inverse || sym) {
      // forward x, forward y per plane
      rc = row_pass<T>(c, ib, ob, lx, ly + lz, rows, false, 1.0, s);
      if (rc == FFTPDE_OK) rc = col_pass<T>(c, ob, nullptr, ob, nullptr, lx, ly, nb * nz, kColForward, unit, 1, s);
    }
    if (rc == FFTPDE_OK) {
      if (sym) {
        rc = col_pass<T>(c, ob, nullptr, ob, nullptr, lx + ly, lz, nb, kColFwdMulInv, *sym, 1, s);
      } else if (!inverse) {
        rc = col_pass<T>(c, ob, nullptr, ob, nullptr, lx + ly, lz, nb, kColForward, unit, 1, s);
      } else {
        SymParams inv = unit;
        inv.scale = 1.0 / (double)pts;
        rc = col_pass<T>(c, ib, nullptr, ob, nullptr, lx + ly, lz, nb, kColInverse, inv, 1, s);
      }
    }
    if (rc == FFTPDE_OK && (inverse || sym)) {
      // inverse y per plane, inverse x
      rc = col_pass<T>(c, ob, nullptr, ob, nullptr, lx, ly, nb * nz, kColInverse, unit, 1, s);
      if (rc == FFTPDE_OK) rc = row_pass<T>(c, ob, ob, lx, ly + lz, rows, true, 1.0, s);
    }
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

int run_transform3d(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int nz, int batch,
                    hipStream_t s) {
  return dtype == FFTPDE_C64 ? pass3d<float>(c, in, out, nx, ny, nz, batch, nullptr, inverse, s)
                             : pass3d<double>(c, in, out, nx, ny, nz, batch, nullptr, inverse, s);
}

int run_solve3d(Context* c, int dtype, int op, const void* in, void* out, int nx, int ny, int nz, int batch, double lx,
                double ly, double lz, double coef, double t, hipStream_t s) {
  const int sop = op == FFTPDE_POISSON ? kSymPoisson : op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave;
  const SymParams sym = make_sym3d(sop, nx, ny, nz, lx, ly, lz, coef, t);
  return dtype == FFTPDE_C64 ? pass3d<float>(c, in, out, nx, ny, nz, batch, &sym, false, s)
                             : pass3d<double>(c, in, out, nx, ny, nz, batch, &sym, false, s);
}

// Solves with a source constant in time: forward row passes of f, g (if
// given) and s into per-stream scratch spectra, one three-field column pass
// (forward, coefficients, inverse), inverse row passes of u (and v).  Complex
// fields, or real fields in pairs (real: see solve_real_pairs).
template <typename T>
int solve_source(Context* c, const void* f, const void* g, const void* src, void* u, void* v, int nx, int ny,
                 int batch, const SymParams& sym, bool real, hipStream_t s) {
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lx = ilog2(nx), ly = ilog2(ny);
  const long long pts = (long long)nx * ny;
  const size_t cfield = sizeof(cx<T>) * (size_t)pts;     // one complex (or pair) field
  const long long units = real ? (batch + 1) / 2 : batch;  // complex fields to transform
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  long long chunk = cb > 0 ? std::max<long long>(1, cb / (long long)cfield) : units;
  chunk = std::min<long long>(chunk, units);
  if (!c->col_variant(dt, ly, 3)) return FFTPDE_EINVAL;
  const bool two = g != nullptr || v != nullptr;  // a second spectrum (G in, V out)
  void* w = nullptr;
  const int rcw = c->workspace(cfield * (size_t)chunk * (two ? 3 : 2), s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  void* mF = w;
  void* mS = static_cast<char*>(w) + cfield * (size_t)chunk;
  void* mG = two ? static_cast<char*>(w) + 2 * cfield * (size_t)chunk : nullptr;
  const size_t elem = real ? sizeof(T) : sizeof(cx<T>);
  for (long long q0 = 0; q0 < units; q0 += chunk) {
    const long long nq = std::min<long long>(chunk, units - q0);
    const long long nrows = (long long)ny * nq;
    const long long f0 = real ? 2 * q0 : q0;
    const long long nreal = real ? std::min<long long>(2 * nq, batch - f0) : 0;
    const size_t off = elem * (size_t)(f0 * pts);
    const int ri = real ? 1 : 0;
    int rc = row_pass<T>(c, at<T>(f, off), mF, lx, ly, nrows, false, 1.0, s, -1, -1, ri, 0, nreal);
    if (rc == FFTPDE_OK && g) rc = row_pass<T>(c, at<T>(g, off), mG, lx, ly, nrows, false, 1.0, s, -1, -1, ri, 0, nreal);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, at<T>(src, off), mS, lx, ly, nrows, false, 1.0, s, -1, -1, ri, 0, nreal);
    if (rc == FFTPDE_OK) {
      const int dtc = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
      const ColVariant* cv = c->col_variant(dtc, ly, 3);
      ColArgs<T> a{static_cast<const cx<T>*>(mF), g ? static_cast<const cx<T>*>(mG) : nullptr,
                   static_cast<const cx<T>*>(mS), static_cast<cx<T>*>(mF), v ? static_cast<cx<T>*>(mG) : nullptr,
                   twiddles<T>(c), nq << lx, lx, kColFwdMulInv, sym, -1,
                   c->stage_tw<T>(ly, cv->maxlr, false), c->stage_tw<T>(ly, cv->maxlr, true)};
      const double bytes = (double)cfield * (double)nq * ((g ? 1 : 0) + 2 + 1 + (v ? 1 : 0));
      const long long maxb = cv->pf ? c->max_blocks(reinterpret_cast<const void*>(cv->occupancy_fused),
                                                   cv->occupancy_fused) : 0;
      hipError_t e = timed_launch(c, cv->name, bytes, s, [&] { return cv->launch_fused(&a, nq << lx, maxb, s); });
      if (e != hipSuccess) {
        set_last_error(cv->name, e);
        rc = FFTPDE_EDEVICE;
      }
    }
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, mF, at<T>(u, off), lx, ly, nrows, true, 1.0, s, -1, -1, 0, ri, nreal);
    if (rc == FFTPDE_OK && v) rc = row_pass<T>(c, mG, at<T>(v, off), lx, ly, nrows, true, 1.0, s, -1, -1, 0, ri, nreal);
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

int run_source(Context* c, int dtype, int op, const void* f, const void* g, const void* src, void* u, void* v, int nx,
               int ny, int batch, double lx, double ly, double coef, double t, hipStream_t s) {
  SymParams sym = make_sym(op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave, nx, ny, lx, ly, coef, t);
  sym.op = op == FFTPDE_DIFFUSION ? kSymDiffSource : kSymWaveSource;
  sym.c = coef;  // kappa or the wave speed
  sym.t = t;
  const bool real = dtype == FFTPDE_R32 || dtype == FFTPDE_R64;
  const bool fp32 = dtype == FFTPDE_C64 || dtype == FFTPDE_R32;
  return fp32 ? solve_source<float>(c, f, g, src, u, v, nx, ny, batch, sym, real, s)
              : solve_source<double>(c, f, g, src, u, v, nx, ny, batch, sym, real, s);
}

int run_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                  hipStream_t s) {
  const SymParams sym = make_sym(kSymScale, nx, ny, 1.0, 1.0, 0.0, 0.0);
  const int mode = inverse ? kColInverse : kColForward;
  const int r = dtype == FFTPDE_C64 ? small_pass<float>(c, in, out, nx, ny, batch, mode, sym, s)
                                    : small_pass<double>(c, in, out, nx, ny, batch, mode, sym, s);
  if (r != -100) return r;
  return dtype == FFTPDE_C64 ? transform<float>(c, in, out, nx, ny, batch, inverse, s)
                             : transform<double>(c, in, out, nx, ny, batch, inverse, s);
}

// fft2d_r2c / fft2d_c2r in two passes (halfrow.hpp): the column pass over
// the real fields read as complex fields of nx/2 columns, then the row pass
// over row pairs (b, -b) that writes whole half-spectrum rows (c2r: the
// reverse), one work field of M x ny complex points per real field between
// them.  Chunks of fields count the real fields and the work fields
// together.
template <typename T>
int half_rows(Context* c, bool inverse, const void* in, void* out, int nx, int ny, int batch, hipStream_t s) {
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int fp64 = sizeof(T) == 8;
  const int lx = ilog2(nx), ly = ilog2(ny), lm = lx - 1;
  const size_t rbytes = sizeof(T) * (size_t)nx * ny;                   // one real field = one work field
  const size_t hbytes = sizeof(cx<T>) * (size_t)(nx / 2 + 1) * ny;    // one half spectrum
  const long long cb = c->chunk_bytes_for(dt, lx, ly);
  long long chunk = cb > 0 ? std::max<long long>(1, cb / (2 * (long long)rbytes)) : batch;
  chunk = std::min<long long>(chunk, batch);
  // work layout: blocks of tiled_bytes per row, at least one column tile wide
  int lt = lm;
  const int tiled_bytes = c->tiled_bytes_for(dt, lx, ly);
  if (tiled_bytes > 0) {
    int bt = 0;
    while ((int)sizeof(cx<T>) << (bt + 1) <= tiled_bytes) bt++;
    lt = std::min(lm, std::max(bt, halfrow_col_logt(fp64, ly)));
  }
  void* w = nullptr;
  const int rcw = c->workspace(rbytes * (size_t)chunk, s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  HalfRowArgs<T> a{};
  a.work = static_cast<cx<T>*>(w);
  a.tw = twiddles<T>(c);
  a.stw = c->stage_tw<T>(ly, halfrow_col_maxlr(fp64), false);
  a.lognx = lx;
  a.logny = ly;
  a.lt = lt;
  a.scale = T(1.0 / ((double)(nx / 2) * (double)ny));
  const char* names[4] = {sizeof(T) == 4 ? "r2c_cols_float" : "r2c_cols_double",
                          sizeof(T) == 4 ? "r2c_rows_float" : "r2c_rows_double",
                          sizeof(T) == 4 ? "c2r_rows_float" : "c2r_rows_double",
                          sizeof(T) == 4 ? "c2r_cols_float" : "c2r_cols_double"};
  for (long long f0 = 0; f0 < batch; f0 += chunk) {
    a.fields = std::min<long long>(chunk, batch - f0);
    const double rb = (double)rbytes * a.fields, hb = (double)hbytes * a.fields;
    auto step = [&](int k, double bytes, hipError_t (*fn)(const HalfRowArgs<T>&, hipStream_t)) {
      const hipError_t e = timed_launch(c, names[k], bytes, s, [&] { return fn(a, s); });
      if (e != hipSuccess) {
        set_last_error(names[k], e);
        return FFTPDE_EDEVICE;
      }
      return FFTPDE_OK;
    };
    int rc;
    if (!inverse) {
      a.rin = static_cast<const T*>(at<T>(in, rbytes * (size_t)f0));
      a.hout = static_cast<cx<T>*>(at<T>(out, hbytes * (size_t)f0));
      rc = step(0, 2 * rb, launch_r2c_cols<T>);
      if (rc == FFTPDE_OK) rc = step(1, rb + hb, launch_r2c_rows<T>);
    } else {
      a.hin = static_cast<const cx<T>*>(at<T>(in, hbytes * (size_t)f0));
      a.rout = static_cast<T*>(at<T>(out, rbytes * (size_t)f0));
      rc = step(2, hb + rb, launch_c2r_rows<T>);
      if (rc == FFTPDE_OK) rc = step(3, 2 * rb, launch_c2r_cols<T>);
    }
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

// fft2d_r2c / fft2d_c2r: real fields in pairs, each pair one complex field
// (row pass with real loads or stores), its spectrum in the per-stream
// scratch, and the half spectra split off (forward) or joined (inverse).
template <typename T>
int half_transform(Context* c, bool inverse, const void* in, void* out, int nx, int ny, int batch, hipStream_t s) {
  // the real side is read (or written) as complex points: it must be aligned like them
  const void* real = inverse ? out : in;
  if (halfrow_supported(sizeof(T) == 8, ilog2(nx), ilog2(ny)) &&
      reinterpret_cast<uintptr_t>(real) % sizeof(cx<T>) == 0)
    return half_rows<T>(c, inverse, in, out, nx, ny, batch, s);
  const int dt = sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128;
  const int lx = ilog2(nx), ly = ilog2(ny);
  const long long pts = (long long)nx * ny, hpts = (long long)(nx / 2 + 1) * ny;
  const size_t pair_bytes = sizeof(cx<T>) * (size_t)pts;
  const long long npairs = (batch + 1) / 2;
  const long long chunk = pair_chunk(c, dt, lx, ly, pair_bytes, npairs, !inverse);
  // the pair spectra in the column passes' tiled layout, as in the solves
  const ColVariant* cv = c->col_variant(dt, ly, 1);
  if (!cv) return FFTPDE_EINVAL;
  int lt = -1;
  const int tiled_bytes = c->tiled_bytes_for(dt, lx, ly);
  if (tiled_bytes > 0) {
    int bt = 0;
    while ((int)sizeof(cx<T>) << (bt + 1) <= tiled_bytes) bt++;
    lt = bt > cv->logt ? bt : cv->logt;
    if (lt >= lx) lt = -1;
  }
  void* w = nullptr;
  const int rcw = c->workspace(pair_bytes * (size_t)chunk, s, &w);
  if (rcw != FFTPDE_OK) return rcw;
  const SymParams sym = make_sym(kSymScale, nx, ny, 1.0, 1.0, 0.0, 0.0);
  const char* name = inverse ? (sizeof(T) == 4 ? "tangle_float" : "tangle_double")
                             : (sizeof(T) == 4 ? "untangle_float" : "untangle_double");
  for (long long p0 = 0; p0 < npairs; p0 += chunk) {
    const long long np = std::min<long long>(chunk, npairs - p0);
    const long long nrows = (long long)ny * np;
    const long long f0 = 2 * p0, nreal = std::min<long long>(2 * np, batch - f0);
    const size_t real_off = sizeof(T) * (size_t)(f0 * pts), half_off = sizeof(cx<T>) * (size_t)(f0 * hpts);
    HalfArgs<T> h{static_cast<cx<T>*>(w), nullptr, nx, ny, np, nreal, lt, ly};
    const double hbytes = (double)sizeof(cx<T>) * (double)(np * pts + nreal * hpts);
    int rc = FFTPDE_OK;
    if (!inverse) {
      h.half = static_cast<cx<T>*>(at<T>(out, half_off));
      rc = row_pass<T>(c, at<T>(in, real_off), w, lx, ly, nrows, false, 1.0, s, -1, lt, 1, 0, nreal);
      if (rc == FFTPDE_OK) rc = col_pass<T>(c, w, nullptr, w, nullptr, lx, ly, np, kColForward, sym, 1, s, lt);
      if (rc == FFTPDE_OK) {
        const hipError_t e = timed_launch(c, name, hbytes, s, [&] { return launch_untangle<T>(h, s); });
        if (e != hipSuccess) {
          set_last_error(name, e);
          rc = FFTPDE_EDEVICE;
        }
      }
    } else {
      h.half = static_cast<cx<T>*>(const_cast<void*>(at<T>(in, half_off)));
      const hipError_t e = timed_launch(c, name, hbytes, s, [&] { return launch_tangle<T>(h, s); });
      if (e != hipSuccess) {
        set_last_error(name, e);
        rc = FFTPDE_EDEVICE;
      }
      if (rc == FFTPDE_OK) rc = col_pass<T>(c, w, nullptr, w, nullptr, lx, ly, np, kColInverse, sym, 1, s, lt);
      if (rc == FFTPDE_OK)
        rc = row_pass<T>(c, w, at<T>(out, real_off), lx, ly, nrows, true, 1.0, s, lt, -1, 0, 1, nreal);
    }
    if (rc != FFTPDE_OK) return rc;
  }
  return FFTPDE_OK;
}

int run_half_transform(Context* c, int dtype, bool inverse, const void* in, void* out, int nx, int ny, int batch,
                       hipStream_t s) {
  return dtype == FFTPDE_R32 ? half_transform<float>(c, inverse, in, out, nx, ny, batch, s)
                             : half_transform<double>(c, inverse, in, out, nx, ny, batch, s);
}

size_t solve_scratch_per_field(Context* c, int dtype, int op, int nx, int ny, bool v0, bool v) {
  const int lx = ilog2(nx), ly = ilog2(ny);
  const size_t field = (dtype == FFTPDE_C64 ? 8 : 16) * (size_t)nx * ny;
  const bool two = op == FFTPDE_WAVE && (v0 || v);
  if (!two && c->small_variant(dtype, lx, ly)) return 0;  // one launch in LDS
  const ColVariant* cv = c->col_variant(dtype, ly, two ? 2 : 1);
  const int tiled_bytes = c->tiled_bytes_for(dtype, lx, ly);
  int lt = -1;
  if (tiled_bytes > 0 && cv) {
    const int b = dtype == FFTPDE_C64 ? 8 : 16;
    int bt = 0;
    while (b << (bt + 1) <= tiled_bytes) bt++;
    lt = bt > cv->logt ? bt : cv->logt;
    if (lt >= lx) lt = -1;
  }
  if (!two) return lt >= 0 ? field : 0;
  if (lt >= 0) return 2 * field;
  return (v0 && !v) ? field : 0;
}

int run_solve(Context* c, int dtype, int op, const void* in, const void* in2, void* out, void* out2, int nx, int ny,
              int batch, double lx, double ly, double coef, double t, hipStream_t s, const SolveScratch& sc) {
  const int sop = op == FFTPDE_POISSON ? kSymPoisson : op == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave;
  const SymParams sym = make_sym(sop, nx, ny, lx, ly, coef, t);
  if (dtype == FFTPDE_R32) return solve_real_pairs<float>(c, in, in2, out, out2, nx, ny, batch, sym, s);
  if (dtype == FFTPDE_R64) return solve_real_pairs<double>(c, in, in2, out, out2, nx, ny, batch, sym, s);
  if (op != FFTPDE_WAVE || (!in2 && !out2)) {
    const int r = dtype == FFTPDE_C64 ? small_pass<float>(c, in, out, nx, ny, batch, kColFwdMulInv, sym, s)
                                      : small_pass<double>(c, in, out, nx, ny, batch, kColFwdMulInv, sym, s);
    if (r != -100) return r;
    return dtype == FFTPDE_C64 ? solve_real_symbol<float>(c, in, out, nx, ny, batch, sym, s, sc)
                               : solve_real_symbol<double>(c, in, out, nx, ny, batch, sym, s, sc);
  }
  return dtype == FFTPDE_C64 ? solve_wave_two<float>(c, in, in2, out, out2, nx, ny, batch, sym, s, sc)
                             : solve_wave_two<double>(c, in, in2, out, out2, nx, ny, batch, sym, s, sc);
}

template <typename T>
static int materialize(Context* c, int kind, const void* F, const void* G, void* u, void* v, int nx, int ny, int batch,
                       double lx, double ly, double coef, double t, hipStream_t s) {
  const int lgx = ilog2(nx), lgy = ilog2(ny);
  const SymParams sym = make_sym(kind == FFTPDE_DIFFUSION ? kSymDiffusion : kSymWave, nx, ny, lx, ly, coef, t);
  const int nf = kind == FFTPDE_WAVE && (G || v) ? 2 : 1;
  return for_chunks<T>(c, nx, ny, batch, [&](long long, long long nb, size_t off) {
    const long long nrows = (long long)ny * nb;
    void* ub = at<T>(u, off);
    void* vb = at<T>(v, off);
    int rc = col_pass<T>(c, at<T>(F, off), nf == 2 ? at<T>(G, off) : nullptr, ub, nf == 2 ? vb : nullptr, lgx, lgy,
                         nb, kColMulInv, sym, nf, s);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, ub, ub, lgx, lgy, nrows, true, 1.0, s);
    if (rc == FFTPDE_OK && vb) rc = row_pass<T>(c, vb, vb, lgx, lgy, nrows, true, 1.0, s);
    return rc;
  });
}

int run_materialize(Context* c, int dtype, int kind, const void* F, const void* G, void* u, void* v, int nx, int ny,
                    int batch, double lx, double ly, double coef, double t, hipStream_t s) {
  return dtype == FFTPDE_C64 ? materialize<float>(c, kind, F, G, u, v, nx, ny, batch, lx, ly, coef, t, s)
                             : materialize<double>(c, kind, F, G, u, v, nx, ny, batch, lx, ly, coef, t, s);
}

template <typename T>
static hipError_t diag_t(int kind, const void* F, const void* G, int nx, int ny, int batch, double lx, double ly,
                         double coef, long long n0, double dt, int nt, double* scratch, double* out, hipStream_t s) {
  DiagArgs<T> a{static_cast<const cx<T>*>(F), static_cast<const cx<T>*>(G), kind == FFTPDE_DIFFUSION ? 0 : 1,
                ilog2(nx), ilog2(ny), 2.0 * kPi / lx, 2.0 * kPi / ly, coef, n0, dt, nt, (lx / nx) * (ly / ny)};
  return launch_diag<T>(a, batch, scratch, out, s);
}

int run_diag(Context* c, int dtype, int kind, const void* F, const void* G, int nx, int ny, int batch, double lx,
             double ly, double coef, long long n0, double dt, int nt, double* scratch, double* out, hipStream_t s) {
  const double bytes = (double)(dtype == FFTPDE_C64 ? 8 : 16) * nx * ny * batch * (G ? 2 : 1);
  hipError_t e = timed_launch(c, dtype == FFTPDE_C64 ? "diag_float" : "diag_double", bytes, s, [&] {
    return dtype == FFTPDE_C64 ? diag_t<float>(kind, F, G, nx, ny, batch, lx, ly, coef, n0, dt, nt, scratch, out, s)
                               : diag_t<double>(kind, F, G, nx, ny, batch, lx, ly, coef, n0, dt, nt, scratch, out, s);
  });
  if (e != hipSuccess) {
    set_last_error("diagnostics", e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

template int row_pass<float>(Context*, const void*, void*, int, int, long long, bool, double, hipStream_t, int, int,
                             int, int, long long);
template int row_pass<double>(Context*, const void*, void*, int, int, long long, bool, double, hipStream_t, int,
                              int, int, int, long long);
template int col_pass<float>(Context*, const void*, const void*, void*, void*, int, int, long long, int,
                             const SymParams&, int, hipStream_t, int);
template int col_pass<double>(Context*, const void*, const void*, void*, void*, int, int, long long, int,
                              const SymParams&, int, hipStream_t, int);

}  // namespace fftpde
