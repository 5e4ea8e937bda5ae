// capi.cpp -- the C ABI of libfftpde.so (declared in include/fftpde.h):
// argument checks, twiddle tables, plan choice and the launch sequences of
// the transforms and solves.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fftpde.h"
#include "context.hpp"
#include "kernels.hpp"

using namespace fftpde;

// ---------------------------------------------------------------------------
// twiddle table: w^e = exp(-2 pi i e / 4096), FP64, by octant symmetry
// ---------------------------------------------------------------------------
namespace {

constexpr int kTw = 1 << kTwLog;
constexpr double kPi = 3.14159265358979323846264338327950288;

// cos and sin of 2 pi e / kTw for 0 <= e <= kTw, from libm on [0, pi/4] and
// exact symmetries elsewhere, so that e.g. w^{1024} is exactly -i and the
// two components of w^{512} are equal.
void cos_sin_turn(int e, double& c, double& s) {
  const int q = kTw / 4, o = kTw / 8;
  if (e <= o) {
    const double a = 2.0 * kPi * (double)e / (double)kTw;
    c = std::cos(a);
    s = std::sin(a);
  } else if (e <= q) {  // theta = pi/2 - phi
    double c2, s2;
    cos_sin_turn(q - e, c2, s2);
    c = s2;
    s = c2;
  } else if (e <= 2 * q) {  // theta = pi - phi
    double c2, s2;
    cos_sin_turn(2 * q - e, c2, s2);
    c = -c2;
    s = s2;
  } else {  // theta = 2 pi - phi
    double c2, s2;
    cos_sin_turn(kTw - e, c2, s2);
    c = c2;
    s = -s2;
  }
}

thread_local char g_last_error[256];

void set_error(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool pow2_side(int n) { return n >= 2 && n <= 4096 && (n & (n - 1)) == 0; }
int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) l++;
  return l;
}
bool aligned(const void* p, int dtype) {
  const uintptr_t a = dtype == FFTPDE_C64 ? 8 : 16;
  return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace fftpde {

const RowVariant* Context::row_variant(int dtype, int logn) const {
  const int k = plan_key(dtype, 0, logn, 1);
  if (row_choice[k]) return row_choice[k];
  int n = 0;
  const RowVariant* t = dtype == FFTPDE_C64 ? row_variants_f32(&n) : row_variants_f64(&n);
  for (int i = 0; i < n; i++)
    if (t[i].logn == logn) return &t[i];
  return nullptr;
}

const ColVariant* Context::col_variant(int dtype, int logn, int nf) const {
  const int k = plan_key(dtype, 1, logn, nf);
  if (col_choice[k]) return col_choice[k];
  int n = 0;
  const ColVariant* t = dtype == FFTPDE_C64 ? (nf == 1 ? col_variants_f32_nf1(&n) : col_variants_f32_nf2(&n))
                                            : (nf == 1 ? col_variants_f64_nf1(&n) : col_variants_f64_nf2(&n));
  for (int i = 0; i < n; i++)
    if (t[i].logn == logn) return &t[i];
  return nullptr;
}

int Context::workspace(size_t bytes, void** p) {
  if (bytes <= work_bytes) {
    *p = work;
    return FFTPDE_OK;
  }
  if (work) {
    // stream-ordered users may still read the old buffer
    (void)hipDeviceSynchronize();
    (void)hipFree(work);
    work = nullptr;
    work_bytes = 0;
  }
  hipError_t e = hipMalloc(&work, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc(workspace)", e);
    work = nullptr;
    return FFTPDE_ENOMEM;
  }
  work_bytes = bytes;
  *p = work;
  return FFTPDE_OK;
}

void set_last_error(const char* what, hipError_t e) { set_error(what, e); }

hipEvent_t Context::take_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

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

}  // namespace fftpde

extern "C" {

const char* fftpde_version(void) { return "fftpde 0.1.0 (gfx950)"; }

const char* fftpde_strerror(int status) {
  switch (status) {
    case FFTPDE_OK: return "ok";
    case FFTPDE_PENDING: return "pending";
    case FFTPDE_EINVAL: return "invalid argument";
    case FFTPDE_ENOMEM: return "out of memory";
    case FFTPDE_EDEVICE: return "device error";
    case FFTPDE_EBUDGET: return "request exceeds the memory budget";
    case FFTPDE_ENOTFOUND: return "not found";
    case FFTPDE_ECANCELED: return "cancelled";
    case FFTPDE_ETIMEOUT: return "deadline exceeded";
    default: return "unknown status";
  }
}

const char* fftpde_last_error(void) { return g_last_error; }

int fftpde_create(fftpde_ctx** out, int device) {
  if (!out) return FFTPDE_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FFTPDE_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return FFTPDE_EDEVICE;
  Context* c = new (std::nothrow) Context();
  if (!c) return FFTPDE_ENOMEM;
  c->device = device;
  std::vector<cx<double>> t64(kTw);
  std::vector<cx<float>> t32(kTw);
  for (int e = 0; e < kTw; e++) {
    double cs, sn;
    cos_sin_turn(e, cs, sn);
    t64[e] = {cs, -sn};
    t32[e] = {(float)cs, (float)(-sn)};
  }
  hipError_t e1 = hipMalloc(&c->tw64, sizeof(cx<double>) * kTw);
  hipError_t e2 = hipMalloc(&c->tw32, sizeof(cx<float>) * kTw);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("hipMalloc(twiddles)", e1 != hipSuccess ? e1 : e2);
    if (e1 == hipSuccess) (void)hipFree(c->tw64);
    if (e2 == hipSuccess) (void)hipFree(c->tw32);
    delete c;
    return FFTPDE_ENOMEM;
  }
  e1 = hipMemcpy(c->tw64, t64.data(), sizeof(cx<double>) * kTw, hipMemcpyHostToDevice);
  e2 = hipMemcpy(c->tw32, t32.data(), sizeof(cx<float>) * kTw, hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("hipMemcpy(twiddles)", e1 != hipSuccess ? e1 : e2);
    (void)hipFree(c->tw64);
    (void)hipFree(c->tw32);
    delete c;
    return FFTPDE_EDEVICE;
  }
  *out = reinterpret_cast<fftpde_ctx*>(c);
  return FFTPDE_OK;
}

int fftpde_profile(fftpde_ctx* ctx, int enable) {
  if (!ctx) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  for (auto& t : c->timed) {
    c->event_pool.push_back(t.start);
    c->event_pool.push_back(t.stop);
  }
  c->timed.clear();
  c->profiling = enable != 0;
  return FFTPDE_OK;
}

int fftpde_profile_read(fftpde_ctx* ctx, char* buf, size_t cap, size_t* needed) {
  if (!ctx || (!buf && cap)) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  struct Agg {
    const char* name;
    long long count;
    double ms, bytes;
  };
  std::vector<Agg> agg;
  for (auto& t : c->timed) {
    if (hipEventSynchronize(t.stop) != hipSuccess) return FFTPDE_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) return FFTPDE_EDEVICE;
    size_t i = 0;
    while (i < agg.size() && std::strcmp(agg[i].name, t.name) != 0) i++;
    if (i == agg.size()) agg.push_back({t.name, 0, 0.0, 0.0});
    agg[i].count++;
    agg[i].ms += ms;
    agg[i].bytes += t.bytes;
  }
  std::string out = "[";
  for (size_t i = 0; i < agg.size(); i++) {
    char line[256];
    std::snprintf(line, sizeof(line), "%s{\"kernel\": \"%s\", \"launches\": %lld, \"total_ms\": %.6f, \"bytes\": %.0f}",
                  i ? ", " : "", agg[i].name, agg[i].count, agg[i].ms, agg[i].bytes);
    out += line;
  }
  out += "]";
  if (needed) *needed = out.size() + 1;
  if (cap < out.size() + 1) return cap ? FFTPDE_ENOMEM : FFTPDE_OK;
  std::memcpy(buf, out.c_str(), out.size() + 1);
  return FFTPDE_OK;
}

int fftpde_destroy(fftpde_ctx* ctx) {
  if (!ctx) return FFTPDE_OK;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  if (c->tw64) (void)hipFree(c->tw64);
  if (c->tw32) (void)hipFree(c->tw32);
  if (c->work) (void)hipFree(c->work);
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
  return FFTPDE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
namespace fftpde {

template <typename T>
static const cx<T>* twiddles(const Context* c) {
  if constexpr (sizeof(T) == 4) return c->tw32;
  else return c->tw64;
}

template <typename T>
int row_pass(Context* c, const void* in, void* out, int lognx, long long nrows, bool inverse, double scale,
             hipStream_t s) {
  const RowVariant* v = c->row_variant(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, lognx);
  if (!v) return FFTPDE_EINVAL;
  RowArgs<T> a{static_cast<const cx<T>*>(in), static_cast<cx<T>*>(out), twiddles<T>(c), nrows, inverse ? 1 : 0,
               T(scale)};
  const double bytes = 2.0 * sizeof(cx<T>) * (double)nrows * (double)(1 << lognx);
  hipError_t e = timed_launch(c, v->name, bytes, s, [&] { return v->launch(&a, nrows, s); });
  if (e != hipSuccess) {
    set_last_error(v->name, e);
    return FFTPDE_EDEVICE;
  }
  return FFTPDE_OK;
}

template <typename T>
int col_pass(Context* c, const void* in0, const void* in1, void* out0, void* out1, int lognx, int logny,
             long long batch, int mode, const SymParams& sym, int nf, hipStream_t s) {
  const ColVariant* v = c->col_variant(sizeof(T) == 4 ? FFTPDE_C64 : FFTPDE_C128, logny, nf);
  if (!v) return FFTPDE_EINVAL;
  ColArgs<T> a{static_cast<const cx<T>*>(in0), static_cast<const cx<T>*>(in1), static_cast<cx<T>*>(out0),
               static_cast<cx<T>*>(out1), twiddles<T>(c), batch << lognx, lognx, mode, sym};
  const double field = sizeof(cx<T>) * (double)batch * (double)(1ll << (lognx + logny));
  const double bytes = field * ((in0 ? 1 : 0) + (in1 ? 1 : 0) + (out0 ? 1 : 0) + (out1 ? 1 : 0));
  hipError_t e = timed_launch(c, v->name, bytes, s, [&] { return v->launch(&a, batch << lognx, s); });
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
  }
  return p;
}

template <typename T>
int transform(Context* c, const void* in, void* out, int nx, int ny, int batch, bool inverse, hipStream_t s) {
  const int lx = ilog2(nx), ly = ilog2(ny);
  SymParams sym = make_sym(kSymScale, nx, ny, 1.0, 1.0, 0.0, 0.0);
  int rc;
  if (!inverse) {
    rc = row_pass<T>(c, in, out, lx, (long long)ny * batch, false, 1.0, s);
    if (rc == FFTPDE_OK) rc = col_pass<T>(c, out, nullptr, out, nullptr, lx, ly, batch, kColForward, sym, 1, s);
  } else {
    rc = col_pass<T>(c, in, nullptr, out, nullptr, lx, ly, batch, kColInverse, sym, 1, s);
    if (rc == FFTPDE_OK) rc = row_pass<T>(c, out, out, lx, (long long)ny * batch, true, 1.0, s);
  }
  return rc;
}

// forward rows -> fused column pass -> inverse rows, for one real symbol
template <typename T>
int solve_real_symbol(Context* c, const void* in, void* out, int nx, int ny, int batch, const SymParams& sym,
                      hipStream_t s) {
  const int lx = ilog2(nx), ly = ilog2(ny);
  const long long nrows = (long long)ny * batch;
  int rc = row_pass<T>(c, in, out, lx, nrows, false, 1.0, s);
  if (rc == FFTPDE_OK) rc = col_pass<T>(c, out, nullptr, out, nullptr, lx, ly, batch, kColFwdMulInv, sym, 1, s);
  if (rc == FFTPDE_OK) rc = row_pass<T>(c, out, out, lx, nrows, true, 1.0, s);
  return rc;
}

template <typename T>
int solve_wave_two(Context* c, const void* u0, const void* v0, void* u, void* v, int nx, int ny, int batch,
                   const SymParams& sym, hipStream_t s) {
  const int lx = ilog2(nx), ly = ilog2(ny);
  const long long nrows = (long long)ny * batch;
  void* vbuf = v;
  if (v0 && !v) {
    const size_t bytes = sizeof(cx<T>) * (size_t)nx * ny * batch;
    int rc = c->workspace(bytes, &vbuf);
    if (rc != FFTPDE_OK) return rc;
  }
  int rc = row_pass<T>(c, u0, u, lx, nrows, false, 1.0, s);
  if (rc == FFTPDE_OK && v0) rc = row_pass<T>(c, v0, vbuf, lx, nrows, false, 1.0, s);
  if (rc == FFTPDE_OK)
    rc = col_pass<T>(c, u, v0 ? vbuf : nullptr, u, v, lx, ly, batch, kColFwdMulInv, sym, 2, s);
  if (rc == FFTPDE_OK) rc = row_pass<T>(c, u, u, lx, nrows, true, 1.0, s);
  if (rc == FFTPDE_OK && v) rc = row_pass<T>(c, v, v, lx, nrows, true, 1.0, s);
  return rc;
}

}  // namespace fftpde

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
namespace {

int check_common(fftpde_ctx* ctx, int nx, int ny, int batch, int dtype) {
  if (!ctx) return FFTPDE_EINVAL;
  if (!pow2_side(nx) || !pow2_side(ny) || batch < 1) return FFTPDE_EINVAL;
  if (dtype != FFTPDE_C64 && dtype != FFTPDE_C128) return FFTPDE_EINVAL;
  return FFTPDE_OK;
}

int check_field(const void* p, int dtype) { return (p && aligned(p, dtype)) ? FFTPDE_OK : FFTPDE_EINVAL; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

int fft2d_forward(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
                  fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(out, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == FFTPDE_C64 ? transform<float>(c, in, out, nx, ny, batch, false, s)
                             : transform<double>(c, in, out, nx, ny, batch, false, s);
}

int fft2d_inverse(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
                  fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(out, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == FFTPDE_C64 ? transform<float>(c, in, out, nx, ny, batch, true, s)
                             : transform<double>(c, in, out, nx, ny, batch, true, s);
}

int solve_poisson(fftpde_ctx* ctx, const void* s_in, void* u, int nx, int ny, int batch, double lx, double ly,
                  int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(s_in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  const SymParams sym = make_sym(kSymPoisson, nx, ny, lx, ly, 0.0, 0.0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == FFTPDE_C64 ? solve_real_symbol<float>(c, s_in, u, nx, ny, batch, sym, s)
                             : solve_real_symbol<double>(c, s_in, u, nx, ny, batch, sym, s);
}

int solve_diffusion(fftpde_ctx* ctx, const void* u0, void* u, int nx, int ny, int batch, double lx, double ly,
                    double kappa, double t, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u0, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(kappa) && kappa >= 0.0 && std::isfinite(t) && t >= 0.0))
    rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  const SymParams sym = make_sym(kSymDiffusion, nx, ny, lx, ly, kappa, t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == FFTPDE_C64 ? solve_real_symbol<float>(c, u0, u, nx, ny, batch, sym, s)
                             : solve_real_symbol<double>(c, u0, u, nx, ny, batch, sym, s);
}

int solve_wave(fftpde_ctx* ctx, const void* u0, const void* v0, void* u, void* v, int nx, int ny, int batch,
               double lx, double ly, double c_speed, double t, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u0, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && v0) rc = check_field(v0, dtype);
  if (rc == FFTPDE_OK && v) rc = check_field(v, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(c_speed) && c_speed >= 0.0 && std::isfinite(t))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && v && (v == u || v == u0)) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && v0 && (v0 == u)) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  const SymParams sym = make_sym(kSymWave, nx, ny, lx, ly, c_speed, t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!v0 && !v)
    return dtype == FFTPDE_C64 ? solve_real_symbol<float>(c, u0, u, nx, ny, batch, sym, s)
                               : solve_real_symbol<double>(c, u0, u, nx, ny, batch, sym, s);
  return dtype == FFTPDE_C64 ? solve_wave_two<float>(c, u0, v0, u, v, nx, ny, batch, sym, s)
                             : solve_wave_two<double>(c, u0, v0, u, v, nx, ny, batch, sym, s);
}

}  // extern "C"
