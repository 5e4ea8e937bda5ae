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
#include "noalloc.hpp"
#include "rk4.hpp"
#include "solve.hpp"

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
  const uintptr_t a = dtype == FFTPDE_R32 ? 4 : (dtype == FFTPDE_C64 || dtype == FFTPDE_R64) ? 8 : 16;
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
  const ColVariant* t = dtype == FFTPDE_C64
                           ? (nf == 1 ? col_variants_f32_nf1(&n) : nf == 2 ? col_variants_f32_nf2(&n) : col_variants_f32_nf3(&n))
                           : (nf == 1 ? col_variants_f64_nf1(&n) : nf == 2 ? col_variants_f64_nf2(&n) : col_variants_f64_nf3(&n));
  for (int i = 0; i < n; i++)
    if (t[i].logn == logn) return &t[i];
  return nullptr;
}

const SmallVariant* Context::small_variant(int dtype, int lognx, int logny) const {
  if (!use_small) return nullptr;
  int n = 0;
  const SmallVariant* t = dtype == FFTPDE_C64 ? small_variants_f32(&n) : small_variants_f64(&n);
  for (int i = 0; i < n; i++)
    if (t[i].lx == lognx && t[i].ly == logny) return &t[i];
  return nullptr;
}

int Context::workspace(size_t bytes, hipStream_t s, void** p) {
  Work& w = work[static_cast<void*>(s)];
  if (bytes <= w.bytes) {
    *p = w.p;
    return FFTPDE_OK;
  }
  if (w.p) {
    // work already enqueued on this stream may still use the old buffer
    (void)hipStreamSynchronize(s);
    (void)hipFree(w.p);
    w.p = nullptr;
    w.bytes = 0;
  }
  hipError_t e = hipMalloc(&w.p, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc(workspace)", e);
    w.p = nullptr;
    return FFTPDE_ENOMEM;
  }
  w.bytes = bytes;
  *p = w.p;
  return FFTPDE_OK;
}

void set_last_error(const char* what, hipError_t e) { set_error(what, e); }

long long Context::max_blocks(const void* variant, OccFn occ) {
  auto it = occupancy.find(variant);
  int per = 0;
  if (it != occupancy.end()) {
    per = it->second;
  } else {
    per = occ ? occ() : 0;
    occupancy[variant] = per;
  }
  if (per <= 0 || num_cus <= 0) return 0;  // unknown: one workgroup per tile
  return (long long)per * num_cus;
}

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
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cus = prop.multiProcessorCount;
  std::vector<cx<double>> t64(kTw);
  std::vector<cx<float>> t32(kTw);
  for (int e = 0; e < kTw; e++) {
    double cs, sn;
    cos_sin_turn(e, cs, sn);
    t64[e] = {cs, -sn};
    t32[e] = {(float)cs, (float)(-sn)};
  }
  // stage tables: copies of table entries, so every twiddle source gives the
  // same values
  for (int logn = 1; logn <= 12; logn++)
    for (int lr = 1; lr <= Context::kStageMaxLr; lr++)
      for (int rev = 0; rev < 2; rev++) {
        c->stage_tw_at[logn][lr][rev] = (int)t64.size();
        const int n = stage_tw_entries(logn, lr, rev != 0);
        for (int i = 0; i < n; i++) {
          const int e = stage_tw_exponent(logn, lr, rev != 0, i);
          const cx<double> w64 = t64[e];
          const cx<float> w32 = t32[e];
          t64.push_back(w64);
          t32.push_back(w32);
        }
      }
  const size_t ntw = t64.size();
  hipError_t e1 = hipMalloc(&c->tw64, sizeof(cx<double>) * ntw);
  hipError_t e2 = hipMalloc(&c->tw32, sizeof(cx<float>) * ntw);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("hipMalloc(twiddles)", e1 != hipSuccess ? e1 : e2);
    if (e1 == hipSuccess) (void)hipFree(c->tw64);
    if (e2 == hipSuccess) (void)hipFree(c->tw32);
    delete c;
    return FFTPDE_ENOMEM;
  }
  e1 = hipMemcpy(c->tw64, t64.data(), sizeof(cx<double>) * ntw, hipMemcpyHostToDevice);
  e2 = hipMemcpy(c->tw32, t32.data(), sizeof(cx<float>) * ntw, hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("hipMemcpy(twiddles)", e1 != hipSuccess ? e1 : e2);
    (void)hipFree(c->tw64);
    (void)hipFree(c->tw32);
    delete c;
    return FFTPDE_EDEVICE;
  }
  // this device's copy of solve_wave_noalloc's fixed scratch (once per
  // device); a failure here only disables that entry point, which then
  // reports FFTPDE_EDEVICE
  (void)noalloc_bind(device);
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

}  // extern "C"

namespace {

struct VariantRef {
  const char* name;
  int dtype, pass, logn, nf;
  const RowVariant* row;
  const ColVariant* col;
};

template <class F>
void for_each_variant(F&& f) {
  int n = 0;
  const RowVariant* r32 = row_variants_f32(&n);
  for (int i = 0; i < n; i++) f(VariantRef{r32[i].name, FFTPDE_C64, 0, r32[i].logn, 1, &r32[i], nullptr});
  const RowVariant* r64 = row_variants_f64(&n);
  for (int i = 0; i < n; i++) f(VariantRef{r64[i].name, FFTPDE_C128, 0, r64[i].logn, 1, &r64[i], nullptr});
  const ColVariant* (*tabs[6])(int*) = {col_variants_f32_nf1, col_variants_f32_nf2, col_variants_f32_nf3,
                                        col_variants_f64_nf1, col_variants_f64_nf2, col_variants_f64_nf3};
  for (int k = 0; k < 6; k++) {
    const ColVariant* t = tabs[k](&n);
    for (int i = 0; i < n; i++)
      f(VariantRef{t[i].name, k < 3 ? FFTPDE_C64 : FFTPDE_C128, 1, t[i].logn, t[i].nf, nullptr, &t[i]});
  }
}

int copy_out(const std::string& text, char* buf, size_t cap, size_t* needed) {
  if (needed) *needed = text.size() + 1;
  if (!buf) return cap ? FFTPDE_EINVAL : FFTPDE_OK;
  if (cap < text.size() + 1) return FFTPDE_ENOMEM;
  std::memcpy(buf, text.c_str(), text.size() + 1);
  return FFTPDE_OK;
}

}  // namespace

extern "C" {

int fftpde_plan_variants(fftpde_ctx* ctx, char* buf, size_t cap, size_t* needed) {
  if (!ctx) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  std::string out = "[";
  bool first = true;
  for_each_variant([&](const VariantRef& v) {
    const int k = plan_key(v.dtype, v.pass, v.logn, v.nf);
    const bool chosen = v.row ? (c->row_variant(v.dtype, v.logn) == v.row)
                              : (c->col_variant(v.dtype, v.logn, v.nf) == v.col);
    (void)k;
    char line[384];
    if (v.row)
      std::snprintf(line, sizeof(line),
                    "%s{\"name\": \"%s\", \"dtype\": %d, \"pass\": \"row\", \"logn\": %d, \"fields\": 1, "
                    "\"e\": %d, \"threads\": %d, \"lines\": %d, \"prefetch\": %d, \"lds\": %d, \"active\": %d}",
                    first ? "" : ", ", v.name, v.dtype, v.logn, v.row->e, v.row->th, v.row->lines, v.row->pf,
                    v.row->lds_bytes, chosen ? 1 : 0);
    else
      std::snprintf(line, sizeof(line),
                    "%s{\"name\": \"%s\", \"dtype\": %d, \"pass\": \"col\", \"logn\": %d, \"fields\": %d, "
                    "\"e\": %d, \"threads\": %d, \"cols\": %d, \"split\": %d, \"prefetch\": %d, \"lds\": %d, "
                    "\"active\": %d}",
                    first ? "" : ", ", v.name, v.dtype, v.logn, v.nf, v.col->e, v.col->th, 1 << v.col->logt,
                    v.col->split, v.col->pf, v.col->lds_bytes, chosen ? 1 : 0);
    out += line;
    first = false;
  });
  for (int d = 0; d < 2; d++) {
    int cnt = 0;
    const SmallVariant* t = d == 0 ? small_variants_f32(&cnt) : small_variants_f64(&cnt);
    for (int i = 0; i < cnt; i++) {
      char line[256];
      std::snprintf(line, sizeof(line),
                    ", {\"name\": \"%s\", \"dtype\": %d, \"pass\": \"small\", \"lognx\": %d, \"logny\": %d, "
                    "\"threads\": %d, \"active\": %d}",
                    t[i].name, d, t[i].lx, t[i].ly, t[i].th, c->use_small ? 1 : 0);
      out += line;
    }
  }
  out += "]";
  return copy_out(out, buf, cap, needed);
}

int fftpde_plan_small(fftpde_ctx* ctx, int enable) {
  if (!ctx) return FFTPDE_EINVAL;
  reinterpret_cast<Context*>(ctx)->use_small = enable != 0;
  return FFTPDE_OK;
}

int fftpde_plan_tiled(fftpde_ctx* ctx, int block_bytes) {
  if (!ctx || block_bytes < 0 || block_bytes > 65536 || (block_bytes & (block_bytes - 1))) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  c->tiled_bytes = block_bytes;
  c->tiled_for.clear();  // an explicit setting overrides tuned ones
  return FFTPDE_OK;
}

int fftpde_plan_chunk(fftpde_ctx* ctx, long long bytes) {
  if (!ctx || bytes < 0) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  c->chunk_bytes = bytes;
  c->chunk_for.clear();  // an explicit setting overrides tuned ones
  return FFTPDE_OK;
}

int fftpde_plan_select(fftpde_ctx* ctx, const char* name) {
  if (!ctx) return FFTPDE_EINVAL;
  Context* c = reinterpret_cast<Context*>(ctx);
  if (!name || !*name) {
    c->tiled_for.clear();
    c->chunk_for.clear();
    for (int k = 0; k < kPlanSlots; k++) {
      c->row_choice[k] = nullptr;
      c->col_choice[k] = nullptr;
    }
    return FFTPDE_OK;
  }
  int rc = FFTPDE_ENOTFOUND;
  for_each_variant([&](const VariantRef& v) {
    if (rc == FFTPDE_OK || std::strcmp(v.name, name) != 0) return;
    const int k = plan_key(v.dtype, v.pass, v.logn, v.nf);
    if (v.row) c->row_choice[k] = v.row;
    else c->col_choice[k] = v.col;
    rc = FFTPDE_OK;
  });
  return rc;
}

int fftpde_destroy(fftpde_ctx* ctx) {
  if (!ctx) return FFTPDE_OK;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  if (c->tw64) (void)hipFree(c->tw64);
  if (c->tw32) (void)hipFree(c->tw32);
  for (auto& w : c->work)
    if (w.second.p) (void)hipFree(w.second.p);
  for (auto& t : c->mr_tw) (void)hipFree(t.second.f64);
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
// entry points
// ---------------------------------------------------------------------------
namespace {

// mixed_ok: sides may also be 7-smooth (the mixed-radix path, with real
// dtypes where real_ok).
int check_common(fftpde_ctx* ctx, int nx, int ny, int batch, int dtype, bool real_ok = false, bool mixed_ok = false) {
  if (!ctx || batch < 1) return FFTPDE_EINVAL;
  const bool real = dtype == FFTPDE_R32 || dtype == FFTPDE_R64;
  if (dtype != FFTPDE_C64 && dtype != FFTPDE_C128 && !(real_ok && real)) return FFTPDE_EINVAL;
  if (pow2_side(nx) && pow2_side(ny)) return FFTPDE_OK;
  if (mixed_ok && mixed_side(nx) && mixed_side(ny)) return FFTPDE_OK;
  return FFTPDE_EINVAL;
}

bool is_mixed(int nx, int ny) { return !pow2_side(nx) || !pow2_side(ny); }


int check_field(const void* p, int dtype) { return (p && aligned(p, dtype)) ? FFTPDE_OK : FFTPDE_EINVAL; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// real fields (R32 / R64) <-> half spectra of the matching complex dtype
int half_checks(fftpde_ctx* ctx, const void* real, const void* half, int nx, int ny, int batch, int dtype) {
  if (dtype != FFTPDE_R32 && dtype != FFTPDE_R64) return FFTPDE_EINVAL;
  int rc = check_common(ctx, nx, ny, batch, dtype, true, true);
  if (rc == FFTPDE_OK) rc = check_field(real, dtype);
  if (rc == FFTPDE_OK) rc = check_field(half, dtype == FFTPDE_R32 ? FFTPDE_C64 : FFTPDE_C128);
  if (rc != FFTPDE_OK) return rc;
  const size_t elem = dtype == FFTPDE_R32 ? 4 : 8;
  const uintptr_t r0 = reinterpret_cast<uintptr_t>(real), h0 = reinterpret_cast<uintptr_t>(half);
  const uintptr_t r1 = r0 + elem * (size_t)nx * ny * batch, h1 = h0 + 2 * elem * (size_t)(nx / 2 + 1) * ny * batch;
  return (r0 < h1 && h0 < r1) ? FFTPDE_EINVAL : FFTPDE_OK;  // no overlap
}

}  // namespace

extern "C" {

int fft2d_forward(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
                  fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, false, true);
  if (rc == FFTPDE_OK) rc = check_field(in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(out, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_transform(c, dtype, false, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
  return run_transform(c, dtype, false, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
}

int fft2d_inverse(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
                  fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, false, true);
  if (rc == FFTPDE_OK) rc = check_field(in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(out, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_transform(c, dtype, true, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
  return run_transform(c, dtype, true, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
}

int fft2d_r2c(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
              fftpde_stream stream) {
  const int rc = half_checks(ctx, in, out, nx, ny, batch, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_half(c, dtype, false, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
  return run_half_transform(c, dtype, false, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
}

int fft2d_c2r(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int batch, int dtype,
              fftpde_stream stream) {
  const int rc = half_checks(ctx, out, in, nx, ny, batch, dtype);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_half(c, dtype, true, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
  return run_half_transform(c, dtype, true, in, out, nx, ny, batch, static_cast<hipStream_t>(stream));
}

int solve_poisson(fftpde_ctx* ctx, const void* s_in, void* u, int nx, int ny, int batch, double lx, double ly,
                  int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, true, true);
  if (rc == FFTPDE_OK) rc = check_field(s_in, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_solve(c, dtype, FFTPDE_POISSON, s_in, nullptr, u, nullptr, nx, ny, batch, lx, ly, 0.0, 0.0,
                           static_cast<hipStream_t>(stream));
  return run_solve(c, dtype, FFTPDE_POISSON, s_in, nullptr, u, nullptr, nx, ny, batch, lx, ly, 0.0, 0.0,
                   static_cast<hipStream_t>(stream));
}

int solve_diffusion(fftpde_ctx* ctx, const void* u0, void* u, int nx, int ny, int batch, double lx, double ly,
                    double kappa, double t, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, true, true);
  if (rc == FFTPDE_OK) rc = check_field(u0, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(kappa) && kappa >= 0.0 && std::isfinite(t) && t >= 0.0))
    rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  if (is_mixed(nx, ny))
    return run_mixed_solve(c, dtype, FFTPDE_DIFFUSION, u0, nullptr, u, nullptr, nx, ny, batch, lx, ly, kappa, t,
                           static_cast<hipStream_t>(stream));
  return run_solve(c, dtype, FFTPDE_DIFFUSION, u0, nullptr, u, nullptr, nx, ny, batch, lx, ly, kappa, t,
                   static_cast<hipStream_t>(stream));
}

int solve_diffusion_source(fftpde_ctx* ctx, const void* f, const void* src, void* u, int nx, int ny, int batch,
                           double lx, double ly, double kappa, double t, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, true);
  if (rc == FFTPDE_OK) rc = check_field(f, dtype);
  if (rc == FFTPDE_OK) rc = check_field(src, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(kappa) && kappa >= 0.0 && std::isfinite(t) && t >= 0.0))
    rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_source(c, dtype, FFTPDE_DIFFUSION, f, nullptr, src, u, nullptr, nx, ny, batch, lx, ly, kappa, t,
                    static_cast<hipStream_t>(stream));
}

int solve_wave_source(fftpde_ctx* ctx, const void* f, const void* g0, const void* src, void* u, void* v, int nx,
                      int ny, int batch, double lx, double ly, double c_speed, double t, int dtype,
                      fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, true);
  if (rc == FFTPDE_OK) rc = check_field(f, dtype);
  if (rc == FFTPDE_OK && g0) rc = check_field(g0, dtype);
  if (rc == FFTPDE_OK) rc = check_field(src, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && v) rc = check_field(v, dtype);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(c_speed) && c_speed >= 0.0 && std::isfinite(t))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && v && v == u) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_source(c, dtype, FFTPDE_WAVE, f, g0, src, u, v, nx, ny, batch, lx, ly, c_speed, t,
                    static_cast<hipStream_t>(stream));
}

namespace {
int check3d(fftpde_ctx* ctx, int nx, int ny, int nz, int batch, int dtype, const void* a, const void* b) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK && (!pow2_side(nz) || (long long)nx * ny > (1ll << 24))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK) rc = check_field(a, dtype);
  if (rc == FFTPDE_OK) rc = check_field(b, dtype);
  return rc;
}
}  // namespace

int fft3d_forward(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int nz, int batch, int dtype,
                  fftpde_stream stream) {
  const int rc = check3d(ctx, nx, ny, nz, batch, dtype, in, out);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_transform3d(c, dtype, false, in, out, nx, ny, nz, batch, static_cast<hipStream_t>(stream));
}

int fft3d_inverse(fftpde_ctx* ctx, const void* in, void* out, int nx, int ny, int nz, int batch, int dtype,
                  fftpde_stream stream) {
  const int rc = check3d(ctx, nx, ny, nz, batch, dtype, in, out);
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_transform3d(c, dtype, true, in, out, nx, ny, nz, batch, static_cast<hipStream_t>(stream));
}

int solve_poisson_3d(fftpde_ctx* ctx, const void* s_in, void* u, int nx, int ny, int nz, int batch, double lx,
                     double ly, double lz, int dtype, fftpde_stream stream) {
  int rc = check3d(ctx, nx, ny, nz, batch, dtype, s_in, u);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly) && finite_pos(lz))) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_solve3d(c, dtype, FFTPDE_POISSON, s_in, u, nx, ny, nz, batch, lx, ly, lz, 0.0, 0.0,
                     static_cast<hipStream_t>(stream));
}

int solve_diffusion_3d(fftpde_ctx* ctx, const void* u0, void* u, int nx, int ny, int nz, int batch, double lx,
                       double ly, double lz, double kappa, double t, int dtype, fftpde_stream stream) {
  int rc = check3d(ctx, nx, ny, nz, batch, dtype, u0, u);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly) && finite_pos(lz))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(kappa) && kappa >= 0.0 && std::isfinite(t) && t >= 0.0)) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_solve3d(c, dtype, FFTPDE_DIFFUSION, u0, u, nx, ny, nz, batch, lx, ly, lz, kappa, t,
                     static_cast<hipStream_t>(stream));
}

int solve_wave_3d(fftpde_ctx* ctx, const void* u0, void* u, int nx, int ny, int nz, int batch, double lx, double ly,
                  double lz, double c_speed, double t, int dtype, fftpde_stream stream) {
  int rc = check3d(ctx, nx, ny, nz, batch, dtype, u0, u);
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly) && finite_pos(lz))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(c_speed) && c_speed >= 0.0 && std::isfinite(t))) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  return run_solve3d(c, dtype, FFTPDE_WAVE, u0, u, nx, ny, nz, batch, lx, ly, lz, c_speed, t,
                     static_cast<hipStream_t>(stream));
}

int fftpde_wave_rk4(fftpde_ctx* ctx, const fftpde_orbit_source* src, const void* f, const void* g0, void* u, void* v,
                    int nx, int ny, int batch, double x0, double y0, double lx, double ly, double c_speed, double t0,
                    double dt, int steps, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype);
  if (rc == FFTPDE_OK) rc = check_field(f, dtype);
  if (rc == FFTPDE_OK && g0) rc = check_field(g0, dtype);
  if (rc == FFTPDE_OK) rc = check_field(u, dtype);
  if (rc == FFTPDE_OK && v) rc = check_field(v, dtype);
  if (rc == FFTPDE_OK && (!src || !(std::isfinite(src->sigma) && src->sigma > 0.0))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK) {
    const double fin[] = {src->amplitude, src->radius, src->omega, src->gamma, src->cx, src->cy, x0, y0, t0, dt};
    for (double x : fin)
      if (!std::isfinite(x)) rc = FFTPDE_EINVAL;
  }
  if (rc == FFTPDE_OK && !(finite_pos(lx) && finite_pos(ly))) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && !(std::isfinite(c_speed) && c_speed >= 0.0) ) rc = FFTPDE_EINVAL;
  if (rc == FFTPDE_OK && (steps < 0 || (v && v == u))) rc = FFTPDE_EINVAL;
  if (rc != FFTPDE_OK) return rc;
  Context* c = reinterpret_cast<Context*>(ctx);
  DeviceGuard g(c->device);
  const OrbitSource os{src->amplitude, src->sigma, src->radius, src->omega, src->gamma, src->cx, src->cy};
  return run_wave_rk4(c, dtype, os, f, g0, u, v, nx, ny, batch, x0, y0, lx, ly, c_speed, t0, dt, steps,
                      static_cast<hipStream_t>(stream));
}

int solve_wave_noalloc(fftpde_ctx* ctx, const void* u0, const void* v0, void* u, void* v, int nx, int ny, int batch,
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
  SolveScratch sc;
  sc.p = noalloc_scratch(c->device);
  sc.bytes = noalloc_scratch_bytes();
  if (!sc.p) {
    std::snprintf(g_last_error, sizeof(g_last_error), "solve_wave_noalloc: no static scratch on device %d",
                  c->device);
    return FFTPDE_EDEVICE;
  }
  const size_t need = solve_scratch_per_field(c, dtype, FFTPDE_WAVE, nx, ny, v0 != nullptr, v != nullptr);
  if (need > sc.bytes) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "solve_wave_noalloc: one %dx%d field needs %zu bytes of scratch, more than the %zu-byte array",
                  nx, ny, need, sc.bytes);
    return FFTPDE_EINVAL;
  }
  return run_solve(c, dtype, FFTPDE_WAVE, u0, v0, u, v, nx, ny, batch, lx, ly, c_speed, t,
                   static_cast<hipStream_t>(stream), sc);
}

int solve_wave(fftpde_ctx* ctx, const void* u0, const void* v0, void* u, void* v, int nx, int ny, int batch,
               double lx, double ly, double c_speed, double t, int dtype, fftpde_stream stream) {
  int rc = check_common(ctx, nx, ny, batch, dtype, true, true);
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
  if (is_mixed(nx, ny))
    return run_mixed_solve(c, dtype, FFTPDE_WAVE, u0, v0, u, v, nx, ny, batch, lx, ly, c_speed, t,
                           static_cast<hipStream_t>(stream));
  return run_solve(c, dtype, FFTPDE_WAVE, u0, v0, u, v, nx, ny, batch, lx, ly, c_speed, t,
                   static_cast<hipStream_t>(stream));
}

}  // extern "C"
