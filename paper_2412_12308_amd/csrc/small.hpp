// small.hpp -- single-pass 2D transforms and solves for small grids: one
// workgroup per field holds the whole field in LDS and registers, so a solve
// reads and writes HBM once and takes one launch.
//   rows forward (x) -> columns forward (y) [-> symbol -> columns inverse ->
//   rows inverse]
// (the row-column order of Sec. II.D; the inverse by the conjugation identity
// of Sec. II.B).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fftpde {

template <typename T>
struct SmallArgs {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* tw;
  long long batch;
  int mode;  // kColForward (2D forward), kColInverse (2D inverse), kColFwdMulInv (solve)
  SymParams sym;
};

template <typename T, int LX, int LY, int TH>
__global__ void __launch_bounds__(TH) small_kernel(SmallArgs<T> a) {
  constexpr int NX = 1 << LX, NY = 1 << LY, P = NX * NY;
  constexpr int E = P / TH;
  static_assert(E * TH == P, "the workgroup holds one whole field");
  using RMap = RowMap<LX, NY, plan_pad(LX, 3, false)>;
  using Row = Engine<T, LX, E, TH, 3, false, RMap, false>;
  using CFMap = ColMap<LY, LX, plan_pad(LY, 3, false)>;
  using CIMap = ColMap<LY, LX, plan_pad(LY, 3, true)>;
  using ColF = Engine<T, LY, E, TH, 3, false, CFMap, false>;
  using ColI = Engine<T, LY, E, TH, 3, true, CIMap, false>;
  // the field between passes: y * FS + x, padded so column reads spread over banks
  constexpr int FS = NX + (NX >= 8 ? NX / 8 : 1);
  constexpr int W0 = NY * FS;
  constexpr int W1 = Row::kLdsWords > ColF::kLdsWords ? Row::kLdsWords : ColF::kLdsWords;
  constexpr int W2 = W1 > ColI::kLdsWords ? W1 : ColI::kLdsWords;
  __shared__ cx<T> lds[W0 > W2 ? W0 : W2];

  const long long f = blockIdx.x;
  if (f >= a.batch) return;
  const cx<T>* in = a.in + f * P;
  cx<T>* out = a.out + f * P;
  const int tid = threadIdx.x;
  const int mode = a.mode;
  const T sgn = mode == kColInverse ? T(-1) : T(1);
  cx<T> x[E];

  // rows: x transforms for every y
  Row::for_each_input(tid, [&](int i, int line, int n) {
    const cx<T> v = in[line * NX + n];
    x[i] = {v.re, sgn * v.im};
  });
  Row::run(x, lds, a.tw, tid);
  Row::for_each_output(tid, [&](int i, int line, int n) { lds[line * FS + n] = x[i]; });
  lds_barrier();
  // columns: y transforms for every x frequency
  ColF::for_each_input(tid, [&](int i, int line, int n) { x[i] = lds[n * FS + line]; });
  lds_barrier();
  ColF::run(x, lds, a.tw, tid);
  if (mode == kColForward || mode == kColInverse) {
    const T sc = mode == kColInverse ? T(a.sym.scale) : T(1);
    ColF::for_each_output(tid, [&](int i, int line, int n) {
      out[n * NX + line] = {x[i].re * sc, sgn * x[i].im * sc};
    });
    return;
  }
  // symbol, then the inverse by conjugation: columns, rows
  auto mul = [&](auto tag) {
    constexpr int OP = decltype(tag)::value;
    ColI::for_each_input(tid, [&](int i, int line, int n) {
      const Symbol<T, OP> sym(a.sym, line);
      const T m = sym(n);
      x[i] = {x[i].re * m, -x[i].im * m};
    });
  };
  switch (a.sym.op) {
    case kSymPoisson: mul(std::integral_constant<int, kSymPoisson>()); break;
    case kSymDiffusion: mul(std::integral_constant<int, kSymDiffusion>()); break;
    case kSymWave: mul(std::integral_constant<int, kSymWave>()); break;
    default: mul(std::integral_constant<int, kSymScale>()); break;
  }
  ColI::run(x, lds, a.tw, tid);
  ColI::for_each_output(tid, [&](int i, int line, int n) { lds[n * FS + line] = x[i]; });
  lds_barrier();
  Row::for_each_input(tid, [&](int i, int line, int n) { x[i] = lds[line * FS + n]; });
  lds_barrier();
  Row::run(x, lds, a.tw, tid);
  Row::for_each_output(tid, [&](int i, int line, int n) { out[line * NX + n] = conjg(x[i]); });
}

struct SmallVariant {
  LaunchFn launch;  // units = batch (fields)
  int lx, ly, th;
  int lds_bytes;
  const char* name;
};

template <typename T, int LX, int LY, int TH>
hipError_t launch_small(const void* args, long long batch, long long, hipStream_t s) {
  if (batch <= 0 || batch > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL((small_kernel<T, LX, LY, TH>), dim3((unsigned)batch), dim3(TH), 0, s,
                     *static_cast<const SmallArgs<T>*>(args));
  return hipGetLastError();
}

#define FFTPDE_SMALL_VARIANT(T, LX, LY, TH)                                                        \
  {&::fftpde::launch_small<T, LX, LY, TH>, LX, LY, TH,                                              \
   int(((1 << (LY)) * ((1 << (LX)) + (1 << (LX)) / 8)) * sizeof(::fftpde::cx<T>)),                 \
   "small_" #T "_x" #LX "_y" #LY "_th" #TH}

const SmallVariant* small_variants_f32(int* count);
const SmallVariant* small_variants_f64(int* count);

}  // namespace fftpde
