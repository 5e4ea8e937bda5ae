// noalloc.cpp -- the fixed device scratch behind solve_wave_noalloc.
//
// A solve keeps the spectrum between its passes in scratch memory.  The
// ordinary entry points take it from the context's per-stream workspace,
// which grows with hipMalloc on demand; solve_wave_noalloc takes it from the
// array below instead, so it never allocates.  The array is a file-scope
// device variable: every GPU the library runs on holds its own copy (made
// when the code object loads) until the process ends.  Its device address is
// looked up once per device, at context creation with that device current,
// and only that address is used from the host (the array's name is a
// host-side stand-in, not a device address).  Calls that overlap on one GPU
// share the one array and race; nothing in it needs to start at zero (the
// forward row pass writes every element a later pass reads).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fftpde.h"
#include "context.hpp"
#include "noalloc.hpp"

namespace fftpde {
namespace {

constexpr size_t kScratchBytes = FFTPDE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_bind(int device) {
  if (device < 0 || device >= kMaxDevices) return FFTPDE_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return FFTPDE_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_last_error("hipGetSymbolAddress(scratch)", e);
    return FFTPDE_EDEVICE;
  }
  g_ptr[device] = p;
  return FFTPDE_OK;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace fftpde
