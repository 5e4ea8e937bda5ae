// noalloc.hpp -- the fixed device scratch of solve_wave_noalloc (noalloc.cpp).
#pragma once

#include <cstddef>

namespace fftpde {

// Looks up this device's copy of the scratch array (the device must be
// current); once per device, later calls return at once.  FFTPDE_OK, or
// FFTPDE_EDEVICE (text in fftpde_last_error) / FFTPDE_EINVAL (device >= 64).
int noalloc_bind(int device);
// The device address found by noalloc_bind, or null before it succeeded.
void* noalloc_scratch(int device);
// Size of the array: FFTPDE_NOALLOC_SCRATCH_BYTES.
size_t noalloc_scratch_bytes();

}  // namespace fftpde
