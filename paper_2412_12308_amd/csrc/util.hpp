// util.hpp -- small device utilities used by the host side: deterministic
// fills of scratch fields and a relative-difference reduction (plan checks).
#pragma once

#include <hip/hip_runtime.h>

namespace fftpde {

// Fill n complex values of dtype (0 = FP32, 1 = FP64) with a deterministic
// pseudo-random pattern in [-1, 1) derived from `seed` and the index.
hipError_t fill_pattern(void* p, long long n, int dtype, unsigned seed, hipStream_t s);

// acc[0] += sum |a - b|^2, acc[1] += sum |b|^2 over n complex values (FP64
// accumulation); acc is a device array of two doubles.
hipError_t diff_norms(const void* a, const void* b, long long n, int dtype, double* acc, hipStream_t s);

// Set n doubles to zero with a kernel (no memset node in captured graphs).
hipError_t zero_doubles(double* p, long long n, hipStream_t s);

}  // namespace fftpde
