// rpass_f64.hip -- the radix-R + power-of-two passes, FP64 complex.
#include "rpass_kernels.hpp"

namespace fftpde {

template <>
hipError_t rp_launch<double>(const RpArgs<double>& a, hipStream_t s) {
  return rp::dispatch<double>(a, s);
}

}  // namespace fftpde
