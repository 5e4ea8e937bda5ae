// Single-pass small-grid kernels, FP64 complex: every (nx, ny) with both sides in
// [32, 256] and at most 8192 points (one workgroup per field).
#include "small.hpp"

namespace fftpde {
namespace {
const SmallVariant kSmall[] = {
    FFTPDE_SMALL_VARIANT(double, 5, 5, 128),
    FFTPDE_SMALL_VARIANT(double, 5, 6, 256),
    FFTPDE_SMALL_VARIANT(double, 5, 7, 512),
    FFTPDE_SMALL_VARIANT(double, 5, 8, 1024),
    FFTPDE_SMALL_VARIANT(double, 6, 5, 256),
    FFTPDE_SMALL_VARIANT(double, 6, 6, 512),
    FFTPDE_SMALL_VARIANT(double, 6, 7, 1024),
    FFTPDE_SMALL_VARIANT(double, 7, 5, 512),
    FFTPDE_SMALL_VARIANT(double, 7, 6, 1024),
    FFTPDE_SMALL_VARIANT(double, 8, 5, 1024),
};
}  // namespace
const SmallVariant* small_variants_f64(int* count) {
  *count = int(sizeof(kSmall) / sizeof(kSmall[0]));
  return kSmall;
}
}  // namespace fftpde
