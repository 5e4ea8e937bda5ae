// Single-pass small-grid kernels, FP32 complex: every (nx, ny) with both sides in
// [32, 512] and at most 16384 points (one workgroup per field).
#include "small.hpp"

namespace fftpde {
namespace {
const SmallVariant kSmall[] = {
    FFTPDE_SMALL_VARIANT(float, 5, 5, 128),
    FFTPDE_SMALL_VARIANT(float, 5, 6, 256),
    FFTPDE_SMALL_VARIANT(float, 5, 7, 512),
    FFTPDE_SMALL_VARIANT(float, 5, 8, 1024),
    FFTPDE_SMALL_VARIANT(float, 5, 9, 1024),
    FFTPDE_SMALL_VARIANT(float, 6, 5, 256),
    FFTPDE_SMALL_VARIANT(float, 6, 6, 512),
    FFTPDE_SMALL_VARIANT(float, 6, 7, 1024),
    FFTPDE_SMALL_VARIANT(float, 6, 8, 1024),
    FFTPDE_SMALL_VARIANT(float, 7, 5, 512),
    FFTPDE_SMALL_VARIANT(float, 7, 6, 1024),
    FFTPDE_SMALL_VARIANT(float, 7, 7, 1024),
    FFTPDE_SMALL_VARIANT(float, 8, 5, 1024),
    FFTPDE_SMALL_VARIANT(float, 8, 6, 1024),
    FFTPDE_SMALL_VARIANT(float, 9, 5, 1024),
};
}  // namespace
const SmallVariant* small_variants_f32(int* count) {
  *count = int(sizeof(kSmall) / sizeof(kSmall[0]));
  return kSmall;
}
}  // namespace fftpde
