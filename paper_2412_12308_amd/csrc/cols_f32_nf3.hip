// Column-pass kernel configurations, FP32 complex, three fields per pass (initial
// value, initial velocity and a source constant in time).
// Tiles of T = 2^LOGT columns: 64-byte row segments or wider.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f32_nf3(int* count);
namespace {
const ColVariant kCols[] = {
    // 512-thread tiles: all three fields stay in registers (up to 256 VGPRs)
    FFTPDE_COL_VARIANT(float, 1, 8, 8, 64, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 2, 8, 8, 128, 3, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 3, 8, 8, 256, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 4, 8, 8, 512, 3, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 5, 7, 8, 512, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 6, 6, 8, 512, 3, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 7, 5, 8, 512, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 8, 4, 8, 512, 3, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 9, 3, 8, 512, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 10, 2, 8, 512, 3, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 11, 1, 8, 512, 3, 3, 0, 0, 3), FFTPDE_COL_VARIANT(float, 12, 0, 8, 512, 3, 3, 0, 0, 3),
};
}  // namespace
const ColVariant* col_variants_f32_nf3(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
