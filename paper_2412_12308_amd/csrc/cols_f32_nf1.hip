// Column-pass kernel configurations, FP32 complex, 1 field(s) per pass.
// Tiles of T = 2^LOGT columns: 64-byte row segments or wider.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f32_nf1(int* count);
namespace {
const ColVariant kCols[] = {
    FFTPDE_COL_VARIANT(float, 1, 8, 8, 64, 3, 1),    FFTPDE_COL_VARIANT(float, 2, 8, 8, 128, 3, 1),
    FFTPDE_COL_VARIANT(float, 3, 8, 8, 256, 3, 1),   FFTPDE_COL_VARIANT(float, 4, 8, 8, 512, 3, 1),
    FFTPDE_COL_VARIANT(float, 5, 8, 8, 1024, 3, 1),  FFTPDE_COL_VARIANT(float, 6, 7, 8, 1024, 3, 1),
    FFTPDE_COL_VARIANT(float, 7, 6, 8, 1024, 3, 1),  FFTPDE_COL_VARIANT(float, 8, 5, 8, 1024, 3, 1),
    FFTPDE_COL_VARIANT(float, 9, 4, 8, 1024, 3, 1),  FFTPDE_COL_VARIANT(float, 10, 3, 8, 1024, 3, 1),
    FFTPDE_COL_VARIANT(float, 10, 3, 16, 512, 3, 1), FFTPDE_COL_VARIANT(float, 11, 3, 16, 1024, 3, 1),
    FFTPDE_COL_VARIANT(float, 11, 3, 16, 1024, 4, 1), FFTPDE_COL_VARIANT(float, 11, 2, 8, 1024, 3, 1),
    FFTPDE_COL_VARIANT(float, 12, 2, 16, 1024, 3, 1), FFTPDE_COL_VARIANT(float, 12, 2, 16, 1024, 4, 1),
};
}  // namespace
const ColVariant* col_variants_f32_nf1(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
