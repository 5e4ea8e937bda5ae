// Row-pass kernel configurations, FP32 complex.  Elements per thread E and
// threads TH; LINES = E*TH/N rows per workgroup.
#include "kernels.hpp"

namespace fftpde {
namespace {
const RowVariant kRows[] = {
    FFTPDE_ROW_VARIANT(float, 1, 8, 64, 3),   FFTPDE_ROW_VARIANT(float, 2, 8, 64, 3),
    FFTPDE_ROW_VARIANT(float, 3, 8, 64, 3),   FFTPDE_ROW_VARIANT(float, 4, 8, 128, 3),
    FFTPDE_ROW_VARIANT(float, 5, 8, 128, 3),  FFTPDE_ROW_VARIANT(float, 6, 8, 256, 3),
    FFTPDE_ROW_VARIANT(float, 7, 8, 256, 3),  FFTPDE_ROW_VARIANT(float, 8, 8, 256, 3),
    FFTPDE_ROW_VARIANT(float, 9, 8, 256, 3),  FFTPDE_ROW_VARIANT(float, 10, 8, 256, 3),
    FFTPDE_ROW_VARIANT(float, 10, 8, 128, 3), FFTPDE_ROW_VARIANT(float, 11, 8, 256, 3),
    FFTPDE_ROW_VARIANT(float, 11, 16, 128, 4), FFTPDE_ROW_VARIANT(float, 11, 16, 256, 4),
    FFTPDE_ROW_VARIANT(float, 12, 8, 512, 3), FFTPDE_ROW_VARIANT(float, 12, 16, 256, 4),
};
}  // namespace
const RowVariant* row_variants_f32(int* count) {
  *count = int(sizeof(kRows) / sizeof(kRows[0]));
  return kRows;
}
}  // namespace fftpde
