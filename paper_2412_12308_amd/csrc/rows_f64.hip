// Row-pass kernel configurations, FP64 complex (fields as for FP32).  The
// first entry of each length is the default plan.
#include "kernels.hpp"

namespace fftpde {
namespace {
const RowVariant kRows[] = {
    FFTPDE_ROW_VARIANT(double, 1, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 2, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 3, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 4, 8, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 5, 8, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 6, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 7, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 8, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 9, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 10, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 10, 8, 256, 3, 0, 0),
    FFTPDE_ROW_VARIANT(double, 11, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 11, 8, 256, 3, 0, 0),
    FFTPDE_ROW_VARIANT(double, 11, 8, 256, 3, 0, 1),
    FFTPDE_ROW_VARIANT(double, 11, 16, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 12, 8, 512, 3, 1, 1),
    FFTPDE_ROW_VARIANT(double, 12, 8, 512, 3, 0, 0),
    FFTPDE_ROW_VARIANT(double, 12, 8, 512, 3, 0, 1),
};
}  // namespace
const RowVariant* row_variants_f64(int* count) {
  *count = int(sizeof(kRows) / sizeof(kRows[0]));
  return kRows;
}
}  // namespace fftpde
