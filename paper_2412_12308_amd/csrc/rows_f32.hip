// Row-pass kernel configurations, FP32 complex.  E elements per thread, TH
// threads, LINES = E*TH/N rows per tile, PF = prefetch the next tile, TW =
// twiddle source (0 global table, 1 registers).  The first entry of each
// length is the default plan.
#include "kernels.hpp"

namespace fftpde {
namespace {
const RowVariant kRows[] = {
    FFTPDE_ROW_VARIANT(float, 1, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 2, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 3, 8, 64, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 4, 8, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 5, 8, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 6, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 7, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 8, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 9, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 10, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 10, 8, 256, 3, 0, 0),
    FFTPDE_ROW_VARIANT(float, 10, 8, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 11, 16, 128, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 11, 8, 256, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 11, 8, 256, 3, 0, 0),
    FFTPDE_ROW_VARIANT(float, 11, 8, 256, 3, 1, 0),
    FFTPDE_ROW_VARIANT(float, 11, 8, 256, 3, 0, 1),
    FFTPDE_ROW_VARIANT(float, 11, 16, 128, 4, 1, 1),
    FFTPDE_ROW_VARIANT(float, 12, 8, 512, 3, 1, 1),
    FFTPDE_ROW_VARIANT(float, 12, 8, 512, 3, 0, 0),
    FFTPDE_ROW_VARIANT(float, 12, 16, 256, 4, 1, 1),
    FFTPDE_ROW_VARIANT(float, 12, 16, 256, 3, 1, 1),
};
}  // namespace
const RowVariant* row_variants_f32(int* count) {
  *count = int(sizeof(kRows) / sizeof(kRows[0]));
  return kRows;
}
}  // namespace fftpde
