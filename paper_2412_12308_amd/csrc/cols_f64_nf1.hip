// Column-pass kernel configurations, FP64 complex, one field per pass (fields
// as for FP32).  The first entry of each length is the default plan.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f64_nf1(int* count);
namespace {
const ColVariant kCols[] = {
    FFTPDE_COL_VARIANT(double, 1, 8, 8, 64, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 2, 7, 8, 64, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 3, 7, 8, 128, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 4, 7, 8, 256, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 5, 7, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 6, 6, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 7, 5, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 8, 4, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 9, 3, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 10, 2, 8, 512, 3, 1, 0, 1, 3),
    FFTPDE_COL_VARIANT(double, 11, 1, 8, 512, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 1, 8, 512, 3, 1, 0, 0, 4),
    FFTPDE_COL_VARIANT(double, 11, 1, 16, 256, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 2, 8, 1024, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 2, 16, 512, 3, 1, 1, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 2, 8, 1024, 3, 1, 1, 0, 2),
    FFTPDE_COL_VARIANT(double, 11, 1, 8, 512, 3, 1, 1, 0, 2),
    FFTPDE_COL_VARIANT(double, 11, 1, 8, 512, 3, 1, 1, 0, 4),
    FFTPDE_COL_VARIANT(double, 12, 1, 8, 1024, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 12, 1, 8, 1024, 3, 1, 1, 0, 3),
};
}  // namespace
const ColVariant* col_variants_f64_nf1(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
