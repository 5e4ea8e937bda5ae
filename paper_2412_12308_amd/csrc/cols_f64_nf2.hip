// Column-pass kernel configurations, FP64 complex, two fields per pass (wave
// displacement and velocity).  Half-width tiles keep 512 threads per
// workgroup so both fields stay in registers.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f64_nf2(int* count);
namespace {
const ColVariant kCols[] = {
    FFTPDE_COL_VARIANT(double, 1, 8, 8, 64, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 2, 7, 8, 64, 3, 2, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 3, 7, 8, 128, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 4, 7, 8, 256, 3, 2, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 5, 7, 8, 512, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 6, 6, 8, 512, 3, 2, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 7, 5, 8, 512, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 8, 4, 8, 512, 3, 2, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 9, 3, 8, 512, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 10, 2, 8, 512, 3, 2, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 1, 8, 512, 3, 2, 0, 0, 3), FFTPDE_COL_VARIANT(double, 12, 0, 8, 512, 3, 2, 0, 0, 3),
};
}  // namespace
const ColVariant* col_variants_f64_nf2(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
