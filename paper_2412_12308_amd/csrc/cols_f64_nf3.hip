// Column-pass kernel configurations, FP64 complex, three fields per pass
// (initial value, initial velocity and a source constant in time).  Four
// points per thread (radix 4) on 512 threads keep the three fields in
// registers up to 2048 rows; 4096 rows take eight points per thread and
// spill some registers to scratch memory.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f64_nf3(int* count);
namespace {
const ColVariant kCols[] = {
    FFTPDE_COL_VARIANT(double, 1, 10, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 2, 9, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 3, 8, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 4, 7, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 5, 6, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 6, 5, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 7, 4, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 8, 3, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 9, 2, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 10, 1, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 11, 0, 4, 512, 2, 3, 0, 0, 3),
    FFTPDE_COL_VARIANT(double, 12, 0, 8, 512, 3, 3, 0, 0, 3),
};
}  // namespace
const ColVariant* col_variants_f64_nf3(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
