// Column-pass kernel configurations, FP32 complex, one field per pass.
// T = 2^LOGT columns per tile (64-byte row segments at T = 8), S = split
// real/imaginary LDS exchange, PF = prefetch the next tile, TW = twiddle
// source (2 LDS copy, 3 per-stage tables, 4 per-stage tables with each value
// loaded by one lane of the tile's columns); _XW: the fused pass with its
// exchanges around the radix-8 stage inside each wavefront.  The first entry
// of each length is the default plan.
#include "kernels.hpp"

namespace fftpde {
const ColVariant* col_variants_f32_nf1(int* count);
namespace {
const ColVariant kCols[] = {
    FFTPDE_COL_VARIANT(float, 1, 8, 8, 64, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 2, 8, 8, 128, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 3, 8, 8, 256, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 4, 8, 8, 512, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 5, 8, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 6, 7, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 7, 6, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 8, 5, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 9, 4, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 10, 3, 8, 1024, 3, 1, 0, 1, 2),
    FFTPDE_COL_VARIANT(float, 10, 3, 8, 1024, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 10, 2, 8, 512, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT_XW(float, 11, 2, 16, 512, 4, 1, 1, 0, 2),
    FFTPDE_COL_VARIANT(float, 11, 2, 16, 512, 4, 1, 1, 0, 2),
    FFTPDE_COL_VARIANT(float, 11, 2, 16, 512, 4, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 11, 2, 16, 512, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 11, 3, 16, 1024, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 11, 3, 16, 1024, 3, 1, 0, 0, 2),
    FFTPDE_COL_VARIANT(float, 11, 3, 16, 1024, 3, 1, 1, 0, 2),
    FFTPDE_COL_VARIANT(float, 11, 3, 32, 512, 3, 1, 1, 0, 3),
    FFTPDE_COL_VARIANT(float, 11, 2, 16, 512, 4, 1, 0, 0, 4),
    FFTPDE_COL_VARIANT(float, 11, 2, 16, 512, 4, 1, 1, 0, 4),
    FFTPDE_COL_VARIANT(float, 12, 2, 16, 1024, 4, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 12, 2, 16, 1024, 3, 1, 0, 0, 3),
    FFTPDE_COL_VARIANT(float, 12, 1, 16, 512, 4, 1, 0, 0, 3),
};
}  // namespace
const ColVariant* col_variants_f32_nf1(int* count) {
  *count = int(sizeof(kCols) / sizeof(kCols[0]));
  return kCols;
}
}  // namespace fftpde
