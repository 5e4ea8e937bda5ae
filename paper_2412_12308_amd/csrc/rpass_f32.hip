// rpass_f32.hip -- the radix-R + power-of-two passes, FP32 complex, and the
// split of a side into R 2^lp.
#include "rpass_kernels.hpp"

namespace fftpde {

bool rp_split(int n, bool col, bool fp64, int* r, int* lp) {
  if (n < 2 || n > kMrMaxSide) return false;
  for (int rr : {1, 3, 5, 7}) {
    if (fp64 && rr > 3) break;
    if (n % rr) continue;
    const int p = n / rr;
    if (p & (p - 1)) continue;
    int l = 0;
    while ((1 << l) < p) l++;
    const int hi = rr == 1 ? (col ? 12 : 11) : rr == 3 ? 10 : 9;
    if (l < 5 || l > hi) return false;
    *r = rr;
    *lp = l;
    return true;
  }
  return false;
}

bool rp_pass_ok(int mode, int n, bool fp64) {
  int r = 0, lp = 0;
  if (!rp_split(n, mode >= kMrColFwd, fp64, &r, &lp)) return false;
  return mode != kMrColSolve || rp_solve_radix(fp64, r);
}

template <>
hipError_t rp_launch<float>(const RpArgs<float>& a, hipStream_t s) {
  return rp::dispatch<float>(a, s);
}

}  // namespace fftpde
