// Host build of the library's rotation fit (the same header the kernels
// use), for CPU checks against the oracle.  Reads "n precision" then n lines of
// 9 cross-covariance entries followed by 9 previous-rotation entries (all
// row-major) from stdin; prints per line the code and the 9 entries of R.
#include <cstdio>

#include "../../paper_1603_08161_amd/csrc/vd_device.h"

int main() {
  long n = 0;
  int prec = 0;
  if (std::scanf("%ld %d", &n, &prec) != 2) return 1;
  for (long i = 0; i < n; ++i) {
    double m[9], rp[9];
    for (int k = 0; k < 9; ++k)
      if (std::scanf("%lf", &m[k]) != 1) return 1;
    for (int k = 0; k < 9; ++k)
      if (std::scanf("%lf", &rp[k]) != 1) return 1;
    int code;
    double out[9];
    if (prec == 1) {
      double R[9];
      code = vd::fit_or_keep<double>(m, rp, R);
      for (int k = 0; k < 9; ++k) out[k] = R[k];
    } else {
      float mf[9], rf[9], R[9];
      for (int k = 0; k < 9; ++k) {
        mf[k] = (float)m[k];
        rf[k] = (float)rp[k];
      }
      code = vd::fit_or_keep<float>(mf, rf, R);
      for (int k = 0; k < 9; ++k) out[k] = R[k];
    }
    std::printf("%d", code);
    for (int k = 0; k < 9; ++k) std::printf(" %.17g", out[k]);
    std::printf("\n");
  }
  return 0;
}
