// Instantiations of the real 16-byte-load A-stream kernel (n <= 256, b <= 2).
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

template <int B, bool DOT2, bool INIT>
static void launch_r2(hipStream_t st, int64_t nb, int64_t rows, const double* A, int64_t lda, int64_t m, int n,
                      const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart,
                      const Ctl* ctl) {
  hipLaunchKernelGGL((k_astream_r2<B, DOT2, INIT>), dim3((unsigned)nb), dim3(256), 0, st, A, lda, m, n, W, AW, AVp,
                     AXp, Gpart, rows, ctl);
}

template <bool DOT2, bool INIT>
static bool by_b(int B, hipStream_t st, int64_t nb, int64_t rows, const double* A, int64_t lda, int64_t m, int n,
                 const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart, const Ctl* ctl) {
  if (B == 1) launch_r2<1, DOT2, INIT>(st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  else if (B == 2) launch_r2<2, DOT2, INIT>(st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  else return false;
  return true;
}

// Workgroups of the r2 pass: about 2048 (two rounds of four per compute unit,
// which balances better than one), at least 64 rows each.
int64_t astream_r2_blocks(int64_t m) {
  int64_t rows = (m + 2047) / 2048;
  if (rows < 64) rows = 64;
  return (m + rows - 1) / rows;
}

// The kernel reads a workgroup's rows through one buffer resource, whose byte
// range is a signed 32-bit count.
bool astream_r2_fits(int B, int n, bool aligned, int64_t m, int64_t lda) {
  if (!(aligned && n % 2 == 0 && n <= 256 && B >= 1 && B <= 2)) return false;
  const int64_t nb = astream_r2_blocks(m);
  const int64_t rows = nb > 0 ? (m + nb - 1) / nb : 0;
  return rows * lda * 8 < ((int64_t)1 << 31);
}

bool dispatch_astream_r2(bool dot2, int init, int B, hipStream_t st, int64_t nb, const double* A, int64_t lda,
                         int64_t m, int n, const double* W, double* AW, const double* AVp, const double* AXp,
                         double* Gpart, const Ctl* ctl) {
  if (n > 256) return false;
  const int64_t rows = (m + nb - 1) / nb;
  if (dot2)
    return init ? by_b<true, true>(B, st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl)
                : by_b<true, false>(B, st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  return init ? by_b<false, true>(B, st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl)
              : by_b<false, false>(B, st, nb, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
}

}  // namespace rl
