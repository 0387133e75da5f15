// Instantiations of the real column-split A-stream kernel (n <= 1024, b <= 10).
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

template <int B, bool DOT2>
static void launch_cs(hipStream_t st, int64_t nb, int nw, int64_t rows, const double* A, int64_t lda, int64_t m,
                      int n, const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart,
                      int init, const Ctl* ctl) {
  hipLaunchKernelGGL((k_astream_cs<B, DOT2>), dim3((unsigned)nb), dim3(64 * nw), 0, st, A, lda, m, n, W, AW, AVp,
                     AXp, Gpart, rows, init, ctl);
}

template <bool DOT2>
static bool cs_by_b(int B, hipStream_t st, int64_t nb, int nw, int64_t rows, const double* A, int64_t lda, int64_t m,
                    int n, const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart, int init,
                    const Ctl* ctl) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: launch_cs<BB, DOT2>(st, nb, nw, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, init, ctl); return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

// waves per workgroup: one 128-column slot each
int astream_cs_waves(int n) { return (n + 127) / 128; }

bool astream_cs_fits(int B, int n, bool aligned) { return aligned && n <= 128 * CS_MAXW && B >= 1 && B <= 10; }

// Workgroups: about 2048 / (waves per workgroup) * 4 row ranges, at least 16
// rows each.
int64_t astream_cs_blocks(int64_t m, int n) {
  const int nw = astream_cs_waves(n);
  int64_t target = 8192 / nw;
  int64_t rows = (m + target - 1) / target;
  if (rows < 16) rows = 16;
  return (m + rows - 1) / rows;
}

bool dispatch_astream_cs(bool dot2, int init, int B, hipStream_t st, int64_t nb, const double* A, int64_t lda,
                         int64_t m, int n, const double* W, double* AW, const double* AVp, const double* AXp,
                         double* Gpart, const Ctl* ctl) {
  const int nw = astream_cs_waves(n);
  if (nw < 1 || nw > CS_MAXW) return false;
  const int64_t rows = (m + nb - 1) / nb;
  if (dot2) return cs_by_b<true>(B, st, nb, nw, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, init, ctl);
  return cs_by_b<false>(B, st, nb, nw, rows, A, lda, m, n, W, AW, AVp, AXp, Gpart, init, ctl);
}

}  // namespace rl
