// Instantiations of the real 16-byte-load A-stream kernel (n <= 256).
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

template <int B, bool DOT2>
static void launch_r2(hipStream_t st, int64_t nb, int init, int aligned, const double* A, int64_t lda, int64_t m,
                      int n, const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart,
                      const Ctl* ctl) {
  const int64_t rows = (m + nb - 1) / nb;
  hipLaunchKernelGGL((k_astream_r2<B, 2, DOT2>), dim3((unsigned)nb), dim3(256), 0, st, A, lda, m, n, W, AW, AVp, AXp,
                     Gpart, rows, init, aligned, ctl);
}

template <bool DOT2>
static bool by_b(int B, hipStream_t st, int64_t nb, int init, int aligned, const double* A, int64_t lda, int64_t m,
                 int n, const double* W, double* AW, const double* AVp, const double* AXp, double* Gpart,
                 const Ctl* ctl) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: launch_r2<BB, DOT2>(st, nb, init, aligned, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl); return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

bool dispatch_astream_r2(bool dot2, int init, int aligned, int B, hipStream_t st, int64_t nb, const double* A,
                         int64_t lda, int64_t m, int n, const double* W, double* AW, const double* AVp,
                         const double* AXp, double* Gpart, const Ctl* ctl) {
  if (n > 256) return false;
  if (dot2) return by_b<true>(B, st, nb, init, aligned, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  return by_b<false>(B, st, nb, init, aligned, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
}

}  // namespace rl
