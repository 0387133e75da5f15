// Instantiations of the generic A-stream kernel for real data.
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

template <int B, int NS, bool DOT2>
static void launch_g(hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n, const void* W,
                     void* AW, const void* AVp, const void* AXp, int init, double* Gpart, const Ctl* ctl) {
  using T = double;
  const int64_t rows = (m + nb - 1) / nb;
  hipLaunchKernelGGL((k_astream<T, B, NS, DOT2>), dim3((unsigned)nb), dim3(256), 0, st, (const T*)A, lda, m, n,
                     (const T*)W, (T*)AW, (const T*)AVp, (const T*)AXp, init, (T*)Gpart, rows, ctl);
}

template <int NS, bool DOT2>
static bool by_b(int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n, const void* W,
                 void* AW, const void* AVp, const void* AXp, int init, double* Gpart, const Ctl* ctl) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: launch_g<BB, NS, DOT2>(st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl); return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

template <bool DOT2>
static bool by_ns(int ns, int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n,
                  const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                  const Ctl* ctl) {
  switch (ns) {
    case 4: return by_b<4, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    case 8: return by_b<8, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    case 16: return by_b<16, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    default: return false;
  }
}

bool dispatch_astream_gd(bool dot2, int ns, int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n,
             const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart, const Ctl* ctl) {
  if (dot2) return by_ns<true>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  return by_ns<false>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
}

}  // namespace rl
