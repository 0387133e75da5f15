// k_orth_reg for real data (see orth_reg.hpp).
#include "orth_reg.hpp"

namespace rl {

bool launch_orth_reg_d(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x,
                       void* W, Ctl* ctl, int check_done, int masked) {
  return orth_reg_dispatch<double>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
}

}  // namespace rl
