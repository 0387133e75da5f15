// One level of the deterministic compensated reduction of the A-stream's
// per-workgroup partial records (k_colsum2 in astream.hip).  The body is a
// device function so that the first level can also run as extra workgroups of
// the first TSQR launch (both read only what the pass wrote).
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace rl {

// Workgroup (bx, by) of 256 threads: 64 elements x 4 record groups, records
// by*64 .. by*64+63 of every element.  fin != nullptr: single group, the
// finished sums s + e; else the group's (sum, error) pair.
__device__ __forceinline__ void colsum2_block(const ColsumJob& J, int bx, int by) {
  if (J.ctl != nullptr && J.ctl->done) return;
  __shared__ double sh_s[256], sh_e[256];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;  // 64 elements x 4 groups
  const int64_t e = (int64_t)bx * 64 + el;
  const int64_t p0 = (int64_t)by * 64;
  // the thread's 16 records are loaded together (one memory latency instead
  // of one per record); records past the end are zeros, which change neither
  // the sum nor its error
  double vs[16], ve[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t p = p0 + g + 4 * u;
    const bool ok = (e < J.len) && (p < J.nparts);
    vs[u] = ok ? J.in_s[p * J.stride + e] : 0.0;
    ve[u] = (ok && e < J.elen) ? J.in_e[p * J.stride + e] : 0.0;
  }
  double S = 0.0, E = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    double t;
    two_sum(S, vs[u], S, t);
    E += t + ve[u];
  }
  sh_s[threadIdx.x] = S;
  sh_e[threadIdx.x] = E;
  __syncthreads();
  if (g == 0 && e < J.len) {
    double s0 = sh_s[el], e0 = sh_e[el], t;
    for (int q = 1; q < 4; ++q) {
      two_sum(s0, sh_s[64 * q + el], s0, t);
      e0 += t + sh_e[64 * q + el];
    }
    if (J.fin != nullptr) {
      J.fin[e] = s0 + e0;  // single group: the finished sums
    } else {
      J.out_s[(int64_t)by * J.len + e] = s0;
      J.out_e[(int64_t)by * J.len + e] = e0;
    }
  }
}

}  // namespace rl
