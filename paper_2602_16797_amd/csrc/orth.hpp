// Orth of the n-side block W against [V X] (BCGS2 + CGS2), shared by the
// kernels of nside.hip and the register-resident variant (orth_reg.hpp).
#pragma once

#include "common.hpp"

namespace rl {

constexpr int NS_THREADS = 256;
constexpr int ORTH_KC = 8;  // Gram entries summed per block reduction (SVQB)
// projections summed per block reduction in orth_project (the per-thread
// partial sums stay in registers)
template <int KM>
struct OrthKC {
  static constexpr int value = 8;
};

// ---------------------------------------------------------------------------
// W (n x B, row-major) <- Orth(W - [V X]([V X]^* W)) with BCGS2; project=0 skips [V X].
// Column j is projected on the columns of [V X W(:, 0:j)] by classical
// Gram-Schmidt passes: two always (BCGS2 then CGS2 inside W), a third when the
// second removed more than half of what was left (the usual "twice is enough"
// safeguard).  A column that vanishes is completed by the first unit vector
// that keeps norm above 1/2 after the same projections.
template <typename T, int KM>
__device__ void orth_project(int n, int B, int j, const T* __restrict__ V, const T* __restrict__ X, int nvx,
                             T* __restrict__ W, T* scratch, T* h, int kw) {
  constexpr int KC = OrthKC<KM>::value;
  const int K = nvx + kw;  // [V X] and the first kw columns of W
  // the K projections are summed in chunks of KC, so the per-thread
  // partial sums stay in registers for any b
  for (int k0 = 0; k0 < K; k0 += KC) {
    T vals[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) vals[kk] = zero<T>();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const T wr = W[(int64_t)r * B + j];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        if (k < K) {
          const T br = (k < nvx) ? ((k < B) ? V[(int64_t)r * B + k] : X[(int64_t)r * B + (k - B)])
                                 : W[(int64_t)r * B + (k - nvx)];
          vals[kk] = cfmac(br, wr, vals[kk]);
        }
      }
    }
    block_sum_many<T, KC>(vals, (K - k0 < KC) ? K - k0 : KC, scratch, h + k0);
  }
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    T wr = W[(int64_t)r * B + j];
    for (int k = 0; k < K; ++k) {
      const T br = (k < nvx) ? ((k < B) ? V[(int64_t)r * B + k] : X[(int64_t)r * B + (k - B)])
                             : W[(int64_t)r * B + (k - nvx)];
      wr = fnmac(br, h[k], wr);
    }
    W[(int64_t)r * B + j] = wr;
  }
  __syncthreads();
}

template <typename T>
__device__ double col_norm(int n, int B, int j, const T* __restrict__ W, double* red) {
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) s += abs2(W[(int64_t)r * B + j]);
  return sqrt(block_sum(s, red));
}

// KM bounds the number of projections of one column, 3B - 1.  Bit j of
// `keep` clear: column j is a locked index's and is set to zero (a zero
// column costs the later projections nothing).
template <typename T, int KM>
__device__ void orth_block(int n, int B, const T* __restrict__ V, const T* __restrict__ X, int project, int with_x,
                           T* __restrict__ W, Ctl* __restrict__ ctl, int keep = -1) {
  __shared__ T scratch[(NS_THREADS / 16) * OrthKC<KM>::value];
  __shared__ T h[KM];
  __shared__ double red[NS_THREADS / 64];
  const int nvx = project ? (with_x ? 2 * B : B) : 0;
  for (int j = 0; j < B; ++j) {
    if (!((keep >> j) & 1)) {
      for (int r = threadIdx.x; r < n; r += blockDim.x) W[(int64_t)r * B + j] = zero<T>();
      __syncthreads();
      continue;
    }
    double nrm = 0.0;
    for (int cand = -1; cand < n; ++cand) {
      if (cand >= 0) {
        for (int r = threadIdx.x; r < n; r += blockDim.x) W[(int64_t)r * B + j] = from_real<T>(r == cand ? 1.0 : 0.0);
        __syncthreads();
      }
      if (nvx + j > 0) {
        orth_project<T, KM>(n, B, j, V, X, nvx, W, scratch, h, j);
        const double n1 = col_norm<T>(n, B, j, W, red);
        orth_project<T, KM>(n, B, j, V, X, nvx, W, scratch, h, j);
        nrm = col_norm<T>(n, B, j, W, red);
        if (nrm < 0.5 * n1) {
          orth_project<T, KM>(n, B, j, V, X, nvx, W, scratch, h, j);
          nrm = col_norm<T>(n, B, j, W, red);
        }
      } else {
        nrm = col_norm<T>(n, B, j, W, red);
      }
      if (cand < 0 && nrm > 0.0 && isfinite(nrm)) break;
      if (cand >= 0 && nrm > 0.5) break;
      if (cand < 0 && threadIdx.x == 0) ctl->degenerate = 1;
    }
    const double inv = 1.0 / nrm;
    for (int r = threadIdx.x; r < n; r += blockDim.x) W[(int64_t)r * B + j] = scal(W[(int64_t)r * B + j], inv);
    __syncthreads();
  }
}

}  // namespace rl
