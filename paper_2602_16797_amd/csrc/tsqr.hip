// TSQR of a tall m x t block (t <= 32), the first half of the Rayleigh-Ritz
// step: the paper computes [~, Theta, C] = svd(A_T) of the m x 3b trial-space
// product (Alg. rlopcg and Alg. rlobpcg, "Rayleigh-Ritz"); with A_T = Q R_T
// the right singular data of A_T are those of the small R_T.
//
// A Gram-matrix route (A_T^* A_T) would square the condition number of A_T,
// whose smallest singular value is the wanted sigma_min; Householder QR keeps
// a column-wise backward error, which is what the small singular values need.
//
// k_tsqr: a workgroup owns a range of rows and walks it in LDS tiles of 256
// rows (one row per thread, column-major in LDS).  Rows 0..t-1 of the tile
// hold the running R; rows t..255 take the next 256-t input rows; a full
// Householder QR of the tile leaves the new R on top.  The input rows are
// [P0(r,:), P1(r,:), P2(r,:)] from up to three row-major panels, so the three
// m x b blocks A_V, A_X, A_W are read in place.  The per-workgroup R factors
// are written row-major (t x t each) and form a (groups*t) x t matrix that the
// same kernel reduces again until one R_T remains.
#include "common.hpp"
#include "kernels.hpp"

namespace rl {

constexpr int TS_TILE = 256;
constexpr int TS_TMAX = 32;

template <typename T>
__device__ inline void ts_block_sum_many(T (&vals)[TS_TMAX], int K, T* scratch, T* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < TS_TMAX; ++k) {
    if (k < K) {
      T v = wave_sum(vals[k]);
      if (lane == 0) scratch[wid * TS_TMAX + k] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    T s = zero<T>();
    for (int w = 0; w < TS_TILE / 64; ++w) s = add(s, scratch[w * TS_TMAX + threadIdx.x]);
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ inline double ts_im(double) { return 0.0; }
__device__ inline double ts_im(cd a) { return a.y; }

template <typename T>
__global__ __launch_bounds__(TS_TILE) void k_tsqr(const T* __restrict__ P0, int b0, const T* __restrict__ P1, int b1,
                                                  const T* __restrict__ P2, int b2, int64_t m, int64_t rows_per_block,
                                                  T* __restrict__ Rout, const Ctl* __restrict__ ctl, int check_done) {
  if (check_done && ctl->done) return;
  extern __shared__ double smem_d[];
  T* tile = reinterpret_cast<T*>(smem_d);  // t columns x TS_TILE rows
  __shared__ T scratch[(TS_TILE / 64) * TS_TMAX];
  __shared__ T outs[TS_TMAX];
  __shared__ double red[TS_TILE / 64];
  const int t = b0 + b1 + b2;
  const int r = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t g1 = (g0 + rows_per_block < m) ? g0 + rows_per_block : m;
  for (int c = 0; c < t; ++c) tile[c * TS_TILE + r] = zero<T>();
  const int fresh = TS_TILE - t;
  for (int64_t g = g0; g < g1; g += fresh) {
    __syncthreads();
    if (r >= t) {
      const int64_t row = g + (r - t);
      if (row < g1) {
        for (int c = 0; c < b0; ++c) tile[c * TS_TILE + r] = P0[row * b0 + c];
        for (int c = 0; c < b1; ++c) tile[(b0 + c) * TS_TILE + r] = P1[row * b1 + c];
        for (int c = 0; c < b2; ++c) tile[(b0 + b1 + c) * TS_TILE + r] = P2[row * b2 + c];
      } else {
        for (int c = 0; c < t; ++c) tile[c * TS_TILE + r] = zero<T>();
      }
    } else {
      // clear the reflector entries left below R's diagonal
      for (int c = 0; c < r; ++c) tile[c * TS_TILE + r] = zero<T>();
    }
    __syncthreads();
    for (int j = 0; j < t; ++j) {
      T* col = tile + j * TS_TILE;
      double xs = (r > j) ? abs2(col[r]) : 0.0;
      xs = block_sum(xs, red);
      const T alpha = col[j];
      const bool noref = (xs == 0.0) && (ts_im(alpha) == 0.0);
      T tau = zero<T>(), sc = zero<T>();
      double beta = re_(alpha);
      if (!noref) {
        const double nrm = sqrt(abs2(alpha) + xs);
        beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
        tau = divs(sub(from_real<T>(beta), alpha), from_real<T>(beta));
        sc = divs(from_real<T>(1.0), sub(alpha, from_real<T>(beta)));
      }
      __syncthreads();
      if (!noref) {
        if (r > j) col[r] = mul(col[r], sc);
        if (r == j) col[j] = from_real<T>(beta);
      }
      __syncthreads();
      const int K = t - j - 1;
      if (K > 0 && !noref) {
        T vals[TS_TMAX];
        const T vr = (r > j) ? col[r] : (r == j ? from_real<T>(1.0) : zero<T>());
#pragma unroll
        for (int k = 0; k < TS_TMAX; ++k) {
          vals[k] = zero<T>();
          if (k < K) vals[k] = cfmac(vr, tile[(j + 1 + k) * TS_TILE + r], zero<T>());
        }
        ts_block_sum_many<T>(vals, K, scratch, outs);
        if (r >= j) {
          const T ct = conj_(tau);
          for (int k = 0; k < K; ++k) {
            T* y = tile + (j + 1 + k) * TS_TILE + r;
            *y = fnmac(mul(ct, outs[k]), vr, *y);
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // write R (t x t row-major), zero below the diagonal
  T* out = Rout + (int64_t)blockIdx.x * t * t;
  for (int i = threadIdx.x; i < t * t; i += blockDim.x) {
    const int rr = i / t, cc = i % t;
    out[i] = (cc >= rr) ? tile[cc * TS_TILE + rr] : zero<T>();
  }
}

int64_t tsqr_groups(int64_t m, int t) {
  const int64_t per = 4 * (int64_t)(TS_TILE - t);
  int64_t g = (m + per - 1) / per;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return g;
}

template <typename T>
static hipError_t tsqr_impl(hipStream_t st, const T* P0, int b0, const T* P1, int b1, const T* P2, int b2, int64_t m,
                            T* bufA, T* bufB, T** Rfinal, const Ctl* ctl, int check_done) {
  const int t = b0 + b1 + b2;
  if (t < 1 || t > TS_TMAX) return hipErrorInvalidValue;
  const size_t lds = (size_t)t * TS_TILE * sizeof(T);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_tsqr<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int64_t groups = tsqr_groups(m, t);
  int64_t rows = (m + groups - 1) / groups;
  hipLaunchKernelGGL(k_tsqr<T>, dim3((unsigned)groups), dim3(TS_TILE), lds, st, P0, b0, P1, b1, P2, b2, m, rows, bufA,
                     ctl, check_done);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  T* cur = bufA;
  T* nxt = bufB;
  while (groups > 1) {
    const int64_t mm = groups * t;
    int64_t g2 = tsqr_groups(mm, t);
    if (g2 >= groups) g2 = groups / 2 > 0 ? groups / 2 : 1;
    const int64_t rows2 = (mm + g2 - 1) / g2;
    hipLaunchKernelGGL(k_tsqr<T>, dim3((unsigned)g2), dim3(TS_TILE), lds, st, (const T*)cur, t, (const T*)nullptr, 0,
                       (const T*)nullptr, 0, mm, rows2, nxt, ctl, check_done);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    T* tmp = cur;
    cur = nxt;
    nxt = tmp;
    groups = g2;
  }
  *Rfinal = cur;
  return hipSuccess;
}

hipError_t launch_tsqr(hipStream_t st, bool cplx, const void* P0, int b0, const void* P1, int b1, const void* P2,
                       int b2, int64_t m, void* bufA, void* bufB, void** Rfinal, const Ctl* ctl, int check_done) {
  if (cplx)
    return tsqr_impl<cd>(st, (const cd*)P0, b0, (const cd*)P1, b1, (const cd*)P2, b2, m, (cd*)bufA, (cd*)bufB,
                         (cd**)Rfinal, ctl, check_done);
  return tsqr_impl<double>(st, (const double*)P0, b0, (const double*)P1, b1, (const double*)P2, b2, m,
                           (double*)bufA, (double*)bufB, (double**)Rfinal, ctl, check_done);
}

}  // namespace rl
