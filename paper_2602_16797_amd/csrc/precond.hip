// The loop preconditioners of the comparison methods (Sec. 1.1, illustrative
// example): LOBPCG with the diagonal preconditioner P = diag(||A(:, i)||^{-1})
// and with none.  The method itself uses P = R^{-1} from the sketch
// (k_trmv in nside.hip); these replace only that step of the loop.
//
// k_colnorm2_part  per-workgroup sums of |A(r, c)|^2 over a range of rows:
//                  a wave takes a row at a time (lane l owns columns l, l+64,
//                  ...; coalesced), the four waves of a workgroup walk
//                  interleaved rows and are combined through LDS in wave
//                  order.  A complex A is read as 2n real columns.
// k_colnorm2_fin   sums the partials in workgroup order (deterministic),
//                  combines the real and imaginary columns, and stores
//                  dscale(i) = 1 / ||A(:, i)||^2 (1 for a zero column).
// k_prec_apply     W = diag(dscale) R (RL_PREC_DIAG) or W = R (RL_PREC_NONE).
#include "common.hpp"
#include "kernels.hpp"

namespace rl {

constexpr int CN_MAXCOLS = 2048;  // doubles per row: n <= 1024 complex
constexpr int CN_MAXG = 1024;     // workgroups of the partial pass

__global__ __launch_bounds__(256) void k_colnorm2_part(const double* __restrict__ A, int64_t lda_d, int64_t m,
                                                       int ncols_d, int64_t rows_per, double* __restrict__ part) {
  __shared__ double red[4][128];
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = (r0 + rows_per < m) ? r0 + rows_per : m;
  double* out = part + (int64_t)blockIdx.x * ncols_d;
  // columns in slices of 512 per lane set (8 per lane), so the accumulators
  // stay in registers for any width
  for (int c0 = 0; c0 < ncols_d; c0 += 512) {
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int64_t r = r0 + wave; r < r1; r += 4) {
      const double* row = A + r * lda_d;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + lane + 64 * u;
        const double x = (c < ncols_d) ? row[c] : 0.0;
        acc[u] = fma(x, x, acc[u]);
      }
    }
    // combine the four waves in wave order, 128 columns at a time
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 2; ++u) red[wave][lane + 64 * u] = acc[2 * h + u];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int c = c0 + lane + 64 * (2 * h + u);
          const int e = lane + 64 * u;
          if (c < ncols_d) out[c] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        }
      }
    }
  }
}

__global__ void k_colnorm2_fin(const double* __restrict__ part, int ng, int n, int es, double* __restrict__ dscale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ncols_d = n * es;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) {
    const double* p = part + (int64_t)g * ncols_d + (int64_t)i * es;
    s += (es == 2) ? p[0] + p[1] : p[0];
  }
  dscale[i] = (s > 0.0) ? 1.0 / s : 1.0;
}

template <typename T>
__global__ void k_prec_apply(int64_t cnt, int B, const double* __restrict__ dscale, const T* __restrict__ R,
                             T* __restrict__ W, const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  W[e] = dscale ? scal(R[e], dscale[e / B]) : R[e];
}

// workgroups of the partial pass: about 64 rows each, at most CN_MAXG
int64_t colnorm_groups(int64_t m) {
  int64_t g = (m + 63) / 64;
  if (g > CN_MAXG) g = CN_MAXG;
  return g < 1 ? 1 : g;
}

hipError_t launch_colnorm_scale(hipStream_t st, bool cplx, const double* A, int64_t lda_d, int64_t m, int n,
                                double* part, double* dscale) {
  const int es = cplx ? 2 : 1;
  const int ncols_d = n * es;
  if (n < 1 || ncols_d > CN_MAXCOLS || lda_d < ncols_d) return hipErrorInvalidValue;
  const int64_t g = colnorm_groups(m);
  const int64_t rows = (m + g - 1) / g;
  hipLaunchKernelGGL(k_colnorm2_part, dim3((unsigned)g), dim3(256), 0, st, A, lda_d, m, ncols_d, rows, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colnorm2_fin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double*)part,
                     (int)g, n, es, dscale);
  return hipGetLastError();
}

hipError_t launch_prec_apply(hipStream_t st, bool cplx, int n, int B, const double* dscale, const void* R, void* W,
                             const Ctl* ctl) {
  const int64_t cnt = (int64_t)n * B;
  const dim3 grid((unsigned)((cnt + 255) / 256));
  if (cplx)
    hipLaunchKernelGGL(k_prec_apply<cd>, grid, dim3(256), 0, st, cnt, B, dscale, (const cd*)R, (cd*)W, ctl);
  else
    hipLaunchKernelGGL(k_prec_apply<double>, grid, dim3(256), 0, st, cnt, B, dscale, (const double*)R, (double*)W,
                       ctl);
  return hipGetLastError();
}

}  // namespace rl
