// Shared device helpers for the RLOBPCG HIP library (gfx950, wave64).
//
// Scalar types: real FP64 (double) and complex FP64 (cd, interleaved re/im,
// layout-compatible with C99 double _Complex and torch.complex128).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rl {

constexpr int WAVE = 64;

struct cd {
  double x, y;
};

// ----- scalar algebra, overloaded for double and cd -------------------------
__device__ __host__ inline double zero_d() { return 0.0; }
template <typename T> __device__ __host__ inline T zero();
template <> __device__ __host__ inline double zero<double>() { return 0.0; }
template <> __device__ __host__ inline cd zero<cd>() { return cd{0.0, 0.0}; }

template <typename T> __device__ __host__ inline T from_real(double a);
template <> __device__ __host__ inline double from_real<double>(double a) { return a; }
template <> __device__ __host__ inline cd from_real<cd>(double a) { return cd{a, 0.0}; }

__device__ __host__ inline double conj_(double a) { return a; }
__device__ __host__ inline cd conj_(cd a) { return cd{a.x, -a.y}; }
__device__ __host__ inline double re_(double a) { return a; }
__device__ __host__ inline double re_(cd a) { return a.x; }
__device__ __host__ inline double abs2(double a) { return a * a; }
__device__ __host__ inline double abs2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ __host__ inline double add(double a, double b) { return a + b; }
__device__ __host__ inline cd add(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __host__ inline double sub(double a, double b) { return a - b; }
__device__ __host__ inline cd sub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __host__ inline double neg(double a) { return -a; }
__device__ __host__ inline cd neg(cd a) { return cd{-a.x, -a.y}; }
__device__ __host__ inline double mul(double a, double b) { return a * b; }
__device__ __host__ inline cd mul(cd a, cd b) {
  return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __host__ inline double scal(double a, double s) { return a * s; }
__device__ __host__ inline cd scal(cd a, double s) { return cd{a.x * s, a.y * s}; }

// a*b + c
__device__ inline double fmac(double a, double b, double c) { return fma(a, b, c); }
__device__ inline cd fmac(cd a, cd b, cd c) {
  return cd{fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
// conj(a)*b + c
__device__ inline double cfmac(double a, double b, double c) { return fma(a, b, c); }
__device__ inline cd cfmac(cd a, cd b, cd c) {
  return cd{fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y))};
}
// c - a*b
__device__ inline double fnmac(double a, double b, double c) { return fma(-a, b, c); }
__device__ inline cd fnmac(cd a, cd b, cd c) {
  return cd{fma(-a.x, b.x, fma(a.y, b.y, c.x)), fma(-a.x, b.y, fma(-a.y, b.x, c.y))};
}
// a / b for cd via Smith's algorithm
__device__ inline double divs(double a, double b) { return a / b; }
__device__ inline cd divs(cd a, cd b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return cd{(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return cd{(a.x * r + a.y) / den, (a.y * r - a.x) / den};
  }
}

// ----- wave-level reductions (64 lanes) --------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline cd wave_sum(cd v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v.x += __shfl_xor(v.x, o, WAVE);
    v.y += __shfl_xor(v.y, o, WAVE);
  }
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ inline double shfl(double v, int src) { return __shfl(v, src, WAVE); }
__device__ inline cd shfl(cd v, int src) { return cd{__shfl(v.x, src, WAVE), __shfl(v.y, src, WAVE)}; }

// Block-wide sum of one value; every thread gets the result.  `red` must hold
// at least blockDim.x/64 values of T.  Contains two __syncthreads.
template <typename T>
__device__ inline T block_sum(T v, T* red) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = zero<T>();
  for (int w = 0; w < nw; ++w) s = add(s, red[w]);
  return s;
}

// ----- error-free transformations (Knuth TwoSum, FMA TwoProduct) -------------
__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ inline void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}

// ----- device control block ---------------------------------------------------
// One per solve, in device memory.  Kernels of the iteration return at once
// when `done` is set, so iterations enqueued past the stop are no-ops.
struct Ctl {
  int32_t done;        // stop rule fired
  int32_t iter;        // loop index i of the next iteration
  int32_t has_x;       // X (and A_X) hold data (t = 3b)
  int32_t status;      // 0 stopped by the rule, 1 max_iter reached
  int32_t degenerate;  // a Normalize/Orth met a zero vector
  int32_t nonfinite;   // NaN or Inf seen in S*A
  int32_t zero_theta;  // a final theta was exactly zero
  int32_t stop_rule;   // 0 paper, 1 tol only, 2 none
  int32_t check_every;
  int32_t max_iter;
  int32_t b;           // block size
  int32_t rr_mode;     // trial basis of the last Rayleigh-Ritz: 0 [V], 1 [V W], 2 [V X W]
  int32_t x_update;    // the last Rayleigh-Ritz produced C_X (X is updated)
  int32_t pad0[3];
  double sigma1;       // Sigma~(1,1) estimate (largest singular value of R)
  double tau;          // tolerance
  double pad1[8];
};

}  // namespace rl
