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
// float (the reduced-precision sketch and QR): the same operations in FP32;
// abs2 widens to double so norms are accumulated in FP64.
template <> __device__ __host__ inline float zero<float>() { return 0.0f; }
template <> __device__ __host__ inline float from_real<float>(double a) { return (float)a; }
__device__ __host__ inline float conj_(float a) { return a; }
__device__ __host__ inline double re_(float a) { return a; }
__device__ __host__ inline double abs2(float a) { return (double)a * (double)a; }
__device__ __host__ inline float add(float a, float b) { return a + b; }
__device__ __host__ inline float sub(float a, float b) { return a - b; }
__device__ __host__ inline float neg(float a) { return -a; }
__device__ __host__ inline float mul(float a, float b) { return a * b; }
__device__ __host__ inline float scal(float a, double s) { return a * (float)s; }
__device__ inline float fmac(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline float cfmac(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline float fnmac(float a, float b, float c) { return fmaf(-a, b, c); }
__device__ inline float divs(float a, float b) { return a / b; }

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
// Within each row of 16 lanes the sums use DPP lane permutations (pairs, quads,
// half-row mirror, row mirror), which run at ALU latency; the four row sums are
// then combined from scalar readlanes, so every lane gets the same value and
// the summation order is fixed.  Callers must have the whole wave active.
// 16-byte streaming loads of A by the kernels that read each element once:
// non-temporal, so the stream does not displace the reused vectors from the
// caches.  (The complex kernels whose vector groups re-read A rely on L2 and
// use ordinary loads.)
typedef double rl_dv2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ld_stream2(const double* p) {
  const rl_dv2 v = __builtin_nontemporal_load(reinterpret_cast<const rl_dv2*>(p));
  return make_double2(v.x, v.y);
}

// Buffer-resource loads.  Word 3 of a raw (stride 0, untyped) gfx9-family
// buffer resource: DATA_FORMAT = 32 bits (bits 15..18 = 4); the hardware
// returns zero for any lane whose access lies past the resource's byte range
// (word 2), so kernels can read a range's tail without branches.
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;
// 16-byte non-temporal load at byte offset voff + soff of a buffer resource
__device__ inline double2 ld_buf_stream2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 2 /* non-temporal */);
  return make_double2(__builtin_bit_cast(double, ((unsigned long long)v[1] << 32) | v[0]),
                      __builtin_bit_cast(double, ((unsigned long long)v[3] << 32) | v[2]));
}

// Index of the calling wave in its workgroup, known to the compiler to be
// wave-uniform (scalar register), so branches on it are scalar branches.
__device__ inline int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ inline double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_1032 = 0xB1;       // quad_perm [1,0,3,2]: partner lane ^ 1
constexpr int DPP_QUAD_2301 = 0x4E;       // quad_perm [2,3,0,1]: partner lane ^ 2
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane 7-j within 8
constexpr int DPP_ROW_MIRROR = 0x140;       // lane 15-j within 16

// sum over the 16 lanes of each row, result in every lane of the row
__device__ inline double row_sum16(double v) {
  v += dpp_d<DPP_QUAD_1032>(v);
  v += dpp_d<DPP_QUAD_2301>(v);
  v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
  v += dpp_d<DPP_ROW_MIRROR>(v);
  return v;
}
__device__ inline cd row_sum16(cd v) { return cd{row_sum16(v.x), row_sum16(v.y)}; }
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ inline float row_sum16(float v) {
  v += dpp_f<DPP_QUAD_1032>(v);
  v += dpp_f<DPP_QUAD_2301>(v);
  v += dpp_f<DPP_ROW_HALF_MIRROR>(v);
  v += dpp_f<DPP_ROW_MIRROR>(v);
  return v;
}
__device__ inline float readlane_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

__device__ inline double wave_sum(double v) {
  v = row_sum16(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ inline cd wave_sum(cd v) { return cd{wave_sum(v.x), wave_sum(v.y)}; }
__device__ inline float wave_sum(float v) {
  v = row_sum16(v);
  return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}
__device__ inline cd readlane_d(cd v, int l) { return cd{readlane_d(v.x, l), readlane_d(v.y, l)}; }
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_d<DPP_QUAD_1032>(v));
  v = fmax(v, dpp_d<DPP_QUAD_2301>(v));
  v = fmax(v, dpp_d<DPP_ROW_HALF_MIRROR>(v));
  v = fmax(v, dpp_d<DPP_ROW_MIRROR>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
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

// Block-wide sums of vals[0..K) (K block-uniform, K <= KMAX); out[k] gets
// sum k.  Each value is reduced over its 16-lane row by DPP, the row sums go
// through LDS.  `scratch` must hold (blockDim.x / 16) * KMAX values of T.
// Contains two __syncthreads.
template <typename T, int KMAX>
__device__ inline void block_sum_many(T (&vals)[KMAX], int K, T* scratch, T* out) {
  const int row = threadIdx.x >> 4;
  const int nrows = blockDim.x >> 4;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      const T v = row_sum16(vals[k]);
      if ((threadIdx.x & 15) == 0) scratch[row * KMAX + k] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < K) {
    T s = zero<T>();
    for (int r = 0; r < nrows; ++r) s = add(s, scratch[r * KMAX + threadIdx.x]);
    out[threadIdx.x] = s;
  }
  __syncthreads();
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
  int32_t lock;        // locking of converged columns is on
  int32_t act;         // bit j set: column j of the block is active (not locked)
  int32_t pad0[1];
  double sigma1;       // Sigma~(1,1) estimate (largest singular value of R)
  double tau;          // tolerance
  double rinv_norm;     // max_j ||R^{-*} V_0(:, j)||, about 1/sigma_min(R) (reduced-precision guard)
  double pad1[7];
};

}  // namespace rl
