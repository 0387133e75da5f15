// Register-resident Orth (k_orth_reg), instantiated per scalar type by
// orth_reg_d.hip and orth_reg_c.hip.
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "orth.hpp"
#include "tr_reduce.hpp"

namespace rl {

// ---------------------------------------------------------------------------
// The same Orth with W held in registers, for n <= NS_THREADS * RPT: thread t
// holds rows t + NS_THREADS i (i < RPT) of W, so every step is one reduction
// round (a wave transpose-reduction of the thread's partial sums, then the sum
// over the waves through LDS in wave order) instead of a pass over W in
// global memory per projection.
//  * BCGS2 against [V X]: two block projections W -= [V X]([V X]^* W), one
//    round each (the second also yields the column norms before it);
//  * Orth(W): CGS2 column by column; column j takes one round for its dots
//    with the earlier columns and its norm, and one for the second pass's
//    dots and the norm after the first; when the first pass removes most of
//    the column (its rounding then leaves parts along [V X] as well, which
//    orth_block's joint passes remove) that round takes the dots with
//    [V X W(:, 0:j)] jointly.  The norm after the second pass follows by
//    Pythagoras (the second pass removes a tiny part whenever the
//    twice-is-enough test passes; a third, joint round runs when it does
//    not).  A column that the block projections shrank below half is
//    projected on [V X] once more, the same test as orth_block applies to its
//    passes (the first column's norm is then formed afresh).
// A column that vanishes (or turns non-finite) hands the block, written back,
// to orth_block, which completes it with a unit vector and sets the
// degenerate flag.  Locked columns (bit clear in `keep`) are zero.
// f(integral_constant<int, J>) for J = J0 .. J1-1, unrolled at compile time
template <int J0, int J1>
struct StaticFor {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    f(std::integral_constant<int, J0>{});
    StaticFor<J0 + 1, J1>::run(f);
  }
};
template <int J1>
struct StaticFor<J1, J1> {
  template <typename F>
  __device__ __forceinline__ static void run(F&&) {}
};
template <typename T>
struct NDbl {
  static constexpr int v = 1;
};
template <>
struct NDbl<cd> {
  static constexpr int v = 2;
};
__device__ inline void put_d(double* d, int i, double a) { d[i] = a; }
__device__ inline void put_d(double* d, int i, cd a) {
  d[2 * i] = a.x;
  d[2 * i + 1] = a.y;
}
template <typename T>
__device__ inline T get_t(const double* d, int i);
template <>
__device__ inline double get_t<double>(const double* d, int i) {
  return d[i];
}
template <>
__device__ inline cd get_t<cd>(const double* d, int i) {
  return cd{d[2 * i], d[2 * i + 1]};
}
template <int N>
struct Pow2Up {
  static constexpr int v = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : N <= 16 ? 16 : N <= 32 ? 32 : 64;
  static constexpr int log = v == 1 ? 0 : v == 2 ? 1 : v == 4 ? 2 : v == 8 ? 3 : v == 16 ? 4 : v == 32 ? 5 : 6;
};
// Wave sums of v[0..nv) (nv <= V2) into dst[0..nv) of this wave's LDS slot.
template <int V2, int LOG2V>
__device__ inline void wave_sums_to(double (&v)[V2], int nv, int lane, double* dst) {
  tr_reduce_plain<V2, LOG2V>(v, lane);
  int idx = 0;
#pragma unroll
  for (int st = 0; st < LOG2V; ++st) idx |= ((lane >> (5 - st)) & 1) << (LOG2V - 1 - st);
  if ((lane & ((64 >> LOG2V) - 1)) == 0 && idx < nv) dst[idx] = v[0];
}
// out[e] = sum over the waves of part[w * stride + e], e < nv; two barriers
__device__ inline void waves_sum(const double* part, int stride, int nv, double* out) {
  __syncthreads();
  for (int e = threadIdx.x; e < nv; e += NS_THREADS) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NS_THREADS / 64; ++w) s += part[w * stride + e];
    out[e] = s;
  }
  __syncthreads();
}

template <typename T, int B, int RPT, int KM>
__global__ __launch_bounds__(NS_THREADS) void k_orth_reg(int n, const T* __restrict__ V, const T* __restrict__ X,
                                                         int project, int with_x, T* __restrict__ W,
                                                         Ctl* __restrict__ ctl, int check_done, int masked) {
  if (check_done && ctl->done) return;
  constexpr int ND = NDbl<T>::v;
  // the second block projection's sums, or a joint round's
  constexpr int NVMAX = (2 * B * B * ND + B) > ((3 * B - 1) * ND + 1) ? (2 * B * B * ND + B) : ((3 * B - 1) * ND + 1);
  constexpr int VB = Pow2Up<B * ND>::v, LB = Pow2Up<B * ND>::log;          // one [V X] column's dots
  constexpr int VJ = Pow2Up<(B - 1) * ND + 1>::v, LJ = Pow2Up<(B - 1) * ND + 1>::log;  // column rounds
  constexpr int VX = Pow2Up<2 * B * ND>::v, LX = Pow2Up<2 * B * ND>::log;  // one column against [V X]
  constexpr int VJX = Pow2Up<(3 * B - 1) * ND + 1>::v, LJX = Pow2Up<(3 * B - 1) * ND + 1>::log;  // joint rounds
  __shared__ double part[(NS_THREADS / 64) * NVMAX];
  __shared__ double sums[NVMAX];
  __shared__ double n1sq[B];
  __shared__ double gsum[2 * B * ND];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int keep = (masked && ctl->lock) ? ctl->act : -1;
  const int nvx = project ? (with_x ? 2 * B : B) : 0;
  double* mypart = part + wave * NVMAX;
  auto yval = [&](int r, int k) __attribute__((always_inline)) -> T { return (k < B) ? V[(int64_t)r * B + k] : X[(int64_t)r * B + (k - B)]; };
  T w[RPT][B];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + NS_THREADS * i;
#pragma unroll
    for (int c = 0; c < B; ++c) w[i][c] = (r < n && ((keep >> c) & 1)) ? W[(int64_t)r * B + c] : zero<T>();
  }
  // --- BCGS2 against [V X] ---------------------------------------------------
  for (int pass = 0; pass < 2 && nvx > 0; ++pass) {
    for (int k = 0; k < nvx; ++k) {
      double v[VB];
#pragma unroll
      for (int e = 0; e < VB; ++e) v[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + NS_THREADS * i;
        if (r < n) {
          const T y = yval(r, k);
#pragma unroll
          for (int c = 0; c < B; ++c) {
            T d = get_t<T>(v, c);
            d = cfmac(y, w[i][c], d);
            put_d(v, c, d);
          }
        }
      }
      wave_sums_to<VB, LB>(v, B * ND, lane, mypart + k * B * ND);
    }
    if (pass == 1) {
      // column norms before the second projection
      double v[Pow2Up<B>::v];
#pragma unroll
      for (int e = 0; e < Pow2Up<B>::v; ++e) v[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int c = 0; c < B; ++c) v[c] += abs2(w[i][c]);
      wave_sums_to<Pow2Up<B>::v, Pow2Up<B>::log>(v, B, lane, mypart + nvx * B * ND);
    }
    waves_sum(part, NVMAX, nvx * B * ND + (pass == 1 ? B : 0), sums);
    if (pass == 1 && tid < B) n1sq[tid] = sums[nvx * B * ND + tid];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = tid + NS_THREADS * i;
      if (r < n) {
        for (int k = 0; k < nvx; ++k) {
          const T y = yval(r, k);
#pragma unroll
          for (int c = 0; c < B; ++c) w[i][c] = fnmac(y, get_t<T>(sums, k * B + c), w[i][c]);
        }
      }
    }
  }
  __syncthreads();  // n1sq visible
  // --- Orth(W): CGS2 column by column (unrolled at compile time, so the
  // register rows are indexed statically) --------------------------------------
  bool degenerate = false;
  StaticFor<0, B>::run([&](auto jc) __attribute__((always_inline)) {
    constexpr int j = decltype(jc)::value;
    if (degenerate || !((keep >> j) & 1)) return;  // a locked column stays zero
    // round: dots of column j with columns c < j, then its squared norm
    auto column_round = [&](double* out) __attribute__((always_inline)) {
      double v[VJ];
#pragma unroll
      for (int e = 0; e < VJ; ++e) v[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int c = 0; c < j; ++c) {
          T d = get_t<T>(v, c);
          d = cfmac(w[i][c], w[i][j], d);
          put_d(v, c, d);
        }
        v[j * ND] += abs2(w[i][j]);
      }
      wave_sums_to<VJ, LJ>(v, j * ND + 1, lane, mypart);
      waves_sum(part, NVMAX, j * ND + 1, out);
    };
    auto project_prev = [&](const double* h) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int c = 0; c < j; ++c) w[i][j] = fnmac(w[i][c], get_t<T>(h, c), w[i][j]);
    };
    // joint round: dots of column j with the columns c < j (out[0 .. j ND)),
    // its squared norm (out[j ND]) and its dots with [V X] (out[j ND + 1 ..),
    // k < nvx); every register offset is fixed at compile time
    auto joint_round = [&](double* out) __attribute__((always_inline)) {
      double v[VJX];
#pragma unroll
      for (int e = 0; e < VJX; ++e) v[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int c = 0; c < j; ++c) {
          T d = get_t<T>(v, c);
          d = cfmac(w[i][c], w[i][j], d);
          put_d(v, c, d);
        }
        v[j * ND] += abs2(w[i][j]);
        const int r = tid + NS_THREADS * i;
        if (r < n) {
#pragma unroll
          for (int k = 0; k < 2 * B; ++k) {
            if (k < nvx) {
              T d = get_t<T>(v + j * ND + 1, k);
              d = cfmac(yval(r, k), w[i][j], d);
              put_d(v + j * ND + 1, k, d);
            }
          }
        }
      }
      wave_sums_to<VJX, LJX>(v, (nvx + j) * ND + 1, lane, mypart);
      waves_sum(part, NVMAX, (nvx + j) * ND + 1, out);
    };
    auto project_joint = [&](const double* h) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + NS_THREADS * i;
        if (r < n) {
          for (int k = 0; k < nvx; ++k) w[i][j] = fnmac(yval(r, k), get_t<T>(h + j * ND + 1, k), w[i][j]);
        }
#pragma unroll
        for (int c = 0; c < j; ++c) w[i][j] = fnmac(w[i][c], get_t<T>(h, c), w[i][j]);
      }
    };
    auto removed = [&](const double* h) __attribute__((always_inline)) {
      double s2 = 0.0;
#pragma unroll
      for (int c = 0; c < j; ++c) s2 += abs2(get_t<T>(h, c));
      return s2;
    };
    auto removed_joint = [&](const double* h) __attribute__((always_inline)) {
      double s2 = 0.0;
#pragma unroll
      for (int c = 0; c < j; ++c) s2 += abs2(get_t<T>(h, c));
      for (int k = 0; k < nvx; ++k) s2 += abs2(get_t<T>(h + j * ND + 1, k));
      return s2;
    };
    column_round(sums);
    double sq = sums[j * ND];
    if (nvx > 0 && sq < 0.25 * n1sq[j]) {
      // the block projections removed most of the column: once more against [V X]
      double v[VX];
#pragma unroll
      for (int e = 0; e < VX; ++e) v[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + NS_THREADS * i;
        if (r < n) {
#pragma unroll
          for (int k = 0; k < 2 * B; ++k) {
            if (k < nvx) {
              T d = get_t<T>(v, k);
              d = cfmac(yval(r, k), w[i][j], d);
              put_d(v, k, d);
            }
          }
        }
      }
      wave_sums_to<VX, LX>(v, nvx * ND, lane, mypart);
      waves_sum(part, NVMAX, nvx * ND, gsum);
      double g2 = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + NS_THREADS * i;
        if (r < n) {
          for (int k = 0; k < nvx; ++k) w[i][j] = fnmac(yval(r, k), get_t<T>(gsum, k), w[i][j]);
        }
      }
      for (int k = 0; k < nvx; ++k) g2 += abs2(get_t<T>(gsum, k));
      sq -= g2;
      // what this pass removed need not be small next to what is left, so the
      // first column's norm is formed afresh (a later column's comes from its
      // own rounds below)
      if (j == 0) {
        column_round(sums);
        sq = sums[0];
      }
    }
    double nrmsq = sq;
    if (j > 0) {
      // first pass against the earlier columns; when it removes most of the
      // column its rounding leaves parts along [V X] as well, and the later
      // passes run against [V X W(:, 0:j)] jointly
      // the first pass's share of the column (by Pythagoras from round one's
      // dots: a decision, not a norm) says whether it cancels
      const bool cancels = sq - removed(sums) < 0.25 * sq;
      project_prev(sums);
      double n1;
      if (cancels) {
        joint_round(sums);
        n1 = sums[j * ND];
        project_joint(sums);
        nrmsq = n1 - removed_joint(sums);
      } else {
        column_round(sums);
        n1 = sums[j * ND];
        project_prev(sums);
        nrmsq = n1 - removed(sums);
      }
      if (nrmsq < 0.25 * n1) {
        joint_round(sums);
        const double n2 = sums[j * ND];
        project_joint(sums);
        nrmsq = n2 - removed_joint(sums);
      }
    }
    if (!(nrmsq > 0.0) || !isfinite(nrmsq)) {
      degenerate = true;
      return;
    }
    const double inv = 1.0 / sqrt(nrmsq);
#pragma unroll
    for (int i = 0; i < RPT; ++i) w[i][j] = scal(w[i][j], inv);
  });
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + NS_THREADS * i;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < B; ++c) W[(int64_t)r * B + c] = w[i][c];
    }
  }
  if (degenerate) {
    __syncthreads();
    orth_block<T, KM>(n, B, V, X, project, with_x, W, ctl, keep);
  }
}

template <typename T, int B, int KM>
static bool orth_reg_go(hipStream_t st, int n, const void* V, const void* X, int project, int with_x, void* W,
                        Ctl* ctl, int check_done, int masked) {
  constexpr int maxr = std::is_same<T, cd>::value ? 4 : 8;
  const int rpt = (n + NS_THREADS - 1) / NS_THREADS;
#define RL_OR(R)                                                                                                    \
  if constexpr (R <= maxr) {                                                                                        \
    if (rpt <= R) {                                                                                                 \
      hipLaunchKernelGGL((k_orth_reg<T, B, R, KM>), dim3(1), dim3(NS_THREADS), 0, st, n, (const T*)V, (const T*)X, \
                         project, with_x, (T*)W, ctl, check_done, masked);                                          \
      return true;                                                                                                  \
    }                                                                                                               \
  }
  RL_OR(1) RL_OR(2) RL_OR(4) RL_OR(8)
#undef RL_OR
  return false;
}

// k_orth_reg for n <= 8 NS_THREADS (real) / 4 NS_THREADS (complex), b <= 10
template <typename T>
static bool orth_reg_dispatch(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x,
                              void* W, Ctl* ctl, int check_done, int masked) {
  switch (B) {
    case 1: return orth_reg_go<T, 1, 4>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 2: return orth_reg_go<T, 2, 8>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 3: return orth_reg_go<T, 3, 16>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 4: return orth_reg_go<T, 4, 16>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 5: return orth_reg_go<T, 5, 16>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 6: return orth_reg_go<T, 6, 32>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 7: return orth_reg_go<T, 7, 32>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 8: return orth_reg_go<T, 8, 32>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 9: return orth_reg_go<T, 9, 32>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    case 10: return orth_reg_go<T, 10, 32>(st, n, V, X, project, with_x, W, ctl, check_done, masked);
    default: return false;
  }
}

}  // namespace rl
