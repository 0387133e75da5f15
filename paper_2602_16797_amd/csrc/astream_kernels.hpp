// Device code of the A-stream pass, shared by the instantiation units
// (astream_r2.hip, astream_gd.hip, astream_gc.hip).  See astream.hip for the
// algorithm.
#pragma once

#include "common.hpp"

namespace rl {

template <int B>
struct RowsPerBatch {
  static constexpr int value = (B >= 8) ? 1 : (B >= 4 ? 2 : (B >= 2 ? 4 : 8));
};

// Dot2 accumulation: s + e carries the running sum to about twice the working
// precision (TwoProduct by FMA, TwoSum by Knuth); the wave butterfly combines
// the lanes' (s, e) pairs the same way.
__device__ inline void dot2_add(double a, double b, double& s, double& e) {
  double p, ep, t;
  two_prod(a, b, p, ep);
  two_sum(s, p, s, t);
  e += t + ep;
}
__device__ inline void dot2_wave(double& s, double& e) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double s2 = __shfl_xor(s, o, WAVE);
    const double e2 = __shfl_xor(e, o, WAVE);
    double t;
    two_sum(s, s2, s, t);
    e = e + e2 + t;
  }
}
template <int NS, int B>
__device__ inline double dot2_row(const double (&a)[NS], const double (&w)[NS][B], int j) {
  double s = 0.0, e = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) dot2_add(a[k], w[k][j], s, e);
  dot2_wave(s, e);
  return s + e;
}
// complex: Re = sum a.x w.x - a.y w.y, Im = sum a.x w.y + a.y w.x, each a real Dot2
template <int NS, int B>
__device__ inline cd dot2_row(const cd (&a)[NS], const cd (&w)[NS][B], int j) {
  double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    dot2_add(a[k].x, w[k][j].x, sr, er);
    dot2_add(-a[k].y, w[k][j].y, sr, er);
    dot2_add(a[k].x, w[k][j].y, si, ei);
    dot2_add(a[k].y, w[k][j].x, si, ei);
  }
  dot2_wave(sr, er);
  dot2_wave(si, ei);
  return cd{sr + er, si + ei};
}
// (s, e) += conj(a) * v as Dot2 pairs (component-wise for complex)
__device__ inline void dot2_cacc(double a, double v, double& s, double& e) { dot2_add(a, v, s, e); }
__device__ inline void dot2_cacc(cd a, cd v, cd& s, cd& e) {
  dot2_add(a.x, v.x, s.x, e.x);
  dot2_add(a.y, v.y, s.x, e.x);
  dot2_add(a.x, v.y, s.y, e.y);
  dot2_add(-a.y, v.x, s.y, e.y);
}

template <typename T, int B, int NS, bool DOT2>
__global__ __launch_bounds__(256) void k_astream(const T* __restrict__ A, int64_t lda, int64_t m, int n,
                                                 const T* __restrict__ W, T* __restrict__ AW,
                                                 const T* __restrict__ AVp, const T* __restrict__ AXp, int init,
                                                 T* __restrict__ Gpart, int64_t rows_per_block,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  constexpr int RB = RowsPerBatch<B>::value;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool has_v = AVp != nullptr, has_x = AXp != nullptr;
  T w[NS][B];
  T g1s[NS][B], g1e[NS][B], gx[NS][B], gw[NS][B];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = lane + 64 * s;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      w[s][j] = (c < n) ? W[(int64_t)c * B + j] : zero<T>();
      g1s[s][j] = zero<T>();
      g1e[s][j] = zero<T>();
      gx[s][j] = zero<T>();
      gw[s][j] = zero<T>();
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  for (int64_t rb = r0 + (int64_t)wave * RB; rb < r1; rb += 4 * RB) {
    T a[RB][NS];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = rb + q;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int c = lane + 64 * s;
        a[q][s] = (row < r1 && c < n) ? A[row * lda + c] : zero<T>();
      }
    }
    T av[RB][B], ax[RB][B];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = rb + q;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        av[q][j] = (has_v && row < r1) ? AVp[row * B + j] : zero<T>();
        ax[q][j] = (has_x && row < r1) ? AXp[row * B + j] : zero<T>();
      }
    }
    T y[RB][B];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        if constexpr (DOT2) {
          y[q][j] = dot2_row(a[q], w, j);
        } else {
          T acc = zero<T>();
#pragma unroll
          for (int s = 0; s < NS; ++s) acc = fmac(a[q][s], w[s][j], acc);
          y[q][j] = wave_sum(acc);
        }
      }
    }
    // lane q*B + j writes y[q][j]: RB*B consecutive elements of A_W
    T out = zero<T>();
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (lane == q * B + j) out = y[q][j];
    if (lane < RB * B) {
      const int64_t row = rb + lane / B;
      if (row < r1) AW[rb * B + lane] = out;
    }
    // column sums: group 1 (Dot2) is A^* A_V, or A^* A_W in the start pass
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const T v1 = init ? y[q][j] : av[q][j];
          if constexpr (DOT2) dot2_cacc(a[q][s], v1, g1s[s][j], g1e[s][j]);
          else g1s[s][j] = cfmac(a[q][s], v1, g1s[s][j]);
          if (!init) {
            gx[s][j] = cfmac(a[q][s], ax[q][j], gx[s][j]);
            gw[s][j] = cfmac(a[q][s], y[q][j], gw[s][j]);
          }
        }
  }
  // per wave: sums [G1 | G_X | G_W] (3 n B) then the G1 errors (n B)
  const int64_t plane = (int64_t)n * B;
  T* gp = Gpart + ((int64_t)blockIdx.x * 4 + wave) * 4 * plane;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = lane + 64 * s;
    if (c < n) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int64_t e = (int64_t)c * B + j;
        gp[e] = g1s[s][j];
        gp[plane + e] = gx[s][j];
        gp[2 * plane + e] = gw[s][j];
        gp[3 * plane + e] = g1e[s][j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Real data, even leading dimension: the same pass with 16-byte loads (lane l
// owns the column pair 2l, 2l+1 of every 128-column slot) and the RB*B row
// sums of a batch reduced together.  The compensated transpose-reduction
// halves the values each lane carries at every butterfly stage, so a batch of
// V values costs about 2V + 6 shuffles instead of 12 per value; the finished
// sums are broadcast to every lane with scalar readlanes.

template <int V2, int LOG2V>
__device__ inline void tr_reduce_dot2(double (&s)[V2], double (&e)[V2], int lane) {
#pragma unroll
  for (int st = 0; st < LOG2V; ++st) {
    const int half = V2 >> (st + 1);
    const int o = 32 >> st;
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const double ks = hi ? s[k + half] : s[k];
      const double ke = hi ? e[k + half] : e[k];
      const double ss = hi ? s[k] : s[k + half];
      const double se = hi ? e[k] : e[k + half];
      const double rs = __shfl_xor(ss, o, WAVE);
      const double re = __shfl_xor(se, o, WAVE);
      double t;
      two_sum(ks, rs, s[k], t);
      e[k] = ke + re + t;
    }
  }
#pragma unroll
  for (int o = 32 >> LOG2V; o >= 1; o >>= 1) {
    const double rs = __shfl_xor(s[0], o, WAVE);
    const double re = __shfl_xor(e[0], o, WAVE);
    double t;
    two_sum(s[0], rs, s[0], t);
    e[0] = e[0] + re + t;
  }
}

template <int V2, int LOG2V>
__device__ inline void tr_reduce_plain(double (&s)[V2], int lane) {
#pragma unroll
  for (int st = 0; st < LOG2V; ++st) {
    const int half = V2 >> (st + 1);
    const int o = 32 >> st;
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const double ks = hi ? s[k + half] : s[k];
      const double ss = hi ? s[k] : s[k + half];
      s[k] = ks + __shfl_xor(ss, o, WAVE);
    }
  }
#pragma unroll
  for (int o = 32 >> LOG2V; o >= 1; o >>= 1) s[0] += __shfl_xor(s[0], o, WAVE);
}

// lane holding value index k after the transpose-reduction
template <int LOG2V>
__device__ constexpr int tr_src_lane(int k) {
  int l = 0;
  for (int st = 0; st < LOG2V; ++st) l |= ((k >> (LOG2V - 1 - st)) & 1) << (5 - st);
  return l;
}

template <int B>
struct BatchShape {
  static constexpr int RB = (B >= 8) ? 2 : (B >= 4 ? 4 : (B >= 2 ? 4 : 8));
  static constexpr int V = RB * B;
  static constexpr int V2 = V <= 1 ? 1 : V <= 2 ? 2 : V <= 4 ? 4 : V <= 8 ? 8 : V <= 16 ? 16 : V <= 32 ? 32 : 64;
  static constexpr int LOG2V = V2 == 1 ? 0 : V2 == 2 ? 1 : V2 == 4 ? 2 : V2 == 8 ? 3 : V2 == 16 ? 4 : V2 == 32 ? 5 : 6;
};

template <int B, int NSP, bool DOT2>
__global__ __launch_bounds__(256) void k_astream_r2(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                    const double* __restrict__ W, double* __restrict__ AW,
                                                    const double* __restrict__ AVp, const double* __restrict__ AXp,
                                                    double* __restrict__ Gpart, int64_t rows_per_block, int INIT,
                                                    int aligned, const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  using SH = BatchShape<B>;
  constexpr int RB = SH::RB, V = SH::V, V2 = SH::V2, LOG2V = SH::LOG2V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool has_x = AXp != nullptr;
  double2 w[NSP][B];
  double2 g1s[NSP][B], g1e[NSP][B], gx[NSP][B], gw[NSP][B];
#pragma unroll
  for (int s = 0; s < NSP; ++s) {
    const int c = 2 * lane + 128 * s;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      w[s][j].x = (c < n) ? W[(int64_t)c * B + j] : 0.0;
      w[s][j].y = (c + 1 < n) ? W[(int64_t)(c + 1) * B + j] : 0.0;
      g1s[s][j] = make_double2(0.0, 0.0);
      g1e[s][j] = make_double2(0.0, 0.0);
      gx[s][j] = make_double2(0.0, 0.0);
      gw[s][j] = make_double2(0.0, 0.0);
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  for (int64_t rb = r0 + (int64_t)wave * RB; rb < r1; rb += 4 * RB) {
    double2 a[RB][NSP];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = rb + q;
#pragma unroll
      for (int s = 0; s < NSP; ++s) {
        const int c = 2 * lane + 128 * s;
        if (aligned && row < r1 && c + 1 < n) {
          a[q][s] = *reinterpret_cast<const double2*>(A + row * lda + c);
        } else if (row < r1 && c + 1 < n) {
          a[q][s].x = A[row * lda + c];
          a[q][s].y = A[row * lda + c + 1];
        } else {
          a[q][s].x = (row < r1 && c < n) ? A[row * lda + c] : 0.0;
          a[q][s].y = 0.0;
        }
      }
    }
    // panel values of the batch: one coalesced load, then scalar broadcasts
    double avl = 0.0, axl = 0.0;
    if (!INIT) {
      if (lane < V && rb + lane / B < r1) {
        avl = AVp[rb * B + lane];
        if (has_x) axl = AXp[rb * B + lane];
      }
    }
    // row sums of A W for the batch
    double ys[V2], ye[V2];
#pragma unroll
    for (int v = 0; v < V2; ++v) {
      ys[v] = 0.0;
      ye[v] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int v = q * B + j;
#pragma unroll
        for (int s = 0; s < NSP; ++s) {
          if constexpr (DOT2) {
            dot2_add(a[q][s].x, w[s][j].x, ys[v], ye[v]);
            dot2_add(a[q][s].y, w[s][j].y, ys[v], ye[v]);
          } else {
            ys[v] = fma(a[q][s].x, w[s][j].x, ys[v]);
            ys[v] = fma(a[q][s].y, w[s][j].y, ys[v]);
          }
        }
      }
    if constexpr (DOT2) tr_reduce_dot2<V2, LOG2V>(ys, ye, lane);
    else tr_reduce_plain<V2, LOG2V>(ys, lane);
    const double mine = DOT2 ? ys[0] + ye[0] : ys[0];
    double y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = readlane_d(mine, tr_src_lane<LOG2V>(v));
    double out = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (lane == v) out = y[v];
    if (lane < V && rb + lane / B < r1) AW[rb * B + lane] = out;
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int v = q * B + j;
        const double yv = y[v];
        const double av = INIT ? yv : readlane_d(avl, v);
        const double ax = INIT ? 0.0 : readlane_d(axl, v);
#pragma unroll
        for (int s = 0; s < NSP; ++s) {
          if constexpr (DOT2) {
            dot2_add(a[q][s].x, av, g1s[s][j].x, g1e[s][j].x);
            dot2_add(a[q][s].y, av, g1s[s][j].y, g1e[s][j].y);
          } else {
            g1s[s][j].x = fma(a[q][s].x, av, g1s[s][j].x);
            g1s[s][j].y = fma(a[q][s].y, av, g1s[s][j].y);
          }
          if (!INIT) {
            gx[s][j].x = fma(a[q][s].x, ax, gx[s][j].x);
            gx[s][j].y = fma(a[q][s].y, ax, gx[s][j].y);
            gw[s][j].x = fma(a[q][s].x, yv, gw[s][j].x);
            gw[s][j].y = fma(a[q][s].y, yv, gw[s][j].y);
          }
        }
      }
  }
  const int64_t plane = (int64_t)n * B;
  double* gp = Gpart + ((int64_t)blockIdx.x * 4 + wave) * 4 * plane;
#pragma unroll
  for (int s = 0; s < NSP; ++s) {
    const int c = 2 * lane + 128 * s;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (c + h < n) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const int64_t e = (int64_t)(c + h) * B + j;
          gp[e] = h ? g1s[s][j].y : g1s[s][j].x;
          gp[plane + e] = h ? gx[s][j].y : gx[s][j].x;
          gp[2 * plane + e] = h ? gw[s][j].y : gw[s][j].x;
          gp[3 * plane + e] = h ? g1e[s][j].y : g1e[s][j].x;
        }
      }
    }
  }
}

}  // namespace rl
