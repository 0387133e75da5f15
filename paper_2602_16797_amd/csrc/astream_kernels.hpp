// Device code of the A-stream pass, shared by the instantiation units
// (astream_r2.hip, astream_cs.hip, astream_ccs.hip, astream_c2.hip,
// astream_gd.hip, astream_gc.hip).  See astream.hip for the algorithm.
#pragma once

#include "common.hpp"
#include "tr_reduce.hpp"

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
  const int lane = threadIdx.x & 63, wave = wave_index();
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


template <int B>
struct BatchShape {
  // rows per wave batch: the transpose-reduction of a batch costs about one
  // butterfly stage per value plus log2(64 / values) stages, so more rows per
  // batch amortise the all-reduce stages
  static constexpr int RB = 4;
  static constexpr int V = RB * B;
  static constexpr int V2 = V <= 1 ? 1 : V <= 2 ? 2 : V <= 4 ? 4 : V <= 8 ? 8 : V <= 16 ? 16 : V <= 32 ? 32 : 64;
  static constexpr int LOG2V = V2 == 1 ? 0 : V2 == 2 ? 1 : V2 == 4 ? 2 : V2 == 8 ? 3 : V2 == 16 ? 4 : V2 == 32 ? 5 : 6;
};

// Real data, even n <= 256, b <= 2, 16-byte aligned rows: lane l owns the column
// pairs (2l, 2l+1) and (2l+128, 2l+129).  Each wave walks batches of RB rows
// with two register buffers: the loads of the next batch are issued before
// the current batch is worked on (the scheduling barrier keeps them there), so
// one batch is always in flight.  A is read through a bounds-checked buffer
// resource that covers the workgroup's rows: rows past its end read as zero,
// so no branch guards the loads, and a lane whose column pair lies past n
// reads pair 0 of the row (its W entries are zero, its column sums are never
// written).  The row values of A_V and A_X are wave-uniform scalar loads (row
// indices clamped into the workgroup's range; the clamped rows multiply zero
// rows of A).  The row sums of a batch are reduced together by the compensated
// transpose-reduction; the lanes that end up holding a finished sum store it
// to A_W, and the sums are broadcast with scalar readlanes for the column sums.
// The four waves' column sums are combined through LDS (compensated for the
// A_V group) and each workgroup writes one record [G_V | G_X | G_W | G_V
// error] of 4 n b doubles.  INIT: the start pass (A_V = A V_0 and A^* A_V
// only).  rows_per_block * lda * 8 must stay below 2^31 (the buffer's range).
template <int B, bool DOT2, bool INIT>
__global__ __launch_bounds__(256) void k_astream_r2(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                    const double* __restrict__ W, double* __restrict__ AW,
                                                    const double* __restrict__ AVp, const double* __restrict__ AXp,
                                                    double* __restrict__ Gpart, int64_t rows_per_block,
                                                    const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  using SH = BatchShape<B>;
  constexpr int RB = SH::RB, V = SH::V, V2 = SH::V2, LOG2V = SH::LOG2V;
  constexpr int STEP = 4 * RB;
  __shared__ double red[4][2][256 * B];
  const int lane = threadIdx.x & 63, wave = wave_index();
  const bool has_x = AXp != nullptr;
  double2 w[2][B];
  double2 g1s[2][B], g1e[2][B], gx[2][B], gw[2][B];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
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
  int64_t rb = r0 + (int64_t)wave * RB;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(A + r0 * lda), 0, (int)((r1 - r0) * lda * 8), BUFFER_RSRC_WORD3);
  const uint32_t rowbytes = (uint32_t)lda * 8u;
  uint32_t voff[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) voff[s] = 16u * (uint32_t)((2 * lane + 128 * s < n) ? lane + 64 * s : 0);
  auto load_rows = [&](double2 (&a)[RB][2], int64_t r) {
    const uint32_t sb = (uint32_t)(r - r0) * rowbytes;
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int s = 0; s < 2; ++s) a[q][s] = ld_buf_stream2(rsrc, voff[s], sb + q * rowbytes);
  };
  auto load_uniform = [&](const double* __restrict__ P, int64_t r, double (&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      int64_t i = r + v / B;
      if (i >= r1) i = r1 - 1;
      o[v] = P[i * B + v % B];
    }
  };
  auto load_av_ax = [&](int64_t r, double (&av)[V], double (&ax)[V]) {
    if constexpr (!INIT) {
      load_uniform(AVp, r, av);
      if (has_x) {
        load_uniform(AXp, r, ax);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) ax[v] = 0.0;
      }
    }
  };
  // after the transpose-reduction lane l holds row sum v when its top LOG2V
  // bits are v bit-reversed; the lane of that group with the low bits clear
  // stores it
  int myv = 0;
#pragma unroll
  for (int st = 0; st < LOG2V; ++st) myv |= ((lane >> (5 - st)) & 1) << (LOG2V - 1 - st);
  const bool writer = (lane & ((1 << (6 - LOG2V)) - 1)) == 0 && myv < V;
  auto batch = [&](const double2 (&a)[RB][2], const double (&avs)[V], const double (&axs)[V], int64_t r) {
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
        for (int s = 0; s < 2; ++s) {
          if constexpr (DOT2) {
            // the first product starts the pair exactly
            if (s == 0) two_prod(a[q][s].x, w[s][j].x, ys[v], ye[v]);
            else dot2_add(a[q][s].x, w[s][j].x, ys[v], ye[v]);
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
    if (writer && r + myv / B < r1) AW[r * B + myv] = mine;
    // column sums: A^* A_V (Dot2; A^* A_W in the start pass), A^* A_X, A^* A_W
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int v = q * B + j;
        const double yv = readlane_d(mine, tr_src_lane<LOG2V>(v));
        const double av = INIT ? yv : avs[v];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          if constexpr (DOT2) {
            dot2_add(a[q][s].x, av, g1s[s][j].x, g1e[s][j].x);
            dot2_add(a[q][s].y, av, g1s[s][j].y, g1e[s][j].y);
          } else {
            g1s[s][j].x = fma(a[q][s].x, av, g1s[s][j].x);
            g1s[s][j].y = fma(a[q][s].y, av, g1s[s][j].y);
          }
          if constexpr (!INIT) {
            const double ax = axs[v];
            gx[s][j].x = fma(a[q][s].x, ax, gx[s][j].x);
            gx[s][j].y = fma(a[q][s].y, ax, gx[s][j].y);
            gw[s][j].x = fma(a[q][s].x, yv, gw[s][j].x);
            gw[s][j].y = fma(a[q][s].y, yv, gw[s][j].y);
          }
        }
      }
  };
  double2 a0[RB][2], a1[RB][2];
  double av0[V], ax0[V], av1[V], ax1[V];
  load_rows(a0, rb);
  load_av_ax(rb, av0, ax0);
  while (rb < r1) {
    load_rows(a1, rb + STEP);
    load_av_ax(rb + STEP, av1, ax1);
    __builtin_amdgcn_sched_barrier(0);
    batch(a0, av0, ax0, rb);
    rb += STEP;
    if (rb >= r1) break;
    load_rows(a0, rb + STEP);
    load_av_ax(rb + STEP, av0, ax0);
    __builtin_amdgcn_sched_barrier(0);
    batch(a1, av1, ax1, rb);
    rb += STEP;
  }
  // combine the four waves through LDS, two planes at a time
  const int64_t plane = (int64_t)n * B;
  double* gp = Gpart + (int64_t)blockIdx.x * 4 * plane;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * lane + 128 * s + h;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        red[wave][0][c * B + j] = h ? g1s[s][j].y : g1s[s][j].x;
        red[wave][1][c * B + j] = h ? g1e[s][j].y : g1e[s][j].x;
      }
    }
  __syncthreads();
  for (int e = threadIdx.x; e < plane; e += 256) {
    double S = red[0][0][e], E = red[0][1][e], t;
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      two_sum(S, red[q][0][e], S, t);
      E += t + red[q][1][e];
    }
    gp[e] = S;
    gp[3 * plane + e] = E;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * lane + 128 * s + h;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        red[wave][0][c * B + j] = h ? gx[s][j].y : gx[s][j].x;
        red[wave][1][c * B + j] = h ? gw[s][j].y : gw[s][j].x;
      }
    }
  __syncthreads();
  for (int e = threadIdx.x; e < plane; e += 256) {
    gp[plane + e] = (red[0][0][e] + red[1][0][e]) + (red[2][0][e] + red[3][0][e]);
    gp[2 * plane + e] = (red[0][1][e] + red[1][1][e]) + (red[2][1][e] + red[3][1][e]);
  }
}

// Real data, n <= 1024, any b <= 10, 16-byte aligned rows: the column-split
// pass.  A workgroup of nw waves (blockDim.x = 64 nw) walks its rows in
// batches of RB rows; wave w owns the column pairs 2 lane + 128 w, so each
// column belongs to exactly one wave and the waves read disjoint parts of
// every row.  Each wave reduces its partial row sums row by row (compensated
// transpose-reduction over the b values of a row) into LDS; after one barrier
// per batch, lane v of every wave combines the nw partials of value v in wave
// order and the finished sums are broadcast with scalar readlanes.  Every wave
// then accumulates the column sums of its own columns, so the per-workgroup
// record needs no cross-wave step.  init (the start pass) is a run-time flag.
template <int B>
struct CsShape {
  static constexpr int RB = (B >= 6) ? 2 : 4;  // rows per batch (one barrier each)
  static constexpr int V = RB * B;             // row sums per batch (<= 20)
  static constexpr int B2 = B <= 1 ? 1 : B <= 2 ? 2 : B <= 4 ? 4 : B <= 8 ? 8 : 16;
  static constexpr int LOG2B = B2 == 1 ? 0 : B2 == 2 ? 1 : B2 == 4 ? 2 : B2 == 8 ? 3 : 4;
};
constexpr int CS_MAXW = 8;

template <int B, bool DOT2>
__global__ __launch_bounds__(512) void k_astream_cs(const double* __restrict__ A, int64_t lda, int64_t m, int n,
                                                    const double* __restrict__ W, double* __restrict__ AW,
                                                    const double* __restrict__ AVp, const double* __restrict__ AXp,
                                                    double* __restrict__ Gpart, int64_t rows_per_block, int init,
                                                    const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  using SH = CsShape<B>;
  constexpr int RB = SH::RB, V = SH::V, B2 = SH::B2, LOG2B = SH::LOG2B;
  __shared__ double sp[2][CS_MAXW][V], ep[2][CS_MAXW][V];
  const int nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const bool has_x = AXp != nullptr;
  const int c = 2 * lane + 128 * wave;
  // value index held by this lane after tr_reduce over B2 values: the top
  // LOG2B lane bits, most significant first; lanes whose lower bits are zero
  // represent their group
  int my_idx = 0;
#pragma unroll
  for (int st = 0; st < LOG2B; ++st) my_idx |= ((lane >> (5 - st)) & 1) << (LOG2B - 1 - st);
  const bool my_rep = (lane & ((1 << (6 - LOG2B)) - 1)) == 0;
  double2 w[B], g1s[B], g1e[B], gx[B], gw[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    w[j].x = (c < n) ? W[(int64_t)c * B + j] : 0.0;
    w[j].y = (c + 1 < n) ? W[(int64_t)(c + 1) * B + j] : 0.0;
    g1s[j] = make_double2(0.0, 0.0);
    g1e[j] = make_double2(0.0, 0.0);
    gx[j] = make_double2(0.0, 0.0);
    gw[j] = make_double2(0.0, 0.0);
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  auto load = [&](double2 (&a)[RB], int64_t rb) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = rb + q;
      if (row < r1 && c + 1 < n) a[q] = ld_stream2(A + row * lda + c);
      else if (row < r1 && c < n) a[q] = make_double2(A[row * lda + c], 0.0);
      else a[q] = make_double2(0.0, 0.0);
    }
  };
  int64_t rb = r0;
  double2 a[RB], an[RB];
  load(an, rb);
  double avn = 0.0, axn = 0.0;
  if (!init && lane < V && rb + lane / B < r1) {
    avn = AVp[rb * B + lane];
    if (has_x) axn = AXp[rb * B + lane];
  }
  int buf = 0;
  for (; rb < r1; rb += RB) {
#pragma unroll
    for (int q = 0; q < RB; ++q) a[q] = an[q];
    const double avl = avn, axl = axn;
    const int64_t rn = rb + RB;
    load(an, rn);
    if (!init) {
      avn = 0.0;
      axn = 0.0;
      if (lane < V && rn + lane / B < r1) {
        avn = AVp[rn * B + lane];
        if (has_x) axn = AXp[rn * B + lane];
      }
    }
    // this wave's partial row sums, one row at a time
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      double ys[B2], ye[B2];
#pragma unroll
      for (int j = 0; j < B2; ++j) {
        ys[j] = 0.0;
        ye[j] = 0.0;
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        if constexpr (DOT2) {
          // the first product starts the pair exactly
          two_prod(a[q].x, w[j].x, ys[j], ye[j]);
          dot2_add(a[q].y, w[j].y, ys[j], ye[j]);
        } else {
          ys[j] = fma(a[q].x, w[j].x, ys[j]);
          ys[j] = fma(a[q].y, w[j].y, ys[j]);
        }
      }
      if constexpr (DOT2) tr_reduce_dot2<B2, LOG2B>(ys, ye, lane);
      else tr_reduce_plain<B2, LOG2B>(ys, lane);
      // after the reduction every lane holds the finished sum of value
      // my_idx; one lane per value writes it
      if (my_rep && my_idx < B) {
        sp[buf][wave][q * B + my_idx] = ys[0];
        ep[buf][wave][q * B + my_idx] = DOT2 ? ye[0] : 0.0;
      }
    }
    __syncthreads();
    // lane v < V combines value v over the waves, in wave order
    double comb = 0.0;
    if (lane < V) {
      double S = sp[buf][0][lane], E = ep[buf][0][lane], t;
      for (int q = 1; q < nw; ++q) {
        two_sum(S, sp[buf][q][lane], S, t);
        E += t + ep[buf][q][lane];
      }
      comb = S + E;
    }
    buf ^= 1;
    if (wave == 0 && lane < V && rb + lane / B < r1) AW[rb * B + lane] = comb;
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int v = q * B + j;
        const double yv = readlane_d(comb, v);
        const double av = init ? yv : readlane_d(avl, v);
        if constexpr (DOT2) {
          dot2_add(a[q].x, av, g1s[j].x, g1e[j].x);
          dot2_add(a[q].y, av, g1s[j].y, g1e[j].y);
        } else {
          g1s[j].x = fma(a[q].x, av, g1s[j].x);
          g1s[j].y = fma(a[q].y, av, g1s[j].y);
        }
        if (!init) {
          const double ax = readlane_d(axl, v);
          gx[j].x = fma(a[q].x, ax, gx[j].x);
          gx[j].y = fma(a[q].y, ax, gx[j].y);
          gw[j].x = fma(a[q].x, yv, gw[j].x);
          gw[j].y = fma(a[q].y, yv, gw[j].y);
        }
      }
  }
  const int64_t plane = (int64_t)n * B;
  double* gp = Gpart + (int64_t)blockIdx.x * 4 * plane;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (c + h < n) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int64_t e = (int64_t)(c + h) * B + j;
        gp[e] = h ? g1s[j].y : g1s[j].x;
        gp[plane + e] = h ? gx[j].y : gx[j].x;
        gp[2 * plane + e] = h ? gw[j].y : gw[j].x;
        gp[3 * plane + e] = h ? g1e[j].y : g1e[j].x;
      }
    }
  }
}

}  // namespace rl
