// TSQR of a tall m x t block (t <= 32), the first half of the Rayleigh-Ritz
// step: the paper computes [~, Theta, C] = svd(A_T) of the m x 3b trial-space
// product (Alg. rlopcg and Alg. rlobpcg, "Rayleigh-Ritz"); with A_T = Q R_T
// the right singular data of A_T are those of the small R_T.
//
// A Gram-matrix route (A_T^* A_T) would square the condition number of A_T,
// whose smallest singular value is the wanted sigma_min; Householder QR keeps
// a column-wise backward error, which is what the small singular values need.
//
// Tiles walk a range of rows: rows 0..t-1 of a tile hold the running R, the
// other rows take the next input rows, and a Householder QR of the tile leaves
// the new R on top.  The input rows are [P0(r,:), P1(r,:), P2(r,:)] from up to
// three row-major panels, so the m x b blocks A_V, A_X, A_W are read in place.
// The per-workgroup R factors are written row-major (t x t each) and form a
// (groups*t) x t matrix that is reduced again until one R_T remains.  Two
// kernel families: one-wave register tiles for t <= 8 (k_tsqr_w), and
// workgroup tiles with the columns dealt out over the waves for 8 < t <= 32
// (k_tsqr_cw).
#include "common.hpp"
#include "householder.hpp"
#include "kernels.hpp"
#include "colsum.hpp"
#include "tr_reduce.hpp"

namespace rl {

constexpr int TS_TMAX = 32;

__device__ inline double ts_im(double) { return 0.0; }
__device__ inline double ts_im(cd a) { return a.y; }


// ---------------------------------------------------------------------------
// Register TSQR for t <= 8: a wave holds a tile of 64*RPL rows, RPL rows per
// lane (t values each in registers).  Rows 0..t-1 of the tile (lanes 0..t-1,
// first register row) carry the running R; the other rows take the next
// 64*RPL-t input rows, loaded one tile ahead.  Householder QR of the tile:
// with x the column below the diagonal, |x|^2 and then each x^* a_k (k > j)
// are summed over the wave, and v^* a_k = a_jk + conj(1/(alpha-beta)) x^* a_k
// gives the reflector products without a second pass.  The waves' R factors
// are stacked in LDS and factored again by wave 0.  k_tsqr_w writes one R per
// workgroup; k_tsqr_w_merge (one workgroup of 16 waves, 8 for complex data,
// the next launch on the stream) reduces those the same way and writes R_T.
constexpr int TW_THREADS = 256;

template <typename T, int TT>
__device__ inline T tw_get(const T (&x)[TT], int j) {
  T r = zero<T>();
#pragma unroll
  for (int q = 0; q < TT; ++q)
    if (q == j) r = x[q];
  return r;
}
template <typename T, int TT>
__device__ inline void tw_set(T (&x)[TT], int j, T v) {
#pragma unroll
  for (int q = 0; q < TT; ++q)
    if (q == j) x[q] = v;
}

// QR of the tile; on return tile rows 0..t-1 hold R (upper triangular) and
// every other entry of columns 0..t-1 is zero.  For column j the reflector
// products v^* a_k are formed column by column (x^* a_k is summed over the
// wave just before a_k is updated), so no array of them is kept.
template <typename T, int TT, int RPL>
__device__ __forceinline__ void tw_tile_qr(T (&x)[RPL][TT], int t, int lane) {
  for (int j = 0; j < t; ++j) {
    T xj[RPL];
    bool below[RPL];
    double n2p = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      xj[s] = tw_get<T, TT>(x[s], j);
      below[s] = (s > 0) || (lane > j);
      if (below[s]) n2p += abs2(xj[s]);
    }
    const double n2 = wave_sum(n2p);
    const T alpha = readlane_d(xj[0], j);
    const bool noref = (n2 == 0.0) && (ts_im(alpha) == 0.0);
    if (noref) continue;  // the column is already zero below the diagonal
    const double nrm = sqrt(abs2(alpha) + n2);
    const double beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
    T tau, sc;
    hh_coef(alpha, beta, tau, sc);
    const T ct = conj_(tau), csc = conj_(sc);
    T v[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s)
      v[s] = (s == 0 && lane == j) ? from_real<T>(1.0) : (below[s] ? mul(sc, xj[s]) : zero<T>());
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      if (k > j && k < t) {
        T acc = zero<T>();
#pragma unroll
        for (int s = 0; s < RPL; ++s)
          if (below[s]) acc = cfmac(xj[s], x[s][k], acc);
        const T dk = wave_sum(acc);
        const T ajk = readlane_d(x[0][k], j);
        const T f = mul(ct, fmac(csc, dk, ajk));
#pragma unroll
        for (int s = 0; s < RPL; ++s) x[s][k] = fnmac(f, v[s], x[s][k]);
      }
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      T nx = xj[s];
      if (s == 0 && lane == j) nx = from_real<T>(beta);
      else if (below[s]) nx = zero<T>();
      tw_set<T, TT>(x[s], j, nx);
    }
  }
}

// Input rows: the row-major panels [P0 | P1 | P2] (b0 + b1 + b2 = t columns).
template <typename T>
struct TwPanels {
  const T* P0;
  const T* P1;
  const T* P2;
  int b0, b1, b2;
  __device__ T get(int64_t row, int c) const {
    if (c < b0) return P0[row * b0 + c];
    if (c < b0 + b1) return P1[row * b1 + (c - b0)];
    return P2[row * b2 + (c - b0 - b1)];
  }
};

// Tile rows t..64*RPL-1 of x <- input rows g + (tile row - t), zero past g1.
template <typename T, int TT, int RPL, typename Src>
__device__ inline void tw_load(T (&x)[RPL][TT], const Src& src, int64_t g, int64_t g1, int t, int lane) {
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int tr = lane + 64 * s;
    const int64_t row = g + tr - t;
    const bool valid = tr >= t && row < g1;
#pragma unroll
    for (int c = 0; c < TT; ++c) x[s][c] = (valid && c < t) ? src.get(row, c) : zero<T>();
  }
}

// Rows [g0, g1) of the input, tiles of 64*RPL-t fresh rows, wave w of nw
// takes tiles w, w+nw, ...; x ends as this wave's R.
template <typename T, int TT, int RPL, typename Src>
__device__ __forceinline__ void tw_rows(T (&x)[RPL][TT], const Src& src, int64_t g0, int64_t g1, int t, int lane, int wave, int nw) {
  const int fresh = 64 * RPL - t;
  const int64_t step = (int64_t)nw * fresh;
  int64_t g = g0 + (int64_t)wave * fresh;
  // the next tile is loaded ahead when the copy fits the register budget
  constexpr bool PF = RPL * TT * (int)(sizeof(T) / 8) <= 32;
  if constexpr (PF) {
    T nx[RPL][TT];
    tw_load<T, TT, RPL>(nx, src, g, g1, t, lane);
    for (; g < g1; g += step) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        if (lane + 64 * s >= t) {
#pragma unroll
          for (int c = 0; c < TT; ++c) x[s][c] = nx[s][c];
        }
      }
      tw_load<T, TT, RPL>(nx, src, g + step, g1, t, lane);
      tw_tile_qr<T, TT, RPL>(x, t, lane);
    }
  } else {
    for (; g < g1; g += step) {
      T nx[RPL][TT];
      tw_load<T, TT, RPL>(nx, src, g, g1, t, lane);
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        if (lane + 64 * s >= t) {
#pragma unroll
          for (int c = 0; c < TT; ++c) x[s][c] = nx[s][c];
        }
      }
      tw_tile_qr<T, TT, RPL>(x, t, lane);
    }
  }
}

template <typename T>
struct TwRows {  // rows of a row-major n x t array (global or LDS)
  const T* P;
  int t;
  __device__ T get(int64_t row, int c) const { return P[row * t + c]; }
};

// Stack the NW waves' R factors in LDS and factor them in wave 0.
template <typename T, int TT, int RPL, int NW>
__device__ __forceinline__ void tw_block_merge(T (&x)[RPL][TT], T* Rs, int t, int lane, int wave) {
  if (lane < t) {
#pragma unroll
    for (int c = 0; c < TT; ++c)
      if (c < t) Rs[(wave * t + lane) * t + c] = x[0][c];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int s = 0; s < RPL; ++s)
#pragma unroll
      for (int c = 0; c < TT; ++c) x[s][c] = zero<T>();
    const TwRows<T> src{Rs, t};
    tw_rows<T, TT, RPL>(x, src, 0, (int64_t)NW * t, t, lane, 0, 1);
  }
}

// Workgroups g_tsqr and up run one level of the partial-sum reduction
// (side), which reads only what the preceding pass wrote.
template <typename T, int TT, int RPL>
__global__ __launch_bounds__(TW_THREADS) void k_tsqr_w(const T* __restrict__ P0, int b0, const T* __restrict__ P1,
                                                       int b1, const T* __restrict__ P2, int b2, int64_t m,
                                                       int64_t rows_per_block, T* __restrict__ Rpart,
                                                       const Ctl* __restrict__ ctl, int check_done, int g_tsqr,
                                                       ColsumJob side) {
  if ((int)blockIdx.x >= g_tsqr) {
    const int b = (int)blockIdx.x - g_tsqr;
    colsum2_block(side, b % side.gx, b / side.gx);
    return;
  }
  if (check_done && ctl->done) return;
  constexpr int NW = TW_THREADS / 64;
  __shared__ T Rs[NW * TT * TT];
  const int t = b0 + b1 + b2;
  const int lane = threadIdx.x & 63, wave = wave_index();
  T x[RPL][TT];
#pragma unroll
  for (int s = 0; s < RPL; ++s)
#pragma unroll
    for (int c = 0; c < TT; ++c) x[s][c] = zero<T>();
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t g1 = (g0 + rows_per_block < m) ? g0 + rows_per_block : m;
  const TwPanels<T> src{P0, P1, P2, b0, b1, b2};
  tw_rows<T, TT, RPL>(x, src, g0, g1, t, lane, wave, NW);
  tw_block_merge<T, TT, RPL, NW>(x, Rs, t, lane, wave);
  if (wave == 0 && lane < t) {
#pragma unroll
    for (int c = 0; c < TT; ++c)
      if (c < t) Rpart[((int64_t)blockIdx.x * t + lane) * t + c] = x[0][c];
  }
}

// R_T of the stacked per-workgroup factors (rows = groups * t), one workgroup.
template <typename T, int TT, int RPL, int NW>
__global__ __launch_bounds__(NW * 64) void k_tsqr_w_merge(const T* __restrict__ Rpart, int t, int64_t rows,
                                                          T* __restrict__ Rout, const Ctl* __restrict__ ctl,
                                                          int check_done) {
  if (check_done && ctl->done) return;
  __shared__ T Rs[NW * TT * TT];
  const int lane = threadIdx.x & 63, wave = wave_index();
  T x[RPL][TT];
#pragma unroll
  for (int s = 0; s < RPL; ++s)
#pragma unroll
    for (int c = 0; c < TT; ++c) x[s][c] = zero<T>();
  const TwRows<T> src{Rpart, t};
  tw_rows<T, TT, RPL>(x, src, 0, rows, t, lane, wave, NW);
  tw_block_merge<T, TT, RPL, NW>(x, Rs, t, lane, wave);
  if (wave == 0 && lane < t) {
#pragma unroll
    for (int c = 0; c < TT; ++c)
      if (c < t) Rout[lane * t + c] = x[0][c];
  }
}

// rows per lane: the tile (RPL x TT values, twice with the prefetch) stays
// within the register budget
template <typename T, int TT>
struct TwRpl {
  static constexpr int real = TT <= 4 ? 4 : (TT <= 8 ? 2 : 1);
  static constexpr int value = sizeof(T) == 16 ? (real > 1 ? real / 2 : 1) : real;
};
template <typename T, int TT>
struct TwMergeWaves {
  static constexpr int value = TT > 16 ? 4 : ((sizeof(T) == 16 || TT > 8) ? 8 : 16);
};

// Workgroups of the first launch: enough for every SIMD (256 workgroups of
// four waves), no more: the first launch's time is set by its total tile count
// over the whole chip, the single-workgroup merge's by the number of stacked
// factors.
static int64_t tsqr_w_groups(int64_t m, int t, bool cplx) {
  const int tt = t <= 4 ? 4 : (t <= 8 ? 8 : (t <= 16 ? 16 : 32));
  int rpl = tt <= 4 ? 4 : (tt <= 8 ? 2 : 1);
  if (cplx) rpl = rpl > 1 ? rpl / 2 : 1;
  const int64_t fresh = 64 * rpl - t;
  int64_t g = (m + 4 * fresh - 1) / (4 * fresh);  // at least one tile per wave
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return g;
}

template <typename T, int TT>
static void tsqr_w_go(hipStream_t st, const T* P0, int b0, const T* P1, int b1, const T* P2, int b2, int64_t m,
                      int64_t g, T* bufA, T* bufB, const Ctl* ctl, int check_done, const ColsumJob* side) {
  constexpr int RPL = TwRpl<T, TT>::value;
  constexpr int NWM = TwMergeWaves<T, TT>::value;
  const int t = b0 + b1 + b2;
  const int64_t rows = (m + g - 1) / g;
  // never-read panels still get a valid pointer
  if (P1 == nullptr) P1 = P0;
  if (P2 == nullptr) P2 = P0;
  ColsumJob sj{};
  int64_t extra = 0;
  if (side != nullptr) {
    sj = *side;
    extra = (int64_t)sj.gx * sj.gy;
  }
  hipLaunchKernelGGL((k_tsqr_w<T, TT, RPL>), dim3((unsigned)(g + extra)), dim3(TW_THREADS), 0, st, P0, b0, P1, b1, P2,
                     b2, m, rows, bufA, ctl, check_done, (int)g, sj);
  hipLaunchKernelGGL((k_tsqr_w_merge<T, TT, RPL, NWM>), dim3(1), dim3(NWM * 64), 0, st, (const T*)bufA, t, g * t,
                     bufB, ctl, check_done);
}

// ---------------------------------------------------------------------------
// Column-wave TSQR for 8 < t <= 32: one tile of 64*RPL rows per workgroup of
// NW waves, held in registers with the columns dealt out over the waves (wave
// w owns columns w, w+NW, ...; lane l holds tile rows l + 64 s, s < RPL).  The
// tile is NW times taller than a one-wave tile, so the t rows of running R
// take a small share of it, and no wave holds more than TT/NW columns.
//
// Column j is factored by its owner wave (one wave reduction for |x|^2), which
// publishes the Householder vector and conj(tau) in LDS; after one barrier
// every wave applies the reflector to its own columns k > j: the products
// v^* a_k of all its columns are summed in one transpose-reduction, broadcast
// with readlanes and used for the rank-one update.  The owner of column j+1
// factors it right after applying reflector j, so one barrier per column
// suffices (the vector buffer alternates between two slots).
//
// The first tile of a row range fills all 64*RPL rows; later tiles keep R in
// rows 0..t-1 and take 64*RPL-t fresh rows.  One R per workgroup is written;
// the stacked R factors are reduced by the same kernel in further launches
// until one remains.
template <typename T, int TT, int NW, int RPL>
struct CwShape {
  static constexpr int CPW = TT / NW;                       // columns per wave
  static constexpr int RT = 64 * RPL;                       // tile rows
  static constexpr int NV = CPW * (int)(sizeof(T) / 8);     // reals reduced per column
  static constexpr int LOG2NV = NV <= 1 ? 0 : NV <= 2 ? 1 : NV <= 4 ? 2 : NV <= 8 ? 3 : NV <= 16 ? 4 : 5;
};

template <typename T, int TT, int NW, int RPL>
__global__ __launch_bounds__(NW * 64) void k_tsqr_cw(const T* __restrict__ P0, int b0, const T* __restrict__ P1,
                                                     int b1, const T* __restrict__ P2, int b2, int64_t m,
                                                     int64_t rows_per_block, T* __restrict__ Rout,
                                                     const Ctl* __restrict__ ctl, int check_done) {
  if (check_done && ctl->done) return;
  using SH = CwShape<T, TT, NW, RPL>;
  constexpr int CPW = SH::CPW, RT = SH::RT, NV = SH::NV, LOG2NV = SH::LOG2NV;
  constexpr int ES = (int)(sizeof(T) / 8);
  __shared__ T vbuf[2][RT];
  __shared__ T tbuf[2];
  const int t = b0 + b1 + b2;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t g1 = (g0 + rows_per_block < m) ? g0 + rows_per_block : m;
  const TwPanels<T> src{P0, P1, P2, b0, b1, b2};
  T x[CPW][RPL];
#pragma unroll
  for (int kc = 0; kc < CPW; ++kc)
#pragma unroll
    for (int s = 0; s < RPL; ++s) x[kc][s] = zero<T>();

  // owner of column j factors it (its slot kc holds column j)
  auto factor = [&](T (&col)[RPL], int j, int slot) {
    double n2p = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s)
      if (lane + 64 * s > j) n2p += abs2(col[s]);
    const double n2 = wave_sum(n2p);
    const T alpha = readlane_d(col[0], j);
    if (n2 == 0.0 && ts_im(alpha) == 0.0) {  // already zero below the diagonal
      if (lane == 0) tbuf[slot] = zero<T>();
      return;
    }
    const double nrm = sqrt(abs2(alpha) + n2);
    const double beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
    T tau, sc;
    hh_coef(alpha, beta, tau, sc);
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = lane + 64 * s;
      const T vs = (r > j) ? mul(sc, col[s]) : (r == j ? from_real<T>(1.0) : zero<T>());
      vbuf[slot][r] = vs;
      if (r > j) col[s] = zero<T>();
      else if (r == j) col[s] = from_real<T>(beta);
    }
    if (lane == 0) tbuf[slot] = conj_(tau);
  };

  bool first = true;
  for (int64_t g = g0; g < g1;) {
    // load the tile: all rows the first time, rows t.. afterwards
    const int r0 = first ? 0 : t;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = lane + 64 * s;
      const int64_t row = g + (r - r0);
      const bool valid = r >= r0 && row < g1;
#pragma unroll
      for (int kc = 0; kc < CPW; ++kc) {
        const int c = wave + NW * kc;
        if (r >= r0) x[kc][s] = (valid && c < t) ? src.get(row, c) : zero<T>();
      }
    }
    g += RT - r0;
    first = false;
    // column 0 belongs to wave 0, slot 0
    if (wave == 0) factor(x[0], 0, 0);
#pragma unroll
    for (int jc = 0; jc < CPW; ++jc) {
      for (int ow = 0; ow < NW; ++ow) {
        const int j = NW * jc + ow;
        if (j >= t) break;
        __syncthreads();
        const T ct = tbuf[j & 1];
        // the reflector is read before the test so the loads overlap; a wave
        // whose columns all lie left of j + 1 has nothing to update
        T v[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) v[s] = vbuf[j & 1][lane + 64 * s];
        if (wave + NW * (CPW - 1) > j && !(re_(ct) == 0.0 && ts_im(ct) == 0.0)) {
          double ys[NV];
#pragma unroll
          for (int q = 0; q < NV; ++q) ys[q] = 0.0;
#pragma unroll
          for (int kc = 0; kc < CPW; ++kc) {
            const int k = wave + NW * kc;
            if (k > j && k < t) {
              T acc = zero<T>();
#pragma unroll
              for (int s = 0; s < RPL; ++s) acc = cfmac(v[s], x[kc][s], acc);
              if constexpr (ES == 2) {
                ys[2 * kc] = re_(acc);
                ys[2 * kc + 1] = ts_im(acc);
              } else {
                ys[kc] = re_(acc);
              }
            }
          }
          tr_reduce_plain<NV, LOG2NV>(ys, lane);
#pragma unroll
          for (int kc = 0; kc < CPW; ++kc) {
            const int k = wave + NW * kc;
            if (k > j && k < t) {
              T d;
              if constexpr (ES == 2) {
                d = T{readlane_d(ys[0], tr_src_lane<LOG2NV>(2 * kc)), readlane_d(ys[0], tr_src_lane<LOG2NV>(2 * kc + 1))};
              } else {
                d = readlane_d(ys[0], tr_src_lane<LOG2NV>(kc));
              }
              const T f = mul(ct, d);
#pragma unroll
              for (int s = 0; s < RPL; ++s) x[kc][s] = fnmac(f, v[s], x[kc][s]);
            }
          }
        }
        // the owner of column j + 1 factors it
        const int j1 = j + 1;
        if (j1 < t && wave == (ow + 1) % NW) {
          if (ow + 1 < NW) factor(x[jc], j1, j1 & 1);
          else if (jc + 1 < CPW) factor(x[jc + 1 < CPW ? jc + 1 : jc], j1, j1 & 1);
        }
      }
    }
    __syncthreads();  // the vector buffer is rewritten by the next tile
  }
  // R: rows 0..t-1 (lanes 0..t-1 of the first register row)
  if (lane < t) {
#pragma unroll
    for (int kc = 0; kc < CPW; ++kc) {
      const int c = wave + NW * kc;
      if (c < t) Rout[((int64_t)blockIdx.x * t + lane) * t + c] = x[kc][0];
    }
  }
}

template <typename T, int TT>
struct CwCfg {  // waves, rows per lane of the column-wave TSQR
  // 16 real values per lane and column (tiles of 1024 real or 512 complex
  // rows); the waves split the columns, fewer per wave the more there are to
  // update (one or two complex columns per wave at t > 16, within the 128
  // registers a 1024-thread workgroup allows)
  static constexpr int NW = sizeof(T) == 16 ? (TT == 32 ? 16 : 8) : (TT == 32 ? 8 : 4);
  static constexpr int RPL = 16 / (int)(sizeof(T) / 8);
};

static int64_t tsqr_cw_fresh(int t, bool cplx) {
  const int rpl = t > 16 ? (cplx ? CwCfg<cd, 32>::RPL : CwCfg<double, 32>::RPL)
                         : (cplx ? CwCfg<cd, 16>::RPL : CwCfg<double, 16>::RPL);
  return 64 * rpl - t;
}

// row ranges of the first launch: two tiles or more each, at most 512
static int64_t tsqr_cw_groups(int64_t m, int t, bool cplx) {
  const int64_t fresh = tsqr_cw_fresh(t, cplx);
  int64_t g = (m + 2 * fresh - 1) / (2 * fresh);
  if (g > 512) g = 512;
  return g < 1 ? 1 : g;
}

template <typename T, int TT>
static hipError_t tsqr_cw_impl(hipStream_t st, const T* P0, int b0, const T* P1, int b1, const T* P2, int b2,
                               int64_t m, T* bufA, T* bufB, T** Rfinal, const Ctl* ctl, int check_done) {
  constexpr int NW = CwCfg<T, TT>::NW, RPL = CwCfg<T, TT>::RPL;
  const int t = b0 + b1 + b2;
  const bool cplx = sizeof(T) == 16;
  if (P1 == nullptr) P1 = P0;
  if (P2 == nullptr) P2 = P0;
  int64_t g = tsqr_cw_groups(m, t, cplx);
  int64_t rows = (m + g - 1) / g;
  hipLaunchKernelGGL((k_tsqr_cw<T, TT, NW, RPL>), dim3((unsigned)g), dim3(NW * 64), 0, st, P0, b0, P1, b1, P2, b2, m,
                     rows, bufA, ctl, check_done);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  T* cur = bufA;
  T* nxt = bufB;
  // reduce the stacked factors until one remains: each workgroup takes as
  // many whole factors as one tile holds, so every launch is one tile deep
  // (a tile's column steps are the latency of a launch)
  const int64_t per = (64 * RPL) / t >= 2 ? (64 * RPL) / t : 2;
  while (g > 1) {
    const int64_t mm = g * t;
    const int64_t g2 = (g + per - 1) / per;
    rows = per * t;
    hipLaunchKernelGGL((k_tsqr_cw<T, TT, NW, RPL>), dim3((unsigned)g2), dim3(NW * 64), 0, st, (const T*)cur, t,
                       (const T*)cur, 0, (const T*)cur, 0, mm, rows, nxt, ctl, check_done);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    T* tmp = cur;
    cur = nxt;
    nxt = tmp;
    g = g2;
  }
  *Rfinal = cur;
  return hipSuccess;
}


// Upper bound on the partial R factors of one TSQR launch (workspace sizing).
int64_t tsqr_groups(int64_t m, int t) {
  const int64_t b = std::max(tsqr_w_groups(m, t, true), tsqr_w_groups(m, t, false));
  const int64_t c = std::max(tsqr_cw_groups(m, t, true), tsqr_cw_groups(m, t, false));
  return std::max(b, c);
}

template <typename T>
static hipError_t tsqr_impl(hipStream_t st, const T* P0, int b0, const T* P1, int b1, const T* P2, int b2, int64_t m,
                            T* bufA, T* bufB, T** Rfinal, Ctl* ctl, int check_done, const ColsumJob* side) {
  const int t = b0 + b1 + b2;
  if (t < 1 || t > TS_TMAX) return hipErrorInvalidValue;
  if (t > 8 && side != nullptr) {
    const hipError_t e = launch_colsum_job(st, *side);
    if (e != hipSuccess) return e;
  }
  if (t > 16) return tsqr_cw_impl<T, 32>(st, P0, b0, P1, b1, P2, b2, m, bufA, bufB, Rfinal, ctl, check_done);
  if (t > 8) return tsqr_cw_impl<T, 16>(st, P0, b0, P1, b1, P2, b2, m, bufA, bufB, Rfinal, ctl, check_done);
  const int64_t g = tsqr_w_groups(m, t, sizeof(T) == 16);
  if (t <= 4) tsqr_w_go<T, 4>(st, P0, b0, P1, b1, P2, b2, m, g, bufA, bufB, ctl, check_done, side);
  else tsqr_w_go<T, 8>(st, P0, b0, P1, b1, P2, b2, m, g, bufA, bufB, ctl, check_done, side);
  *Rfinal = bufB;
  return hipGetLastError();
}

hipError_t launch_tsqr(hipStream_t st, bool cplx, const void* P0, int b0, const void* P1, int b1, const void* P2,
                       int b2, int64_t m, void* bufA, void* bufB, void** Rfinal, Ctl* ctl, int check_done,
                       const ColsumJob* side) {
  if (cplx)
    return tsqr_impl<cd>(st, (const cd*)P0, b0, (const cd*)P1, b1, (const cd*)P2, b2, m, (cd*)bufA, (cd*)bufB,
                         (cd**)Rfinal, ctl, check_done, side);
  return tsqr_impl<double>(st, (const double*)P0, b0, (const double*)P1, b1, (const double*)P2, b2, m,
                           (double*)bufA, (double*)bufB, (double**)Rfinal, ctl, check_done, side);
}

}  // namespace rl
