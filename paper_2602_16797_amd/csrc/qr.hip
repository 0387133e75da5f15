// Householder QR of the sketch S*A (d x n), keeping only R, and R^{-1}.
//
// The preconditioner of RLOBPCG only needs P with P P^* = ((S A)^* S A)^{-1}.
// The paper builds it from the SVD of S*A (Alg. rlopcg, sketch-and-SVD); its
// footnote to Sec. 1 step 3 names the QR route as the traditional one.  With
// S A = Q R, P = R^{-1} gives the same operator, P P^* = (R^* R)^{-1}, so the
// GPU path factors S*A by Householder QR and inverts the triangular R once.
//
// Layout: Y is column-major (ld = d), as written by the sketch reduction.
// Blocked right-looking QR with panel width QR_NB:
//   k_qr_panel   one workgroup factors a (d-p) x nb panel column by column
//                (LAPACK's larfg conventions: real beta, tau = (beta-alpha)/beta,
//                H^* = I - conj(tau) v v^*) and builds the compact-WY T factor
//                with H_1 ... H_nb = I - V T V^* (forward, column-wise).
//   k_qr_update  applies I - V T^* V^* to the trailing columns, CB per block.
//   k_qr_extract writes R row-major and R^* row-major (for the products).
//   k_trinv      R^{-1} by column-oriented back substitution, one wave per
//                column of the identity; writes R^{-1} and R^{-*} row-major.
#include "common.hpp"
#include "householder.hpp"
#include "kernels.hpp"
#include "tr_reduce.hpp"

namespace rl {

constexpr int QR_NB = 32;
constexpr int QR_THREADS = 256;
constexpr int QR_CB = 8;

__device__ inline double im_(double) { return 0.0; }
__device__ inline double im_(cd a) { return a.y; }
__device__ inline double im_(float) { return 0.0; }

// Round a float to the nearest bfloat16 (ties to even), kept in a float: the
// inputs of the BF16 trailing update.
__device__ inline float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u) return x;  // Inf / NaN unchanged
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// V(r, q) of the current panel: unit lower trapezoidal, stored below the diagonal.
template <typename T>
__device__ inline T vpanel(const T* Y, int ld, int p, int q, int r) {
  const int j = p + q;
  if (r < j) return zero<T>();
  if (r == j) return from_real<T>(1.0);
  return Y[(int64_t)j * ld + r];
}

template <typename T>
__global__ __launch_bounds__(QR_THREADS) void k_qr_panel(T* Y, int ld, int d, int n, int p, int nb, T* Tm) {
  __shared__ T scratch[(QR_THREADS / 16) * QR_NB];
  __shared__ T outs[QR_NB];
  __shared__ T taus[QR_NB];
  __shared__ T Tl[QR_NB * QR_NB];  // column-major nb x nb
  __shared__ double red[QR_THREADS / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < QR_NB * QR_NB; i += blockDim.x) Tl[i] = zero<T>();
  __syncthreads();
  for (int jj = 0; jj < nb; ++jj) {
    const int j = p + jj;
    T* col = Y + (int64_t)j * ld;
    double xs = 0.0;
    for (int r = j + 1 + tid; r < d; r += blockDim.x) xs += abs2(col[r]);
    xs = block_sum(xs, red);
    const T alpha = col[j];
    const bool noref = (xs == 0.0) && (im_(alpha) == 0.0);
    T tau = zero<T>(), sc = zero<T>();
    double beta = re_(alpha);
    if (!noref) {
      const double nrm = sqrt(abs2(alpha) + xs);
      beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
      hh_coef(alpha, beta, tau, sc);
    }
    __syncthreads();  // alpha read by all before it is overwritten
    if (!noref) {
      for (int r = j + 1 + tid; r < d; r += blockDim.x) col[r] = mul(col[r], sc);
      if (tid == 0) col[j] = from_real<T>(beta);
    }
    if (tid == 0) taus[jj] = tau;
    __syncthreads();
    // One batched reduction over rows r >= j:
    //   k < K1: s_k = v^* Y(:, j+1+k)           (apply H^* to the rest of the panel)
    //   k >= K1: g_q = V(:, q)^* v, q = k - K1  (column jj of the T factor)
    const int K1 = nb - jj - 1, K2 = jj, K = K1 + K2;
    if (K > 0) {
      T vals[QR_NB];
#pragma unroll
      for (int k = 0; k < QR_NB; ++k) vals[k] = zero<T>();
      for (int r = j + tid; r < d; r += blockDim.x) {
        const T vr = (r == j) ? from_real<T>(1.0) : col[r];
#pragma unroll
        for (int k = 0; k < QR_NB; ++k) {
          if (k < K1) vals[k] = cfmac(vr, Y[(int64_t)(j + 1 + k) * ld + r], vals[k]);
          else if (k < K) vals[k] = cfmac(vpanel(Y, ld, p, k - K1, r), vr, vals[k]);
        }
      }
      block_sum_many<T, QR_NB>(vals, K, scratch, outs);
      if (K1 > 0 && !noref) {
        const T ct = conj_(tau);
        for (int r = j + tid; r < d; r += blockDim.x) {
          const T vr = (r == j) ? from_real<T>(1.0) : col[r];
          for (int k = 0; k < K1; ++k) {
            T* yk = Y + (int64_t)(j + 1 + k) * ld + r;
            *yk = fnmac(mul(ct, outs[k]), vr, *yk);
          }
        }
      }
      if (tid == 0) {
        // T(0:jj, jj) = -tau * T(0:jj, 0:jj) * g
        for (int q = 0; q < jj; ++q) {
          T s = zero<T>();
          for (int l = q; l < jj; ++l) s = fmac(Tl[q + l * QR_NB], outs[K1 + l], s);
          Tl[q + jj * QR_NB] = neg(mul(tau, s));
        }
      }
    }
    if (tid == 0) Tl[jj + jj * QR_NB] = tau;
    __syncthreads();
  }
  for (int i = tid; i < QR_NB * QR_NB; i += blockDim.x) Tm[i] = Tl[i];
}

// Register-resident panel factorisation: 1024 threads, thread t holds rows
// p + t + 1024 s (s < RPT) of the nb <= NBT panel columns in registers, so a
// column step touches no memory except two block reductions.  The reduction
// of column jj is one batched sum of NBT values: entries k > jj are v^* Y(:, k)
// (to apply H^* to the rest of the panel), entries k < jj are V(:, k)^* v
// (column jj of the T factor); both only involve rows >= p + jj.
constexpr int QRP_THREADS = 1024;

template <typename T, int RPT, int NBT>
__global__ __launch_bounds__(QRP_THREADS) void k_qr_panel_reg(T* Y, int ld, int d, int p, int nb, T* Tm) {
  constexpr int NROW = QRP_THREADS / 16;  // DPP rows of the workgroup
  constexpr int NW = QRP_THREADS / 64;
  __shared__ T scratch[NROW * NBT];
  __shared__ T outs[NBT];
  __shared__ T Gm[QR_NB * QR_NB];  // Gm[l * QR_NB + jj] = V(:, l)^* v_jj, l < jj
  __shared__ T taus[QR_NB];
  __shared__ T Tl[QR_NB * QR_NB];  // column-major, leading dimension QR_NB
  __shared__ double red[NW];
  __shared__ T sh_alpha;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T P[RPT][NBT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int row = p + tid + QRP_THREADS * s;
#pragma unroll
    for (int q = 0; q < NBT; ++q) P[s][q] = (row < d && q < nb) ? Y[(int64_t)(p + q) * ld + row] : zero<T>();
  }
  // The column loop is not unrolled: column jj of the register panel is read
  // and written through selects over the compile-time column index.
  for (int jj = 0; jj < nb; ++jj) {
    T pj[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      pj[s] = zero<T>();
#pragma unroll
      for (int q = 0; q < NBT; ++q)
        if (q == jj) pj[s] = P[s][q];
    }
    if (tid == jj) sh_alpha = pj[0];
    double xs = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int rel = tid + QRP_THREADS * s;
      if (rel > jj && p + rel < d) xs += abs2(pj[s]);
    }
    xs = block_sum(xs, red);
    const T alpha = sh_alpha;
    const bool noref = (xs == 0.0) && (im_(alpha) == 0.0);
    T tau = zero<T>(), sc = from_real<T>(1.0);
    double beta = re_(alpha);
    if (!noref) {
      const double nrm = sqrt(abs2(alpha) + xs);
      beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
      hh_coef(alpha, beta, tau, sc);
    }
    // v (the reflector), row by row: 1 at rel == jj, scaled entries below, 0 above
    T v[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int rel = tid + QRP_THREADS * s;
      if (rel > jj && p + rel < d) {
        pj[s] = mul(pj[s], sc);
        v[s] = pj[s];
      } else if (rel == jj) {
        v[s] = from_real<T>(1.0);
        pj[s] = from_real<T>(beta);
      } else {
        v[s] = zero<T>();
      }
#pragma unroll
      for (int q = 0; q < NBT; ++q)
        if (q == jj) P[s][q] = pj[s];
    }
    // one batched sum: k > jj: v^* Y(:, k);  k < jj: V(:, k)^* v
#pragma unroll
    for (int k = 0; k < NBT; ++k) {
      T val = zero<T>();
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        if (k > jj) val = cfmac(v[s], P[s][k], val);
        else if (k < jj) val = cfmac(P[s][k], v[s], val);
      }
      val = row_sum16(val);
      if ((tid & 15) == 0) scratch[(tid >> 4) * NBT + k] = val;
    }
    __syncthreads();
    // wave w finishes sums w, w + NW, ... over the NROW row partials
    for (int k = wid; k < NBT; k += NW) {
      T acc = zero<T>();
      for (int r = lane; r < NROW; r += 64) acc = add(acc, scratch[r * NBT + k]);
      acc = wave_sum(acc);
      if (lane == 0) outs[k] = acc;
    }
    __syncthreads();
    if (!noref) {
      const T ct = conj_(tau);
#pragma unroll
      for (int k = 0; k < NBT; ++k) {
        if (k > jj) {
          const T f = mul(ct, outs[k]);
#pragma unroll
          for (int s = 0; s < RPT; ++s) P[s][k] = fnmac(f, v[s], P[s][k]);
        }
      }
    }
    if (tid < jj) Gm[tid * QR_NB + jj] = outs[tid];
    if (tid == jj) taus[jj] = tau;
  }
  __syncthreads();
  // T factor, row q by thread q: T(q, q) = tau_q,
  // T(q, jj) = -tau_jj sum_{l = q}^{jj-1} T(q, l) (V(:, l)^* v_jj)
  // (the reads of eight terms are issued together: the sum is a chain of
  // LDS reads otherwise)
  if (tid < QR_NB) {
    const int q = tid;
    for (int jj = 0; jj < QR_NB; ++jj) {
      T val = zero<T>();
      if (jj < nb) {
        if (jj == q) {
          val = taus[q];
        } else if (jj > q) {
          T acc = zero<T>();
#pragma unroll 8
          for (int l = q; l < jj; ++l) acc = fmac(Tl[q + l * QR_NB], Gm[l * QR_NB + jj], acc);
          val = neg(mul(taus[jj], acc));
        }
      }
      Tl[q + jj * QR_NB] = val;
    }
  }
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int row = p + tid + QRP_THREADS * s;
#pragma unroll
    for (int q = 0; q < NBT; ++q)
      if (row < d && q < nb) Y[(int64_t)(p + q) * ld + row] = P[s][q];
  }
  __syncthreads();
  for (int i = tid; i < QR_NB * QR_NB; i += QRP_THREADS) Tm[i] = Tl[i];
}

// Column-wave panel factorisation (FP64 up to 1024 rows [p, d), complex up
// to 512): the nb <= 32 panel columns are dealt out over NW waves (wave w owns
// columns w, w+NW, ...) and lane l holds rows p + l + 64 s of them, so every
// column lives in one wave.  Column jj is factored by its owner alone (one
// wave reduction for the norm), which publishes the reflector and conj(tau)
// in LDS; after one barrier each wave, in one batched transpose-reduction,
// forms v^* Y(:, k) for its columns k > jj (then applies H^*) and
// V(:, k)^* v for its columns k < jj (column jj of the T factor).  The owner
// of column jj+1 factors it right after, so a column costs one barrier.
template <typename T, int NW, int RPL>
__global__ __launch_bounds__(NW * 64) void k_qr_panel_cw(T* Y, int ld, int d, int p, int nb, T* Tm) {
  constexpr int CPW = QR_NB / NW;
  constexpr int ES = (int)(sizeof(T) / 8);
  constexpr int NV = CPW * ES;  // reals reduced per column step
  constexpr int LOG2NV = NV <= 2 ? 1 : NV <= 4 ? 2 : NV <= 8 ? 3 : 4;
  static_assert(NV >= 2 && NV <= 16, "batched reduction of 2..16 reals");
  __shared__ T vbuf[2][64 * RPL];
  __shared__ T tbuf[2];
  __shared__ T taus[QR_NB];
  __shared__ T Gm[QR_NB * QR_NB];  // Gm[l * QR_NB + jj] = V(:, l)^* v_jj, l < jj
  __shared__ T Tl[QR_NB * QR_NB];  // column-major, leading dimension QR_NB
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_index();
  T x[CPW][RPL];
#pragma unroll
  for (int kc = 0; kc < CPW; ++kc) {
    const int col = wave + NW * kc;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int row = p + lane + 64 * s;
      x[kc][s] = (col < nb && row < d) ? Y[(int64_t)(p + col) * ld + row] : zero<T>();
    }
  }
  // column jj by its owner: Householder vector below the diagonal, beta on it
  auto factor = [&](T (&c)[RPL], int jj, int slot) {
    double n2p = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s)
      if (lane + 64 * s > jj) n2p += abs2(c[s]);
    const double n2 = wave_sum(n2p);
    const T alpha = readlane_d(c[0], jj);
    const bool noref = (n2 == 0.0) && (im_(alpha) == 0.0);
    T tau = zero<T>(), sc = from_real<T>(1.0);
    double beta = re_(alpha);
    if (!noref) {
      const double nrm = sqrt(abs2(alpha) + n2);
      beta = (re_(alpha) >= 0.0) ? -nrm : nrm;
      hh_coef(alpha, beta, tau, sc);
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int rel = lane + 64 * s;
      T vs = zero<T>();
      if (rel > jj) {
        if (!noref) c[s] = mul(c[s], sc);
        vs = c[s];
      } else if (rel == jj) {
        vs = from_real<T>(1.0);
        if (!noref) c[s] = from_real<T>(beta);
      }
      vbuf[slot][rel] = vs;
    }
    if (lane == 0) {
      tbuf[slot] = conj_(tau);
      taus[jj] = tau;
    }
  };
  if (wave == 0) factor(x[0], 0, 0);
#pragma unroll
  for (int jc = 0; jc < CPW; ++jc) {
    for (int ow = 0; ow < NW; ++ow) {
      const int jj = NW * jc + ow;
      if (jj >= nb) break;
      __syncthreads();
      const T ct = tbuf[jj & 1];
      T v[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) v[s] = vbuf[jj & 1][lane + 64 * s];
      double ys[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) ys[q] = 0.0;
#pragma unroll
      for (int kc = 0; kc < CPW; ++kc) {
        const int k = wave + NW * kc;
        if (k < nb && k != jj) {
          T acc = zero<T>();
          if (k > jj) {
#pragma unroll
            for (int s = 0; s < RPL; ++s) acc = cfmac(v[s], x[kc][s], acc);
          } else {
#pragma unroll
            for (int s = 0; s < RPL; ++s) acc = cfmac(x[kc][s], v[s], acc);
          }
          if constexpr (ES == 2) {
            ys[2 * kc] = re_(acc);
            ys[2 * kc + 1] = im_(acc);
          } else {
            ys[kc] = re_(acc);
          }
        }
      }
      tr_reduce_plain<NV, LOG2NV>(ys, lane);
#pragma unroll
      for (int kc = 0; kc < CPW; ++kc) {
        const int k = wave + NW * kc;
        if (k < nb && k != jj) {
          T dk;
          if constexpr (ES == 2) {
            dk = T{readlane_d(ys[0], tr_src_lane<LOG2NV>(2 * kc)), readlane_d(ys[0], tr_src_lane<LOG2NV>(2 * kc + 1))};
          } else {
            dk = readlane_d(ys[0], tr_src_lane<LOG2NV>(kc));
          }
          if (k > jj) {
            const T f = mul(ct, dk);
#pragma unroll
            for (int s = 0; s < RPL; ++s) x[kc][s] = fnmac(f, v[s], x[kc][s]);
          } else if (lane == 0) {
            Gm[k * QR_NB + jj] = dk;
          }
        }
      }
      const int j1 = jj + 1;
      if (j1 < nb && wave == (ow + 1) % NW) {
        if (ow + 1 < NW) factor(x[jc], j1, j1 & 1);
        else if (jc + 1 < CPW) factor(x[jc + 1 < CPW ? jc + 1 : jc], j1, j1 & 1);
      }
    }
  }
  __syncthreads();
  // T factor, row q by thread q: T(q, q) = tau_q,
  // T(q, jj) = -tau_jj sum_{l = q}^{jj-1} T(q, l) (V(:, l)^* v_jj)
  // (the reads of eight terms are issued together: the sum is a chain of
  // LDS reads otherwise)
  if (tid < QR_NB) {
    const int q = tid;
    for (int jj = 0; jj < QR_NB; ++jj) {
      T val = zero<T>();
      if (jj < nb) {
        if (jj == q) {
          val = taus[q];
        } else if (jj > q) {
          T acc = zero<T>();
#pragma unroll 8
          for (int l = q; l < jj; ++l) acc = fmac(Tl[q + l * QR_NB], Gm[l * QR_NB + jj], acc);
          val = neg(mul(taus[jj], acc));
        }
      }
      Tl[q + jj * QR_NB] = val;
    }
  }
#pragma unroll
  for (int kc = 0; kc < CPW; ++kc) {
    const int col = wave + NW * kc;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int row = p + lane + 64 * s;
      if (col < nb && row < d) Y[(int64_t)(p + col) * ld + row] = x[kc][s];
    }
  }
  __syncthreads();
  for (int i = tid; i < QR_NB * QR_NB; i += NW * 64) Tm[i] = Tl[i];
}

// rows per lane of the column-wave panel for `rows` rows, or 0 when the panel
// is too tall for it
template <typename T>
static int qr_cw_rpl(int rows) {
  if constexpr (sizeof(T) == 4) return 0;  // FP32 panels keep their own kernels
  // the panel stays in registers: 4 x 16 doubles or 2 x 8 complex per lane
  const int r = (rows + 63) / 64;
  const int rmax = sizeof(T) == 16 ? 8 : 16;
  if (r > rmax) return 0;
  return r <= 4 ? 4 : r <= 8 ? 8 : 16;
}

template <typename T>
static void qr_panel_cw_launch(hipStream_t st, T* Y, int d, int p, int nb, int rpl, T* Tm) {
  if constexpr (sizeof(T) == 8) {
    const dim3 g(1);
    if (rpl == 4) hipLaunchKernelGGL((k_qr_panel_cw<T, 8, 4>), g, dim3(512), 0, st, Y, d, d, p, nb, Tm);
    else if (rpl == 8) hipLaunchKernelGGL((k_qr_panel_cw<T, 8, 8>), g, dim3(512), 0, st, Y, d, d, p, nb, Tm);
    else hipLaunchKernelGGL((k_qr_panel_cw<T, 8, 16>), g, dim3(512), 0, st, Y, d, d, p, nb, Tm);
  } else if constexpr (sizeof(T) == 16) {
    const dim3 g(1), b(1024);
    if (rpl == 4) hipLaunchKernelGGL((k_qr_panel_cw<T, 16, 4>), g, b, 0, st, Y, d, d, p, nb, Tm);
    else hipLaunchKernelGGL((k_qr_panel_cw<T, 16, 8>), g, b, 0, st, Y, d, d, p, nb, Tm);
  }
}

// Panel width and register rows per thread for the rows [p, d): the panel
// must fit in about 64 registers per thread.
template <typename T>
static int qr_pick_panel(int rows, int* rpt) {
  const int r = (rows + QRP_THREADS - 1) / QRP_THREADS;
  *rpt = r;
  const int cw = (sizeof(T) == 16) ? 2 : 1;  // FP32 panels use the FP64 shapes
  if (r <= 1) return 32 / cw;
  if (r <= 2) return 16 / cw;
  if (r <= 4) return 8 / cw;
  return 0;  // too tall for the register panel: generic kernel
}

template <typename T>
static void qr_panel_launch(hipStream_t st, T* Y, int d, int p, int nb, int rpt, T* Tm) {
  const dim3 g(1), b(QRP_THREADS);
  if constexpr (sizeof(T) <= 8) {
    if (rpt <= 1) hipLaunchKernelGGL((k_qr_panel_reg<T, 1, 32>), g, b, 0, st, Y, d, d, p, nb, Tm);
    else if (rpt <= 2) hipLaunchKernelGGL((k_qr_panel_reg<T, 2, 16>), g, b, 0, st, Y, d, d, p, nb, Tm);
    else hipLaunchKernelGGL((k_qr_panel_reg<T, 4, 8>), g, b, 0, st, Y, d, d, p, nb, Tm);
  } else {
    if (rpt <= 1) hipLaunchKernelGGL((k_qr_panel_reg<T, 1, 16>), g, b, 0, st, Y, d, d, p, nb, Tm);
    else if (rpt <= 2) hipLaunchKernelGGL((k_qr_panel_reg<T, 2, 8>), g, b, 0, st, Y, d, d, p, nb, Tm);
    else hipLaunchKernelGGL((k_qr_panel_reg<T, 4, 4>), g, b, 0, st, Y, d, d, p, nb, Tm);
  }
}

// C <- (I - V T V^*)^* C = C - V T^* (V^* C) on columns [p+nb, n)
// BF16IN (float only): the panel V and the trailing columns enter both
// products rounded to bfloat16; products and sums stay in FP32.
template <typename T, bool BF16IN = false>
__global__ __launch_bounds__(QR_THREADS) void k_qr_update(T* Y, int ld, int d, int n, int p, int nb,
                                                          const T* __restrict__ Tm) {
  // rows per chunk of V and C staged in LDS (under 52 KB for either type)
  constexpr int RCH = sizeof(T) == 16 ? 64 : 128;
  constexpr int NV = RCH * QR_NB / QR_THREADS;  // V values per thread and chunk
  constexpr int NC = RCH * QR_CB / QR_THREADS;  // C values per thread and chunk
  __shared__ T Vs[RCH][QR_NB + 1];
  __shared__ T Cs[RCH][QR_CB + 1];
  __shared__ T Wt[QR_NB][QR_CB];
  __shared__ T Wt2[QR_NB][QR_CB];
  const int tid = threadIdx.x;
  const int c0 = p + nb + blockIdx.x * QR_CB;
  const int ncb = min(QR_CB, n - c0);
  const int q = tid / QR_CB, cb = tid % QR_CB;  // 32 x 8 = 256
  // a chunk's values are loaded into registers together, the next chunk's
  // while the current one is summed
  T vv[NV], cv[NC];
  auto load_chunk = [&](int r0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int i = tid + k * QR_THREADS;
      const int rr = i % RCH, qq = i / RCH, r = r0 + rr;
      vv[k] = (qq < nb && r < d) ? vpanel(Y, ld, p, qq, r) : zero<T>();
      if constexpr (BF16IN) vv[k] = bf16_round(vv[k]);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = tid + k * QR_THREADS;
      const int rr = i % RCH, cc = i / RCH, r = r0 + rr;
      cv[k] = (cc < ncb && r < d) ? Y[(int64_t)(c0 + cc) * ld + r] : zero<T>();
      if constexpr (BF16IN) cv[k] = bf16_round(cv[k]);
    }
  };
  T acc = zero<T>();
  load_chunk(p);
  for (int r0 = p; r0 < d; r0 += RCH) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int i = tid + k * QR_THREADS;
      Vs[i % RCH][i / RCH] = vv[k];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = tid + k * QR_THREADS;
      Cs[i % RCH][i / RCH] = cv[k];
    }
    __syncthreads();
    if (r0 + RCH < d) load_chunk(r0 + RCH);
#pragma unroll 8
    for (int rr = 0; rr < RCH; ++rr) acc = cfmac(Vs[rr][q], Cs[rr][cb], acc);
  }
  Wt[q][cb] = acc;
  __syncthreads();
  {
    T s = zero<T>();
    for (int l = 0; l <= q && l < nb; ++l) s = cfmac(Tm[l + q * QR_NB], Wt[l][cb], s);
    Wt2[q][cb] = (q < nb) ? s : zero<T>();
  }
  __syncthreads();
  for (int r = p + tid; r < d; r += blockDim.x) {
    T vr[QR_NB];
#pragma unroll
    for (int qq = 0; qq < QR_NB; ++qq) {
      vr[qq] = (qq < nb) ? vpanel(Y, ld, p, qq, r) : zero<T>();
      if constexpr (BF16IN) vr[qq] = bf16_round(vr[qq]);
    }
    // the row's QR_CB trailing entries are loaded together, updated, stored
    T yv[QR_CB];
#pragma unroll
    for (int c = 0; c < QR_CB; ++c) yv[c] = (c < ncb) ? Y[(int64_t)(c0 + c) * ld + r] : zero<T>();
    // the column loop stays rolled (so the 8 x 32 coefficients are read
    // from LDS per column, not held in registers); yv is indexed by selects
#pragma unroll 1
    for (int c = 0; c < QR_CB; ++c) {
      T v = zero<T>();
#pragma unroll
      for (int k = 0; k < QR_CB; ++k)
        if (k == c) v = yv[k];
#pragma unroll
      for (int qq = 0; qq < QR_NB; ++qq) {
        if constexpr (BF16IN) v = fnmac(vr[qq], bf16_round(Wt2[qq][c]), v);
        else v = fnmac(vr[qq], Wt2[qq][c], v);
      }
#pragma unroll
      for (int k = 0; k < QR_CB; ++k)
        if (k == c) yv[k] = v;
    }
#pragma unroll
    for (int c = 0; c < QR_CB; ++c)
      if (c < ncb) Y[(int64_t)(c0 + c) * ld + r] = yv[c];
  }
}

// The trailing update of the reduced-precision (FP32) factorisation on the
// FP32 matrix cores: C <- C - V T^T (V^T C) on 16 trailing columns per
// workgroup, the rows walked in chunks of QRM_RC staged in LDS.  First V^T C
// (32 x 16; wave w takes V columns 16 (w & 1) .. + 15 over the chunk's row
// half w >> 1, the halves summed at the end), then W2 = T^T (V^T C) on the
// vector units, then C -= V W2 chunk by chunk (wave w takes rows 16 w ..
// 16 w + 15 of the chunk).  BF16IN: V, C and W2 enter the products rounded
// to bfloat16 (v_mfma_f32_16x16x16bf16), the sums and C stay FP32; else FP32
// inputs (v_mfma_f32_16x16x4f32).  Lane layouts (checked on gfx950): FP32:
// lane 16 k + i supplies A(i, k), lane 16 k + j supplies B(k, j); BF16:
// lane 16 (k / 4) + i supplies A(i, k) in its element k % 4, and B alike;
// both: register r of lane l holds D(4 (l / 16) + r, l % 16).
typedef float qrm_v4f __attribute__((ext_vector_type(4)));
typedef short qrm_v4s __attribute__((ext_vector_type(4)));
constexpr int QRM_RC = 64;  // rows per staged chunk
constexpr int QRM_CB = 16;  // trailing columns per workgroup

__device__ inline short qrm_bf16(float x) { return (short)(__float_as_uint(bf16_round(x)) >> 16); }

template <bool BF16IN>
__device__ inline qrm_v4f qrm_mma(const float* a4, const float* b4, qrm_v4f c) {
  // a4 / b4: this lane's 4 (BF16) or 1 (FP32) operand values
  if constexpr (BF16IN) {
    qrm_v4s a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a[e] = qrm_bf16(a4[e]);
      b[e] = qrm_bf16(b4[e]);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a4[0], b4[0], c, 0, 0, 0);
  }
}

template <bool BF16IN>
__global__ __launch_bounds__(256) void k_qr_update_mfma(float* __restrict__ Y, int ld, int d, int n, int p, int nb,
                                                        const float* __restrict__ Tm) {
  __shared__ float Vs[QRM_RC][QR_NB + 1];
  __shared__ float Cs[QRM_RC][QRM_CB + 1];
  __shared__ float Wh[2][QR_NB][QRM_CB];  // the two row halves' V^T C
  __shared__ float W2[QR_NB][QRM_CB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int c0 = p + nb + blockIdx.x * QRM_CB;
  const int ncb = min(QRM_CB, n - c0);
  // K steps per MFMA: 16 rows (BF16, 4 per lane) or 4 rows (FP32, 1 per lane)
  constexpr int KS = BF16IN ? 16 : 4;
  auto stage = [&](int r0) {
    for (int e = tid; e < QRM_RC * QR_NB; e += 256) {
      const int rr = e % QRM_RC, q = e / QRM_RC, r = r0 + rr;
      Vs[rr][q] = (q < nb && r < d) ? vpanel(Y, ld, p, q, r) : 0.0f;
    }
    for (int e = tid; e < QRM_RC * QRM_CB; e += 256) {
      const int rr = e % QRM_RC, c = e / QRM_RC, r = r0 + rr;
      Cs[rr][c] = (c < ncb && r < d) ? Y[(int64_t)(c0 + c) * ld + r] : 0.0f;
    }
  };
  // pass 1: V^T C
  qrm_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
  const int mi = wave & 1, kh = wave >> 1;
  for (int r0 = p; r0 < d; r0 += QRM_RC) {
    __syncthreads();
    stage(r0);
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < QRM_RC / 2; k0 += KS) {
      float a4[4], b4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // A(i, k) = V(row k, column 16 mi + i), B(k, j) = C(row k, column j)
        const int kk = BF16IN ? 4 * lk + e : lk;
        const int row = kh * (QRM_RC / 2) + k0 + kk;
        a4[e] = (BF16IN || e == 0) ? Vs[row][16 * mi + li] : 0.0f;
        b4[e] = (BF16IN || e == 0) ? Cs[row][li] : 0.0f;
      }
      acc = qrm_mma<BF16IN>(a4, b4, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Wh[kh][16 * mi + 4 * lk + r][li] = acc[r];
  __syncthreads();
  // W2 = T^T (V^T C): W2[q][c] = sum over l <= q of T(l, q) (V^T C)[l][c]
  for (int e = tid; e < QR_NB * QRM_CB; e += 256) {
    const int q = e / QRM_CB, c = e % QRM_CB;
    float sacc = 0.0f;
    for (int l = 0; l <= q && l < nb; ++l) sacc = fmaf(Tm[l + q * QR_NB], Wh[0][l][c] + Wh[1][l][c], sacc);
    W2[q][c] = (q < nb) ? sacc : 0.0f;
  }
  // pass 2: C -= V W2, wave w on rows 16 w .. 16 w + 15 of each chunk
  for (int r0 = p; r0 < d; r0 += QRM_RC) {
    __syncthreads();
    stage(r0);
    __syncthreads();
    qrm_v4f dv = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < QR_NB; k0 += KS) {
      float a4[4], b4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // A(i, k) = V(row 16 w + i, column k), B(k, j) = W2(k, j)
        const int kk = k0 + (BF16IN ? 4 * lk + e : lk);
        a4[e] = (BF16IN || e == 0) ? Vs[16 * wave + li][kk] : 0.0f;
        b4[e] = (BF16IN || e == 0) ? W2[kk][li] : 0.0f;
      }
      dv = qrm_mma<BF16IN>(a4, b4, dv);
    }
    // lane l, register r: row 16 w + 4 (l / 16) + r of the chunk, column l % 16
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 16 * wave + 4 * lk + r;
      const int row = r0 + rr;
      if (row < d && li < ncb) Y[(int64_t)(c0 + li) * ld + row] = Cs[rr][li] - dv[r];
    }
  }
}

template <typename T>
__global__ void k_qr_extract(const T* __restrict__ Y, int ld, int n, T* __restrict__ Rrow, T* __restrict__ RH) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  Rrow[idx] = (j >= i) ? Y[(int64_t)j * ld + i] : zero<T>();
  RH[idx] = (j <= i) ? conj_(Y[(int64_t)i * ld + j]) : zero<T>();
}

template <typename T>
__global__ __launch_bounds__(256) void k_trinv(const T* __restrict__ Y, int ld, int n, T* __restrict__ Rinv,
                                               T* __restrict__ RinvH) {
  extern __shared__ double smem_d[];
  const int lane = threadIdx.x & 63, wave = wave_index();
  T* xs = reinterpret_cast<T*>(smem_d) + (int64_t)wave * n;
  const int k = blockIdx.x * 4 + wave;
  if (k >= n) return;
  for (int i = lane; i < n; i += 64) xs[i] = (i == k) ? from_real<T>(1.0) : zero<T>();
  __builtin_amdgcn_wave_barrier();
  for (int i = k; i >= 0; --i) {
    const T* coli = Y + (int64_t)i * ld;
    const T xi = divs(xs[i], coli[i]);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) xs[i] = xi;
    for (int l = lane; l < i; l += 64) xs[l] = fnmac(coli[l], xi, xs[l]);
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = lane; i < n; i += 64) {
    const T x = (i <= k) ? xs[i] : zero<T>();
    Rinv[(int64_t)i * n + k] = x;
    RinvH[(int64_t)k * n + i] = conj_(x);
  }
}

// Panels taller than the register-resident panel holds (over 4096 rows):
// leaves of LW columns (8 rows per thread of a 1024-thread workgroup, up to
// 8192 rows), each followed by the update of the panel's remaining columns,
// then the compact-WY T factor of the whole panel, so the trailing update
// keeps its QR_NB-wide panels.  The T factor is rebuilt from the Gram matrix
// of the panel's reflectors, Gm(l, j) = V(:, l)^* V(:, j) over rows [p, d),
// and the leaves' tau_q (their T factors' diagonals), by the same recurrence
// the panel kernels use.
constexpr int QRT_THREADS = 512;  // one thread per pair l < j of a 32-column panel
constexpr int QRT_RC = 64;        // rows per LDS chunk

constexpr int QRL_ROWS = 1024;  // rows per workgroup of the row-split panel kernels (256 threads x 4)
constexpr int QRL_MAXBLK = QRP_THREADS * 8 / QRL_ROWS;

__device__ inline void qr_pair_of(int tid, int nb, int& pl, int& pj) {
  pl = -1;
  pj = -1;
  int c = tid;
  for (int j = 1; j < nb; ++j) {
    if (c < j) {
      pl = c;
      pj = j;
      return;
    }
    c -= j;
  }
}

// Partial Gram matrices of the panel's reflectors, one per block of
// QRL_ROWS rows: Gpart[blk * 512 + pair] = sum over the block's rows of
// V(r, l)^* V(r, j) (pair -> (l, j), l < j < nb).
template <typename T>
__global__ __launch_bounds__(QRT_THREADS) void k_qr_gram_part(const T* __restrict__ Y, int ld, int d, int p, int nb,
                                                              T* __restrict__ Gpart) {
  __shared__ T Vs[QRT_RC][QR_NB + 1];
  const int tid = threadIdx.x;
  int pl, pj;
  qr_pair_of(tid, nb, pl, pj);
  const int rb0 = p + blockIdx.x * QRL_ROWS;
  const int rb1 = min(rb0 + QRL_ROWS, d);
  T acc = zero<T>();
  for (int r0 = rb0; r0 < rb1; r0 += QRT_RC) {
    __syncthreads();
    for (int e = tid; e < QRT_RC * QR_NB; e += QRT_THREADS) {
      const int rr = e % QRT_RC, q = e / QRT_RC, r = r0 + rr;
      Vs[rr][q] = (q < nb && r < rb1) ? vpanel(Y, ld, p, q, r) : zero<T>();
    }
    __syncthreads();
    if (pl >= 0) {
#pragma unroll 8
      for (int rr = 0; rr < QRT_RC; ++rr) acc = cfmac(Vs[rr][pl], Vs[rr][pj], acc);
    }
  }
  Gpart[(int64_t)blockIdx.x * QRT_THREADS + tid] = acc;
}

template <typename T>
__global__ __launch_bounds__(QRT_THREADS) void k_qr_tfactor(const T* __restrict__ Gpart, int nblk, int nb,
                                                            const T* __restrict__ Tleaf, int lw,
                                                            T* __restrict__ Tm) {
  __shared__ T Gm[QR_NB * QR_NB];
  __shared__ T taus[QR_NB];
  __shared__ T Tl[QR_NB * QR_NB];
  const int tid = threadIdx.x;
  int pl, pj;
  qr_pair_of(tid, nb, pl, pj);
  if (pl >= 0) {
    T acc = zero<T>();
    for (int b = 0; b < nblk; ++b) acc = add(acc, Gpart[(int64_t)b * QRT_THREADS + tid]);
    Gm[pl * QR_NB + pj] = acc;
  }
  if (tid < nb) {
    const int q = tid % lw;
    taus[tid] = Tleaf[(int64_t)(tid / lw) * QR_NB * QR_NB + q + q * QR_NB];
  }
  __syncthreads();
  if (tid < QR_NB) {
    const int q = tid;
    for (int jj = 0; jj < QR_NB; ++jj) {
      T val = zero<T>();
      if (jj < nb) {
        if (jj == q) {
          val = taus[q];
        } else if (jj > q) {
          T a = zero<T>();
          for (int l = q; l < jj; ++l) a = fmac(Tl[q + l * QR_NB], Gm[l * QR_NB + jj], a);
          val = neg(mul(taus[jj], a));
        }
      }
      Tl[q + jj * QR_NB] = val;
    }
  }
  __syncthreads();
  for (int i = tid; i < QR_NB * QR_NB; i += QRT_THREADS) Tm[i] = Tl[i];
}

// The update of a leaf's panel columns [c0, c1) by its reflectors (rows from
// pl on; lw <= LW columns of V), split over row blocks: part[blk][c][q] =
// sum over the block's rows of V(r, q)^* C(r, c), then C -= V T^* W with W
// the blocks' partials summed in block order (the same arithmetic as
// k_qr_update, with the rows spread over the grid).
template <typename T, int LW>
__global__ __launch_bounds__(256) void k_qr_leafupd_part(const T* __restrict__ Y, int ld, int d, int pl, int lw,
                                                         int c0, int c1, T* __restrict__ part) {
  constexpr int G = 4;  // columns per batched reduction
  __shared__ T scratch[(256 / 16) * LW * G];
  __shared__ T outs[LW * G];
  const int tid = threadIdx.x;
  const int rb0 = pl + blockIdx.x * QRL_ROWS;
  T v[4][LW];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int r = rb0 + tid + 256 * s;
#pragma unroll
    for (int q = 0; q < LW; ++q) v[s][q] = (r < d && q < lw) ? vpanel(Y, ld, pl, q, r) : zero<T>();
  }
  const int ncol = c1 - c0;
  for (int g0 = 0; g0 < ncol; g0 += G) {
    T vals[LW * G];
#pragma unroll
    for (int e = 0; e < LW * G; ++e) vals[e] = zero<T>();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = rb0 + tid + 256 * s;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const T cv = (r < d && g0 + g < ncol) ? Y[(int64_t)(c0 + g0 + g) * ld + r] : zero<T>();
#pragma unroll
        for (int q = 0; q < LW; ++q) vals[g * LW + q] = cfmac(v[s][q], cv, vals[g * LW + q]);
      }
    }
    block_sum_many<T, LW * G>(vals, LW * G, scratch, outs);
    if (tid < LW * G && g0 + tid / LW < ncol)
      part[((int64_t)blockIdx.x * QR_NB + g0 + tid / LW) * LW + tid % LW] = outs[tid];
  }
}

template <typename T, int LW>
__global__ __launch_bounds__(256) void k_qr_leafupd_apply(T* __restrict__ Y, int ld, int d, int pl, int lw, int c0,
                                                          int c1, const T* __restrict__ part, int nblk,
                                                          const T* __restrict__ Tq) {
  __shared__ T Wt[QR_NB][LW];
  __shared__ T Wt2[QR_NB][LW];
  const int tid = threadIdx.x;
  const int ncol = c1 - c0;
  if (tid < ncol * LW) {
    const int c = tid / LW, q = tid % LW;
    T acc = zero<T>();
    for (int b = 0; b < nblk; ++b) acc = add(acc, part[((int64_t)b * QR_NB + c) * LW + q]);
    Wt[c][q] = acc;
  }
  __syncthreads();
  if (tid < ncol * LW) {
    const int c = tid / LW, q = tid % LW;
    T sacc = zero<T>();
    for (int l = 0; l <= q && l < lw; ++l) sacc = cfmac(Tq[l + q * QR_NB], Wt[c][l], sacc);
    Wt2[c][q] = (q < lw) ? sacc : zero<T>();
  }
  __syncthreads();
  const int rb0 = pl + blockIdx.x * QRL_ROWS;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int r = rb0 + tid + 256 * s;
    if (r >= d) continue;
    T vr[LW];
#pragma unroll
    for (int q = 0; q < LW; ++q) vr[q] = (q < lw) ? vpanel(Y, ld, pl, q, r) : zero<T>();
    for (int c = 0; c < ncol; ++c) {
      T y = Y[(int64_t)(c0 + c) * ld + r];
#pragma unroll
      for (int q = 0; q < LW; ++q) y = fnmac(vr[q], Wt2[c][q], y);
      Y[(int64_t)(c0 + c) * ld + r] = y;
    }
  }
}

template <typename T>
static bool qr_leaf_fits(int rows) {
  return rows <= QRP_THREADS * 8;
}

// The T workspace (QR_TM_ELEMS elements): the panel's T factor, the
// leaves' T factors, the leaf updates' partial sums, the Gram partials.
constexpr int QR_TM_LEAVES = QR_NB * QR_NB;                       // offset of the leaves' T factors
constexpr int QR_TM_UPD = QR_TM_LEAVES + 16 * QR_NB * QR_NB;      // leaf-update partials
constexpr int QR_TM_GRAM = QR_TM_UPD + QRL_MAXBLK * QR_NB * 4;    // Gram partials
static_assert(QR_TM_GRAM + QRL_MAXBLK * QRT_THREADS <= QR_TM_ELEMS, "T workspace");

template <typename T, int LW, int RPT>
static void qr_panel_leaves_go(hipStream_t st, T* Y, int d, int p, int nb, T* Tm) {
  static_assert(QR_NB / LW <= 16 && LW <= 4, "leaf T factors and partials fit the T workspace");
  T* Tleaf = Tm + QR_TM_LEAVES;
  T* upd = Tm + QR_TM_UPD;
  T* gram = Tm + QR_TM_GRAM;
  for (int q = 0; q < nb; q += LW) {
    const int lw = min(LW, nb - q);
    T* Tq = Tleaf + (int64_t)(q / LW) * QR_NB * QR_NB;
    hipLaunchKernelGGL((k_qr_panel_reg<T, RPT, LW>), dim3(1), dim3(QRP_THREADS), 0, st, Y, d, d, p + q, lw, Tq);
    const int c0 = p + q + lw, c1 = p + nb;
    if (c1 > c0) {  // the panel's own columns: full precision, as the panel kernels
      const int nblk = (d - (p + q) + QRL_ROWS - 1) / QRL_ROWS;
      hipLaunchKernelGGL((k_qr_leafupd_part<T, LW>), dim3(nblk), dim3(256), 0, st, (const T*)Y, d, d, p + q, lw, c0,
                         c1, upd);
      hipLaunchKernelGGL((k_qr_leafupd_apply<T, LW>), dim3(nblk), dim3(256), 0, st, Y, d, d, p + q, lw, c0, c1,
                         (const T*)upd, nblk, (const T*)Tq);
    }
  }
  const int nblk = (d - p + QRL_ROWS - 1) / QRL_ROWS;
  hipLaunchKernelGGL(k_qr_gram_part<T>, dim3(nblk), dim3(QRT_THREADS), 0, st, (const T*)Y, d, d, p, nb, gram);
  hipLaunchKernelGGL(k_qr_tfactor<T>, dim3(1), dim3(QRT_THREADS), 0, st, (const T*)gram, nblk, nb, (const T*)Tleaf,
                     LW, Tm);
}

// Leaves of 4 columns (complex: of 2 where the rows need 8 per thread, the
// register budget of a 1024-thread workgroup): each leaf costs three launches
// whatever its width.
template <typename T>
static void qr_panel_leaves(hipStream_t st, T* Y, int d, int p, int nb, T* Tm) {
  if constexpr (sizeof(T) == 16) {
    if (d - p <= QRP_THREADS * 4) qr_panel_leaves_go<T, 4, 4>(st, Y, d, p, nb, Tm);
    else qr_panel_leaves_go<T, 2, 8>(st, Y, d, p, nb, Tm);
  } else {
    qr_panel_leaves_go<T, 4, 8>(st, Y, d, p, nb, Tm);
  }
}

// Blocked Householder factorization of the d x n column-major Y in place.
template <typename T, bool BF16IN = false>
static void qr_factor(hipStream_t st, T* Y, int d, int n, T* Tm) {
  for (int p = 0; p < n;) {
    int rpt = 0, nb;
    const int rpl = qr_cw_rpl<T>(d - p);
    if (rpl > 0) {
      nb = min(QR_NB, n - p);
      qr_panel_cw_launch<T>(st, Y, d, p, nb, rpl, Tm);
    } else {
      int nbr = qr_pick_panel<T>(d - p, &rpt);
      // a register panel narrower than half a block would cost a trailing
      // update (a full pass over the rest of the sketch) every few columns:
      // such heights take 32-column panels factored in leaves instead
      if constexpr (sizeof(T) != 4)
        if (nbr > 0 && nbr < QR_NB / 2 && qr_leaf_fits<T>(d - p)) nbr = 0;
      nb = min(nbr > 0 ? nbr : QR_NB, n - p);
      if (nbr > 0)
        qr_panel_launch<T>(st, Y, d, p, nb, rpt, Tm);
      else if (qr_leaf_fits<T>(d - p))
        qr_panel_leaves<T>(st, Y, d, p, nb, Tm);
      else
        hipLaunchKernelGGL(k_qr_panel<T>, dim3(1), dim3(QR_THREADS), 0, st, Y, d, d, n, p, nb, Tm);
    }
    const int rest = n - p - nb;
    if (rest > 0) {
      if constexpr (sizeof(T) == 4)  // the reduced-precision factorisation: on the matrix cores
        hipLaunchKernelGGL((k_qr_update_mfma<BF16IN>), dim3((rest + QRM_CB - 1) / QRM_CB), dim3(256), 0, st,
                           (float*)Y, d, d, n, p, nb, (const float*)Tm);
      else
        hipLaunchKernelGGL((k_qr_update<T, BF16IN>), dim3((rest + QR_CB - 1) / QR_CB), dim3(QR_THREADS), 0, st, Y,
                           d, d, n, p, nb, (const T*)Tm);
    }
    p += nb;
  }
}

// R (upper triangle of Y) in row-major form and R^{-1}, R^{-*}.
template <typename T>
static hipError_t qr_finish(hipStream_t st, const T* Y, int d, int n, T* Rrow, T* RH, T* Rinv, T* RinvH,
                            hipEvent_t r_ready) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_qr_extract<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, Y, d, n, Rrow, RH);
  // R is complete here (in Y and Rrow); the inverses follow
  if (r_ready != nullptr) {
    const hipError_t e = hipEventRecord(r_ready, st);
    if (e != hipSuccess) return e;
  }
  const size_t lds = (size_t)4 * n * sizeof(T);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_trinv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_trinv<T>, dim3((n + 3) / 4), dim3(256), lds, st, Y, d, n, Rinv, RinvH);
  return hipGetLastError();
}

template <typename T>
static hipError_t qr_impl(hipStream_t st, T* Y, int d, int n, T* Tm, T* Rrow, T* RH, T* Rinv, T* RinvH,
                          hipEvent_t r_ready) {
  qr_factor<T>(st, Y, d, n, Tm);
  return qr_finish<T>(st, Y, d, n, Rrow, RH, Rinv, RinvH, r_ready);
}

// Upper triangle (rows 0..n-1) of the FP32 factor into the FP64 Y (ld d).
__global__ void k_promote_upper(const float* __restrict__ Yf, int d, int n, double* __restrict__ Y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int j = (int)(idx / n), i = (int)(idx % n);  // column j, row i
  Y[(int64_t)j * d + i] = (i <= j) ? (double)Yf[(int64_t)j * d + i] : 0.0;
}

hipError_t launch_qr(hipStream_t st, bool cplx, void* Y, int d, int n, void* Tm, void* Rrow, void* RH, void* Rinv,
                     void* RinvH, hipEvent_t r_ready) {
  if (cplx)
    return qr_impl<cd>(st, (cd*)Y, d, n, (cd*)Tm, (cd*)Rrow, (cd*)RH, (cd*)Rinv, (cd*)RinvH, r_ready);
  return qr_impl<double>(st, (double*)Y, d, n, (double*)Tm, (double*)Rrow, (double*)RH, (double*)Rinv,
                         (double*)RinvH, r_ready);
}

// Reduced-precision QR of a real sketch: factor the FP32 Yf (trailing updates
// in FP32, or with bfloat16 inputs and FP32 accumulation), promote R to FP64
// into Y, then R^{-1} and the row-major copies in FP64.
hipError_t launch_qr_lowp(hipStream_t st, float* Yf, int d, int n, float* Tmf, double* Y, double* Rrow, double* RH,
                          double* Rinv, double* RinvH, bool bf16, hipEvent_t r_ready) {
  if (bf16) qr_factor<float, true>(st, Yf, d, n, Tmf);
  else qr_factor<float, false>(st, Yf, d, n, Tmf);
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_promote_upper, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, (const float*)Yf, d, n,
                     Y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return qr_finish<double>(st, Y, d, n, Rrow, RH, Rinv, RinvH, r_ready);
}

}  // namespace rl
