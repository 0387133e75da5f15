// A-stream kernels: the m-long products of RLOBPCG (paper Alg. rlopcg and
// Alg. rlobpcg: the product with the trial space and the residual's A^*).
//
// k_astream   one pass over the tall A (m x n, row-major, leading dim lda):
//               A_W = A W                                   (m x B)
//               G_T = A^* [A_V A_X A_W]                     (n x 3B, partial sums)
//             The residual R = A^* A_V(new) - V Theta^2 needs A^* of the
//             updated A_V = A_T C_V.  Since A^* A_T C_V = G_T C_V, computing
//             G_T fresh in the pass that forms A_W gives the residual with one
//             read of A per iteration; A_V and A_X (known before the pass) are
//             streamed beside A.  Nothing is carried from iteration to
//             iteration, so no drift builds up in G.
//             Mapping: a wave owns a batch of RB rows; lane l owns columns
//             l, l+64, ...; W and the G accumulators stay in registers; the
//             row dot products of A W are wave reductions.
//             With DOT2 the row products of A W and the column sums of A^* A_V
//             are Dot2 (TwoProduct by FMA, TwoSum, compensated butterfly across
//             lanes; Ogita, Rump and Oishi): A_W is accurate to about one
//             rounding of its own size and A^* A_V likewise, which is what the
//             residual of a converged block needs.  A^* A_X and A^* A_W enter
//             the residual through coefficients that vanish at convergence and
//             stay plain FP64.  In the start pass (init) the new column is
//             A V_0 itself, and its A^* sum is the Dot2 one.
//             Per-wave partials: planes [G1 sum, G1 error, G_X, G_W], n x B each.
// k_colsum2   deterministic compensated sum of the partial planes.
// k_panel     A_V <- A_T C_V, A_X <- A_T C_X (row-local, in place).
// k_final_u   U(:, j) = (A_T C_V)(:, b-1-j) / theta_{b-1-j} for the outputs.
#include "common.hpp"
#include "kernels.hpp"

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

// Compensated, deterministic sum over parts.  Input part p has sums at
// in_s[p*stride + e] and, for e < elen, errors at in_e[p*stride + e];
// block y of the grid sums parts [64y, 64y+64) and writes (sum, error) to
// out_s/out_e[y*len + e].
__global__ __launch_bounds__(256) void k_colsum2(const double* __restrict__ in_s, const double* __restrict__ in_e,
                                                 int64_t stride, int64_t elen, int64_t nparts, int64_t len,
                                                 double* __restrict__ out_s, double* __restrict__ out_e,
                                                 const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  __shared__ double sh_s[256], sh_e[256];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;  // 64 elements x 4 groups
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  const int64_t p0 = (int64_t)blockIdx.y * 64;
  double S = 0.0, E = 0.0;
  if (e < len) {
    for (int k = g; k < 64; k += 4) {
      const int64_t p = p0 + k;
      if (p < nparts) {
        double t;
        two_sum(S, in_s[p * stride + e], S, t);
        E += t + (e < elen ? in_e[p * stride + e] : 0.0);
      }
    }
  }
  sh_s[threadIdx.x] = S;
  sh_e[threadIdx.x] = E;
  __syncthreads();
  if (g == 0 && e < len) {
    double s0 = sh_s[el], e0 = sh_e[el], t;
    for (int q = 1; q < 4; ++q) {
      two_sum(s0, sh_s[64 * q + el], s0, t);
      e0 += t + sh_e[64 * q + el];
    }
    out_s[(int64_t)blockIdx.y * len + e] = s0;
    out_e[(int64_t)blockIdx.y * len + e] = e0;
  }
}

__global__ void k_pair_finish(const double* __restrict__ s, const double* __restrict__ e, int64_t len,
                              double* __restrict__ out, const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = s[i] + e[i];
}

// Row-local panel update.  mode: 0 A_T = [A_V] (t = B), 1 [A_V A_W] (t = 2B),
// 2 [A_V A_X A_W] (t = 3B).  C_V, C_X are t x B row-major.
template <typename T>
__global__ __launch_bounds__(256) void k_panel(T* __restrict__ AV, T* __restrict__ AX, const T* __restrict__ AW,
                                               int64_t m, int B, const T* __restrict__ CVg,
                                               const T* __restrict__ CXg, const Ctl* __restrict__ ctl) {
  if (ctl->done) return;
  const int mode = ctl->rr_mode;
  const int xupd = ctl->x_update;
  const int t = (mode == 0) ? B : (mode == 1 ? 2 * B : 3 * B);
  __shared__ T CV[32 * 16];
  __shared__ T CX[32 * 16];
  for (int i = threadIdx.x; i < t * B; i += blockDim.x) {
    CV[i] = CVg[i];
    CX[i] = xupd ? CXg[i] : zero<T>();
  }
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    T at[32];
    for (int j = 0; j < B; ++j) at[j] = AV[r * B + j];
    if (mode == 2) {
      for (int j = 0; j < B; ++j) at[B + j] = AX[r * B + j];
      for (int j = 0; j < B; ++j) at[2 * B + j] = AW[r * B + j];
    } else if (mode == 1) {
      for (int j = 0; j < B; ++j) at[B + j] = AW[r * B + j];
    }
    for (int j = 0; j < B; ++j) {
      T sv = zero<T>(), sx = zero<T>();
      for (int c = 0; c < t; ++c) {
        sv = fmac(at[c], CV[c * B + j], sv);
        sx = fmac(at[c], CX[c * B + j], sx);
      }
      AV[r * B + j] = sv;
      if (xupd) AX[r * B + j] = sx;
    }
  }
}

// U(:, j) = (A_T C_V)(:, B-1-j) / theta_{B-1-j} for j < k (ascending order).
template <typename T>
__global__ __launch_bounds__(256) void k_final_u(const T* __restrict__ AV, const T* __restrict__ AX,
                                                 const T* __restrict__ AW, int64_t m, int B, int k,
                                                 const T* __restrict__ CVg, const double* __restrict__ thb,
                                                 T* __restrict__ U, int64_t ldu, const Ctl* __restrict__ ctl) {
  const int mode = ctl->rr_mode;
  const int t = (mode == 0) ? B : (mode == 1 ? 2 * B : 3 * B);
  __shared__ T CV[32 * 16];
  __shared__ double inv[16];
  for (int i = threadIdx.x; i < t * B; i += blockDim.x) CV[i] = CVg[i];
  if (threadIdx.x < B) inv[threadIdx.x] = (thb[threadIdx.x] != 0.0) ? 1.0 / thb[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    T at[32];
    for (int j = 0; j < B; ++j) at[j] = AV[r * B + j];
    if (mode == 2) {
      for (int j = 0; j < B; ++j) at[B + j] = AX[r * B + j];
      for (int j = 0; j < B; ++j) at[2 * B + j] = AW[r * B + j];
    } else if (mode == 1) {
      for (int j = 0; j < B; ++j) at[B + j] = AW[r * B + j];
    }
    for (int jo = 0; jo < k; ++jo) {
      const int j = B - 1 - jo;
      T s = zero<T>();
      for (int c = 0; c < t; ++c) s = fmac(at[c], CV[c * B + j], s);
      U[r * ldu + jo] = scal(s, inv[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Blocks: about 1024, fewer when the per-wave partial planes (4 n B values per
// wave) would exceed about 2% of the bytes of A.
int64_t astream_blocks(int64_t m, int n, int B, int es_d) {
  int64_t nb = (m + 255) / 256;
  if (nb > 1024) nb = 1024;
  const double abytes = (double)m * n * es_d * 8.0;
  const double per_block = 4.0 * 4.0 * n * B * es_d * 8.0;
  int64_t cap = (int64_t)(0.02 * abytes / per_block);
  if (cap < 64) cap = 64;
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : nb;
}

int astream_ns(int n) {
  if (n <= 256) return 4;
  if (n <= 512) return 8;
  if (n <= 1024) return 16;
  return 0;
}

int64_t astream_part_doubles(int64_t m, int n, int B, int es_d) {
  return astream_blocks(m, n, B, es_d) * 4 * 4 * (int64_t)n * B * es_d;
}

int64_t astream_tmp_doubles(int64_t m, int n, int B, int es_d) {
  const int64_t parts = astream_blocks(m, n, B, es_d) * 4;
  const int64_t groups = (parts + 63) / 64;
  return 4 * groups * 3 * (int64_t)n * B * es_d;
}

template <typename T, int B, int NS, bool DOT2>
static void launch_as(hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n, const void* W,
                      void* AW, const void* AVp, const void* AXp, int init, void* Gpart, const Ctl* ctl) {
  const int64_t rows = (m + nb - 1) / nb;
  hipLaunchKernelGGL((k_astream<T, B, NS, DOT2>), dim3((unsigned)nb), dim3(256), 0, st, (const T*)A, lda, m, n,
                     (const T*)W, (T*)AW, (const T*)AVp, (const T*)AXp, init, (T*)Gpart, rows, ctl);
}

template <typename T, int NS, bool DOT2>
static bool dispatch_b(int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n,
                       const void* W, void* AW, const void* AVp, const void* AXp, int init, void* Gpart,
                       const Ctl* ctl) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: launch_as<T, BB, NS, DOT2>(st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl); return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

template <typename T, bool DOT2>
static bool dispatch_ns(int ns, int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m, int n,
                        const void* W, void* AW, const void* AVp, const void* AXp, int init, void* Gpart,
                        const Ctl* ctl) {
  switch (ns) {
    case 4: return dispatch_b<T, 4, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    case 8: return dispatch_b<T, 8, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    case 16: return dispatch_b<T, 16, DOT2>(B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
    default: return false;
  }
}

// One pass: AW = A W and G3 = A^* [AVp AXp AW] (n x 3B, contiguous; init: G3[:, 0:B] = A^* AW).
hipError_t launch_astream(hipStream_t st, bool cplx, int B, bool dot2, const void* A, int64_t lda, int64_t m, int n,
                          const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                          double* tmp, double* G3, const Ctl* ctl) {
  const int es_d = cplx ? 2 : 1;
  const int ns = astream_ns(n);
  const int64_t nb = astream_blocks(m, n, B, es_d);
  bool ok;
  if (cplx && dot2)
    ok = dispatch_ns<cd, true>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  else if (cplx)
    ok = dispatch_ns<cd, false>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  else if (dot2)
    ok = dispatch_ns<double, true>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  else
    ok = dispatch_ns<double, false>(ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  if (!ok) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // compensated reduction of the per-wave partials
  const int64_t plen = (int64_t)n * B * es_d;
  const int64_t len = 3 * plen;
  int64_t np = nb * 4;
  const int64_t g1 = (np + 63) / 64;
  const double* cur_s = Gpart;
  const double* cur_e = Gpart + len;
  int64_t stride = 4 * plen, elen = plen;
  int flip = 0;
  while (true) {
    const int64_t groups = (np + 63) / 64;
    double* ds = tmp + (int64_t)flip * 2 * g1 * len;
    double* de = ds + g1 * len;
    hipLaunchKernelGGL(k_colsum2, dim3((unsigned)((len + 63) / 64), (unsigned)groups), dim3(256), 0, st, cur_s,
                       cur_e, stride, elen, np, len, ds, de, ctl);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (groups == 1) {
      hipLaunchKernelGGL(k_pair_finish, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, ds, de, len, G3, ctl);
      return hipGetLastError();
    }
    cur_s = ds;
    cur_e = de;
    stride = len;
    elen = len;
    np = groups;
    flip ^= 1;
  }
}

hipError_t launch_panel(hipStream_t st, bool cplx, void* AV, void* AX, const void* AW, int64_t m, int B,
                        const void* CV, const void* CX, const Ctl* ctl) {
  int64_t nb = (m + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (cplx)
    hipLaunchKernelGGL(k_panel<cd>, dim3((unsigned)nb), dim3(256), 0, st, (cd*)AV, (cd*)AX, (const cd*)AW, m, B,
                       (const cd*)CV, (const cd*)CX, ctl);
  else
    hipLaunchKernelGGL(k_panel<double>, dim3((unsigned)nb), dim3(256), 0, st, (double*)AV, (double*)AX,
                       (const double*)AW, m, B, (const double*)CV, (const double*)CX, ctl);
  return hipGetLastError();
}

hipError_t launch_final_u(hipStream_t st, bool cplx, const void* AV, const void* AX, const void* AW, int64_t m,
                          int B, int k, const void* CV, const double* thb, void* U, int64_t ldu, const Ctl* ctl) {
  int64_t nb = (m + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (cplx)
    hipLaunchKernelGGL(k_final_u<cd>, dim3((unsigned)nb), dim3(256), 0, st, (const cd*)AV, (const cd*)AX,
                       (const cd*)AW, m, B, k, (const cd*)CV, thb, (cd*)U, ldu, ctl);
  else
    hipLaunchKernelGGL(k_final_u<double>, dim3((unsigned)nb), dim3(256), 0, st, (const double*)AV,
                       (const double*)AX, (const double*)AW, m, B, k, (const double*)CV, thb, (double*)U, ldu, ctl);
  return hipGetLastError();
}

}  // namespace rl
