// n-side steps of RLOBPCG: everything whose size is n x (a few b), run by one
// or a few workgroups (latency-bound, not bandwidth-bound).
//
// k_trmv     Y = M X with M an n x n triangular matrix (row-major, upper or
//            lower) and X an n x B block; the preconditioner application
//            W = P (P^* R) of eq:search-direction is two of these with
//            P = R^{-1} (upper) and P^* = R^{-*} (lower).
// k_orth     BCGS2 of W against [V X] (two classical Gram-Schmidt passes,
//            Alg. rlobpcg) followed by Orth(W) as column-wise CGS2 (b = 1:
//            Normalize, Alg. rlopcg).
// k_orth_svqb the same two block projections, then Orth(W) by SVQB (the
//            faster, less stable choice the paper names for this step).
// k_rr       Rayleigh-Ritz from R_T (the TSQR factor of A_T): one-sided Jacobi
//            SVD of R_T gives Theta and C (descending, as MATLAB's svd); then
//            V = T C(:, t-b+1:t), the residual R = G_T C(:, t-b+1:t) - V Theta_b^2
//            with G_T = A^* [A_V A_X A_W] from the same iteration's A-stream
//            pass (= A^* A_V(new) - V Theta^2), its column norms, the stopping
//            rule (eq:est_conv_criterion and eq:stagnation-check), and
//            Q = Orth(C(1:b, 1:t-b)^*), X = T C(:, 1:t-b) Q (eq:x-defining).
// k_lanczos  Sigma~(1,1) = ||R||_2 by Golub-Kahan-Lanczos bidiagonalisation
//            with full reorthogonalisation and a Sturm-bisection of B^T B.
// k_randblk  deterministic start block for inverse subspace iteration.
// k_final_n  sigma (ascending) and V outputs.
#include "common.hpp"
#include "kernels.hpp"
#include "orth.hpp"

#include <type_traits>

namespace rl {

constexpr int RR_TMAX = 32;
constexpr int RR_BMAX = 16;
static_assert(RR_CST_DOUBLES >= RR_TMAX * 32 * 2 + 2 * RR_TMAX, "saved Rayleigh-Ritz data of k_rr's phases");
constexpr int RR_PRE_B = 4;  // k_rr loads a trial row's 3B values together up to this B

__device__ inline double absval(double a) { return fabs(a); }
__device__ inline double absval(cd a) { return hypot(a.x, a.y); }

// ---------------------------------------------------------------------------
template <typename T, int B>
__global__ __launch_bounds__(NS_THREADS) void k_trmv(const T* __restrict__ M, int n, int lower,
                                                     const T* __restrict__ X, T* __restrict__ Y,
                                                     const Ctl* __restrict__ ctl, int check_done) {
  if (check_done && ctl->done) return;
  __shared__ T xs[256 * B];
  const int ri = threadIdx.x >> 4, kk = threadIdx.x & 15;
  const int i = blockIdx.x * 16 + ri;
  const int ib0 = blockIdx.x * 16;
  const int ib1 = (ib0 + 16 < n) ? ib0 + 16 : n;
  const int lstart = lower ? 0 : ib0;
  const int lend = lower ? ib1 : n;
  T acc[B];
#pragma unroll
  for (int j = 0; j < B; ++j) acc[j] = zero<T>();
  for (int l0 = lstart; l0 < lend; l0 += 256) {
    const int cnt = (lend - l0 < 256) ? lend - l0 : 256;
    __syncthreads();
    // the chunk of X, zero past its end (the products there are zero)
    for (int e = threadIdx.x; e < 256 * B; e += blockDim.x) xs[e] = (e < cnt * B) ? X[(int64_t)l0 * B + e] : zero<T>();
    __syncthreads();
    const int lo = lower ? l0 : (i > l0 ? i : l0);
    const int hi = (i >= n) ? lo : (lower ? ((i + 1 < l0 + cnt) ? i + 1 : l0 + cnt) : l0 + cnt);
    // a thread's 16 entries of the chunk are loaded together (one memory
    // latency per chunk instead of one per entry); entries outside the
    // triangle are zeros
    T mv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int l = l0 + kk + 16 * u;
      mv[u] = (l >= lo && l < hi) ? M[(int64_t)i * n + l] : zero<T>();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
#pragma unroll
      for (int j = 0; j < B; ++j) acc[j] = fmac(mv[u], xs[(kk + 16 * u) * B + j], acc[j]);
    }
  }
  // the 16 threads of a row are one DPP row of the wave
#pragma unroll
  for (int j = 0; j < B; ++j) acc[j] = row_sum16(acc[j]);
  if (kk == 0 && i < n) {
#pragma unroll
    for (int j = 0; j < B; ++j) Y[(int64_t)i * B + j] = acc[j];
  }
}

template <typename T, int KM>
__global__ __launch_bounds__(NS_THREADS) void k_orth(int n, int B, const T* __restrict__ V, const T* __restrict__ X,
                                                     int project, int with_x, T* __restrict__ W, Ctl* __restrict__ ctl,
                                                     int check_done, int masked) {
  if (check_done && ctl->done) return;
  orth_block<T, KM>(n, B, V, X, project, with_x, W, ctl, (masked && ctl->lock) ? ctl->act : -1);
}

template <typename T>
__device__ void jacobi_block(T* M, T* Vj, int t);

// W <- Orth(W - [V X]([V X]^* W)) with the two block projections of BCGS2
// and SVQB (Stathopoulos and Wu) for Orth: G = W^* W, D = diag(G)^{-1/2},
// D G D = Z Lambda Z^* by one-sided Jacobi on D G D (Hermitian positive
// semidefinite, so its singular vectors are its eigenvectors and the column
// norms after the rotations its eigenvalues), eigenvalues below
// eps * max raised to it, W <- W D Z Lambda^{-1/2}.  A column that vanishes
// after the projections (zero diagonal of G) hands the block to orth_block.
template <typename T, int KM>
__global__ __launch_bounds__(NS_THREADS) void k_orth_svqb(int n, int B, const T* __restrict__ V,
                                                          const T* __restrict__ X, int project, int with_x,
                                                          T* __restrict__ W, Ctl* __restrict__ ctl, int check_done) {
  if (check_done && ctl->done) return;
  __shared__ T scratch[(NS_THREADS / 16) * ORTH_KC];
  __shared__ T h[KM];
  __shared__ T M[RR_TMAX * 32];   // D G D, rotated in place (column-major, ld 32)
  __shared__ T Vj[RR_TMAX * 32];  // Z
  __shared__ T Gs[RR_BMAX * RR_BMAX];
  __shared__ T Fm[RR_BMAX * RR_BMAX];  // D Z Lambda^{-1/2}, row-major B x B
  __shared__ double dsc[RR_BMAX], lam[RR_BMAX];
  __shared__ int fallback;
  const int tid = threadIdx.x;
  const int nvx = project ? (with_x ? 2 * B : B) : 0;
  if (nvx > 0) {
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < B; ++j) orth_project<T, KM>(n, B, j, V, X, nvx, W, scratch, h, 0);
  }
  // Gram matrix G(p, q) = W(:, p)^* W(:, q), in chunks of ORTH_KC entries
  const int npair = B * B;
  for (int e0 = 0; e0 < npair; e0 += ORTH_KC) {
    T vals[ORTH_KC];
#pragma unroll
    for (int kk = 0; kk < ORTH_KC; ++kk) vals[kk] = zero<T>();
    for (int r = tid; r < n; r += blockDim.x) {
#pragma unroll
      for (int kk = 0; kk < ORTH_KC; ++kk) {
        const int e = e0 + kk;
        if (e < npair) vals[kk] = cfmac(W[(int64_t)r * B + e / B], W[(int64_t)r * B + e % B], vals[kk]);
      }
    }
    block_sum_many<T, ORTH_KC>(vals, (npair - e0 < ORTH_KC) ? npair - e0 : ORTH_KC, scratch, Gs + e0);
  }
  if (tid == 0) {
    fallback = 0;
    for (int p = 0; p < B; ++p) {
      const double g = re_(Gs[p * B + p]);
      if (!(g > 0.0) || !isfinite(g)) fallback = 1;
      dsc[p] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
    }
  }
  __syncthreads();
  if (fallback) {
    if (tid == 0) ctl->degenerate = 1;
    orth_block<T, KM>(n, B, V, X, project, with_x, W, ctl);
    return;
  }
  for (int e = tid; e < RR_TMAX * 32; e += blockDim.x) {
    const int c = e / 32, r = e % 32;
    M[e] = (r < B && c < B) ? scal(Gs[r * B + c], dsc[r] * dsc[c]) : zero<T>();
    Vj[e] = from_real<T>((r == c) ? 1.0 : 0.0);
  }
  __syncthreads();
  jacobi_block<T>(M, Vj, B);
  if (tid < 64) {
    const int lane = tid;
    double lmax = 0.0;
    for (int c = 0; c < B; ++c) {
      const T v = (lane < B) ? M[c * 32 + lane] : zero<T>();
      const double l = sqrt(wave_sum(abs2(v)));
      if (lane == 0) lam[c] = l;
      lmax = fmax(lmax, l);
    }
    if (lane == 0)
      for (int c = 0; c < B; ++c) lam[c] = fmax(lam[c], 2.220446049250313e-16 * lmax);
  }
  __syncthreads();
  for (int e = tid; e < B * B; e += blockDim.x) {
    const int p = e / B, q = e % B;
    Fm[e] = scal(Vj[q * 32 + p], dsc[p] / sqrt(lam[q]));
  }
  __syncthreads();
  for (int r = tid; r < n; r += blockDim.x) {
    T wr[RR_BMAX];
    for (int p = 0; p < B; ++p) wr[p] = W[(int64_t)r * B + p];
    for (int q = 0; q < B; ++q) {
      T acc = zero<T>();
      for (int p = 0; p < B; ++p) acc = fmac(wr[p], Fm[p * B + q], acc);
      W[(int64_t)r * B + q] = acc;
    }
  }
}


// ---------------------------------------------------------------------------
__device__ bool dev_should_stop(int i, const double* __restrict__ ht, const double* __restrict__ hr, int B,
                                const Ctl* __restrict__ c) {
  if (c->stop_rule == 2) return false;
  double rmax = 0.0;
  bool nan = false;
  for (int j = 0; j < B; ++j) {
    const double v = hr[(int64_t)(i + 1) * B + j];
    if (!(v == v)) nan = true;
    rmax = fmax(rmax, v);
  }
  const bool tol = !nan && (rmax <= c->sigma1 * c->sigma1 * c->tau);
  if (c->stop_rule == 1) return tol;
  if (i % c->check_every != 0) return false;
  if (!tol) return false;
  const int jn = i + 1, jm = i + 1 - 5, jo = i + 1 - 10;
  if (jm < 0 || jo < 0) return false;
  for (int j = 0; j < B; ++j) {
    const double rn = hr[(int64_t)jn * B + j], rm = hr[(int64_t)jm * B + j];
    if (!(1.1 * rn >= rm)) return false;
    const double tn = ht[(int64_t)jn * B + j], tm = ht[(int64_t)jm * B + j], to = ht[(int64_t)jo * B + j];
    if (tn == 0.0) continue;
    const double lhs = 1.1 * (tm - tn) / tn;
    const double rhs = (tm == 0.0) ? INFINITY : (to - tm) / tm;
    if (!(lhs >= rhs)) return false;
  }
  return true;
}

// One-sided (Hestenes) Jacobi on the t x t matrix M (column-major, ld 32) by a
// workgroup of 256 threads, in parallel (round-robin) order: the columns,
// padded to an even count tp, meet in tp - 1 rounds of tp/2 disjoint pairs
// per sweep, and the 16 lanes of one DPP row take one pair (lane i holds rows
// i and i + 16), so a round is three 16-lane sums and one rotation per pair
// with one barrier.  Vj accumulates the rotations.  Same rotation formulas as
// the cyclic order; the test |gamma|^2 > tol^2 alpha beta is the usual
// |gamma| > tol sqrt(alpha beta) without its square roots, and 1/|gamma| is
// formed once; the sweep stops when no pair was rotated.
template <typename T>
__device__ void jacobi_block(T* M, T* Vj, int t) {
  const double tol = sqrt((double)t) * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  const int grp = threadIdx.x >> 4, li = threadIdx.x & 15;
  const int tp = t + (t & 1);
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < tp - 1; ++r) {
      if (grp < tp / 2) {
        int a, b;
        if (grp == 0) {
          a = r;
          b = tp - 1;
        } else {
          a = (r + grp) % (tp - 1);
          b = (r - grp + tp - 1) % (tp - 1);
        }
        const int p = a < b ? a : b, q = a < b ? b : a;
        if (q < t) {
          const bool r0 = li < t, r1 = li + 16 < t;
          const T mp0 = r0 ? M[p * 32 + li] : zero<T>(), mp1 = r1 ? M[p * 32 + li + 16] : zero<T>();
          const T mq0 = r0 ? M[q * 32 + li] : zero<T>(), mq1 = r1 ? M[q * 32 + li + 16] : zero<T>();
          const double al = row_sum16(abs2(mp0) + abs2(mp1));
          const double be = row_sum16(abs2(mq0) + abs2(mq1));
          const T ga = row_sum16(cfmac(mp1, mq1, cfmac(mp0, mq0, zero<T>())));
          const double g2 = abs2(ga);
          if (g2 > tol2 * al * be && g2 != 0.0) {
            rotated = 1;
            const double ig = 1.0 / sqrt(g2);
            const T eg = scal(ga, ig);  // unit phase of gamma
            const double zeta = (be - al) * 0.5 * ig;
            const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + tn * tn), s = c * tn;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int row = li + 16 * h;
              if (row < t) {
                const T mp = h ? mp1 : mp0;
                const T mq2 = mul(conj_(eg), h ? mq1 : mq0);
                M[p * 32 + row] = sub(scal(mp, c), scal(mq2, s));
                M[q * 32 + row] = add(scal(mp, s), scal(mq2, c));
                const T vp = Vj[p * 32 + row];
                const T vq2 = mul(conj_(eg), Vj[q * 32 + row]);
                Vj[p * 32 + row] = sub(scal(vp, c), scal(vq2, s));
                Vj[q * 32 + row] = add(scal(vp, s), scal(vq2, c));
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
}

template <typename T, int B>
__global__ __launch_bounds__(NS_THREADS) void k_rr(int n, int init_mode, int with_x, const T* __restrict__ Rt,
                                                   T* __restrict__ V, T* __restrict__ X, const T* __restrict__ W,
                                                   const T* __restrict__ G3, T* __restrict__ Vn,
                                                   T* __restrict__ Rres, T* __restrict__ CVout, T* __restrict__ CXout,
                                                   double* __restrict__ thb, double* __restrict__ hist_theta,
                                                   double* __restrict__ hist_rnorm, Ctl* __restrict__ ctl, int phase,
                                                   double* __restrict__ Cst) {
  if (ctl->done) return;
  __shared__ T M[RR_TMAX * 32];
  __shared__ T Vj[RR_TMAX * 32];
  __shared__ T C[RR_TMAX * 32];       // sorted right singular vectors, column-major ld 32
  __shared__ T CV[RR_TMAX * RR_BMAX];  // t x B row-major
  __shared__ T CX[RR_TMAX * RR_BMAX];
  __shared__ T Qm[RR_TMAX * RR_BMAX];  // (t-B) x B row-major
  __shared__ double th[RR_TMAX];
  __shared__ double sig[RR_TMAX];
  __shared__ double rn[RR_BMAX];
  __shared__ T scratch[(NS_THREADS / 16) * RR_BMAX];
  __shared__ T hsum[RR_BMAX];
  __shared__ int stop_s;
  __shared__ int newact_s;
  __shared__ int padsorted[RR_TMAX];  // sorted column c is a locked index's zero column
  __shared__ int rank_s[RR_TMAX];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int mode = init_mode ? 0 : (with_x ? 2 : 1);
  const int t = (mode == 0) ? B : (mode == 1 ? 2 * B : 3 * B);
  const int iter = ctl->iter;
  // Locking (Sec. 2.3): the X and W columns of locked indices are zero, so
  // their columns of R_T are zero, the Jacobi sweeps never rotate them and
  // they come out as unit singular vectors of value 0.  They rank above every
  // real Ritz value here, so they are never selected and never enter X.
  const int lockon = ctl->lock;
  const int act0 = lockon ? ctl->act : (1 << B) - 1;
  auto padded = [&](int c) { return lockon && c >= B && !((act0 >> ((c - B) % B)) & 1); };
  // phase 0: the whole step; 1: the Rayleigh-Ritz and V_new only, with C,
  // Theta and the padding flags saved to Cst; 2: the rest from Cst, the
  // residual from G3's first block = A^* A_{V_new} (the late-residual form)
  T* Cs = reinterpret_cast<T*>(Cst);
  double* ths = Cst + RR_TMAX * 32 * (sizeof(T) / sizeof(double));
  double* pads = ths + RR_TMAX;
  if (phase == 2) {
    for (int e = tid; e < RR_TMAX * 32; e += blockDim.x) C[e] = Cs[e];
    for (int c = tid; c < RR_TMAX; c += blockDim.x) {
      th[c] = ths[c];
      padsorted[c] = pads[c] != 0.0 ? 1 : 0;
    }
    __syncthreads();
  } else {
  for (int e = tid; e < RR_TMAX * 32; e += blockDim.x) {
    const int c = e / 32, r = e % 32;
    M[e] = (r < t && c < t) ? Rt[r * t + c] : zero<T>();
    Vj[e] = from_real<T>((r == c) ? 1.0 : 0.0);
  }
  __syncthreads();
  jacobi_block<T>(M, Vj, t);
  // column norms (thread c), then the descending order: column c goes to
  // the number of columns ranked before it (larger key, or an equal key and
  // a lower index: the order a stable selection sort gives)
  if (tid < t) {
    double s2 = 0.0;
    for (int r = 0; r < t; ++r) s2 += abs2(M[tid * 32 + r]);
    sig[tid] = sqrt(s2);
  }
  __syncthreads();
  if (tid < t) {
    const double kc = padded(tid) ? INFINITY : sig[tid];
    int rk = 0;
    for (int q = 0; q < t; ++q) {
      const double kq = padded(q) ? INFINITY : sig[q];
      rk += (kq > kc || (kq == kc && q < tid)) ? 1 : 0;
    }
    rank_s[tid] = rk;
    th[rk] = sig[tid];
    padsorted[rk] = padded(tid) ? 1 : 0;
  }
  __syncthreads();
  for (int e = tid; e < t * 32; e += blockDim.x) {
    const int c = e / 32, r = e % 32;
    if (r < t) C[rank_s[c] * 32 + r] = Vj[c * 32 + r];
  }
  __syncthreads();
  }
  for (int e = tid; e < t * B; e += blockDim.x) {
    const int r = e / B, j = e % B;
    CV[e] = C[(t - B + j) * 32 + r];
  }
  if (tid < B && phase != 2) thb[tid] = th[t - B + tid];
  if (phase == 1) {
    // C is complete only in the rows and columns below t; the rest is unused
    for (int e = tid; e < RR_TMAX * 32; e += blockDim.x) Cs[e] = C[e];
    for (int c = tid; c < RR_TMAX; c += blockDim.x) {
      ths[c] = c < t ? th[c] : 0.0;
      pads[c] = (c < t && padsorted[c]) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  if (phase == 1) {
    // V_new = T C_V into Vn (V, X, W stay as they are for phase 2's X)
    const T* T1 = (mode == 2) ? X : W;
    for (int r = tid; r < n; r += blockDim.x) {
      T v[B];
#pragma unroll
      for (int j = 0; j < B; ++j) v[j] = zero<T>();
      // a block's B row values are loaded together, then consumed one at a
      // time from the front of the (rotated) register array, so only one
      // coefficient row is live at once
      for (int blk = 0; blk * B < t; ++blk) {
        const T* P = (blk == 0) ? V : ((blk == 1) ? T1 : W);
        T tr[B];
#pragma unroll
        for (int jc = 0; jc < B; ++jc) tr[jc] = P[(int64_t)r * B + jc];
#pragma unroll 1
        for (int jc = 0; jc < B; ++jc) {
          const T a = tr[0];
#pragma unroll
          for (int q = 0; q + 1 < B; ++q) tr[q] = tr[q + 1];
#pragma unroll
          for (int j = 0; j < B; ++j) v[j] = fmac(a, CV[(blk * B + jc) * B + j], v[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < B; ++j) Vn[(int64_t)r * B + j] = v[j];
    }
    for (int e = tid; e < t * B; e += blockDim.x) CVout[e] = CV[e];
    if (tid == 0) ctl->rr_mode = mode;
    return;
  }
  // pass 1: V_new = T C_V and the residual G_T C_V - V_new Theta_b^2, with its column norms
  {
    const T* GV = G3;
    const T* GX = G3 + (int64_t)n * B;
    const T* GW = G3 + 2 * (int64_t)n * B;
    const T* T1 = (mode == 2) ? X : W;  // second block of the trial space
    const T* G1 = (mode == 2) ? GX : GW;
    T vals[RR_BMAX];
#pragma unroll
    for (int j = 0; j < RR_BMAX; ++j) vals[j] = zero<T>();
    // phase 2: V_new is in Vn and the first block of G3 is A^* A_{V_new}
    for (int r = tid; phase == 2 && r < n; r += blockDim.x) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const double th2 = th[t - B + j] * th[t - B + j];
        const int64_t e = (int64_t)r * B + j;
        const T res = sub(GV[e], scal(Vn[e], th2));
        Rres[e] = res;
        vals[j] = add(vals[j], from_real<T>(abs2(res)));
      }
    }
    for (int r = tid; phase != 2 && r < n; r += blockDim.x) {
      // [V X W](r, :) C_V and G_T(r, :) C_V, one trial-space column at a time
      T v[B], g[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        v[j] = zero<T>();
        g[j] = zero<T>();
      }
      if constexpr (B <= RR_PRE_B) {
        // the row's 3B trial values and their G_T rows are loaded together
        // (every block is a valid n x B array; blocks past t are not used)
        T trv[3 * B], grv[3 * B];
#pragma unroll
        for (int c = 0; c < 3 * B; ++c) {
          const int64_t e = (int64_t)r * B + (c % B);
          trv[c] = (c < B) ? V[e] : ((c < 2 * B) ? T1[e] : W[e]);
          grv[c] = (c < B) ? GV[e] : ((c < 2 * B) ? G1[e] : GW[e]);
        }
#pragma unroll
        for (int c = 0; c < 3 * B; ++c) {
          if (c < t) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
              v[j] = fmac(trv[c], CV[c * B + j], v[j]);
              g[j] = fmac(grv[c], CV[c * B + j], g[j]);
            }
          }
        }
      } else {
        // a block's B row values (and their G_T rows) are loaded together and
        // consumed from the front of the rotated register arrays
        for (int blk = 0; blk * B < t; ++blk) {
          const T* P = (blk == 0) ? V : ((blk == 1) ? T1 : W);
          const T* Gb = (blk == 0) ? GV : ((blk == 1) ? G1 : GW);
          T tr[B], gr[B];
#pragma unroll
          for (int jc = 0; jc < B; ++jc) {
            tr[jc] = P[(int64_t)r * B + jc];
            gr[jc] = Gb[(int64_t)r * B + jc];
          }
#pragma unroll 1
          for (int jc = 0; jc < B; ++jc) {
            const T a = tr[0], ga = gr[0];
#pragma unroll
            for (int q = 0; q + 1 < B; ++q) {
              tr[q] = tr[q + 1];
              gr[q] = gr[q + 1];
            }
#pragma unroll
            for (int j = 0; j < B; ++j) {
              v[j] = fmac(a, CV[(blk * B + jc) * B + j], v[j]);
              g[j] = fmac(ga, CV[(blk * B + jc) * B + j], g[j]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const double th2 = th[t - B + j] * th[t - B + j];
        const T res = sub(g[j], scal(v[j], th2));
        Vn[(int64_t)r * B + j] = v[j];
        Rres[(int64_t)r * B + j] = res;
        vals[j] = add(vals[j], from_real<T>(abs2(res)));
      }
    }
    block_sum_many<T, RR_BMAX>(vals, B, scratch, hsum);
    if (tid < B) rn[tid] = sqrt(re_(hsum[tid]));
    __syncthreads();
  }
  if (tid == 0) {
    const int idx = init_mode ? 0 : iter + 1;
    for (int j = 0; j < B; ++j) {
      hist_theta[(int64_t)idx * B + j] = (init_mode && B == 1) ? INFINITY : th[t - B + j];
      hist_rnorm[(int64_t)idx * B + j] = rn[j];
    }
    __threadfence_block();
    stop_s = init_mode ? 0 : (dev_should_stop(iter, hist_theta, hist_rnorm, B, ctl) ? 1 : 0);
    // the lock update: a column whose residual meets Sigma~(1,1)^2 tau is
    // locked for good (after the rule's check, as the oracle orders them)
    int na = act0;
    if (lockon && !stop_s) {
      const double thr = ctl->sigma1 * ctl->sigma1 * ctl->tau;
      for (int j = 0; j < B; ++j)
        if (rn[j] <= thr) na &= ~(1 << j);
    }
    newact_s = na;
  }
  __syncthreads();
  const int newact = newact_s;
  const bool all_locked = lockon && newact == 0;
  const bool xupd = !init_mode && !stop_s && !all_locked;
  if (xupd && wid == 0) {
    // Q = Orth(C(1:B, 1:t-B)^*), (t-B) x B, by modified Gram-Schmidt applied
    // twice, row a of Q held by lane a.  A column that vanishes (at full
    // convergence C(1:B, 1:t-B) can be exactly 0) is completed, as Householder
    // QR would, by the first unit vector that keeps norm above 1/2 after
    // projection on the earlier ones.
    // With locking only the active rows of C enter (X gets one column per
    // active index; the others are zero).
    const int tb = t - B;
    const int a = lane;
    const bool own = a < tb;
    for (int j = 0; j < B; ++j)
      if (own) Qm[a * B + j] = ((newact >> j) & 1) ? conj_(C[a * 32 + j]) : zero<T>();
    for (int j = 0; j < B; ++j) {
      if (!((newact >> j) & 1)) continue;
      double nrm = 0.0;
      for (int cand = -1; cand < tb; ++cand) {
        if (cand >= 0 && padsorted[cand]) continue;  // a zero column of T
        if (cand >= 0 && own) Qm[a * B + j] = from_real<T>(a == cand ? 1.0 : 0.0);
        for (int pass = 0; pass < 2; ++pass) {
          for (int q = 0; q < j; ++q) {
            const T sp = wave_sum(own ? cfmac(Qm[a * B + q], Qm[a * B + j], zero<T>()) : zero<T>());
            if (own) Qm[a * B + j] = fnmac(Qm[a * B + q], sp, Qm[a * B + j]);
          }
        }
        nrm = sqrt(wave_sum(own ? abs2(Qm[a * B + j]) : 0.0));
        if (cand < 0 && nrm > 0.0 && isfinite(nrm)) break;
        if (cand >= 0 && nrm > 0.5) break;
        if (cand < 0 && lane == 0) ctl->degenerate = 1;
      }
      if (own) Qm[a * B + j] = scal(Qm[a * B + j], 1.0 / nrm);
    }
  }
  __syncthreads();
  if (xupd) {
    // C_X = C(:, 1:t-B) Q  (t x B), one entry per thread
    const int tb = t - B;
    for (int e = tid; e < t * B; e += blockDim.x) {
      const int c = e / B, j = e - (e / B) * B;
      T sx = zero<T>();
      for (int a = 0; a < tb; ++a) sx = fmac(C[a * 32 + c], Qm[a * B + j], sx);
      CX[e] = sx;
    }
  }
  __syncthreads();
  // pass 2: X = T C_X from the old T, then V <- V_new
  for (int r = tid; r < n; r += blockDim.x) {
    if (xupd) {
      T x[B];
#pragma unroll
      for (int j = 0; j < B; ++j) x[j] = zero<T>();
      const T* T1 = (mode == 2) ? X : W;
      if constexpr (B <= RR_PRE_B) {
        T trv[3 * B];
#pragma unroll
        for (int c = 0; c < 3 * B; ++c) {
          const int64_t e = (int64_t)r * B + (c % B);
          trv[c] = (c < B) ? V[e] : ((c < 2 * B) ? T1[e] : W[e]);
        }
#pragma unroll
        for (int c = 0; c < 3 * B; ++c) {
          if (c < t) {
#pragma unroll
            for (int j = 0; j < B; ++j) x[j] = fmac(trv[c], CX[c * B + j], x[j]);
          }
        }
      } else {
        for (int blk = 0; blk * B < t; ++blk) {
          const T* P = (blk == 0) ? V : ((blk == 1) ? T1 : W);
          T tr[B];
#pragma unroll
          for (int jc = 0; jc < B; ++jc) tr[jc] = P[(int64_t)r * B + jc];
#pragma unroll 1
          for (int jc = 0; jc < B; ++jc) {
            const T a = tr[0];
#pragma unroll
            for (int q = 0; q + 1 < B; ++q) tr[q] = tr[q + 1];
#pragma unroll
            for (int j = 0; j < B; ++j) x[j] = fmac(a, CX[(blk * B + jc) * B + j], x[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < B; ++j) X[(int64_t)r * B + j] = x[j];
    }
    for (int j = 0; j < B; ++j) V[(int64_t)r * B + j] = Vn[(int64_t)r * B + j];
  }
  for (int e = tid; e < t * B; e += blockDim.x) {
    CVout[e] = CV[e];
    CXout[e] = xupd ? CX[e] : zero<T>();
  }
  __syncthreads();
  if (tid == 0) {
    ctl->rr_mode = mode;
    ctl->x_update = xupd ? 1 : 0;
    if (lockon) ctl->act = newact;
    if (!init_mode) {
      ctl->iter = iter + 1;
      if (stop_s || all_locked) {
        ctl->done = 1;
        ctl->status = 0;
      } else {
        ctl->has_x = 1;
        if (iter + 1 >= ctl->max_iter) ctl->status = 1;
      }
    } else if (all_locked) {  // every column met the tolerance at the start
      ctl->done = 1;
      ctl->status = 0;
    }
  }
}

// ---------------------------------------------------------------------------
__device__ inline uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double unif_pm1(uint64_t h) { return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0; }

template <typename T>
__global__ void k_randblk(T* __restrict__ Wb, int64_t count, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  T v;
  if constexpr (sizeof(T) == sizeof(double)) {
    v = from_real<T>(unif_pm1(mix64(seed ^ (uint64_t)(2 * i))));
  } else {
    cd c{unif_pm1(mix64(seed ^ (uint64_t)(2 * i))), unif_pm1(mix64(seed ^ (uint64_t)(2 * i + 1)))};
    v = *reinterpret_cast<T*>(&c);
  }
  Wb[i] = v;
}

// Golub-Kahan-Lanczos on R (upper triangular, R(i,l) = Ycol[l*ld + i] = Rrow[i*n + l]).
// One workgroup of 1024 threads (16 waves); thread t keeps entry t of the
// current u and v in registers (n <= 1024).  R v and R^* u are computed one
// row (one column) of R per wave at a time, lanes running along the row
// (column) so loads are coalesced; the operand vector is broadcast from LDS.
// Both new vectors are reorthogonalised twice against all earlier ones.
// The largest eigenvalue of B^T B (B the bidiagonal) is found by multisection
// of its Sturm count over the 64 lanes of one wave.
constexpr int LZ_THREADS = 1024;
constexpr int LZ_WAVES = LZ_THREADS / 64;
constexpr int LZ_MAXK = 64;

// y = M x for the n x n triangular M held both ways: rows (`byrow`, row i is
// M[i*ldr + l], l in [lo(i), hi(i))) -- the caller supplies the row access.
template <typename T, bool CONJ>
__device__ inline void lz_rows(int n, const T* __restrict__ M, int64_t ld, bool upper, const T* xs, T* ys) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i0 = wid * 4; i0 < n; i0 += LZ_WAVES * 4) {
    T acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = zero<T>();
    const int lo = upper ? i0 : 0;
    const int hi = upper ? n : ((i0 + 4 < n) ? i0 + 4 : n);
    // LS 64-column slices per step: their 4 LS loads are issued together
    // (the terms are still added in column order)
    constexpr int LS = sizeof(T) == 16 ? 1 : 4;  // complex: within 128 registers
    for (int l0 = lo; l0 < hi; l0 += 64 * LS) {
      T mv[LS][4], xv[LS];
      bool ok[LS][4];
#pragma unroll
      for (int c = 0; c < LS; ++c) {
        const int l = l0 + 64 * c + lane;
        xv[c] = (l < hi) ? xs[l] : zero<T>();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r;
          ok[c][r] = l < hi && i < n && (upper ? l >= i : l <= i);
          mv[c][r] = ok[c][r] ? M[(int64_t)i * ld + l] : zero<T>();
        }
      }
#pragma unroll
      for (int c = 0; c < LS; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (ok[c][r]) acc[r] = CONJ ? cfmac(mv[c][r], xv[c], acc[r]) : fmac(mv[c][r], xv[c], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T t = wave_sum(acc[r]);
      if (lane == 0 && i0 + r < n) ys[i0 + r] = t;
    }
  }
}

// x <- x - Basis(:, 0:cnt) (Basis(:, 0:cnt)^* x), twice; the thread holds the
// entries tid + LZ_THREADS e (e < NPT) of the vector, Basis columns have
// stride n.  xs and hq are LDS work arrays (xs holds n entries).
template <typename T, int NPT>
__device__ inline void lz_reorth(int n, int cnt, const T* __restrict__ Basis, T (&x)[NPT], T* xs, T* hq) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
      const int i = threadIdx.x + LZ_THREADS * e;
      if (i < n) xs[i] = x[e];
    }
    __syncthreads();
    for (int q = wid; q < cnt; q += LZ_WAVES) {
      T acc = zero<T>();
#pragma unroll 4
      for (int l = lane; l < n; l += 64) acc = cfmac(Basis[(int64_t)q * n + l], xs[l], acc);
      acc = wave_sum(acc);
      if (lane == 0) hq[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
      const int i = threadIdx.x + LZ_THREADS * e;
      if (i < n) {
        // eight independent loads in flight per step of the loop
        T acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = zero<T>();
        int q = 0;
        for (; q + 8 <= cnt; q += 8) {
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] = fmac(Basis[(int64_t)(q + u) * n + i], hq[q + u], acc[u]);
        }
        for (; q < cnt; ++q) acc[0] = fmac(Basis[(int64_t)q * n + i], hq[q], acc[0]);
        T tot = zero<T>();
#pragma unroll
        for (int u = 0; u < 8; ++u) tot = add(tot, acc[u]);
        x[e] = sub(x[e], tot);
      }
    }
    __syncthreads();
  }
}

// Largest eigenvalue of the k x k symmetric tridiagonal (dg, of) by
// multisection of its Sturm count over the 64 lanes of the calling wave.
__device__ double tridiag_top(const double* dg, const double* of, int k);

// number of eigenvalues of the symmetric tridiagonal (dg, of) below x
__device__ inline int sturm_count(const double* dg, const double* of, int k, double x) {
  int cnt = 0;
  double q = dg[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    if (q == 0.0) q = 1e-300;
    q = (dg[i] - x) - of[i - 1] * of[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

__device__ double tridiag_top(const double* dg, const double* of, int k) {
  const int lane = threadIdx.x & 63;
  double hi = 0.0;
  for (int q = 0; q < k; ++q) {
    const double rad = fabs(of[q]) + (q > 0 ? fabs(of[q - 1]) : 0.0);
    hi = fmax(hi, dg[q] + rad);
  }
  double lo = 0.0;
  // lane l tests lo + (l+1) (hi-lo)/65; keep the sub-interval where the count
  // of eigenvalues below reaches k
  for (int it = 0; it < 12 && hi - lo > 1e-17 * hi; ++it) {
    const double w = (hi - lo) / 65.0;
    const double x = lo + (lane + 1) * w;
    const int below = sturm_count(dg, of, k, x);
    const uint64_t full = __ballot(below == k);
    const int first = full ? __builtin_ctzll(full) : 64;
    const double nlo = lo + first * w;
    const double nhi = (first < 64) ? lo + (first + 1) * w : hi;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// B^T B of the first k Lanczos steps: diagonal alpha_q^2 + beta_{q-1}^2,
// off-diagonal alpha_q beta_q.
__device__ inline void lz_tridiag(const double* alpha, const double* beta, int k, double* dg, double* of) {
  for (int q = threadIdx.x; q < k; q += blockDim.x) {
    dg[q] = alpha[q] * alpha[q] + (q > 0 ? beta[q - 1] * beta[q - 1] : 0.0);
    of[q] = (q + 1 < k) ? alpha[q] * beta[q] : 0.0;
  }
}

// NPT vector entries per thread (n <= LZ_THREADS NPT); xs and ys (n entries
// each) are dynamic LDS.
template <typename T, int NPT>
__global__ __launch_bounds__(LZ_THREADS) void k_lanczos(int n, const T* __restrict__ Ycol, int ld,
                                                        const T* __restrict__ Rrow, T* __restrict__ Ub,
                                                        T* __restrict__ Vb, int KL, uint64_t seed,
                                                        Ctl* __restrict__ ctl) {
  extern __shared__ double lz_lds[];
  T* xs = reinterpret_cast<T*>(lz_lds);
  T* ys = xs + LZ_THREADS * NPT;
  __shared__ T hq[LZ_MAXK + 1];
  __shared__ double alpha[LZ_MAXK + 1], beta[LZ_MAXK + 1];
  __shared__ double dg[LZ_MAXK + 1], of[LZ_MAXK + 1];
  __shared__ double red[LZ_WAVES];
  __shared__ double est[2];  // previous top Ritz value, converged flag
  const int tid = threadIdx.x;
  bool own[NPT];
#pragma unroll
  for (int e = 0; e < NPT; ++e) own[e] = tid + LZ_THREADS * e < n;
  if (tid == 0) {
    est[0] = -1.0;
    est[1] = 0.0;
  }
  // v_0: deterministic random unit vector
  T v[NPT], u[NPT], uprev[NPT];
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    v[e] = zero<T>();
    u[e] = zero<T>();
    uprev[e] = zero<T>();
    if (own[e]) {
      const double x = unif_pm1(mix64(seed ^ (uint64_t)(0x5bd1e995ull + tid + LZ_THREADS * e)));
      v[e] = from_real<T>(x);
      s += x * x;
    }
  }
  s = block_sum(s, red);
#pragma unroll
  for (int e = 0; e < NPT; ++e) {
    v[e] = scal(v[e], 1.0 / sqrt(s));
    if (own[e]) Vb[tid + LZ_THREADS * e] = v[e];
  }
  int k = 0;
  for (int j = 0; j < KL; ++j) {
    // u = R v_j - beta_{j-1} u_{j-1}
#pragma unroll
    for (int e = 0; e < NPT; ++e)
      if (own[e]) xs[tid + LZ_THREADS * e] = v[e];
    __syncthreads();
    lz_rows<T, false>(n, Rrow, n, true, xs, ys);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
      u[e] = own[e] ? ys[tid + LZ_THREADS * e] : zero<T>();
      if (j > 0) u[e] = sub(u[e], scal(uprev[e], beta[j - 1]));
    }
    lz_reorth<T, NPT>(n, j, Ub, u, xs, hq);
    s = 0.0;
#pragma unroll
    for (int e = 0; e < NPT; ++e) s += own[e] ? abs2(u[e]) : 0.0;
    s = block_sum(s, red);
    const double a = sqrt(s);
    if (tid == 0) alpha[j] = a;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
      u[e] = scal(u[e], (a > 0.0) ? 1.0 / a : 0.0);
      if (own[e]) Ub[(int64_t)j * n + tid + LZ_THREADS * e] = u[e];
    }
    k = j + 1;
    if (!(a > 0.0)) break;
    // v = R^* u - alpha_j v_j   (column l of R is Ycol[l*ld + 0..l])
#pragma unroll
    for (int e = 0; e < NPT; ++e)
      if (own[e]) xs[tid + LZ_THREADS * e] = u[e];
    __syncthreads();
    lz_rows<T, true>(n, Ycol, ld, false, xs, ys);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NPT; ++e) v[e] = own[e] ? sub(ys[tid + LZ_THREADS * e], scal(v[e], a)) : zero<T>();
    lz_reorth<T, NPT>(n, j + 1, Vb, v, xs, hq);
    s = 0.0;
#pragma unroll
    for (int e = 0; e < NPT; ++e) s += own[e] ? abs2(v[e]) : 0.0;
    s = block_sum(s, red);
    const double bta = sqrt(s);
    if (tid == 0) beta[j] = bta;
    __syncthreads();
    if (!(bta > 1e-15 * a) || j + 1 >= n) break;
#pragma unroll
    for (int e = 0; e < NPT; ++e) {
      v[e] = scal(v[e], 1.0 / bta);
      if (own[e]) Vb[(int64_t)(j + 1) * n + tid + LZ_THREADS * e] = v[e];
      uprev[e] = u[e];
    }
    // every 8 steps from step 16: stop once the top Ritz value of B^T B has
    // settled to 1e-15 relative (k = j + 1 steps so far)
    if (j + 1 >= 16 && (j + 1) % 8 == 0 && j + 1 < KL) {
      lz_tridiag(alpha, beta, j + 1, dg, of);
      __syncthreads();
      if (tid < 64) {
        const double top = tridiag_top(dg, of, j + 1);
        if (tid == 0) {
          est[1] = (fabs(top - est[0]) <= 1e-15 * top) ? 1.0 : 0.0;
          est[0] = top;
        }
      }
      __syncthreads();
      if (est[1] != 0.0) break;
    }
  }
  __syncthreads();
  lz_tridiag(alpha, beta, k, dg, of);
  __syncthreads();
  if (tid < 64) {
    const double top = tridiag_top(dg, of, k);
    if (tid == 0) ctl->sigma1 = sqrt(top);
  }
}

template <typename T>
__global__ void k_final_n(int n, int B, int k, const T* __restrict__ V, const double* __restrict__ thb,
                          double* __restrict__ sigma, T* __restrict__ Vout, int64_t ldv, Ctl* __restrict__ ctl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < k) {
    const double s = thb[B - 1 - idx];
    sigma[idx] = s;
    if (s == 0.0) ctl->zero_theta = 1;
  }
  if (idx < (int64_t)n * k) {
    const int64_t r = idx / k, jo = idx % k;
    Vout[r * ldv + jo] = V[r * B + (B - 1 - jo)];
  }
}

// ---------------------------------------------------------------------------
template <typename T, int B>
static void trmv_b(hipStream_t st, const void* M, int n, int lower, const void* X, void* Y, const Ctl* ctl, int cd_) {
  hipLaunchKernelGGL((k_trmv<T, B>), dim3((n + 15) / 16), dim3(NS_THREADS), 0, st, (const T*)M, n, lower, (const T*)X,
                     (T*)Y, ctl, cd_);
}

template <typename T>
static bool trmv_t(int B, hipStream_t st, const void* M, int n, int lower, const void* X, void* Y, const Ctl* ctl,
                   int cd_) {
  switch (B) {
#define RL_TB(BB) \
  case BB: trmv_b<T, BB>(st, M, n, lower, X, Y, ctl, cd_); return true;
    RL_TB(1) RL_TB(2) RL_TB(3) RL_TB(4) RL_TB(5) RL_TB(6) RL_TB(7) RL_TB(8) RL_TB(9) RL_TB(10)
#undef RL_TB
    default: return false;
  }
}

hipError_t launch_trmv(hipStream_t st, bool cplx, int B, const void* M, int n, int lower, const void* X, void* Y,
                       const Ctl* ctl, int check_done) {
  const bool ok = cplx ? trmv_t<cd>(B, st, M, n, lower, X, Y, ctl, check_done)
                       : trmv_t<double>(B, st, M, n, lower, X, Y, ctl, check_done);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int KM>
static void orth_go(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x, void* W,
                    Ctl* ctl, int check_done, int masked) {
  hipLaunchKernelGGL((k_orth<T, KM>), dim3(1), dim3(NS_THREADS), 0, st, n, B, (const T*)V, (const T*)X, project,
                     with_x, (T*)W, ctl, check_done, masked);
}

template <typename T>
static void orth_dispatch(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x,
                          void* W, Ctl* ctl, int check_done, int masked) {
  if (std::is_same<T, cd>::value ? launch_orth_reg_c(st, n, B, V, X, project, with_x, W, ctl, check_done, masked)
                                  : launch_orth_reg_d(st, n, B, V, X, project, with_x, W, ctl, check_done, masked))
    return;
  const int need = 3 * B;
  if (need <= 4) orth_go<T, 4>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  else if (need <= 8) orth_go<T, 8>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  else if (need <= 16) orth_go<T, 16>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  else if (need <= 32) orth_go<T, 32>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  else orth_go<T, 3 * RR_BMAX>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
}

template <typename T, int KM>
static void svqb_go(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x, void* W,
                    Ctl* ctl, int check_done) {
  hipLaunchKernelGGL((k_orth_svqb<T, KM>), dim3(1), dim3(NS_THREADS), 0, st, n, B, (const T*)V, (const T*)X, project,
                     with_x, (T*)W, ctl, check_done);
}

template <typename T>
static void svqb_dispatch(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x,
                          void* W, Ctl* ctl, int check_done) {
  const int need = 3 * B;
  if (need <= 4) svqb_go<T, 4>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  else if (need <= 8) svqb_go<T, 8>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  else if (need <= 16) svqb_go<T, 16>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  else if (need <= 32) svqb_go<T, 32>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  else svqb_go<T, 3 * RR_BMAX>(st, n, B, V, X, project, with_x, W, ctl, check_done);
}

hipError_t launch_orth_svqb(hipStream_t st, bool cplx, int n, int B, const void* V, const void* X, int project,
                            int with_x, void* W, Ctl* ctl, int check_done) {
  if (B < 1 || B > RR_BMAX) return hipErrorInvalidValue;
  if (cplx) svqb_dispatch<cd>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  else svqb_dispatch<double>(st, n, B, V, X, project, with_x, W, ctl, check_done);
  return hipGetLastError();
}

hipError_t launch_orth(hipStream_t st, bool cplx, int n, int B, const void* V, const void* X, int project, int with_x,
                       void* W, Ctl* ctl, int check_done, int masked) {
  if (B < 1 || B > RR_BMAX) return hipErrorInvalidValue;
  if (cplx) orth_dispatch<cd>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  else orth_dispatch<double>(st, n, B, V, X, project, with_x, W, ctl, check_done, masked);
  return hipGetLastError();
}

template <typename T, int B>
static void rr_go(hipStream_t st, int n, int init_mode, int with_x, const void* Rt, void* V, void* X, const void* W,
                  const void* G3, void* Vn, void* Rres, void* CV, void* CX, double* thb, double* ht, double* hr,
                  Ctl* ctl, int phase, double* Cst) {
  hipLaunchKernelGGL((k_rr<T, B>), dim3(1), dim3(NS_THREADS), 0, st, n, init_mode, with_x, (const T*)Rt, (T*)V,
                     (T*)X, (const T*)W, (const T*)G3, (T*)Vn, (T*)Rres, (T*)CV, (T*)CX, thb, ht, hr, ctl, phase, Cst);
}

template <typename T>
static bool rr_by_b(int B, hipStream_t st, int n, int init_mode, int with_x, const void* Rt, void* V, void* X,
                    const void* W, const void* G3, void* Vn, void* Rres, void* CV, void* CX, double* thb, double* ht,
                    double* hr, Ctl* ctl, int phase, double* Cst) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: rr_go<T, BB>(st, n, init_mode, with_x, Rt, V, X, W, G3, Vn, Rres, CV, CX, thb, ht, hr, ctl, phase, Cst); \
    return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

hipError_t launch_rr(hipStream_t st, bool cplx, int n, int B, int init_mode, int with_x, const void* Rt, void* V,
                     void* X, const void* W, const void* G3, void* Vn, void* Rres, void* CV, void* CX, double* thb,
                     double* ht, double* hr, Ctl* ctl, int phase, double* Cst) {
  if (phase < 0 || phase > 2 || (phase != 0 && (Cst == nullptr || init_mode))) return hipErrorInvalidValue;
  const bool ok = cplx ? rr_by_b<cd>(B, st, n, init_mode, with_x, Rt, V, X, W, G3, Vn, Rres, CV, CX, thb, ht, hr, ctl,
                                     phase, Cst)
                       : rr_by_b<double>(B, st, n, init_mode, with_x, Rt, V, X, W, G3, Vn, Rres, CV, CX, thb, ht, hr,
                                         ctl, phase, Cst);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

__global__ void k_publish(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_publish(hipStream_t st, const Ctl* src, Ctl* dst) {
  static_assert(sizeof(Ctl) % 4 == 0, "Ctl is copied in 32-bit words");
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, st, (const int32_t*)src, (int32_t*)dst, (int)(sizeof(Ctl) / 4));
  return hipGetLastError();
}

hipError_t launch_randblk(hipStream_t st, bool cplx, void* Wb, int64_t count, uint64_t seed) {
  const unsigned g = (unsigned)((count + 255) / 256);
  if (cplx)
    hipLaunchKernelGGL(k_randblk<cd>, dim3(g), dim3(256), 0, st, (cd*)Wb, count, seed);
  else
    hipLaunchKernelGGL(k_randblk<double>, dim3(g), dim3(256), 0, st, (double*)Wb, count, seed);
  return hipGetLastError();
}

template <typename T, int NPT>
static hipError_t lanczos_go(hipStream_t st, int n, const void* Ycol, int ld, const void* Rrow, void* Ub, void* Vb,
                             int KL, uint64_t seed, Ctl* ctl) {
  const size_t lds = 2 * sizeof(T) * (size_t)LZ_THREADS * NPT;
  const hipError_t e =
      hipFuncSetAttribute((const void*)k_lanczos<T, NPT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_lanczos<T, NPT>), dim3(1), dim3(LZ_THREADS), lds, st, n, (const T*)Ycol, ld, (const T*)Rrow,
                     (T*)Ub, (T*)Vb, KL, seed, ctl);
  return hipGetLastError();
}

// n <= 1024 (one entry per thread) or n <= 2048 (two)
hipError_t launch_lanczos(hipStream_t st, bool cplx, int n, const void* Ycol, int ld, const void* Rrow, void* Ub,
                          void* Vb, int KL, uint64_t seed, Ctl* ctl) {
  if (n <= LZ_THREADS)
    return cplx ? lanczos_go<cd, 1>(st, n, Ycol, ld, Rrow, Ub, Vb, KL, seed, ctl)
                : lanczos_go<double, 1>(st, n, Ycol, ld, Rrow, Ub, Vb, KL, seed, ctl);
  if (n <= 2 * LZ_THREADS)
    return cplx ? lanczos_go<cd, 2>(st, n, Ycol, ld, Rrow, Ub, Vb, KL, seed, ctl)
                : lanczos_go<double, 2>(st, n, Ycol, ld, Rrow, Ub, Vb, KL, seed, ctl);
  return hipErrorInvalidValue;
}

hipError_t launch_final_n(hipStream_t st, bool cplx, int n, int B, int k, const void* V, const double* thb,
                          double* sigma, void* Vout, int64_t ldv, Ctl* ctl) {
  const int64_t cnt = (int64_t)n * k > k ? (int64_t)n * k : k;
  const unsigned g = (unsigned)((cnt + 255) / 256);
  if (cplx)
    hipLaunchKernelGGL(k_final_n<cd>, dim3(g), dim3(256), 0, st, n, B, k, (const cd*)V, thb, sigma, (cd*)Vout, ldv, ctl);
  else
    hipLaunchKernelGGL(k_final_n<double>, dim3(g), dim3(256), 0, st, n, B, k, (const double*)V, thb, sigma,
                       (double*)Vout, ldv, ctl);
  return hipGetLastError();
}

}  // namespace rl

namespace rl {

// Singular values (descending) and right singular vectors of a t x t R
// (row-major), for the tall-SVD step entry point.
template <typename T>
__global__ __launch_bounds__(NS_THREADS) void k_rt_svd(int t, const T* __restrict__ Rt, double* __restrict__ sigma,
                                                       T* __restrict__ Cout) {
  __shared__ T M[RR_TMAX * 32];
  __shared__ T Vj[RR_TMAX * 32];
  __shared__ double sig[RR_TMAX];
  const int lane = threadIdx.x;
  for (int e = lane; e < RR_TMAX * 32; e += blockDim.x) {
    const int c = e / 32, r = e % 32;
    M[e] = (r < t && c < t) ? Rt[r * t + c] : zero<T>();
    Vj[e] = from_real<T>((r == c) ? 1.0 : 0.0);
  }
  __syncthreads();
  jacobi_block<T>(M, Vj, t);
  // column norms, then each column's place in the descending order (the
  // number ranked before it: larger, or equal with a lower index)
  __shared__ int rank_s[RR_TMAX];
  const int tid = threadIdx.x;
  if (tid < t) {
    double s2 = 0.0;
    for (int r = 0; r < t; ++r) s2 += abs2(M[tid * 32 + r]);
    sig[tid] = sqrt(s2);
  }
  __syncthreads();
  if (tid < t) {
    int rk = 0;
    for (int q = 0; q < t; ++q) rk += (sig[q] > sig[tid] || (sig[q] == sig[tid] && q < tid)) ? 1 : 0;
    rank_s[tid] = rk;
    sigma[rk] = sig[tid];
  }
  __syncthreads();
  for (int e = tid; e < t * 32; e += blockDim.x) {
    const int c = e / 32, r = e % 32;
    if (r < t) Cout[r * t + rank_s[c]] = Vj[c * 32 + r];
  }
}

hipError_t launch_rt_svd(hipStream_t st, bool cplx, int t, const void* Rt, double* sigma, void* C) {
  if (cplx)
    hipLaunchKernelGGL(k_rt_svd<cd>, dim3(1), dim3(NS_THREADS), 0, st, t, (const cd*)Rt, sigma, (cd*)C);
  else
    hipLaunchKernelGGL(k_rt_svd<double>, dim3(1), dim3(NS_THREADS), 0, st, t, (const double*)Rt, sigma, (double*)C);
  return hipGetLastError();
}

// out = max_j ||Z(:, j)||_2 over the B columns of the n x B block Z (one
// workgroup; the reduced-precision guard's 1 / sigma_min(R) estimate).
template <typename T>
__global__ __launch_bounds__(NS_THREADS) void k_max_colnorm(int n, int B, const T* __restrict__ Z,
                                                            double* __restrict__ out) {
  __shared__ double red[NS_THREADS / 64];
  double best = 0.0;
  for (int j = 0; j < B; ++j) {
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) s += abs2(Z[(int64_t)r * B + j]);
    const double nrm = sqrt(block_sum(s, red));
    best = (nrm > best || !(nrm == nrm)) ? nrm : best;
  }
  if (threadIdx.x == 0) *out = best;
}

hipError_t launch_max_colnorm(hipStream_t st, bool cplx, int n, int B, const void* Z, double* out) {
  if (cplx)
    hipLaunchKernelGGL(k_max_colnorm<cd>, dim3(1), dim3(NS_THREADS), 0, st, n, B, (const cd*)Z, out);
  else
    hipLaunchKernelGGL(k_max_colnorm<double>, dim3(1), dim3(NS_THREADS), 0, st, n, B, (const double*)Z, out);
  return hipGetLastError();
}

}  // namespace rl
