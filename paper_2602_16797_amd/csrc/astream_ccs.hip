// Complex column-split A-stream pass (n <= 1024, any b): the fused product of
// the LOBPCG iteration, A_W = A W and G = A^* [A_V A_X A_W] (Section 3.3, the
// single pass over A of each iteration), for complex128 data.
//
// Lane l of wave w owns column c = l + 64 w (one 16-byte load per row), so a
// workgroup of ceil(n / 64) waves covers a whole row.  The b block vectors are
// split into groups of at most BS: the per-lane state is 4 BS complex
// accumulators plus BS entries of W, and a 1024-thread workgroup leaves 128
// registers per lane, which a whole block of b = 10 complex vectors does not
// fit.  The groups of one row range run as neighbouring workgroups of the same
// XCD (block index b -> XCD b mod 8), so the second read of the rows is served
// by that XCD's L2 while the first is still streaming them.
//
// Per batch of RB rows each wave reduces its partial sums of the 2 BS real
// components (re, im per vector) with the transpose-reduction and writes them
// to LDS; after one barrier every wave combines the waves' partials
// (compensated), its 64 lanes splitting the work over components and waves,
// and the finished row sums are broadcast with readlanes and used at once for
// the column sums.
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

template <int BS, bool DOT2>
struct CcsShape {
  static constexpr int RB = DOT2 ? 1 : 2;  // rows per batch (one barrier each)
  static constexpr int T = 2 * BS;      // real components per row
  static constexpr int V = RB * T;      // row sums per batch (<= 20)
  static constexpr int T2 = T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16;
  static constexpr int LOG2T = T2 == 2 ? 1 : T2 == 4 ? 2 : T2 == 8 ? 3 : 4;
};
constexpr int CCS_MAXW = 16;

// (s, e) += conj(a) * v, component-wise Dot2 sums
__device__ inline void ccs_dot2_cacc(const cd& a, double vr, double vi, cd& s, cd& e) {
  dot2_add(a.x, vr, s.x, e.x);
  dot2_add(a.y, vi, s.x, e.x);
  dot2_add(a.x, vi, s.y, e.y);
  dot2_add(-a.y, vr, s.y, e.y);
}
__device__ inline void ccs_cacc(const cd& a, double vr, double vi, cd& s) {
  s.x = fma(a.x, vr, s.x);
  s.x = fma(a.y, vi, s.x);
  s.y = fma(a.x, vi, s.y);
  s.y = fma(-a.y, vr, s.y);
}

template <int BS, bool DOT2>
__global__ __launch_bounds__(1024) void k_astream_ccs(const cd* __restrict__ A, int64_t lda, int64_t m, int n, int B,
                                                      const cd* __restrict__ W, cd* __restrict__ AW,
                                                      const cd* __restrict__ AVp, const cd* __restrict__ AXp,
                                                      double* __restrict__ Gpart, int64_t rows_per_block,
                                                      int64_t nrb, int ng, int init, const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  using SH = CcsShape<BS, DOT2>;
  constexpr int RB = SH::RB, T = SH::T, V = SH::V, T2 = SH::T2, LOG2T = SH::LOG2T;
  constexpr int VP = V <= 2 ? 2 : V <= 4 ? 4 : V <= 8 ? 8 : V <= 16 ? 16 : 32;
  constexpr int CQ = 64 / VP;  // lanes per component in the cross-wave combine
  // block -> (row range, vector group): the ng groups of a row range are
  // consecutive blocks of one XCD
  const int64_t bid = blockIdx.x;
  const int64_t kx = bid >> 3;
  const int grp = (int)(kx % ng);
  const int64_t rbi = (kx / ng) * 8 + (bid & 7);
  if (rbi >= nrb) return;
  const int j0 = grp * BS;
  const int bsr = (B - j0 < BS) ? B - j0 : BS;
  __shared__ double sp[2][CCS_MAXW][V];
  __shared__ double ep[DOT2 ? 2 : 1][DOT2 ? CCS_MAXW : 1][DOT2 ? V : 1];
  const int nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const bool has_x = AXp != nullptr;
  const int c = lane + 64 * wave;
  int my_idx = 0;
#pragma unroll
  for (int st = 0; st < LOG2T; ++st) my_idx |= ((lane >> (5 - st)) & 1) << (LOG2T - 1 - st);
  const bool my_rep = (lane & ((1 << (6 - LOG2T)) - 1)) == 0;
  cd w[BS], g1s[BS], g1e[BS], gx[BS], gw[BS];
#pragma unroll
  for (int j = 0; j < BS; ++j) {
    w[j] = (c < n && j < bsr) ? W[(int64_t)c * B + j0 + j] : cd{0.0, 0.0};
    g1s[j] = cd{0.0, 0.0};
    g1e[j] = cd{0.0, 0.0};
    gx[j] = cd{0.0, 0.0};
    gw[j] = cd{0.0, 0.0};
  }
  const int64_t r0 = rbi * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  auto load = [&](cd (&a)[RB], int64_t rb) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int64_t row = rb + q;
      a[q] = (row < r1 && c < n) ? A[row * lda + c] : cd{0.0, 0.0};
    }
  };
  // lane v < V carries real component v of the batch: row v / T, component
  // v mod T (2 j + 0 for Re, 2 j + 1 for Im of vector j0 + j)
  const int vq = lane / T, vt = lane - (lane / T) * T;
  const bool vlane = lane < V && vt < 2 * bsr;
  const int ccv = lane / CQ, ccq = lane - (lane / CQ) * CQ;
  const double* AVd = reinterpret_cast<const double*>(AVp);
  const double* AXd = reinterpret_cast<const double*>(AXp);
  double* AWd = reinterpret_cast<double*>(AW);
  const int64_t ldv = 2 * (int64_t)B;  // doubles per row of A_V, A_X, A_W
  int64_t rb = r0;
  cd a[RB], an[RB];
  load(an, rb);
  double avn = 0.0, axn = 0.0;
  if (!init && vlane && rb + vq < r1) {
    avn = AVd[(rb + vq) * ldv + 2 * j0 + vt];
    if (has_x) axn = AXd[(rb + vq) * ldv + 2 * j0 + vt];
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
      if (vlane && rn + vq < r1) {
        avn = AVd[(rn + vq) * ldv + 2 * j0 + vt];
        if (has_x) axn = AXd[(rn + vq) * ldv + 2 * j0 + vt];
      }
    }
    // this wave's partial row sums of A W, one row at a time
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      double ys[T2], ye[T2];
#pragma unroll
      for (int t = 0; t < T2; ++t) {
        ys[t] = 0.0;
        ye[t] = 0.0;
      }
#pragma unroll
      for (int j = 0; j < BS; ++j) {
        if (j < bsr) {
          if constexpr (DOT2) {
            // the first product of each component starts its pair exactly
            two_prod(a[q].x, w[j].x, ys[2 * j], ye[2 * j]);
            dot2_add(-a[q].y, w[j].y, ys[2 * j], ye[2 * j]);
            two_prod(a[q].x, w[j].y, ys[2 * j + 1], ye[2 * j + 1]);
            dot2_add(a[q].y, w[j].x, ys[2 * j + 1], ye[2 * j + 1]);
          } else {
            ys[2 * j] = fma(a[q].x, w[j].x, ys[2 * j]);
            ys[2 * j] = fma(-a[q].y, w[j].y, ys[2 * j]);
            ys[2 * j + 1] = fma(a[q].x, w[j].y, ys[2 * j + 1]);
            ys[2 * j + 1] = fma(a[q].y, w[j].x, ys[2 * j + 1]);
          }
        }
      }
      if constexpr (DOT2) tr_reduce_dot2<T2, LOG2T>(ys, ye, lane);
      else tr_reduce_plain<T2, LOG2T>(ys, lane);
      if (my_rep && my_idx < T) {
        sp[buf][wave][q * T + my_idx] = ys[0];
        if constexpr (DOT2) ep[buf][wave][q * T + my_idx] = ye[0];
      }
    }
    __syncthreads();
    // the wave partials are combined by all 64 lanes: lane l takes component
    // l / CQ and the waves congruent to l mod CQ, then the CQ lanes of a
    // component finish the sum with compensated butterfly stages
    double S = 0.0, E = 0.0;
    if (ccv < V) {
      for (int q = ccq; q < nw; q += CQ) {
        double t;
        two_sum(S, sp[buf][q][ccv], S, t);
        E += t;
        if constexpr (DOT2) E += ep[buf][q][ccv];
      }
    }
    if constexpr (CQ > 16) ar_stage_dot2<16>(S, E);
    if constexpr (CQ > 8) ar_stage_dot2<8>(S, E);
    if constexpr (CQ > 4) ar_stage_dot2<4>(S, E);
    if constexpr (CQ > 2) ar_stage_dot2<2>(S, E);
    if constexpr (CQ > 1) ar_stage_dot2<1>(S, E);
    const double comb = S + E;  // component lane / CQ
    buf ^= 1;
    if (wave == 0 && ccq == 0 && ccv < V) {
      const int wq = ccv / T, wt = ccv - (ccv / T) * T;
      if (wt < 2 * bsr && rb + wq < r1) AWd[(rb + wq) * ldv + 2 * j0 + wt] = comb;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
      for (int j = 0; j < BS; ++j) {
        if (j < bsr) {
          const int v = q * T + 2 * j;
          const double yr = readlane_d(comb, v * CQ), yi = readlane_d(comb, (v + 1) * CQ);
          const double vr = init ? yr : readlane_d(avl, v), vi = init ? yi : readlane_d(avl, v + 1);
          if constexpr (DOT2) ccs_dot2_cacc(a[q], vr, vi, g1s[j], g1e[j]);
          else ccs_cacc(a[q], vr, vi, g1s[j]);
          if (!init) {
            if (has_x) ccs_cacc(a[q], readlane_d(axl, v), readlane_d(axl, v + 1), gx[j]);
            ccs_cacc(a[q], yr, yi, gw[j]);
          }
        }
      }
  }
  // partial record of this row range: planes [G1 | G_X | G_W | G1 errors],
  // each n x B complex; this group fills its B-columns j0 .. j0 + bsr - 1
  const int64_t plane = 2 * (int64_t)n * B;
  double* gp = Gpart + rbi * 4 * plane;
  if (c < n) {
#pragma unroll
    for (int j = 0; j < BS; ++j) {
      if (j < bsr) {
        const int64_t e = 2 * ((int64_t)c * B + j0 + j);
        gp[e] = g1s[j].x;
        gp[e + 1] = g1s[j].y;
        gp[plane + e] = gx[j].x;
        gp[plane + e + 1] = gx[j].y;
        gp[2 * plane + e] = gw[j].x;
        gp[2 * plane + e + 1] = gw[j].y;
        gp[3 * plane + e] = g1e[j].x;
        gp[3 * plane + e + 1] = g1e[j].y;
      }
    }
  }
}

template <int BS, bool DOT2>
static void launch_ccs(hipStream_t st, int64_t nblk, int nw, int64_t rows, int64_t nrb, int ng, const cd* A,
                       int64_t lda, int64_t m, int n, int B, const cd* W, cd* AW, const cd* AVp, const cd* AXp,
                       double* Gpart, int init, const Ctl* ctl) {
  hipLaunchKernelGGL((k_astream_ccs<BS, DOT2>), dim3((unsigned)nblk), dim3(64 * nw), 0, st, A, lda, m, n, B, W, AW,
                     AVp, AXp, Gpart, rows, nrb, ng, init, ctl);
}

template <bool DOT2>
static bool ccs_by_bs(int BS, hipStream_t st, int64_t nblk, int nw, int64_t rows, int64_t nrb, int ng, const cd* A,
                      int64_t lda, int64_t m, int n, int B, const cd* W, cd* AW, const cd* AVp, const cd* AXp,
                      double* Gpart, int init, const Ctl* ctl) {
  switch (BS) {
#define RL_CASE(S)                                                                                         \
  case S:                                                                                                  \
    launch_ccs<S, DOT2>(st, nblk, nw, rows, nrb, ng, A, lda, m, n, B, W, AW, AVp, AXp, Gpart, init, ctl); \
    return true;
    RL_CASE(1) RL_CASE(2)
#undef RL_CASE
    default: break;
  }
  if constexpr (!DOT2) {  // Dot2 groups hold at most two vectors
    switch (BS) {
      case 3: launch_ccs<3, DOT2>(st, nblk, nw, rows, nrb, ng, A, lda, m, n, B, W, AW, AVp, AXp, Gpart, init, ctl); return true;
      case 4: launch_ccs<4, DOT2>(st, nblk, nw, rows, nrb, ng, A, lda, m, n, B, W, AW, AVp, AXp, Gpart, init, ctl); return true;
      default: break;
    }
  }
  return false;
}

int astream_ccs_waves(int n) { return (n + 63) / 64; }

bool astream_ccs_fits(int B, int n, bool aligned) { return aligned && n >= 1 && n <= 64 * CCS_MAXW && B >= 1; }

// vector groups: at most 4 vectors per group (2 with Dot2 sums), split evenly
void astream_ccs_groups(int B, bool dot2, int* ng, int* bs) {
  const int cap = dot2 ? 2 : 4;
  *ng = (B + cap - 1) / cap;
  *bs = (B + *ng - 1) / *ng;
}

// Row ranges: about 2048 workgroups in all over the groups, at least 16 rows
// each; the partial records (one per row range) stay within about 4% of the
// bytes of A.
int64_t astream_ccs_ranges(int64_t m, int n, int B, bool dot2) {
  int ng, bs;
  astream_ccs_groups(B, dot2, &ng, &bs);
  int64_t target = 2048 / ng;
  const double abytes = 16.0 * (double)m * n;
  const double rec = 4.0 * 16.0 * n * B;
  const int64_t cap = (int64_t)(0.04 * abytes / rec);
  if (target > cap) target = cap;
  if (target < 8) target = 8;
  int64_t rows = (m + target - 1) / target;
  if (rows < 16) rows = 16;
  return (m + rows - 1) / rows;
}

bool dispatch_astream_ccs(bool dot2, int init, int B, hipStream_t st, int64_t nrb, const void* A, int64_t lda,
                          int64_t m, int n, const void* W, void* AW, const void* AVp, const void* AXp,
                          double* Gpart, const Ctl* ctl) {
  const int nw = astream_ccs_waves(n);
  if (nw < 1 || nw > CCS_MAXW) return false;
  int ng, bs;
  astream_ccs_groups(B, dot2, &ng, &bs);
  const int64_t rows = (m + nrb - 1) / nrb;
  const int64_t nblk = ((nrb + 7) / 8) * 8 * ng;
  if (dot2)
    return ccs_by_bs<true>(bs, st, nblk, nw, rows, nrb, ng, (const cd*)A, lda, m, n, B, (const cd*)W, (cd*)AW,
                           (const cd*)AVp, (const cd*)AXp, Gpart, init, ctl);
  return ccs_by_bs<false>(bs, st, nblk, nw, rows, nrb, ng, (const cd*)A, lda, m, n, B, (const cd*)W, (cd*)AW,
                          (const cd*)AVp, (const cd*)AXp, Gpart, init, ctl);
}

}  // namespace rl
