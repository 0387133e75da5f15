// Complex A-stream in two reads of A, for wide problems (256 < n <= 1024).
//
// The fused single-read form (astream_ccs.hip) needs every row's sums of A W
// reduced across all ceil(n/64) waves of a workgroup before the row can enter
// A^* [A_V A_X A_W]; for wide complex rows that cross-wave traffic and the
// readlane broadcasts cost more issue slots than the arithmetic.  Here the two
// products of the iteration's pass (Section 3.3) take one read of A each:
//
//   k_c2_rows  A_W = A W.  A wave owns whole rows (lane l holds columns
//              l + 64 s, s < NS); the group's slice of W sits in LDS
//              vector-major, so every lane reads its own entries without bank
//              conflicts, and a row's 2 BS sums need one transpose-reduction
//              inside the wave and no barrier.  Vectors are split into groups
//              of BS <= 5 (the W slice must fit LDS: 80 KB for 1024 columns);
//              the groups of one row range are neighbouring workgroups of one
//              XCD.
//   k_c2_cols  G = A^* [A_V A_X A_W].  Lane l of wave w in column slab s owns
//              column 256 s + 64 w + l.  A row's values of A_V (A_X, A_W) are
//              the same for every lane and are read through the scalar cache
//              into scalar registers, so the column sums are plain FMAs (Dot2
//              pairs for the A_V block) with no cross-lane work and no LDS.
//              The three planes are three workgroups (neighbours on one XCD),
//              which keeps the accumulators of b = 10 vectors to b complex
//              pairs per lane.
//              Each workgroup writes its plane of its slab of the row range's
//              partial record [G_V | G_X | G_W | G_V errors].
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

constexpr int C2_THREADS = 256;
template <bool DOT2>
struct C2Cols {
  static constexpr int RC = DOT2 ? 4 : 8;  // rows loaded ahead by the column kernel
};

template <int BS>
struct C2RowShape {
  static constexpr int T = 2 * BS;  // real sums per row
  static constexpr int T2 = T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16;
  static constexpr int LOG2T = T2 == 2 ? 1 : T2 == 4 ? 2 : T2 == 8 ? 3 : 4;
};

template <int BS, int NS, bool DOT2>
__global__ __launch_bounds__(C2_THREADS, 2) void k_c2_rows(const cd* __restrict__ A, int64_t lda, int64_t m, int n,
                                                          int B, const cd* __restrict__ W, cd* __restrict__ AW,
                                                          int64_t rows_per_block, int64_t nrb, int ng,
                                                          const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  using SH = C2RowShape<BS>;
  constexpr int T = SH::T, T2 = SH::T2, LOG2T = SH::LOG2T;
  constexpr int NC = 64 * NS;
  extern __shared__ double c2_lds[];
  cd* Ws = reinterpret_cast<cd*>(c2_lds);  // Ws[j * NC + c], the group's vectors
  // block -> (row range, vector group): the groups of a row range are
  // consecutive blocks of one XCD
  const int64_t bid = blockIdx.x;
  const int64_t kx = bid >> 3;
  const int grp = (int)(kx % ng);
  const int64_t rbi = (kx / ng) * 8 + (bid & 7);
  if (rbi >= nrb) return;
  const int j0 = grp * BS;
  const int bsr = (B - j0 < BS) ? B - j0 : BS;
  const int lane = threadIdx.x & 63, wave = wave_index();
  for (int e = threadIdx.x; e < BS * NC; e += C2_THREADS) {
    const int j = e / NC, c = e - (e / NC) * NC;
    Ws[e] = (c < n && j < bsr) ? W[(int64_t)c * B + j0 + j] : cd{0.0, 0.0};
  }
  __syncthreads();
  int my_idx = 0;
#pragma unroll
  for (int st = 0; st < LOG2T; ++st) my_idx |= ((lane >> (5 - st)) & 1) << (LOG2T - 1 - st);
  const bool my_rep = (lane & ((1 << (6 - LOG2T)) - 1)) == 0;
  const int64_t r0 = rbi * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  auto load = [&](cd (&a)[NS], int64_t row) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = lane + 64 * s;
      a[s] = (row < r1 && c < n) ? A[row * lda + c] : cd{0.0, 0.0};
    }
  };
  double* AWd = reinterpret_cast<double*>(AW);
  cd an[NS];
  int64_t row = r0 + wave;
  load(an, row);
  for (; row < r1; row += C2_THREADS / 64) {
    cd a[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) a[s] = an[s];
    load(an, row + C2_THREADS / 64);
    double ys[T2], ye[T2];
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      ys[t] = 0.0;
      ye[t] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int j = 0; j < BS; ++j) {
        if (j < bsr) {
          const cd w = Ws[j * NC + lane + 64 * s];
          if constexpr (DOT2) {
            // the first product of each component starts its pair exactly
            if (s == 0) {
              two_prod(a[s].x, w.x, ys[2 * j], ye[2 * j]);
              two_prod(a[s].x, w.y, ys[2 * j + 1], ye[2 * j + 1]);
            } else {
              dot2_add(a[s].x, w.x, ys[2 * j], ye[2 * j]);
              dot2_add(a[s].x, w.y, ys[2 * j + 1], ye[2 * j + 1]);
            }
            dot2_add(-a[s].y, w.y, ys[2 * j], ye[2 * j]);
            dot2_add(a[s].y, w.x, ys[2 * j + 1], ye[2 * j + 1]);
          } else {
            ys[2 * j] = fma(a[s].x, w.x, ys[2 * j]);
            ys[2 * j] = fma(-a[s].y, w.y, ys[2 * j]);
            ys[2 * j + 1] = fma(a[s].x, w.y, ys[2 * j + 1]);
            ys[2 * j + 1] = fma(a[s].y, w.x, ys[2 * j + 1]);
          }
        }
      }
    }
    if constexpr (DOT2) tr_reduce_dot2<T2, LOG2T>(ys, ye, lane);
    else tr_reduce_plain<T2, LOG2T>(ys, lane);
    if (my_rep && my_idx < 2 * bsr) AWd[row * 2 * (int64_t)B + 2 * j0 + my_idx] = DOT2 ? ys[0] + ye[0] : ys[0];
  }
}

template <int B, bool DOT2>
__global__ __launch_bounds__(C2_THREADS) void k_c2_cols(const cd* __restrict__ A, int64_t lda, int64_t m, int n,
                                                       const cd* __restrict__ AVp, const cd* __restrict__ AXp,
                                                       const cd* __restrict__ AW, int init,
                                                       double* __restrict__ Gpart, int64_t rows_per_block,
                                                       int64_t nrb, int nslab, int npg, const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  // plane group 0: G_V (Dot2 pairs with DOT2; A_W in the start pass), 1: G_X,
  // 2: G_W.  The groups of one (row range, slab) are neighbouring blocks of
  // one XCD.
  const int64_t bid = blockIdx.x;
  const int64_t kx = bid >> 3;
  const int pg = (int)(kx % npg);
  const int slab = (int)((kx / npg) % nslab);
  const int64_t rbi = (kx / npg / nslab) * 8 + (bid & 7);
  if (rbi >= nrb) return;
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int c = slab * C2_THREADS + wave * 64 + lane;
  constexpr int RC = C2Cols<DOT2>::RC;
  const int64_t r0 = rbi * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < m) ? r0 + rows_per_block : m;
  // the group's row values: wave-uniform, read through the scalar cache
  const cd* Vg = (pg == 0) ? (init ? AW : AVp) : (pg == 1 ? AXp : AW);
  cd gs[B], ge[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    gs[j] = cd{0.0, 0.0};
    ge[j] = cd{0.0, 0.0};
  }
  auto loada = [&](cd (&a)[RC], int64_t rb) {
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      const int64_t rr = rb + q;
      a[q] = (rr < r1 && c < n) ? A[rr * lda + c] : cd{0.0, 0.0};
    }
  };
  if (Vg != nullptr) {
    cd an[RC];
    loada(an, r0);
    for (int64_t rb = r0; rb < r1; rb += RC) {
      cd a[RC];
#pragma unroll
      for (int q = 0; q < RC; ++q) a[q] = an[q];
      loada(an, rb + RC);
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        const int64_t rr = rb + q;
        if (rr < r1) {
#pragma unroll
          for (int j = 0; j < B; ++j) {
            const cd v = Vg[rr * B + j];
            if (DOT2 && pg == 0) {
              dot2_add(a[q].x, v.x, gs[j].x, ge[j].x);
              dot2_add(a[q].y, v.y, gs[j].x, ge[j].x);
              dot2_add(a[q].x, v.y, gs[j].y, ge[j].y);
              dot2_add(-a[q].y, v.x, gs[j].y, ge[j].y);
            } else {
              gs[j] = cfmac(a[q], v, gs[j]);
            }
          }
        }
      }
    }
  }
  const int64_t plane = 2 * (int64_t)n * B;
  double* gp = Gpart + rbi * 4 * plane;
  if (c < n) {
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int64_t e = 2 * ((int64_t)c * B + j);
      double* dst = gp + (int64_t)pg * plane + e;
      dst[0] = gs[j].x;
      dst[1] = gs[j].y;
      if (pg == 0) {
        gp[3 * plane + e] = ge[j].x;
        gp[3 * plane + e + 1] = ge[j].y;
        if (npg == 1) {  // start pass: no G_X, G_W
          gp[plane + e] = 0.0;
          gp[plane + e + 1] = 0.0;
          gp[2 * plane + e] = 0.0;
          gp[2 * plane + e + 1] = 0.0;
        }
      }
    }
  }
}

// vector groups of the row kernel: at most 5 vectors (the W slice of 5
// vectors x 1024 columns is 80 KB of LDS, two workgroups per CU)
static void c2_groups(int B, int* ng, int* bs) {
  *ng = (B + 4) / 5;
  *bs = (B + *ng - 1) / *ng;
}

bool astream_c2_fits(int B, int n, bool aligned) { return aligned && n > 256 && n <= 1024 && B >= 1 && B <= 10; }

// Row ranges: about 2048 workgroups over the column slabs, at least 16 rows
// each; the partial records (one per row range) stay within about 4% of the
// bytes of A.
int64_t astream_c2_ranges(int64_t m, int n, int B) {
  const int nslab = (n + C2_THREADS - 1) / C2_THREADS;
  int64_t target = 2048 / nslab;
  const double abytes = 16.0 * (double)m * n;
  const double rec = 4.0 * 16.0 * n * B;
  const int64_t cap = (int64_t)(0.04 * abytes / rec);
  if (target > cap) target = cap;
  if (target < 8) target = 8;
  int64_t rows = (m + target - 1) / target;
  if (rows < 16) rows = 16;
  return (m + rows - 1) / rows;
}

template <int BS, int NS, bool DOT2>
static void c2_rows_go(hipStream_t st, int64_t nblk, int64_t rows, int64_t nrb, int ng, const cd* A, int64_t lda,
                       int64_t m, int n, int B, const cd* W, cd* AW, const Ctl* ctl) {
  const size_t lds = sizeof(cd) * BS * 64 * NS;
  hipFuncSetAttribute((const void*)k_c2_rows<BS, NS, DOT2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_c2_rows<BS, NS, DOT2>), dim3((unsigned)nblk), dim3(C2_THREADS), lds, st, A, lda, m, n, B, W,
                     AW, rows, nrb, ng, ctl);
}

template <int NS, bool DOT2>
static bool c2_rows_bs(int bs, hipStream_t st, int64_t nblk, int64_t rows, int64_t nrb, int ng, const cd* A,
                       int64_t lda, int64_t m, int n, int B, const cd* W, cd* AW, const Ctl* ctl) {
  switch (bs) {
    case 1: c2_rows_go<1, NS, DOT2>(st, nblk, rows, nrb, ng, A, lda, m, n, B, W, AW, ctl); return true;
    case 2: c2_rows_go<2, NS, DOT2>(st, nblk, rows, nrb, ng, A, lda, m, n, B, W, AW, ctl); return true;
    case 3: c2_rows_go<3, NS, DOT2>(st, nblk, rows, nrb, ng, A, lda, m, n, B, W, AW, ctl); return true;
    case 4: c2_rows_go<4, NS, DOT2>(st, nblk, rows, nrb, ng, A, lda, m, n, B, W, AW, ctl); return true;
    case 5: c2_rows_go<5, NS, DOT2>(st, nblk, rows, nrb, ng, A, lda, m, n, B, W, AW, ctl); return true;
    default: return false;
  }
}

template <bool DOT2>
static bool c2_cols_b(int B, hipStream_t st, int64_t nblk, int64_t rows, int64_t nrb, int nslab, int npg, const cd* A,
                      int64_t lda, int64_t m, int n, const cd* AVp, const cd* AXp, const cd* AW, int init,
                      double* Gpart, const Ctl* ctl) {
  switch (B) {
#define RL_CASE(BB)                                                                                              \
  case BB:                                                                                                       \
    hipLaunchKernelGGL((k_c2_cols<BB, DOT2>), dim3((unsigned)nblk), dim3(C2_THREADS), 0, st, A, lda, m, n, AVp, \
                       AXp, AW, init, Gpart, rows, nrb, nslab, npg, ctl);                                        \
    return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

// A_W = A W (row kernel), then the column sums (column kernel); nrb partial
// records as for the other paths.
bool dispatch_astream_c2(bool dot2, int init, int B, hipStream_t st, int64_t nrb, const void* A, int64_t lda,
                         int64_t m, int n, const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart,
                         const Ctl* ctl) {
  if (n <= 256 || n > 1024 || B < 1 || B > 10) return false;
  int ng, bs;
  c2_groups(B, &ng, &bs);
  const int ns = (n + 63) / 64;
  // row kernel: the same row ranges as the partial records, ng groups each
  const int64_t rows = (m + nrb - 1) / nrb;
  const int64_t nblk_r = ((nrb + 7) / 8) * 8 * ng;
  const cd* Ac = (const cd*)A;
  bool ok;
  // NS templates: 8 (n <= 512) or 16 (n <= 1024) column slots per lane
  if (ns <= 8)
    ok = dot2 ? c2_rows_bs<8, true>(bs, st, nblk_r, rows, nrb, ng, Ac, lda, m, n, B, (const cd*)W, (cd*)AW, ctl)
              : c2_rows_bs<8, false>(bs, st, nblk_r, rows, nrb, ng, Ac, lda, m, n, B, (const cd*)W, (cd*)AW, ctl);
  else
    ok = dot2 ? c2_rows_bs<16, true>(bs, st, nblk_r, rows, nrb, ng, Ac, lda, m, n, B, (const cd*)W, (cd*)AW, ctl)
              : c2_rows_bs<16, false>(bs, st, nblk_r, rows, nrb, ng, Ac, lda, m, n, B, (const cd*)W, (cd*)AW, ctl);
  if (!ok) return false;
  const int nslab = (n + C2_THREADS - 1) / C2_THREADS;
  const int npg = init ? 1 : 3;
  const int64_t nblk_c = ((nrb + 7) / 8) * 8 * nslab * npg;
  if (dot2)
    return c2_cols_b<true>(B, st, nblk_c, rows, nrb, nslab, npg, Ac, lda, m, n, (const cd*)AVp, (const cd*)AXp,
                           (const cd*)AW, init, Gpart, ctl);
  return c2_cols_b<false>(B, st, nblk_c, rows, nrb, nslab, npg, Ac, lda, m, n, (const cd*)AVp, (const cd*)AXp,
                          (const cd*)AW, init, Gpart, ctl);
}

}  // namespace rl
