// Complex A-stream on the FP64 matrix cores (v_mfma_f64_16x16x4f64), for
// wide problems (256 < n <= 1024, b <= 10), with plain FP64 accumulation.
//
// The iteration's pass (Alg. rlobpcg: the product A W of the new search block
// and the Gram data A^* [A_V A_X A_W] of the Rayleigh-Ritz step) is two dense
// contractions with a 1e6-long dimension.  In real form, with
//   Ar (m x 2n)  = A with (re, im) interleaved, exactly A's memory layout,
//   Wr (2n x 2b) = [[Re W, Im W], [-Im W, Re W]] interleaved the same way,
//   Tr (m x 6b)  = [A_V A_X A_W] with (re, im) interleaved,
// they read  A_W = Ar Wr  (rows of A against a small matrix) and
// Gr = Ar^T Tr  (a 2n x 6b Gram block summed over all rows), whose 2 x 2
// blocks combine into A^* T:  Re = Gr(2c, 2v) + Gr(2c+1, 2v+1),
// Im = Gr(2c, 2v+1) - Gr(2c+1, 2v).  A_W must be complete for a row before
// the row can enter Gr, and a row of A (16 KB at n = 1000) is too wide to keep
// on chip next to the accumulators of all of Gr, so each product takes one
// read of A:
//
//   k_zm_aw  A_W = Ar Wr.  W (n x b complex, at most 160 KB) sits in LDS; a
//            wave owns 32 rows (two 16-row M tiles) and walks k in blocks of
//            16 real columns.  Lane (q, t) = (lane / 16, lane % 16) loads 32
//            bytes, columns k0 + 4q .. k0 + 4q + 3 of row t; the four MFMA
//            steps of the block use k = k0 + 4q + s (a permutation of the
//            contraction index, applied to both operands), so one wide load
//            feeds all four steps and a wave load covers 128 contiguous bytes
//            of 16 rows.  The B operand Wr(k, j) is read from W in LDS with
//            the sign pattern of Wr.
//   k_zm_g   Gr = Ar^T Tr over a row range, written as one partial record
//            [G_V | G_X | G_W | 0] per row range (the layout every pass
//            writes; the compensated reduction of the records follows).  A
//            wave owns 64 real columns of A: lane (q, t) loads 32 bytes of
//            row i0 + q, columns kw + 4t .. kw + 4t + 3, and each of the four
//            values feeds its own M tile (tile u holds the columns
//            kw + 4t + u), so the 16 x 16 accumulator tiles are 4 M tiles by
//            up to 4 N tiles.  Tr's rows are staged in LDS per 32-row chunk,
//            double buffered, with the column order chosen so a lane reads
//            its N tiles' values in one access.  Tiles u and u + 1 hold the
//            real and imaginary parts of the same complex column at the same
//            lane and register, so the 2 x 2 combination needs only a swap
//            of neighbouring lanes before the record is written.
//
// Matrix-core operand layout of v_mfma_f64_16x16x4f64 (checked on gfx950):
// lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16), and register r of
// the result holds D(4 r + l / 16, l % 16).
#include "astream_kernels.hpp"
#include "kernels.hpp"

namespace rl {

typedef double zm_v4d __attribute__((ext_vector_type(4)));

__device__ inline zm_v4d zm_mfma(double a, double b, zm_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// v_mfma_f64_4x4x4f64: four independent 4 x 4 x 4 products, block beta =
// (lane / 4) % 4; lane 16 k + 4 beta + i supplies A_beta(i, k), lane
// 16 k + 4 beta + j supplies B_beta(k, j), and lane 16 i + 4 beta + j holds
// D_beta(i, j) (checked on gfx950).  With the same A operand as a 16 x 16 x 4
// tile (lane (q, t) = (lane / 16, lane % 16) supplies row t of the tile at
// contraction index q), block beta takes the tile's rows 4 beta .. 4 beta + 3,
// so one instruction forms a 16 x 4 tail tile: the last 1..4 columns of an
// N dimension of 16 NT + 1..4 without a padded 16-column tile.
__device__ inline double zm_mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

constexpr int ZM_AW_THREADS = 1024;  // 16 waves: one workgroup per CU holds W in LDS
constexpr int ZM_G_THREADS = 256;    // 4 waves: 256 real columns per workgroup
constexpr int ZM_G_RC = 32;          // rows of Tr per LDS chunk

// ----------------------------------------------------------------------------
// A_W = A W (real form Ar Wr).  NT = N tiles of 16 real output columns (2b);
// KH = 16-byte loads per lane, M tile and k block (a k block is 8 KH real
// columns, so each of a tile's 16 rows is read KH * 64 contiguous bytes at a
// time).
//
// CPLX = false is the same kernel for real A (lda2 = lda, Ar = A, Wr = W):
// the 16-byte pair a lane loads holds two consecutive columns k, k + 1, and
// the B operands are W(k, j) and W(k + 1, j).
//
// TAIL: the output columns 16 NT .. 16 NT + 3 form a 4-column tail tile
// (zm_mfma4) instead of a padded 16-column tile.
template <bool CPLX, int NT, int KH, bool TAIL = false>
__global__ __launch_bounds__(ZM_AW_THREADS) void k_zm_aw(const double* __restrict__ A, int64_t lda2, int64_t m,
                                                         int n, int B, const double* __restrict__ W,
                                                         double* __restrict__ AW, const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  extern __shared__ double zm_lds[];
  // W in LDS: complex Ws[2 (c B + v) + part], real Ws[k B + j]
  const int nwb = (CPLX ? 2 : 1) * n * B;
  for (int e = threadIdx.x; e < nwb; e += ZM_AW_THREADS) zm_lds[e] = W[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int q = lane >> 4, t = lane & 15;
  const int n2 = CPLX ? 2 * n : n, B2 = CPLX ? 2 * B : B;
  constexpr int KBW = 8 * KH;  // real columns per k block
  const int nkb = (n2 + KBW - 1) / KBW;
  // this lane's output columns per N tile: complex: vector v, part r (Wr's
  // sign pattern); real: vector 16 nt + t
  constexpr int NTS = NT + (TAIL ? 1 : 0);  // B operands per step (the tail's last)
  int vcol[NTS];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) vcol[nt] = CPLX ? (16 * nt + t) >> 1 : 16 * nt + t;
  if constexpr (TAIL) vcol[NT] = CPLX ? (16 * NT + (t & 3)) >> 1 : 16 * NT + (t & 3);
  const int rpart = t & 1;
  const int64_t ntile = (m + 31) / 32;
  const int64_t gw = (int64_t)blockIdx.x * (ZM_AW_THREADS / 64) + wave;
  const int64_t nwave = (int64_t)gridDim.x * (ZM_AW_THREADS / 64);
  for (int64_t tile = gw; tile < ntile; tile += nwave) {
    const int64_t r0 = tile * 32;
    // Loads are unconditional (addresses clamped into A, so no branch or
    // exec mask sits between a load and its use and the compiler can keep
    // them in flight), and ordinary: a row's 128-byte line is read by two
    // 16-byte loads per lane, and a non-temporal first load let the line go
    // before the second (21 % more HBM traffic measured).  Lane (q, t) reads columns k0 + 2 KH q .. + 2 KH - 1
    // of row t of each M tile; each 16-byte pair is valid or invalid as a
    // whole (2n is even).
    const double* rowp[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int64_t row = r0 + 16 * mt + t;
      rowp[mt] = A + (row < m ? row : m - 1) * lda2;
    }
    auto load = [&](double2 (&a)[2][KH], int kb) {
      const int k = KBW * kb + 2 * KH * q;
#pragma unroll
      for (int i = 0; i < KH; ++i) {
        const int kc = k + 2 * i < n2 - 2 ? k + 2 * i : n2 - 2;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) a[mt][i] = *reinterpret_cast<const double2*>(rowp[mt] + kc);
      }
    };
    zm_v4d acc[2][NT];
    double acct[2] = {0.0, 0.0};  // the tail tile (TAIL)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = zm_v4d{0.0, 0.0, 0.0, 0.0};
    // one k block of MFMA steps on the values of buffer a: step s uses
    // k = k0 + 2 KH q + s (a permutation of the contraction index, the same
    // for both operands), i.e. complex column c = k0 / 2 + KH q + s / 2, part s % 2
    auto step = [&](const double2 (&a)[2][KH], int kb) {
#pragma unroll
      for (int h = 0; h < KH; ++h) {
        double b_re[NTS], b_im[NTS];
        if constexpr (CPLX) {
          const int c = (KBW / 2) * kb + KH * q + h;
          const cd* Ws = reinterpret_cast<const cd*>(zm_lds);
#pragma unroll
          for (int nt = 0; nt < NTS; ++nt) {
            const bool wok = c < n && vcol[nt] < B;
            const int wi = wok ? c * B + vcol[nt] : 0;
            const cd w = Ws[wi];
            // Wr(2c, 2v) = Re w, Wr(2c, 2v+1) = Im w, Wr(2c+1, 2v) = -Im w, Wr(2c+1, 2v+1) = Re w
            b_re[nt] = wok ? (rpart ? w.y : w.x) : 0.0;
            b_im[nt] = wok ? (rpart ? w.x : -w.y) : 0.0;
          }
        } else {
          // the pair holds columns k and k + 1 (n may be odd: k + 1 < n is checked on its own)
          const int k = KBW * kb + 2 * KH * q + 2 * h;
#pragma unroll
          for (int nt = 0; nt < NTS; ++nt) {
            const bool ok0 = k < n && vcol[nt] < B, ok1 = k + 1 < n && vcol[nt] < B;
            const double w0 = zm_lds[ok0 ? k * B + vcol[nt] : 0];
            const double w1 = zm_lds[ok1 ? (k + 1) * B + vcol[nt] : 0];
            b_re[nt] = ok0 ? w0 : 0.0;
            b_im[nt] = ok1 ? w1 : 0.0;
          }
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          // no mask on A: a clamped row's results are never stored, and a
          // clamped column meets a zero of Wr
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            acc[mt][nt] = zm_mfma(a[mt][h].x, b_re[nt], acc[mt][nt]);
            acc[mt][nt] = zm_mfma(a[mt][h].y, b_im[nt], acc[mt][nt]);
          }
          if constexpr (TAIL) {
            acct[mt] = zm_mfma4(a[mt][h].x, b_re[NT], acct[mt]);
            acct[mt] = zm_mfma4(a[mt][h].y, b_im[NT], acct[mt]);
          }
        }
      }
    };
    // two buffers, each refilled two k blocks ahead right after its use (no
    // register copies between a load and its use, so the loads stay in flight)
    double2 a0[2][KH], a1[2][KH];
    load(a0, 0);
    load(a1, 1);
    for (int kb = 0; kb < nkb; kb += 2) {
      step(a0, kb);
      load(a0, kb + 2);
      if (kb + 1 < nkb) {
        step(a1, kb + 1);
        load(a1, kb + 3);
      }
    }
    // register r of a tile holds output row 4r + q, column 16 nt + t
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t orow = r0 + 16 * mt + 4 * r + q;
          const int col = 16 * nt + t;
          if (orow < m && col < B2) AW[orow * B2 + col] = acc[mt][nt][r];
        }
    if constexpr (TAIL) {
      // the tail tile: lane (q, t) holds row 4 (t / 4) + q, column 16 NT + t % 4
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int64_t orow = r0 + 16 * mt + 4 * (t >> 2) + q;
        const int col = 16 * NT + (t & 3);
        if (orow < m && col < B2) AW[orow * B2 + col] = acct[mt];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Partial records of A^* [P0 P1 P2] over row ranges (real form Ar^T Tr).
// NT = N tiles over the used columns of Tr (np planes of 2b real columns).
// Tr plane g goes to record plane g (init: the single plane A_W to plane 0).
//
// CPLX = false is the same kernel for real A (Ar = A, Tr = [A_V A_X A_W], no
// 2 x 2 combination: Gr is A^T T itself).  TAIL: the Tr columns 16 NT ..
// 16 NT + 3 form a 4-column tail tile (zm_mfma4) instead of a padded one.
template <bool CPLX, int NT, bool TAIL = false>
__global__ __launch_bounds__(ZM_G_THREADS, 2) void k_zm_g(const double* __restrict__ A, int64_t lda2, int64_t m, int n,
                                                       int B, const double* __restrict__ P0,
                                                       const double* __restrict__ P1, const double* __restrict__ P2,
                                                       int np, int init, double* __restrict__ Gpart,
                                                       int64_t rows_per_range, int64_t nrr, int nslice,
                                                       const Ctl* __restrict__ ctl) {
  if (ctl != nullptr && ctl->done) return;
  constexpr int NTS = NT + (TAIL ? 1 : 0);  // staged 16-column groups (the tail's last)
  constexpr int TW = 16 * NTS;               // Tr columns staged per row
  __shared__ double Ts[2][ZM_G_RC * TW];
  // block -> (row range, column slice): the slices of a row range are
  // neighbouring blocks of one XCD, so the staged rows of Tr come from L2
  const int64_t bid = blockIdx.x;
  const int64_t kx = bid >> 3;
  const int slice = (int)(kx % nslice);
  const int64_t rr = (kx / nslice) * 8 + (bid & 7);
  if (rr >= nrr) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int q = lane >> 4, t = lane & 15;
  const int n2 = CPLX ? 2 * n : n, B2 = CPLX ? 2 * B : B;
  const int kw = 256 * slice + 64 * wave;  // this wave's first real column of A
  const bool active = kw < n2;
  const int64_t r0 = rr * rows_per_range;
  const int64_t r1 = (r0 + rows_per_range < m) ? r0 + rows_per_range : m;
  const int ncol = np * B2;
  const double* Pg[3] = {P0, P1, P2};
  // staging: element e of a chunk is (row e / TW, Tr column e % TW); it is
  // stored at row * TW + (col % 16) * NT + col / 16 so that lane t finds its
  // NT values (columns t, 16 + t, ...) side by side
  constexpr int PER = (ZM_G_RC * TW + ZM_G_THREADS - 1) / ZM_G_THREADS;
  // fetch(v, cb): this thread's share of the chunk's rows of Tr, loaded
  // unconditionally from clamped addresses (no branch between a load and its
  // use); stage() zeroes what lies outside Tr when it writes the chunk to LDS
  auto fetch = [&](double (&v)[PER], int64_t cb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * ZM_G_THREADS;
      const int rw = e / TW, col = e - (e / TW) * TW;
      const int64_t grow = cb + rw;
      const int g = col < ncol ? col / B2 : 0;
      const double* P = Pg[g] != nullptr ? Pg[g] : P0;
      const int64_t gr = grow < r1 ? grow : r1 - 1;
      const int cw = col < ncol ? col - g * B2 : 0;
      v[i] = P[gr * B2 + cw];
    }
  };
  auto valid = [&](int e, int64_t cb) {
    const int rw = e / TW, col = e - (e / TW) * TW;
    return e < ZM_G_RC * TW && cb + rw < r1 && col < ncol && Pg[col < ncol ? col / B2 : 0] != nullptr;
  };
  auto stage = [&](const double (&v)[PER], int buf, int64_t cb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * ZM_G_THREADS;
      if (e < ZM_G_RC * TW) {
        const int rw = e / TW, col = e - (e / TW) * TW;
        Ts[buf][rw * TW + (col & 15) * NTS + (col >> 4)] = valid(e, cb) ? v[i] : 0.0;
      }
    }
  };
  zm_v4d acc[4][NT];
  double acct[4] = {0.0, 0.0, 0.0, 0.0};  // the tail tile (TAIL)
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[u][nt] = zm_v4d{0.0, 0.0, 0.0, 0.0};
  const int kcol = kw + 4 * t;  // this lane's four columns of A: kcol .. kcol + 3
  // unconditional loads from clamped addresses (rows past r1 read row
  // r1 - 1)
  // (each 16-byte half is clamped on its own: a half past 2n reads the last
  // pair, and its rows of Gr, c >= n, are never written)
  const int kc0 = kcol < n2 - 2 ? kcol : n2 - 2;
  const int kc1 = kcol + 2 < n2 - 2 ? kcol + 2 : n2 - 2;
  auto loada = [&](double2 (&a)[2], int64_t grow) {
    const double* p = A + (grow < r1 ? grow : r1 - 1) * lda2;
    a[0] = ld_stream2(p + kc0);
    a[1] = ld_stream2(p + kc1);
  };
  {
    double v[PER];
    fetch(v, r0);
    stage(v, 0, r0);
  }
  // four buffers of A rows, each refilled four K steps (16 rows) ahead
  // right after its use, across chunk boundaries (a chunk is 8 K steps)
  double2 ab[4][2];
#pragma unroll
  for (int j = 0; j < 4; ++j) loada(ab[j], r0 + 4 * j + q);
  __syncthreads();
  int buf = 0;
  for (int64_t cb = r0; cb < r1; cb += ZM_G_RC) {
    double v[PER];
    const bool more = cb + ZM_G_RC < r1;
    if (more) fetch(v, cb + ZM_G_RC);
    if (active) {
      const double* Tb = Ts[buf];
#pragma unroll
      for (int ks = 0; ks < ZM_G_RC / 4; ++ks) {
        const double* tr = Tb + (4 * ks + q) * TW + t * NTS;
        double bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bv[nt] = tr[nt];
        // no mask on A: a clamped row meets the zero rows of Tr staged past
        // r1, and the rows of Gr of clamped columns are never written
        const double2* a0 = ab[ks & 3];
        const double av[4] = {a0[0].x, a0[0].y, a0[1].x, a0[1].y};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[u][nt] = zm_mfma(av[u], bv[nt], acc[u][nt]);
        if constexpr (TAIL) {
          // Tr column 16 NT + t % 4, the same for the four blocks
          const double bt = Tb[(4 * ks + q) * TW + (t & 3) * NTS + NT];
#pragma unroll
          for (int u = 0; u < 4; ++u) acct[u] = zm_mfma4(av[u], bt, acct[u]);
        }
        loada(ab[ks & 3], cb + 4 * ks + 16 + q);
      }
    }
    if (more) stage(v, buf ^ 1, cb + ZM_G_RC);
    __syncthreads();
    buf ^= 1;
  }
  if (!active) return;
  if constexpr (CPLX) {
    // 2 x 2 combination: tile u (even) holds Gr(2c, .), tile u + 1 Gr(2c + 1, .)
    // at the same lane and register; columns 2v and 2v + 1 are lanes t and t + 1.
    const int64_t plane = 2 * (int64_t)n * B;
    double* gp = Gpart + rr * 4 * plane;
    const int rp = t & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double x0 = acc[2 * h][nt][r], x1 = acc[2 * h + 1][nt][r];
          const double y0 = dpp_d<0xB1>(x0), y1 = dpp_d<0xB1>(x1);  // the neighbour lane t ^ 1
          // output row 4r + q of the tile is the column group kcol' = kw + 4 (4r + q)
          const int c = (kw + 4 * (4 * r + q)) / 2 + h;
          const int colr = 16 * nt + t;  // Tr column of this lane (even t: re part)
          if (rp == 0 && c < n && colr < ncol) {
            const int g = colr / B2, vv = (colr - g * B2) >> 1;
            const double re = x0 + y1;  // Gr(2c, 2v) + Gr(2c+1, 2v+1)
            const double im = y0 - x1;  // Gr(2c, 2v+1) - Gr(2c+1, 2v)
            const int pl = init ? 0 : g;
            double* dst = gp + (int64_t)pl * plane + 2 * ((int64_t)c * B + vv);
            dst[0] = re;
            dst[1] = im;
          }
        }
    if constexpr (TAIL) {
      // tail tile: lane (q, t) holds real column kw + 16 (t / 4) + 4 q + u of
      // A against Tr column 16 NT + t % 4; u = 2h, 2h + 1 are the re and im
      // rows of complex column c, and Tr columns 2v, 2v + 1 lanes t, t + 1
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double x0 = acct[2 * h], x1 = acct[2 * h + 1];
        const double y0 = dpp_d<0xB1>(x0), y1 = dpp_d<0xB1>(x1);
        const int c = (kw + 16 * (t >> 2) + 4 * q) / 2 + h;
        const int colr = 16 * NT + (t & 3);
        if (rp == 0 && c < n && colr < ncol) {
          const int g = colr / B2, vv = (colr - g * B2) >> 1;
          const int pl = init ? 0 : g;
          double* dst = gp + (int64_t)pl * plane + 2 * ((int64_t)c * B + vv);
          dst[0] = x0 + y1;
          dst[1] = y0 - x1;
        }
      }
    }
    // the planes this pass does not form, and the error plane, are zero
    // (init 2: the Gram pass alone, whose reduction reads plane 0 only)
    for (int cc = lane; init != 2 && cc < 32 * B; cc += 64) {
      const int c = kw / 2 + cc / B, vv = cc - (cc / B) * B;
      if (c < n) {
        const int64_t e = 2 * ((int64_t)c * B + vv);
        for (int pl = (init ? 1 : 3); pl < 4; ++pl) {
          gp[pl * plane + e] = 0.0;
          gp[pl * plane + e + 1] = 0.0;
        }
      }
    }
  } else {
    // tile u, register r holds G(c, col) for column c = kw + 4 (4r + q) + u of
    // A and column col = 16 nt + t of Tr
    const int64_t plane = (int64_t)n * B;
    double* gp = Gpart + rr * 4 * plane;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = kw + 4 * (4 * r + q) + u;
          const int colr = 16 * nt + t;
          if (c < n && colr < ncol) {
            const int g = colr / B2, vv = colr - g * B2;
            gp[(int64_t)(init ? 0 : g) * plane + (int64_t)c * B + vv] = acc[u][nt][r];
          }
        }
    if constexpr (TAIL) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = kw + 16 * (t >> 2) + 4 * q + u;
        const int colr = 16 * NT + (t & 3);
        if (c < n && colr < ncol) {
          const int g = colr / B2, vv = colr - g * B2;
          gp[(int64_t)(init ? 0 : g) * plane + (int64_t)c * B + vv] = acct[u];
        }
      }
    }
    for (int cc = lane; init != 2 && cc < 64 * B; cc += 64) {
      const int c = kw + cc / B, vv = cc - (cc / B) * B;
      if (c < n) {
        const int64_t e = (int64_t)c * B + vv;
        for (int pl = (init ? 1 : 3); pl < 4; ++pl) gp[pl * plane + e] = 0.0;
      }
    }
  }
}

bool astream_zm_fits(int B, int n, bool aligned, int64_t lds_max) {
  return aligned && n > 256 && n <= 1024 && B >= 1 && B <= 10 && (int64_t)n * B * 16 <= lds_max;
}

// Real A: even n (each lane's 16-byte pairs are whole columns pairs), W in LDS.
bool astream_rm_fits(int B, int n, bool aligned, int64_t lds_max) {
  return aligned && n % 2 == 0 && n > 1024 && n <= 2048 && B >= 1 && B <= 10 && (int64_t)n * B * 8 <= lds_max;
}

constexpr int ZM_AW_KH = 2;  // 32 contiguous bytes per row and lane per k block

template <bool CPLX, int NT, bool TAIL = false>
static hipError_t zm_aw_go(hipStream_t st, int grid, const double* A, int64_t lda2, int64_t m, int n, int B,
                           const double* W, double* AW, const Ctl* ctl) {
  const size_t lds = (CPLX ? 16 : 8) * (size_t)n * B;
  const hipError_t e = hipFuncSetAttribute((const void*)k_zm_aw<CPLX, NT, ZM_AW_KH, TAIL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zm_aw<CPLX, NT, ZM_AW_KH, TAIL>), dim3((unsigned)grid), dim3(ZM_AW_THREADS), lds, st, A,
                     lda2, m, n, B, W, AW, ctl);
  return hipGetLastError();
}

// A W for B2 output columns: one 16-column tile, one and a 4-column tail
// (17..20), or two tiles
template <bool CPLX>
static hipError_t zm_aw_cols(hipStream_t st, int grid, const double* A, int64_t lda2, int64_t m, int n, int B,
                             const double* W, double* AW, const Ctl* ctl) {
  const int B2 = CPLX ? 2 * B : B;
  if (B2 <= 16) return zm_aw_go<CPLX, 1>(st, grid, A, lda2, m, n, B, W, AW, ctl);
  if (B2 <= 20) return zm_aw_go<CPLX, 1, true>(st, grid, A, lda2, m, n, B, W, AW, ctl);
  return zm_aw_go<CPLX, 2>(st, grid, A, lda2, m, n, B, W, AW, ctl);
}

template <bool CPLX, int NT, bool TAIL = false>
static void zm_g_go(hipStream_t st, int64_t nblk, const double* A, int64_t lda2, int64_t m, int n, int B,
                    const double* P0, const double* P1, const double* P2, int np, int init, double* Gpart,
                    int64_t rows, int64_t nrr, int nslice, const Ctl* ctl) {
  hipLaunchKernelGGL((k_zm_g<CPLX, NT, TAIL>), dim3((unsigned)nblk), dim3(ZM_G_THREADS), 0, st, A, lda2, m, n, B, P0,
                     P1, P2, np, init, Gpart, rows, nrr, nslice, ctl);
}

// The Gram kernel for ncol used Tr columns: full 16-column tiles, and a
// 4-column tail tile when 1..4 columns are left past at least one full tile.
template <bool CPLX>
static bool zm_g_cols(hipStream_t st, int64_t nblk, const double* A, int64_t lda2, int64_t m, int n, int B,
                      const double* P0, const double* P1, const double* P2, int np, int init, double* Gpart,
                      int64_t rows, int64_t nrr, int nslice, const Ctl* ctl) {
  const int ncol = np * (CPLX ? 2 * B : B);
  const int full = ncol / 16, rest = ncol % 16;
#define RL_ZMG(NTV, TL) \
  zm_g_go<CPLX, NTV, TL>(st, nblk, A, lda2, m, n, B, P0, P1, P2, np, init, Gpart, rows, nrr, nslice, ctl)
  if (full >= 1 && rest >= 1 && rest <= 4) {
    switch (full) {
      case 1: RL_ZMG(1, true); break;
      case 2: RL_ZMG(2, true); break;
      case 3: RL_ZMG(3, true); break;
      default: return false;
    }
  } else {
    switch ((ncol + 15) / 16) {
      case 1: RL_ZMG(1, false); break;
      case 2: RL_ZMG(2, false); break;
      case 3: RL_ZMG(3, false); break;
      case 4: RL_ZMG(4, false); break;
      default: return false;
    }
  }
#undef RL_ZMG
  return true;
}

// A_W = A W, then the partial records of A^* [A_V A_X A_W] (init: A^* A_W in
// the first plane) over nrr row ranges; cplx selects the complex real form.
template <bool CPLX>
static bool zm_dispatch(int init, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                        const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart, int n_cu,
                        const Ctl* ctl, hipEvent_t mid) {
  const double* Ad = (const double*)A;
  const int64_t lda2 = CPLX ? 2 * lda : lda;
  const int n2 = CPLX ? 2 * n : n, B2 = CPLX ? 2 * B : B;
  // one workgroup per CU (W fills the LDS), at most one per 32-row tile per wave
  const int64_t tiles = (m + 31) / 32;
  int grid = n_cu > 0 ? n_cu : 256;
  if ((int64_t)grid * (ZM_AW_THREADS / 64) > tiles) grid = (int)((tiles + 15) / 16);
  if (grid < 1) grid = 1;
  const hipError_t e = zm_aw_cols<CPLX>(st, grid, Ad, lda2, m, n, B, (const double*)W, (double*)AW, ctl);
  if (e != hipSuccess) return false;
  // the second kernel's start, for timing the Gram contraction on its own
  if (mid != nullptr && hipEventRecord(mid, st) != hipSuccess) return false;
  const int64_t rows = (m + nrr - 1) / nrr;
  const int nslice = (n2 + 255) / 256;
  const int64_t nblk = ((nrr + 7) / 8) * 8 * nslice;
  const double* P0 = init ? (const double*)AW : (const double*)AVp;
  const double* P1 = init ? nullptr : (const double*)AXp;
  const double* P2 = init ? nullptr : (const double*)AW;
  const int np = init ? 1 : 3;
  if (!zm_g_cols<CPLX>(st, nblk, Ad, lda2, m, n, B, P0, P1, P2, np, init, Gpart, rows, nrr, nslice, ctl))
    return false;
  return hipGetLastError() == hipSuccess;
}

// The Gram contraction alone: the partial records of A^* P0 over nrr row
// ranges (plane 0 only: the other planes are not written, and the reduction
// of these records reads plane 0 alone), for the late residual
// A^* A_{V_{i+1}} of an iteration whose A W came from its own pass.
template <bool CPLX>
static bool zm_gram(int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n, const void* P0,
                    double* Gpart, const Ctl* ctl) {
  const double* Ad = (const double*)A;
  const int64_t lda2 = CPLX ? 2 * lda : lda;
  const int n2 = CPLX ? 2 * n : n, B2 = CPLX ? 2 * B : B;
  const int64_t rows = (m + nrr - 1) / nrr;
  const int nslice = (n2 + 255) / 256;
  const int64_t nblk = ((nrr + 7) / 8) * 8 * nslice;
  const double* P = (const double*)P0;
  (void)B2;
  if (!zm_g_cols<CPLX>(st, nblk, Ad, lda2, m, n, B, P, nullptr, nullptr, 1, 2, Gpart, rows, nrr, nslice, ctl))
    return false;
  return hipGetLastError() == hipSuccess;
}

// A W alone (the first read of an iteration on the late-residual path).
template <bool CPLX>
static bool zm_aw_only(int B, hipStream_t st, const void* A, int64_t lda, int64_t m, int n, const void* W, void* AW,
                       int n_cu, const Ctl* ctl) {
  const double* Ad = (const double*)A;
  const int64_t lda2 = CPLX ? 2 * lda : lda;
  const int B2 = CPLX ? 2 * B : B;
  const int64_t tiles = (m + 31) / 32;
  int grid = n_cu > 0 ? n_cu : 256;
  if ((int64_t)grid * (ZM_AW_THREADS / 64) > tiles) grid = (int)((tiles + 15) / 16);
  if (grid < 1) grid = 1;
  (void)B2;
  return zm_aw_cols<CPLX>(st, grid, Ad, lda2, m, n, B, (const double*)W, (double*)AW, ctl) == hipSuccess;
}

bool dispatch_zm_aw_only(bool cplx, int B, hipStream_t st, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, int n_cu, const Ctl* ctl) {
  if (B < 1 || B > 10) return false;
  return cplx ? zm_aw_only<true>(B, st, A, lda, m, n, W, AW, n_cu, ctl)
              : zm_aw_only<false>(B, st, A, lda, m, n, W, AW, n_cu, ctl);
}

bool dispatch_zm_gram(bool cplx, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                      const void* P0, double* Gpart, const Ctl* ctl) {
  if (B < 1 || B > 10 || nrr < 1) return false;
  return cplx ? zm_gram<true>(B, st, nrr, A, lda, m, n, P0, Gpart, ctl)
              : zm_gram<false>(B, st, nrr, A, lda, m, n, P0, Gpart, ctl);
}

bool dispatch_astream_zm(int init, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart, int n_cu,
                         const Ctl* ctl, hipEvent_t mid) {
  if (n <= 256 || n > 1024 || B < 1 || B > 10 || nrr < 1) return false;
  return zm_dispatch<true>(init, B, st, nrr, A, lda, m, n, W, AW, AVp, AXp, Gpart, n_cu, ctl, mid);
}

bool dispatch_astream_rm(int init, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart, int n_cu,
                         const Ctl* ctl, hipEvent_t mid) {
  if (n <= 1024 || n > 2048 || (n & 1) || B < 1 || B > 10 || nrr < 1) return false;
  return zm_dispatch<false>(init, B, st, nrr, A, lda, m, n, W, AW, AVp, AXp, Gpart, n_cu, ctl, mid);
}

}  // namespace rl
