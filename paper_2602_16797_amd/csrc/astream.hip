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
// k_colsum2   deterministic compensated sum of the partial planes (the last
//             level writes the finished sums).
// k_panel     A_V <- A_T C_V, A_X <- A_T C_X (row-local, in place).
// k_final_u   U(:, j) = (A_T C_V)(:, b-1-j) / theta_{b-1-j} for the outputs.
#include <algorithm>

#include "common.hpp"
#include "astream_kernels.hpp"
#include "kernels.hpp"
#include "colsum.hpp"

namespace rl {

// Compensated, deterministic sum over parts.  Input part p has sums at
// in_s[p*stride + e] and, for e < elen, errors at in_e[p*stride + e];
// block y of the grid sums parts [64y, 64y+64) and writes (sum, error) to
// out_s/out_e[y*len + e].
__global__ __launch_bounds__(256) void k_colsum2(ColsumJob J) { colsum2_block(J, blockIdx.x, blockIdx.y); }


// Row-local panel update.  mode: 0 A_T = [A_V] (t = B), 1 [A_V A_W] (t = 2B),
// 2 [A_V A_X A_W] (t = 3B).  C_V, C_X are t x B row-major.  pmode 0:
// A_V <- A_T C_V and A_X <- A_T C_X in place (AVout == AV); 1: AVout <- A_T C_V
// only, A_T left as it is; 2: A_X <- A_T C_X only (the late-residual form,
// whose new A_V was formed by pmode 1 before the Gram pass).
// Each wave takes chunks of 64 rows: a panel's chunk (64 B contiguous values)
// is read with coalesced loads into the wave's LDS slot and each lane picks
// its row out of it; the lane's output row goes back through the slot and
// out with coalesced stores.  (A lane reading its own B-value row straight
// from memory touches 64 scattered rows per load instruction.)  A chunk is
// read in full before any of it is written, so the in-place forms are safe.
// Lanes of one wave exchange values through LDS: a compiler fence at wave
// scope between the writes and the other lanes' reads (DS instructions of a
// wave execute in order, so no wait is needed beyond it).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T, int B, bool ONE>
__global__ __launch_bounds__(256) void k_panel(const T* AV, T* AVout, T* AX, const T* AW, int64_t m,
                                               const T* __restrict__ CVg, const T* __restrict__ CXg,
                                               const Ctl* __restrict__ ctl, int pmode) {
  if (ctl->done) return;
  const int mode = ctl->rr_mode;
  const int xupd = (pmode != 1) && ctl->x_update;
  const bool vupd = pmode != 2;
  const int t = (mode == 0) ? B : (mode == 1 ? 2 * B : 3 * B);
  __shared__ T CV[3 * B * B];
  __shared__ T CX[3 * B * B];
  __shared__ T stage[4][64 * B];
  for (int i = threadIdx.x; i < 3 * B * B; i += blockDim.x) {
    CV[i] = (i < t * B) ? CVg[i] : zero<T>();
    CX[i] = (xupd && i < t * B) ? CXg[i] : zero<T>();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = wave_index();
  T* slot = stage[wave];
  const int64_t nchunk = (m + 63) / 64;
  if constexpr (ONE) {
    // one output block (pmode 1 or 2): the panels are consumed one at a time
    // into B accumulators, so only B values of the row are live, and the
    // next (chunk, panel) unit is loaded while the current one is added
    const T* Cm = vupd ? CV : CX;
    T* out = vupd ? AVout : AX;
    if (!vupd && !xupd) return;
    const int np = (mode == 0) ? 1 : (mode == 1 ? 2 : 3);
    const T* P1 = mode == 2 ? AX : AW;
    const T* P2 = AW;
    const int64_t stride = (int64_t)gridDim.x * 4;
    int64_t ch = (int64_t)blockIdx.x * 4 + wave;
    if (ch >= nchunk) return;
    auto load = [&](T (&v)[B], int64_t c, const T* P) __attribute__((always_inline)) {
      const int64_t r0 = c * 64;
      const int cnt = (int)((m - r0 < 64 ? m - r0 : 64) * B);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = lane + 64 * u;
        v[u] = (e < cnt) ? P[r0 * B + e] : zero<T>();
      }
    };
    T cur[B], acc[B];
    load(cur, ch, AV);
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = zero<T>();
    int p = 0;
    for (;;) {
      // the unit's values go to the slot, and the registers take the next
      // unit's loads, which stay in flight while this one is added
#pragma unroll
      for (int u = 0; u < B; ++u) slot[lane + 64 * u] = cur[u];
      int pn = p + 1;
      int64_t chn = ch;
      if (pn == np) {
        pn = 0;
        chn = ch + stride;
      }
      const bool more = chn < nchunk;
      if (more) load(cur, chn, pn == 0 ? AV : (pn == 1 ? P1 : P2));
      wave_lds_sync();
      // row values read back one at a time (a rolled loop keeps the
      // coefficient reads from being hoisted into registers)
      const T* Cp = Cm + p * B * B;
#pragma unroll 1
      for (int c = 0; c < B; ++c) {
        const T a = slot[lane * B + c];
#pragma unroll
        for (int j = 0; j < B; ++j) acc[j] = fmac(a, Cp[c * B + j], acc[j]);
      }
      wave_lds_sync();
      if (p == np - 1) {
        // the lane's output row through the slot, then coalesced stores
        const int64_t r0 = ch * 64;
        const int cnt = (int)((m - r0 < 64 ? m - r0 : 64) * B);
#pragma unroll
        for (int j = 0; j < B; ++j) slot[lane * B + j] = acc[j];
        wave_lds_sync();
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int e = lane + 64 * u;
          if (e < cnt) out[r0 * B + e] = slot[e];
        }
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < B; ++j) acc[j] = zero<T>();
      }
      if (!more) break;
      p = pn;
      ch = chn;
    }
  } else {
  const T* panels[3] = {AV, mode == 2 ? AX : (mode == 1 ? AW : nullptr), mode == 2 ? AW : nullptr};
  for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunk; ch += (int64_t)gridDim.x * 4) {
    const int64_t r0 = ch * 64;
    const int cnt = (int)((m - r0 < 64 ? m - r0 : 64) * B);  // values of the chunk per panel
    T at[3 * B];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const T* P = panels[p];
      if (P != nullptr) {
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int e = lane + 64 * u;
          slot[e] = (e < cnt) ? P[r0 * B + e] : zero<T>();
        }
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < B; ++j) at[p * B + j] = slot[lane * B + j];
        wave_lds_sync();
      } else {
#pragma unroll
        for (int j = 0; j < B; ++j) at[p * B + j] = zero<T>();
      }
    }
    // the lane's output row through the slot, then coalesced stores
    auto emit = [&](const T* Cm, T* out) {
#pragma unroll(B <= 2 ? B : 1)
      for (int j = 0; j < B; ++j) {
        T sv = zero<T>();
#pragma unroll
        for (int c = 0; c < 3 * B; ++c) sv = fmac(at[c], Cm[c * B + j], sv);
        slot[lane * B + j] = sv;
      }
      wave_lds_sync();
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = lane + 64 * u;
        if (e < cnt) out[r0 * B + e] = slot[e];
      }
      wave_lds_sync();
    };
    if (vupd) emit(CV, AVout);
    if (xupd) emit(CX, AX);
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

// Partial records: the r2 pass writes one per workgroup, the generic passes
// one per wave; the workspace holds the larger of the two.
static int64_t astream_max_parts(int64_t m, int n, int B, int es_d) {
  const int64_t g = astream_blocks(m, n, B, es_d) * 4;
  const int64_t r = astream_r2_blocks(m);
  const int64_t c = astream_cs_blocks(m, n);
  const int64_t cc = std::max(std::max(astream_ccs_ranges(m, n, B, true), astream_ccs_ranges(m, n, B, false)),
                              astream_c2_ranges(m, n, B));
  return std::max(std::max(g, cc), std::max(r, c));
}

// Compute units and the largest dynamic LDS a workgroup may take, per device
// (queried once per device).
static int g_cu[64];
static int64_t g_lds[64];
static void device_caps(int* cu, int64_t* lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    *cu = 256;
    *lds = 64 * 1024;
    return;
  }
  if (g_cu[dev] == 0) {
    int c = 0, l = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
    if (hipDeviceGetAttribute(&l, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || l < 1)
      l = 64 * 1024;
    g_lds[dev] = std::min<int64_t>(l, 160 * 1024);
    g_cu[dev] = c;
  }
  *cu = g_cu[dev];
  *lds = g_lds[dev];
}
int device_cu_count() {
  int c;
  int64_t l;
  device_caps(&c, &l);
  return c;
}
int64_t device_lds_max() {
  int c;
  int64_t l;
  device_caps(&c, &l);
  return l;
}

// Whether a pass kernel takes the shape: all of them cover n <= 1024 with
// b <= 10; the real matrix-core pass also covers even n <= 2048 with plain
// sums and 16-byte aligned rows (W in LDS: n b doubles, at most 160 KB).
bool astream_shape_ok(bool cplx, bool dot2, int64_t n, int B, const void* A, int64_t lda) {
  if (n < 1 || B < 1 || B > 10) return false;
  if (n <= 1024) return true;
  const bool aligned = (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  return !cplx && !dot2 && n <= 2048 && astream_rm_fits(B, (int)n, aligned, 160 * 1024);
}

// The pass kernels of this shape read A twice (the matrix-core pair), so the
// loop takes the late-residual form: A W alone, the Rayleigh-Ritz, then
// A^* A_{V_{i+1}} alone.
bool astream_late_residual(bool cplx, bool dot2, int n, int B, const void* A, int64_t lda) {
  if (dot2) return false;
  const bool aligned16 = ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool aligned = (lda % 2 == 0) && aligned16;
  if (cplx) return astream_zm_fits(B, n, aligned16, device_lds_max());
  return astream_rm_fits(B, n, aligned, device_lds_max());
}

// A W alone on the late-residual path.
hipError_t launch_astream_aw(hipStream_t st, bool cplx, int B, const void* A, int64_t lda, int64_t m, int n,
                             const void* W, void* AW, const Ctl* ctl) {
  if (!dispatch_zm_aw_only(cplx, B, st, A, lda, m, n, W, AW, device_cu_count(), ctl)) return hipErrorInvalidValue;
  return hipGetLastError();
}

// A^* P0 alone (plane 0 of the partial records; *np_out records).
hipError_t launch_astream_gram(hipStream_t st, bool cplx, int B, const void* A, int64_t lda, int64_t m, int n,
                               const void* P0, double* Gpart, const Ctl* ctl, int64_t* np_out) {
  const int64_t nb = astream_c2_ranges(m, n, B);
  if (!dispatch_zm_gram(cplx, B, st, nb, A, lda, m, n, P0, Gpart, ctl)) return hipErrorInvalidValue;
  *np_out = nb;
  return hipGetLastError();
}

int64_t astream_part_doubles(int64_t m, int n, int B, int es_d) {
  return astream_max_parts(m, n, B, es_d) * 4 * (int64_t)n * B * es_d;
}

int64_t astream_tmp_doubles(int64_t m, int n, int B, int es_d) {
  const int64_t groups = (astream_max_parts(m, n, B, es_d) + 63) / 64;
  return 4 * groups * 3 * (int64_t)n * B * es_d;
}

// One pass: AW = A W and G3 = A^* [AVp AXp AW] (n x 3B, contiguous; init: G3[:, 0:B] = A^* AW).
// The pass kernels: AW = A W and the per-workgroup partial column sums of
// A^* [AVp AXp AW] (init: A^* AW); *np_out receives the number of partial
// records for launch_astream_reduce.
hipError_t launch_astream_pass(hipStream_t st, bool cplx, int B, bool dot2, const void* A, int64_t lda, int64_t m,
                               int n, const void* W, void* AW, const void* AVp, const void* AXp, int init,
                               double* Gpart, const Ctl* ctl, int64_t* np_out, hipEvent_t mid,
                               bool* mid_recorded) {
  if (mid_recorded != nullptr) *mid_recorded = false;
  const int es_d = cplx ? 2 : 1;
  const int ns = astream_ns(n);
  int64_t nb = astream_blocks(m, n, B, es_d);
  int64_t np = nb * 4;  // partial records
  bool ok;
  const bool aligned = (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (!cplx && astream_r2_fits(B, n, aligned, m, lda)) {
    nb = astream_r2_blocks(m);
    np = nb;
    ok = dispatch_astream_r2(dot2, init, B, st, nb, (const double*)A, lda, m, n, (const double*)W, (double*)AW,
                             (const double*)AVp, (const double*)AXp, Gpart, ctl);
  } else if (!cplx && astream_cs_fits(B, n, aligned)) {
    nb = astream_cs_blocks(m, n);
    np = nb;
    ok = dispatch_astream_cs(dot2, init, B, st, nb, (const double*)A, lda, m, n, (const double*)W, (double*)AW,
                             (const double*)AVp, (const double*)AXp, Gpart, ctl);
  } else if (cplx && !dot2 && astream_zm_fits(B, n, ((reinterpret_cast<uintptr_t>(A) & 15) == 0),
                                                device_lds_max())) {
    // plain sums: the two contractions on the FP64 matrix cores
    nb = astream_c2_ranges(m, n, B);
    np = nb;
    ok = dispatch_astream_zm(init, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, Gpart, device_cu_count(), ctl, mid);
    if (ok && mid != nullptr && mid_recorded != nullptr) *mid_recorded = true;
  } else if (!cplx && !dot2 && astream_rm_fits(B, n, aligned, device_lds_max())) {
    // real, 1024 < n <= 2048, plain sums: the same two matrix-core kernels
    nb = astream_c2_ranges(m, n, B);
    np = nb;
    ok = dispatch_astream_rm(init, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, Gpart, device_cu_count(), ctl, mid);
    if (ok && mid != nullptr && mid_recorded != nullptr) *mid_recorded = true;
  } else if (cplx && astream_c2_fits(B, n, ((reinterpret_cast<uintptr_t>(A) & 15) == 0))) {
    nb = astream_c2_ranges(m, n, B);
    np = nb;
    ok = dispatch_astream_c2(dot2, init, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  } else if (cplx && astream_ccs_fits(B, n, ((reinterpret_cast<uintptr_t>(A) & 15) == 0))) {
    nb = astream_ccs_ranges(m, n, B, dot2);
    np = nb;
    ok = dispatch_astream_ccs(dot2, init, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, Gpart, ctl);
  } else if (cplx)
    ok = dispatch_astream_gc(dot2, ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  else
    ok = dispatch_astream_gd(dot2, ns, B, st, nb, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl);
  if (!ok) return hipErrorInvalidValue;
  *np_out = np;
  return hipGetLastError();
}

// The levels of the compensated reduction of the np partial records into G3
// (n x 3B): level 0 reads the records, each later level the previous level's
// (sum, error) pairs, the last writes G3.  Returns the number of levels.
// first_only: only the first plane of each record is read (its error plane
// is not), and only G3's first block is written (the Gram pass alone).
int astream_reduce_plan(bool cplx, int B, int n, int64_t np, const double* Gpart, double* tmp, double* G3,
                        const Ctl* ctl, ColsumJob* lev, int maxlev, bool first_only) {
  const int es_d = cplx ? 2 : 1;
  const int64_t plen = (int64_t)n * B * es_d;
  const int64_t len = first_only ? plen : 3 * plen;
  const int64_t g1 = (np + 63) / 64;
  const double* cur_s = Gpart;
  const double* cur_e = Gpart + 3 * plen;
  int64_t stride = 4 * plen, elen = first_only ? 0 : plen;
  int flip = 0, nl = 0;
  while (nl < maxlev) {
    const int64_t groups = (np + 63) / 64;
    double* ds = tmp + (int64_t)flip * 2 * g1 * len;
    double* de = ds + g1 * len;
    ColsumJob& J = lev[nl++];
    J = ColsumJob{cur_s, cur_e, stride, elen, np, len, ds, de, groups == 1 ? G3 : nullptr, ctl,
                  (int)((len + 63) / 64), (int)groups};
    if (groups == 1) return nl;
    cur_s = ds;
    cur_e = de;
    stride = len;
    elen = len;
    np = groups;
    flip ^= 1;
  }
  return -1;
}

hipError_t launch_colsum_job(hipStream_t st, const ColsumJob& J) {
  hipLaunchKernelGGL(k_colsum2, dim3((unsigned)J.gx, (unsigned)J.gy), dim3(256), 0, st, J);
  return hipGetLastError();
}

hipError_t launch_astream_reduce(hipStream_t st, bool cplx, int B, int n, int64_t np, const double* Gpart,
                                 double* tmp, double* G3, const Ctl* ctl, bool first_only) {
  ColsumJob lev[16];
  const int nl = astream_reduce_plan(cplx, B, n, np, Gpart, tmp, G3, ctl, lev, 16, first_only);
  if (nl < 1) return hipErrorInvalidValue;
  for (int i = 0; i < nl; ++i) {
    const hipError_t e = launch_colsum_job(st, lev[i]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_astream(hipStream_t st, bool cplx, int B, bool dot2, const void* A, int64_t lda, int64_t m, int n,
                          const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                          double* tmp, double* G3, const Ctl* ctl, hipEvent_t pass_done) {
  int64_t np = 0;
  hipError_t e = launch_astream_pass(st, cplx, B, dot2, A, lda, m, n, W, AW, AVp, AXp, init, Gpart, ctl, &np);
  if (e != hipSuccess) return e;
  // the pass itself ends here (timing of the pass kernels alone)
  if (pass_done != nullptr) {
    e = hipEventRecord(pass_done, st);
    if (e != hipSuccess) return e;
  }
  return launch_astream_reduce(st, cplx, B, n, np, Gpart, tmp, G3, ctl);
}

template <typename T, int B>
static void panel_go(hipStream_t st, int64_t nb, const void* AV, void* AVout, void* AX, const void* AW, int64_t m,
                     const void* CV, const void* CX, const Ctl* ctl, int pmode) {
  if (pmode == 0)
    hipLaunchKernelGGL((k_panel<T, B, false>), dim3((unsigned)nb), dim3(256), 0, st, (const T*)AV, (T*)AVout,
                       (T*)AX, (const T*)AW, m, (const T*)CV, (const T*)CX, ctl, pmode);
  else
    hipLaunchKernelGGL((k_panel<T, B, true>), dim3((unsigned)nb), dim3(256), 0, st, (const T*)AV, (T*)AVout,
                       (T*)AX, (const T*)AW, m, (const T*)CV, (const T*)CX, ctl, pmode);
}

template <typename T>
static bool panel_by_b(int B, hipStream_t st, int64_t nb, const void* AV, void* AVout, void* AX, const void* AW,
                       int64_t m, const void* CV, const void* CX, const Ctl* ctl, int pmode) {
  switch (B) {
#define RL_CASE(BB) \
  case BB: panel_go<T, BB>(st, nb, AV, AVout, AX, AW, m, CV, CX, ctl, pmode); return true;
    RL_CASE(1) RL_CASE(2) RL_CASE(3) RL_CASE(4) RL_CASE(5)
    RL_CASE(6) RL_CASE(7) RL_CASE(8) RL_CASE(9) RL_CASE(10)
#undef RL_CASE
    default: return false;
  }
}

hipError_t launch_panel(hipStream_t st, bool cplx, void* AV, void* AX, const void* AW, int64_t m, int B,
                        const void* CV, const void* CX, const Ctl* ctl, int pmode, void* AVout) {
  int64_t nb = (m + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (pmode == 1 && (AVout == nullptr || AVout == AV)) return hipErrorInvalidValue;
  void* out = (pmode == 1) ? AVout : AV;
  const bool ok = cplx ? panel_by_b<cd>(B, st, nb, AV, out, AX, AW, m, CV, CX, ctl, pmode)
                       : panel_by_b<double>(B, st, nb, AV, out, AX, AW, m, CV, CX, ctl, pmode);
  if (!ok) return hipErrorInvalidValue;
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

// Outputs of the refresh step (the fresh A V-hat and its thin SVD,
// A V-hat = U_r diag(s) C^*): V-hat C, sigma = s and U-hat = (A V-hat) C / s,
// the k smallest in ascending order (s and C come descending from the SVD of
// the TSQR factor: column B-1-j holds the j-th smallest).
template <typename T>
__global__ __launch_bounds__(256) void k_refresh_v(int n, int B, int k, const T* __restrict__ V,
                                                   const T* __restrict__ C, const double* __restrict__ s,
                                                   double* __restrict__ sigma, T* __restrict__ Vout, int64_t ldv,
                                                   Ctl* __restrict__ ctl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < k) {
    const double sj = s[B - 1 - idx];
    sigma[idx] = sj;
    if (sj == 0.0) ctl->zero_theta = 1;
  }
  if (idx < (int64_t)n * k) {
    const int64_t r = idx / k;
    const int j = B - 1 - (int)(idx % k);
    T acc = zero<T>();
    for (int c = 0; c < B; ++c) acc = fmac(V[r * B + c], C[c * B + j], acc);
    Vout[r * ldv + (idx % k)] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_refresh_u(int64_t m, int B, int k, const T* __restrict__ AVf,
                                                   const T* __restrict__ Cg, const double* __restrict__ s,
                                                   T* __restrict__ U, int64_t ldu) {
  __shared__ T C[16 * 16];
  __shared__ double inv[16];
  for (int i = threadIdx.x; i < B * B; i += blockDim.x) C[i] = Cg[i];
  if (threadIdx.x < B) inv[threadIdx.x] = (s[threadIdx.x] != 0.0) ? 1.0 / s[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    T a[16];
    for (int c = 0; c < B; ++c) a[c] = AVf[r * B + c];
    for (int jo = 0; jo < k; ++jo) {
      const int j = B - 1 - jo;
      T acc = zero<T>();
      for (int c = 0; c < B; ++c) acc = fmac(a[c], C[c * B + j], acc);
      U[r * ldu + jo] = scal(acc, inv[j]);
    }
  }
}

hipError_t launch_refresh_out(hipStream_t st, bool cplx, int n, int64_t m, int B, int k, const void* V,
                              const void* AVf, const void* C, const double* s, double* sigma, void* Vout,
                              int64_t ldv, void* U, int64_t ldu, Ctl* ctl) {
  if (B < 1 || B > 16 || k < 1 || k > B) return hipErrorInvalidValue;
  const int gv = (int)(((int64_t)n * k + 255) / 256);
  int64_t gu = (m + 255) / 256;
  if (gu > 2048) gu = 2048;
  if (cplx) {
    hipLaunchKernelGGL(k_refresh_v<cd>, dim3(gv), dim3(256), 0, st, n, B, k, (const cd*)V, (const cd*)C, s, sigma,
                       (cd*)Vout, ldv, ctl);
    if (U != nullptr)
      hipLaunchKernelGGL(k_refresh_u<cd>, dim3((unsigned)gu), dim3(256), 0, st, m, B, k, (const cd*)AVf,
                         (const cd*)C, s, (cd*)U, ldu);
  } else {
    hipLaunchKernelGGL(k_refresh_v<double>, dim3(gv), dim3(256), 0, st, n, B, k, (const double*)V,
                       (const double*)C, s, sigma, (double*)Vout, ldv, ctl);
    if (U != nullptr)
      hipLaunchKernelGGL(k_refresh_u<double>, dim3((unsigned)gu), dim3(256), 0, st, m, B, k, (const double*)AVf,
                         (const double*)C, s, (double*)U, ldu);
  }
  return hipGetLastError();
}

}  // namespace rl
