// Host orchestration of RLOBPCG on one gfx950 GPU and the C-ABI of
// include/rlobpcg.h.
//
// One solve (paper Sec. 1 steps 1-4; Alg. rlopcg / Alg. rlobpcg):
//   setup  sketch S*A (one pass over A) -> Householder QR -> R, R^{-1}
//          -> Sigma~(1,1) by Golub-Kahan-Lanczos on R
//          -> start block: the smallest-b right singular subspace of R (= of
//             S*A) by inverse subspace iteration with R^{-1} R^{-*}
//          -> A_V = A V_0 and G_V = A^* A_V (one pass over A)
//          -> Rayleigh-Ritz of A_V (b > 1 rotates V_0, A_V; b = 1 keeps v_0)
//          -> R_0 = G_V - V_0 Theta^2
//   loop   i = 0, 1, ...:
//            A_V, A_X <- A_T C (coefficients of the previous Rayleigh-Ritz)
//            W = R^{-1} (R^{-*} R_i)                       (eq:search-direction)
//            BCGS2 of W against [V X], Orth(W)
//            A_W = A W and G_W = A^* A_W                   (one pass over A)
//            TSQR of A_T = [A_V A_X A_W] -> R_T; Jacobi SVD -> Theta, C
//            V, G_V, R_{i+1}, stop rule, Q, X, G_X         (k_rr)
//          The stop decision lives on the device (Ctl::done); every kernel of
//          later iterations returns at once once it is set.  The host reads the
//          flag only at iterations where the rule can fire.
//   final  sigma ascending, V, and U = A_T C_V / theta.
//
// All device memory besides the caller's A and outputs is one workspace per
// handle, grown on demand.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rlobpcg.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace rl;

struct rl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Ctl* host_ctl = nullptr;      // pinned, mapped host memory
  Ctl* host_ctl_dev = nullptr;  // its device address
  int64_t lds_budget = 64 * 1024;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> prof;  // triples around A-stream launches: start, mid (two-kernel passes), end
  std::vector<char> prof_mid;    // the launch recorded its mid event
  bool ws_async = false;         // workspace from the stream-ordered allocator (server slots)
  hipStream_t aux = nullptr;     // second stream: Sigma~(1,1) beside the start block
  hipEvent_t fork = nullptr, join = nullptr;
};

// The second stream and its fork/join events, created on first use.
static int ensure_aux(rl_ctx* h) {
  if (h->aux) return RL_OK;
  if (hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join, hipEventDisableTiming) != hipSuccess)
    return RL_ERR_DEVICE;
  if (hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) {
    h->aux = nullptr;
    return RL_ERR_DEVICE;
  }
  return RL_OK;
}

static int ensure_prof_events(rl_ctx* h, size_t launches) {
  if (h->prof_mid.size() < launches) h->prof_mid.resize(launches);
  while (h->prof.size() < 4 * launches) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return RL_ERR_DEVICE;
    h->prof.push_back(e);
  }
  return RL_OK;
}

static int rl_hip_fail(hipError_t, const char*) { return RL_ERR_DEVICE; }

namespace {

struct Arena {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    const size_t o = off;
    off += bytes;
    return o;
  }
};

struct Layout {
  size_t ctl, ht, hr, Y, Yf, Tmf, part, Tm, Rrow, RH, Rinv, RinvH;
  size_t V, X, W, Z, Vn, G3, Rres;
  size_t AV, AX, AW, Gpart, Gtmp, tsA, tsB, CV, CX, thb, Ub, Vb;
  size_t AV2, Cst;  // late-residual form: the other A_V buffer and the saved Rayleigh-Ritz data
  size_t dsc, cnp;  // diagonal preconditioner scales and their partial sums
  size_t total;
  int KL;
};

struct Problem {
  int64_t m, n, d;
  int B, k, zeta;
  bool cplx;
  size_t es;
  int max_iter;
  int sketch_prec;
  int loop_precond;
  bool late = false;  // the loop may take the late-residual form (two reads of A per iteration)
};

// Shapes whose loop may take the late-residual form (the pass kernels read A
// twice there); the workspace holds its second A_V buffer for all of them.
static bool late_shape(bool cplx, bool dot2, int64_t n) {
  return !dot2 && (cplx ? (n > 256 && n <= 1024) : (n > 1024 && n <= 2048));
}

static Layout plan(const Problem& p, int64_t lds_budget) {
  Layout L{};
  Arena a;
  const size_t es = p.es;
  const int64_t n = p.n, m = p.m, B = p.B;
  const int64_t ncols_d = n * (int64_t)(es / 8);
  int nchunk;
  int64_t rows;
  int64_t partd = sketch_partial_doubles(m, ncols_d, (int)p.d, lds_budget, &nchunk, &rows, 8);
  if (p.sketch_prec != RL_SKETCH_F64) {
    const int64_t pf = sketch_partial_doubles(m, ncols_d, (int)p.d, lds_budget, &nchunk, &rows, 4);
    partd = std::max<int64_t>(partd, (pf + 1) / 2);
  }
  L.ctl = a.take(sizeof(Ctl));
  L.ht = a.take(sizeof(double) * (size_t)(p.max_iter + 2) * B);
  L.hr = a.take(sizeof(double) * (size_t)(p.max_iter + 2) * B);
  L.Y = a.take(es * (size_t)p.d * n);
  if (p.sketch_prec != RL_SKETCH_F64) {
    L.Yf = a.take(sizeof(float) * (size_t)p.d * n);
    L.Tmf = a.take(sizeof(float) * QR_TM_ELEMS);
  }
  L.part = a.take(sizeof(double) * (size_t)std::max<int64_t>(partd, 1));
  L.Tm = a.take(es * QR_TM_ELEMS);
  L.Rrow = a.take(es * (size_t)n * n);
  L.RH = a.take(es * (size_t)n * n);
  L.Rinv = a.take(es * (size_t)n * n);
  L.RinvH = a.take(es * (size_t)n * n);
  const size_t nb = es * (size_t)n * B;
  L.V = a.take(nb);
  L.X = a.take(nb);
  L.W = a.take(nb);
  L.Z = a.take(nb);
  L.Vn = a.take(nb);
  L.G3 = a.take(3 * nb);
  L.Rres = a.take(nb);
  const size_t mb = es * (size_t)m * B;
  L.AV = a.take(mb);
  L.AX = a.take(mb);
  L.AW = a.take(mb);
  const int es_d = (int)(es / 8);
  L.Gpart = a.take(sizeof(double) * (size_t)astream_part_doubles(m, (int)n, (int)B, es_d));
  L.Gtmp = a.take(sizeof(double) * (size_t)astream_tmp_doubles(m, (int)n, (int)B, es_d));
  const int t = 3 * p.B;
  const int64_t g = tsqr_groups(std::max<int64_t>(m, 1), t);
  L.tsA = a.take(es * (size_t)g * t * t);
  L.tsB = a.take(es * (size_t)g * t * t);
  L.CV = a.take(es * 32 * 16);
  L.CX = a.take(es * 32 * 16);
  const bool diag = p.loop_precond == RL_PREC_DIAG;
  L.dsc = a.take(sizeof(double) * (size_t)(diag ? n : 1));
  L.cnp = a.take(sizeof(double) * (size_t)(diag ? colnorm_groups(m) * ncols_d : 1));
  L.thb = a.take(sizeof(double) * 32);
  L.AV2 = a.take(p.late ? mb : 256);
  L.Cst = a.take(sizeof(double) * RR_CST_DOUBLES);
  L.KL = (int)std::min<int64_t>(n, 64);
  L.Ub = a.take(es * (size_t)(L.KL + 1) * n);
  L.Vb = a.take(es * (size_t)(L.KL + 1) * n);
  L.total = a.off + 256;
  return L;
}

static int ensure_ws(rl_ctx* h, size_t bytes) {
  if (h->ws_bytes >= bytes) return RL_OK;
  if (h->ws_async) {
    // server slots: stream-ordered, so other slots' work is never waited on
    if (h->ws) (void)hipFreeAsync(h->ws, h->stream);
    h->ws = nullptr;
    h->ws_bytes = 0;
    if (hipMallocAsync(&h->ws, bytes, h->stream) != hipSuccess) {
      h->ws = nullptr;
      return RL_ERR_NOMEM;
    }
    h->ws_bytes = bytes;
    return RL_OK;
  }
  if (h->ws) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  if (hipMalloc(&h->ws, bytes) != hipSuccess) {
    h->ws = nullptr;
    return RL_ERR_NOMEM;
  }
  h->ws_bytes = bytes;
  return RL_OK;
}

static void release_ws(rl_ctx* h) {
  if (!h->ws) return;
  // work left on the second stream (a solve that returned early) finishes first
  if (h->aux) (void)hipStreamWaitEvent(h->stream, h->join, 0);
  if (h->ws_async) {
    (void)hipFreeAsync(h->ws, h->stream);
  } else {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->ws);
  }
  h->ws = nullptr;
  h->ws_bytes = 0;
}

template <typename P>
static inline P* at(void* base, size_t off) {
  return reinterpret_cast<P*>(static_cast<char*>(base) + off);
}

static int check_opts(int64_t m, int64_t n, int32_t k, const rl_opts& o) {
  if (m < 1 || n < 1 || k < 1) return RL_ERR_ARG;
  if (o.block < k || 3 * (int64_t)o.block > n || n > m) return RL_ERR_ARG;
  if (o.d < n || o.zeta < 1 || o.zeta > o.d) return RL_ERR_ARG;
  if (o.max_iter < 0 || o.check_every < 1) return RL_ERR_ARG;
  if (o.stop_rule < 0 || o.stop_rule > 2) return RL_ERR_ARG;
  if (o.init_iters < 0 || o.lanczos_steps < 1) return RL_ERR_ARG;
  if (o.sketch_prec < RL_SKETCH_F64 || o.sketch_prec > RL_SKETCH_BF16) return RL_ERR_ARG;
  if (o.loop_precond < RL_PREC_SKETCH || o.loop_precond > RL_PREC_NONE) return RL_ERR_ARG;
  if (o.orth < RL_ORTH_CGS2 || o.orth > RL_ORTH_SVQB) return RL_ERR_ARG;
  if (o.refresh < 0 || o.refresh > 1) return RL_ERR_ARG;
  if (o.prec_guard < 0 || o.prec_guard > 1) return RL_ERR_ARG;
  if (o.lock < 0 || o.lock > 1) return RL_ERR_ARG;
  if (o.lock && o.orth == RL_ORTH_SVQB) return RL_ERR_UNSUPPORTED;
  if (n > 2048 || o.block > 10) return RL_ERR_UNSUPPORTED;
  if (o.d > INT32_MAX / 2) return RL_ERR_ARG;
  return RL_OK;
}

#define CK(expr)                                 \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return RL_ERR_DEVICE;  \
  } while (0)

// Flags NaN/Inf among n doubles (R^{-1} of a numerically singular sketch).
__global__ void k_flag_nonfinite(const double* __restrict__ x, int64_t n, Ctl* __restrict__ ctl) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) {
      atomicOr(&ctl->nonfinite, 1);
      return;
    }
}

static int solve(rl_ctx* h, bool cplx, int64_t m, int64_t n, const void* A, int64_t lda, int32_t k,
                 const rl_opts* opts_in, double* sigma, void* Vout, int64_t ldv, void* Uout, int64_t ldu,
                 rl_info* info) {
  if (!h || !A || !sigma || !Vout) return RL_ERR_ARG;
  rl_opts o;
  if (opts_in) o = *opts_in;
  else rl_default_opts(&o, m, n, k);
  int rc = check_opts(m, n, k, o);
  if (rc != RL_OK) return rc;
  if (lda < n || ldv < k || (Uout && ldu < k)) return RL_ERR_ARG;
  if (cplx && o.sketch_prec != RL_SKETCH_F64) return RL_ERR_UNSUPPORTED;
  if (!astream_shape_ok(cplx, o.dot2 != 0, n, o.block, A, lda)) return RL_ERR_UNSUPPORTED;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  Problem p{m, n, o.d, o.block, k, o.zeta, cplx, (size_t)(cplx ? 16 : 8), o.max_iter, o.sketch_prec,
            o.loop_precond};
  p.late = late_shape(cplx, o.dot2 != 0, n);
  const Layout L = plan(p, h->lds_budget);
  // the pass reads A twice (matrix-core kernels): A W, the Rayleigh-Ritz, then
  // A^* A_{V_{i+1}} alone (a third of the Gram work of A^* [A_V A_X A_W])
  const bool late = p.late && astream_late_residual(cplx, o.dot2 != 0, (int)n, o.block, A, lda);
  // a previous solve that returned early may have left work on the second stream
  if (h->aux) CK(hipStreamWaitEvent(h->stream, h->join, 0));
  rc = ensure_ws(h, L.total);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  void* ws = h->ws;
  Ctl* ctl = at<Ctl>(ws, L.ctl);
  const int B = o.block;
  const bool dot2 = (o.dot2 != 0);
  const int es_d = cplx ? 2 : 1;

  // control block
  Ctl hc;
  memset(&hc, 0, sizeof(hc));
  hc.stop_rule = o.stop_rule;
  hc.check_every = o.check_every;
  hc.max_iter = o.max_iter;
  hc.b = B;
  hc.tau = o.tau;
  hc.status = 1;
  hc.lock = o.lock;
  hc.act = (1 << B) - 1;
  *h->host_ctl = hc;
  CK(hipEventRecord(h->ev[0], st));
  CK(launch_publish(st, h->host_ctl_dev, ctl));

  // Step 1-2: sketch and QR (fork: recorded once R is complete)
  rc = ensure_aux(h);
  if (rc != RL_OK) return rc;
  const double scale = 1.0 / sqrt((double)o.zeta);
  if (o.sketch_prec == RL_SKETCH_F64) {
    CK(launch_sketch(st, (const double*)A, lda * es_d, m, n * es_d, es_d, (int)o.d, o.zeta, o.seed, scale,
                     at<void>(ws, L.part), at<void>(ws, L.Y), ctl, h->lds_budget, false));
    CK(launch_qr(st, cplx, at<void>(ws, L.Y), (int)o.d, (int)n, at<void>(ws, L.Tm), at<void>(ws, L.Rrow),
                 at<void>(ws, L.RH), at<void>(ws, L.Rinv), at<void>(ws, L.RinvH), h->fork));
  } else {
    // reduced-precision sketch and QR; R is promoted to FP64 for everything after
    CK(launch_sketch(st, (const double*)A, lda, m, n, 1, (int)o.d, o.zeta, o.seed, scale, at<void>(ws, L.part),
                     at<void>(ws, L.Yf), ctl, h->lds_budget, true));
    CK(launch_qr_lowp(st, at<float>(ws, L.Yf), (int)o.d, (int)n, at<float>(ws, L.Tmf), at<double>(ws, L.Y),
                      at<double>(ws, L.Rrow), at<double>(ws, L.RH), at<double>(ws, L.Rinv), at<double>(ws, L.RinvH),
                      o.sketch_prec == RL_SKETCH_BF16, h->fork));
  }
  {
    const int64_t cnt = n * n * es_d;
    hipLaunchKernelGGL(k_flag_nonfinite, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 1024)), dim3(256), 0,
                       st, at<double>(ws, L.Rinv), cnt, ctl);
    CK(hipGetLastError());
  }
  // Sigma~(1,1) on the second stream from the moment R is complete (beside
  // the inverses and the start block): it only reads R and writes sigma1,
  // which the first stopping test needs
  CK(hipStreamWaitEvent(h->aux, h->fork, 0));
  const int KL = std::min<int>(L.KL, o.lanczos_steps);
  CK(launch_lanczos(h->aux, cplx, (int)n, at<void>(ws, L.Y), (int)o.d, at<void>(ws, L.Rrow), at<void>(ws, L.Ub),
                    at<void>(ws, L.Vb), KL, o.seed ^ 0xA5A5A5A5ull, ctl));
  CK(hipEventRecord(h->join, h->aux));
  // Step 3: start block from the smallest right singular subspace of R
  CK(launch_randblk(st, cplx, at<void>(ws, L.W), n * B, o.seed ^ 0x3C3C3C3Cull));
  CK(launch_orth(st, cplx, (int)n, B, nullptr, nullptr, 0, 0, at<void>(ws, L.W), ctl, 0));
  for (int it = 0; it < o.init_iters; ++it) {
    CK(launch_trmv(st, cplx, B, at<void>(ws, L.RinvH), (int)n, 1, at<void>(ws, L.W), at<void>(ws, L.Z), ctl, 0));
    CK(launch_trmv(st, cplx, B, at<void>(ws, L.Rinv), (int)n, 0, at<void>(ws, L.Z), at<void>(ws, L.W), ctl, 0));
    CK(launch_orth(st, cplx, (int)n, B, nullptr, nullptr, 0, 0, at<void>(ws, L.W), ctl, 0));
  }
  CK(hipMemcpyAsync(at<void>(ws, L.V), at<void>(ws, L.W), p.es * n * B, hipMemcpyDeviceToDevice, st));
  double kappa_est = 0.0;
  if (o.sketch_prec != RL_SKETCH_F64 && o.prec_guard) {
    // Reduced-precision guard: kappa(R) ~ ||R||_2 max_j ||R^{-*} V_0(:, j)||
    // (V_0 spans the smallest right singular vectors of R, so the second
    // factor estimates 1 / sigma_min(R)).  A reduced-precision R resolves the
    // directions of A only down to about u_low sqrt(n) ||A|| (its own
    // condition number saturates there), so once kappa u_low sqrt(n) > 0.1 it
    // no longer preconditions the bottom of the spectrum reliably, and the
    // sketch and QR are redone in FP64 before any pass of the loop is spent
    // on it.
    CK(launch_trmv(st, cplx, B, at<void>(ws, L.RinvH), (int)n, 1, at<void>(ws, L.V), at<void>(ws, L.Z), ctl, 0));
    CK(launch_max_colnorm(st, cplx, (int)n, B, at<void>(ws, L.Z), &ctl->rinv_norm));
    CK(hipStreamWaitEvent(st, h->join, 0));
    CK(launch_publish(st, ctl, h->host_ctl_dev));
    CK(hipStreamSynchronize(st));
    const double u_low = (o.sketch_prec == RL_SKETCH_BF16) ? 0x1p-8 : 0x1p-24;
    kappa_est = h->host_ctl->sigma1 * h->host_ctl->rinv_norm;
    if (!(kappa_est * u_low * sqrt((double)n) <= 0.1)) {
      float ms_low = 0.f;
      CK(hipEventRecord(h->ev[1], st));
      CK(hipEventSynchronize(h->ev[1]));
      (void)hipEventElapsedTime(&ms_low, h->ev[0], h->ev[1]);
      rl_opts o64 = o;
      o64.sketch_prec = RL_SKETCH_F64;
      const int r64 = solve(h, cplx, m, n, A, lda, k, &o64, sigma, Vout, ldv, Uout, ldu, info);
      if (info) {
        info->sketch_prec_used = RL_SKETCH_F64;
        info->kappa_est = kappa_est;
        info->a_passes += 1;                // the reduced-precision sketch
        info->t_setup_us += 1e3 * ms_low;  // and the rest of its setup
        info->bytes_a = (int64_t)info->a_passes * m * n * (int64_t)p.es;
      }
      return r64;
    }
  }
  const bool prof = o.profile != 0;
  int nprof = 0;
  if (prof) {
    rc = ensure_prof_events(h, (size_t)o.max_iter + 1);
    if (rc != RL_OK) return rc;
    CK(hipEventRecord(h->prof[4 * nprof], st));
    h->prof_mid[nprof] = 0;
  }
  // start pass: A_V = A V_0 and A^* A_V (into the first block of G3)
  CK(launch_astream(st, cplx, B, dot2, A, lda, m, (int)n, at<void>(ws, L.V), at<void>(ws, L.AV), nullptr, nullptr, 1,
                    at<double>(ws, L.Gpart), at<double>(ws, L.Gtmp), at<double>(ws, L.G3), ctl,
                    prof ? h->prof[4 * nprof + 3] : nullptr));
  if (prof) ++nprof;
  void* Rt = nullptr;
  CK(launch_tsqr(st, cplx, at<void>(ws, L.AV), B, nullptr, 0, nullptr, 0, m, at<void>(ws, L.tsA),
                 at<void>(ws, L.tsB), &Rt, ctl, 0));
  CK(launch_rr(st, cplx, (int)n, B, 1, 0, Rt, at<void>(ws, L.V), at<void>(ws, L.X), at<void>(ws, L.W),
               at<void>(ws, L.G3), at<void>(ws, L.Vn), at<void>(ws, L.Rres), at<void>(ws, L.CV), at<void>(ws, L.CX),
               at<double>(ws, L.thb), at<double>(ws, L.ht), at<double>(ws, L.hr), ctl));
  // diagonal loop preconditioner: one more pass over A for the column norms
  if (o.loop_precond == RL_PREC_DIAG)
    CK(launch_colnorm_scale(st, cplx, (const double*)A, lda * es_d, m, (int)n, at<double>(ws, L.cnp),
                            at<double>(ws, L.dsc)));
  CK(hipStreamWaitEvent(st, h->join, 0));
  CK(launch_publish(st, ctl, h->host_ctl_dev));
  CK(hipEventRecord(h->ev[1], st));
  CK(hipStreamSynchronize(st));
  if (h->host_ctl->nonfinite) return RL_ERR_NONFINITE;

  // Step 4: LOBPCG
  int it = 0;
  // late-residual form: A_V alternates between two buffers (the new one is
  // formed before the Gram pass, while the old one is still part of A_T)
  void* AVcur = at<void>(ws, L.AV);
  void* AVoth = at<void>(ws, L.AV2);
  for (; it < o.max_iter; ++it) {
    const bool x_beside = late && it > 0;
    if (x_beside) {
      // A_X <- A_T C_X with the previous iteration's A_T (its A_V is AVoth),
      // on the second stream beside the preconditioner and Orth, which touch
      // only n-side blocks; A W overwrites A_W, so it waits for the join
      CK(hipEventRecord(h->fork, st));
      CK(hipStreamWaitEvent(h->aux, h->fork, 0));
      CK(launch_panel(h->aux, cplx, AVoth, at<void>(ws, L.AX), at<void>(ws, L.AW), m, B, at<void>(ws, L.CV),
                      at<void>(ws, L.CX), ctl, 2));
      CK(hipEventRecord(h->join, h->aux));
    } else {
      CK(launch_panel(st, cplx, AVcur, at<void>(ws, L.AX), at<void>(ws, L.AW), m, B, at<void>(ws, L.CV),
                      at<void>(ws, L.CX), ctl));
    }
    if (o.loop_precond == RL_PREC_SKETCH) {
      CK(launch_trmv(st, cplx, B, at<void>(ws, L.RinvH), (int)n, 1, at<void>(ws, L.Rres), at<void>(ws, L.Z), ctl,
                     1));
      CK(launch_trmv(st, cplx, B, at<void>(ws, L.Rinv), (int)n, 0, at<void>(ws, L.Z), at<void>(ws, L.W), ctl, 1));
    } else {
      CK(launch_prec_apply(st, cplx, (int)n, B,
                           o.loop_precond == RL_PREC_DIAG ? at<double>(ws, L.dsc) : (const double*)nullptr,
                           at<void>(ws, L.Rres), at<void>(ws, L.W), ctl));
    }
    const int with_x = it > 0 ? 1 : 0;
    if (o.orth == RL_ORTH_SVQB)
      CK(launch_orth_svqb(st, cplx, (int)n, B, at<void>(ws, L.V), at<void>(ws, L.X), 1, with_x, at<void>(ws, L.W),
                          ctl, 1));
    else
      CK(launch_orth(st, cplx, (int)n, B, at<void>(ws, L.V), at<void>(ws, L.X), 1, with_x, at<void>(ws, L.W), ctl,
                     1, 1));
    if (x_beside) CK(hipStreamWaitEvent(st, h->join, 0));
    if (prof) CK(hipEventRecord(h->prof[4 * nprof], st));
    if (late) {
      // A W; TSQR of [A_V A_X A_W]; the Rayleigh-Ritz and V_new; the new
      // A_V = A_T C_V; A^* A_V (the Gram pass) reduced into G3's first block;
      // then the residual, the stopping rule, X and V <- V_new
      CK(launch_astream_aw(st, cplx, B, A, lda, m, (int)n, at<void>(ws, L.W), at<void>(ws, L.AW), ctl));
      if (prof) CK(hipEventRecord(h->prof[4 * nprof + 1], st));
      CK(launch_tsqr(st, cplx, AVcur, B, with_x ? at<void>(ws, L.AX) : nullptr, with_x ? B : 0, at<void>(ws, L.AW),
                     B, m, at<void>(ws, L.tsA), at<void>(ws, L.tsB), &Rt, ctl, 1));
      CK(launch_rr(st, cplx, (int)n, B, 0, with_x, Rt, at<void>(ws, L.V), at<void>(ws, L.X), at<void>(ws, L.W),
                   at<void>(ws, L.G3), at<void>(ws, L.Vn), at<void>(ws, L.Rres), at<void>(ws, L.CV),
                   at<void>(ws, L.CX), at<double>(ws, L.thb), at<double>(ws, L.ht), at<double>(ws, L.hr), ctl, 1,
                   at<double>(ws, L.Cst)));
      CK(launch_panel(st, cplx, AVcur, at<void>(ws, L.AX), at<void>(ws, L.AW), m, B, at<void>(ws, L.CV),
                      at<void>(ws, L.CX), ctl, 1, AVoth));
      int64_t np = 0;
      if (prof) CK(hipEventRecord(h->prof[4 * nprof + 2], st));
      CK(launch_astream_gram(st, cplx, B, A, lda, m, (int)n, AVoth, at<double>(ws, L.Gpart), ctl, &np));
      if (prof) {
        CK(hipEventRecord(h->prof[4 * nprof + 3], st));
        h->prof_mid[nprof] = 2;
        ++nprof;
      }
      CK(launch_astream_reduce(st, cplx, B, (int)n, np, at<double>(ws, L.Gpart), at<double>(ws, L.Gtmp),
                               at<double>(ws, L.G3), ctl, true));
      CK(launch_rr(st, cplx, (int)n, B, 0, with_x, Rt, at<void>(ws, L.V), at<void>(ws, L.X), at<void>(ws, L.W),
                   at<void>(ws, L.G3), at<void>(ws, L.Vn), at<void>(ws, L.Rres), at<void>(ws, L.CV),
                   at<void>(ws, L.CX), at<double>(ws, L.thb), at<double>(ws, L.ht), at<double>(ws, L.hr), ctl, 2,
                   at<double>(ws, L.Cst)));
      std::swap(AVcur, AVoth);
    } else {
    // the pass, then its partial sums reduced beside the TSQR of [A_V A_X A_W]
    // (the first reduction level runs inside the first TSQR launch)
    int64_t np = 0;
    bool mid = false;
    CK(launch_astream_pass(st, cplx, B, dot2, A, lda, m, (int)n, at<void>(ws, L.W), at<void>(ws, L.AW),
                           AVcur, with_x ? at<void>(ws, L.AX) : nullptr, 0, at<double>(ws, L.Gpart),
                           ctl, &np, prof ? h->prof[4 * nprof + 1] : nullptr, &mid));
    if (prof) {
      CK(hipEventRecord(h->prof[4 * nprof + 3], st));
      h->prof_mid[nprof] = mid ? 1 : 0;
      ++nprof;
    }
    ColsumJob lev[16];
    const int nlev = astream_reduce_plan(cplx, B, (int)n, np, at<double>(ws, L.Gpart), at<double>(ws, L.Gtmp),
                                         at<double>(ws, L.G3), ctl, lev, 16);
    if (nlev < 1) return RL_ERR_DEVICE;
    CK(launch_tsqr(st, cplx, at<void>(ws, L.AV), B, with_x ? at<void>(ws, L.AX) : nullptr, with_x ? B : 0,
                   at<void>(ws, L.AW), B, m, at<void>(ws, L.tsA), at<void>(ws, L.tsB), &Rt, ctl, 1, &lev[0]));
    for (int q = 1; q < nlev; ++q) CK(launch_colsum_job(st, lev[q]));
    CK(launch_rr(st, cplx, (int)n, B, 0, with_x, Rt, at<void>(ws, L.V), at<void>(ws, L.X), at<void>(ws, L.W),
                 at<void>(ws, L.G3), at<void>(ws, L.Vn), at<void>(ws, L.Rres), at<void>(ws, L.CV), at<void>(ws, L.CX),
                 at<double>(ws, L.thb), at<double>(ws, L.ht), at<double>(ws, L.hr), ctl));
    }
    const bool can_stop = (o.stop_rule == RL_STOP_TOL) || (o.stop_rule == RL_STOP_PAPER && it % o.check_every == 0);
    if (can_stop) {
      CK(launch_publish(st, ctl, h->host_ctl_dev));
      CK(hipStreamSynchronize(st));
      if (h->host_ctl->done) {
        ++it;
        break;
      }
    }
  }
  CK(hipEventRecord(h->ev[2], st));
  // outputs
  if (o.refresh) {
    // Refresh: A V-hat afresh in one pass (no accumulated drift of the
    // maintained products), the thin SVD of that m x b block (TSQR, then
    // one-sided Jacobi of its b x b factor), and (V-hat, sigma, U-hat)
    // rotated by its right singular vectors.  The loop's kernels stop at the
    // device stop flag, so this pass and its TSQR run without it.
    CK(launch_astream(st, cplx, B, dot2, A, lda, m, (int)n, at<void>(ws, L.V), at<void>(ws, L.AW), nullptr, nullptr,
                      1, at<double>(ws, L.Gpart), at<double>(ws, L.Gtmp), at<double>(ws, L.G3), nullptr));
    void* Rr = nullptr;
    CK(launch_tsqr(st, cplx, at<void>(ws, L.AW), B, nullptr, 0, nullptr, 0, m, at<void>(ws, L.tsA),
                   at<void>(ws, L.tsB), &Rr, ctl, 0));
    CK(launch_rt_svd(st, cplx, B, Rr, at<double>(ws, L.thb), at<void>(ws, L.CV)));
    CK(launch_refresh_out(st, cplx, (int)n, m, B, k, at<void>(ws, L.V), at<void>(ws, L.AW), at<void>(ws, L.CV),
                          at<double>(ws, L.thb), sigma, Vout, ldv, Uout, ldu, ctl));
  } else {
    CK(launch_final_n(st, cplx, (int)n, B, k, at<void>(ws, L.V), at<double>(ws, L.thb), sigma, Vout, ldv, ctl));
    void* AVlast = at<void>(ws, L.AV);
    if (late && Uout) {
      // the A_V of the last Rayleigh-Ritz's A_T: iteration j (counted on the
      // device; iterations queued after the stop flag did nothing) used
      // L.AV for even j and L.AV2 for odd j
      CK(launch_publish(st, ctl, h->host_ctl_dev));
      CK(hipStreamSynchronize(st));
      const int done_iters = h->host_ctl->iter;
      if (done_iters > 0 && ((done_iters - 1) & 1)) AVlast = at<void>(ws, L.AV2);
    }
    if (Uout)
      CK(launch_final_u(st, cplx, AVlast, at<void>(ws, L.AX), at<void>(ws, L.AW), m, B, k,
                        at<void>(ws, L.CV), at<double>(ws, L.thb), Uout, ldu, ctl));
  }
  CK(hipEventRecord(h->ev[3], st));
  CK(launch_publish(st, ctl, h->host_ctl_dev));
  CK(hipStreamSynchronize(st));
  const Ctl& fc = *h->host_ctl;
  const int status = fc.done ? RL_OK : RL_NOT_CONVERGED;
  if (info) {
    info->status = status;
    info->iters = fc.iter;
    info->a_passes = 2 + fc.iter + (o.loop_precond == RL_PREC_DIAG ? 1 : 0) + (o.refresh ? 1 : 0);
    info->degenerate = fc.degenerate;
    info->zero_theta = fc.zero_theta;
    info->block = B;
    info->sigma1 = fc.sigma1;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
    info->t_setup_us = 1e3 * ms;
    (void)hipEventElapsedTime(&ms, h->ev[1], h->ev[2]);
    info->t_iter_us = 1e3 * ms;
    (void)hipEventElapsedTime(&ms, h->ev[2], h->ev[3]);
    info->t_final_us = 1e3 * ms;
    info->bytes_a = (int64_t)info->a_passes * m * n * (int64_t)p.es;
    info->sketch_prec_used = o.sketch_prec;
    info->kappa_est = kappa_est;
    info->act_mask = fc.act;
    info->n_locked = o.lock ? B - __builtin_popcount((unsigned)fc.act) : 0;
    info->n_astream = prof ? nprof : 0;
    info->t_astream_us = 0.0;
    info->n_pass_g = 0;
    info->t_pass_g_us = 0.0;
    // events per launch: start, after A W, before the Gram kernel (late
    // form), end; prof_mid 0: one kernel, 1: A W then the Gram kernel back to
    // back, 2: the late form (its two reads apart)
    for (int q = 0; prof && q < nprof; ++q) {
      float ka = 0.f, kg = 0.f;
      if (h->prof_mid[q] == 2) {
        float k1 = 0.f;
        (void)hipEventElapsedTime(&k1, h->prof[4 * q], h->prof[4 * q + 1]);
        (void)hipEventElapsedTime(&kg, h->prof[4 * q + 2], h->prof[4 * q + 3]);
        ka = k1 + kg;
      } else {
        (void)hipEventElapsedTime(&ka, h->prof[4 * q], h->prof[4 * q + 3]);
        if (h->prof_mid[q]) (void)hipEventElapsedTime(&kg, h->prof[4 * q + 1], h->prof[4 * q + 3]);
      }
      info->t_astream_us += 1e3 * ka;
      if (h->prof_mid[q]) {
        info->t_pass_g_us += 1e3 * kg;
        ++info->n_pass_g;
      }
    }
    if (info->hist_cap > 0) {
      const int rowsh = std::min<int>(info->hist_cap, fc.iter + 1);
      if (info->theta_hist)
        CK(hipMemcpy(info->theta_hist, at<double>(ws, L.ht), sizeof(double) * rowsh * B, hipMemcpyDeviceToHost));
      if (info->rnorm_hist)
        CK(hipMemcpy(info->rnorm_hist, at<double>(ws, L.hr), sizeof(double) * rowsh * B, hipMemcpyDeviceToHost));
    }
  }
  return status;
}

// Workspace bytes one solve of this shape and these options needs (the
// server's admission unit).
static int64_t planned_bytes(bool cplx, int64_t m, int64_t n, int32_t k, const rl_opts& o, int64_t lds_budget) {
  Problem p{m, n, o.d, o.block, k, o.zeta, cplx, (size_t)(cplx ? 16 : 8), o.max_iter, o.sketch_prec,
            o.loop_precond};
  p.late = late_shape(cplx, o.dot2 != 0, n);
  return (int64_t)plan(p, lds_budget).total;
}

// Transpose a row-major d x n block (doubles per element es) into column-major.
__global__ void k_rowmajor_to_col_f(const float* __restrict__ Y, int64_t ldy, int64_t d, int64_t n,
                                    float* __restrict__ Yc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * n) return;
  const int64_t r = idx / n, c = idx % n;
  Yc[c * d + r] = Y[r * ldy + c];
}
__global__ void k_col_to_rowmajor_f(const float* __restrict__ Yc, int64_t d, int64_t n, float* __restrict__ Y,
                                    int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * n) return;
  const int64_t r = idx / n, c = idx % n;
  Y[r * ldy + c] = Yc[c * d + r];
}
__global__ void k_rowmajor_to_col(const double* __restrict__ Y, int64_t ldy, int64_t d, int64_t n, int es,
                                  double* __restrict__ Yc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * n * es) return;
  const int64_t comp = idx % es, e = idx / es;
  const int64_t r = e / n, c = e % n;
  Yc[(c * d + r) * es + comp] = Y[(r * ldy + c) * es + comp];
}
__global__ void k_col_to_rowmajor(const double* __restrict__ Yc, int64_t d, int64_t n, int es, double* __restrict__ Y,
                                  int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * n * es) return;
  const int64_t comp = idx % es, e = idx / es;
  const int64_t r = e / n, c = e % n;
  Y[(r * ldy + c) * es + comp] = Yc[(c * d + r) * es + comp];
}

}  // namespace

// ---------------------------------------------------------------------------
// Served form: continuous admission of solves of different shapes.
//
// A server owns `slots` worker threads; each has its own stream (default
// priority) and handle, so the solves in flight overlap on the device: the
// small latency-bound kernels of one solve run beside the A passes of
// another.  A submitted request waits in a FIFO queue; a free slot takes the
// head of the queue as soon as the planned workspaces of the solves in flight
// plus the head's fit the HBM budget.  Workspaces come from the
// stream-ordered allocator and are returned when the solve ends, so memory
// freed by one solve admits the next without a device-wide synchronisation.
// Every solve runs the same kernels in the same configuration as alone, so its
// results do not depend on what else is in flight.
struct rl_job {
  uint64_t ticket = 0;
  bool cplx = false;
  int64_t m = 0, n = 0, lda = 0, ldv = 0, ldu = 0;
  int32_t k = 0;
  const void* A = nullptr;
  double* sigma = nullptr;
  void* V = nullptr;
  void* U = nullptr;
  rl_opts opts{};
  int64_t bytes = 0;
  int status = RL_PENDING;
  bool done = false;
  rl_info info{};
  std::chrono::steady_clock::time_point t_submit, t_start, t_end;
};

struct rl_server {
  int device = 0;
  int64_t budget = 0;
  int64_t in_use = 0;
  int64_t lds_budget = 64 * 1024;
  bool stopping = false;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work;  // workers: a job may be admissible
  std::condition_variable cv_done;  // waiters: a job finished
  std::deque<rl_job*> queue;
  std::unordered_map<uint64_t, rl_job*> jobs;
  std::vector<std::thread> workers;
  std::vector<rl_ctx*> ctxs;
  std::vector<hipStream_t> streams;
};

static void server_worker(rl_server* s, int slot) {
  (void)hipSetDevice(s->device);
  rl_ctx* h = s->ctxs[slot];
  for (;;) {
    rl_job* job = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        if (s->queue.empty()) return s->stopping;
        return s->in_use + s->queue.front()->bytes <= s->budget;
      });
      if (s->queue.empty()) return;  // stopping and drained
      job = s->queue.front();
      s->queue.pop_front();
      s->in_use += job->bytes;
      job->t_start = std::chrono::steady_clock::now();
    }
    s->cv_work.notify_all();  // the next head may fit too
    rl_info info{};
    const int rc = solve(h, job->cplx, job->m, job->n, job->A, job->lda, job->k, &job->opts, job->sigma, job->V,
                         job->ldv, job->U, job->ldu, &info);
    release_ws(h);
    (void)hipStreamSynchronize(h->stream);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      job->info = info;
      job->status = rc;
      job->done = true;
      job->t_end = std::chrono::steady_clock::now();
      s->in_use -= job->bytes;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
}

static void fill_times(const rl_job* j, rl_job_times* t) {
  if (!t) return;
  using us = std::chrono::duration<double, std::micro>;
  t->queued_us = us(j->t_start - j->t_submit).count();
  t->run_us = us(j->t_end - j->t_start).count();
  t->latency_us = us(j->t_end - j->t_submit).count();
  t->workspace_bytes = j->bytes;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free pass (rl_step_astream_iter_noalloc): the
// per-workgroup partial records of one pass and the levels of their
// reduction.  Every GPU the library runs on holds its own copy from module
// load until the process ends.  In host code the symbol is only a stand-in:
// each device's address comes from hipGetSymbolAddress (resolved by
// rl_create with that device current) and only that address is ever passed
// to kernels.  No part of it needs to start at zero: each pass writes every
// record it later reads.
#define RL_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
#define RL_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[RL_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[RL_MAX_DEVICES] = {};

// Resolves the current device's scratch address once per device.
static int resolve_scratch(int device) {
  if (device < 0 || device >= RL_MAX_DEVICES) return RL_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return RL_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return RL_ERR_DEVICE;
  g_scratch_ptr[device] = p;
  return RL_OK;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= RL_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

extern "C" {

int rl_create(rl_handle* out, int device, void* stream) {
  if (!out) return RL_ERR_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return RL_ERR_DEVICE;
  const int src = resolve_scratch(device);
  if (src != RL_OK) return src;
  rl_ctx* h = new (std::nothrow) rl_ctx();
  if (!h) return RL_ERR_NOMEM;
  h->device = device;
  h->stream = (hipStream_t)stream;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    h->lds_budget = std::min<int64_t>(lds, 160 * 1024);
  if (hipHostMalloc((void**)&h->host_ctl, sizeof(Ctl), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete h;
    return RL_ERR_NOMEM;
  }
  if (hipHostGetDevicePointer((void**)&h->host_ctl_dev, h->host_ctl, 0) != hipSuccess) {
    (void)hipHostFree(h->host_ctl);
    delete h;
    return RL_ERR_DEVICE;
  }
  for (int i = 0; i < 4; ++i)
    if (hipEventCreate(&h->ev[i]) != hipSuccess) {
      rl_destroy(h);
      return RL_ERR_DEVICE;
    }
  *out = h;
  return RL_OK;
}

int rl_destroy(rl_handle h) {
  if (!h) return RL_OK;
  (void)hipSetDevice(h->device);
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->ws) (void)hipFree(h->ws);
  if (h->host_ctl) (void)hipHostFree(h->host_ctl);
  for (int i = 0; i < 4; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  for (hipEvent_t e : h->prof) (void)hipEventDestroy(e);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->fork) (void)hipEventDestroy(h->fork);
  if (h->join) (void)hipEventDestroy(h->join);
  delete h;
  return RL_OK;
}

int rl_set_stream(rl_handle h, void* stream) {
  if (!h) return RL_ERR_ARG;
  h->stream = (hipStream_t)stream;
  return RL_OK;
}

int rl_default_opts(rl_opts* o, int64_t m, int64_t n, int32_t k) {
  (void)m;
  if (!o) return RL_ERR_ARG;
  memset(o, 0, sizeof(*o));
  o->d = 4 * n;
  o->zeta = 8;
  o->block = k;
  o->seed = 0;
  o->tau = 2.0 * sqrt((double)n) * 2.220446049250313e-16;
  o->max_iter = (k == 1) ? 200 : 100;
  o->check_every = 5;
  o->stop_rule = RL_STOP_PAPER;
  o->dot2 = (n <= 1024) ? 1 : 0;  // wider real shapes run the plain-sum matrix-core pass
  o->init_iters = 10;
  o->lanczos_steps = 64;
  o->refresh = 1;
  o->prec_guard = 1;
  return RL_OK;
}

int rl_svds_smallest_d(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int32_t k,
                       const rl_opts* opts, double* sigma, double* V, int64_t ldv, double* U, int64_t ldu,
                       rl_info* info) {
  return solve(h, false, m, n, A, lda, k, opts, sigma, V, ldv, U, ldu, info);
}

int rl_svds_smallest_z(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int32_t k,
                       const rl_opts* opts, double* sigma, double* V, int64_t ldv, double* U, int64_t ldu,
                       rl_info* info) {
  return solve(h, true, m, n, A, lda, k, opts, sigma, V, ldv, U, ldu, info);
}

int rl_step_sketch(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t d,
                   int32_t zeta, uint64_t seed, double* Y, int64_t ldy) {
  if (!h || !A || !Y || m < 1 || n < 1 || lda < n || ldy < n || d < 1 || zeta < 1 || zeta > d) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  const int es = is_complex ? 2 : 1;
  int nchunk;
  int64_t rows;
  const int64_t partd = sketch_partial_doubles(m, n * es, (int)d, h->lds_budget, &nchunk, &rows, 8);
  if (partd < 0) return RL_ERR_UNSUPPORTED;
  Arena a;
  const size_t o_ctl = a.take(sizeof(Ctl)), o_part = a.take(sizeof(double) * partd),
               o_yc = a.take(sizeof(double) * (size_t)d * n * es);
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  CK(hipMemsetAsync(at<void>(h->ws, o_ctl), 0, sizeof(Ctl), st));
  CK(launch_sketch(st, A, lda * es, m, n * es, es, (int)d, zeta, seed, 1.0 / sqrt((double)zeta),
                   at<void>(h->ws, o_part), at<void>(h->ws, o_yc), at<Ctl>(h->ws, o_ctl), h->lds_budget, false));
  const int64_t tot = d * n * es;
  hipLaunchKernelGGL(k_col_to_rowmajor, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     at<double>(h->ws, o_yc), d, n, es, Y, ldy);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_qr(rl_handle h, int is_complex, int64_t d, int64_t n, const double* Y, int64_t ldy, double* R,
               double* Rinv) {
  if (!h || !Y || !R || !Rinv || n < 1 || d < n || ldy < n || n > 4096) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  const int es = is_complex ? 2 : 1;
  const size_t esb = 8 * (size_t)es;
  Arena a;
  const size_t o_yc = a.take(esb * d * n), o_tm = a.take(esb * QR_TM_ELEMS), o_rh = a.take(esb * n * n),
               o_rih = a.take(esb * n * n);
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  const int64_t tot = d * n * es;
  hipLaunchKernelGGL(k_rowmajor_to_col, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, ldy, d, n, es,
                     at<double>(h->ws, o_yc));
  CK(hipGetLastError());
  CK(launch_qr(st, is_complex != 0, at<void>(h->ws, o_yc), (int)d, (int)n, at<void>(h->ws, o_tm), R,
               at<void>(h->ws, o_rh), Rinv, at<void>(h->ws, o_rih)));
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_sketch_f32(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int64_t d, int32_t zeta,
                       uint64_t seed, float* Y, int64_t ldy) {
  if (!h || !A || !Y || m < 1 || n < 1 || lda < n || ldy < n || d < 1 || zeta < 1 || zeta > d) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  int nchunk;
  int64_t rows;
  const int64_t partf = sketch_partial_doubles(m, n, (int)d, h->lds_budget, &nchunk, &rows, 4);
  if (partf < 0) return RL_ERR_UNSUPPORTED;
  Arena a;
  const size_t o_ctl = a.take(sizeof(Ctl)), o_part = a.take(sizeof(float) * partf),
               o_yc = a.take(sizeof(float) * (size_t)d * n);
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  CK(hipMemsetAsync(at<void>(h->ws, o_ctl), 0, sizeof(Ctl), st));
  CK(launch_sketch(st, A, lda, m, n, 1, (int)d, zeta, seed, 1.0 / sqrt((double)zeta), at<void>(h->ws, o_part),
                   at<void>(h->ws, o_yc), at<Ctl>(h->ws, o_ctl), h->lds_budget, true));
  const int64_t tot = d * n;
  hipLaunchKernelGGL(k_col_to_rowmajor_f, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     at<float>(h->ws, o_yc), d, n, Y, ldy);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_qr_lowp(rl_handle h, int64_t d, int64_t n, const float* Y, int64_t ldy, int32_t sketch_prec, double* R,
                    double* Rinv) {
  if (!h || !Y || !R || !Rinv || n < 1 || d < n || ldy < n || n > 4096) return RL_ERR_ARG;
  if (sketch_prec != RL_SKETCH_F32 && sketch_prec != RL_SKETCH_BF16) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  Arena a;
  const size_t o_yf = a.take(sizeof(float) * d * n), o_tm = a.take(sizeof(float) * QR_TM_ELEMS),
               o_y = a.take(sizeof(double) * d * n), o_rh = a.take(sizeof(double) * n * n),
               o_rih = a.take(sizeof(double) * n * n);
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  const int64_t tot = d * n;
  hipLaunchKernelGGL(k_rowmajor_to_col_f, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, ldy, d, n,
                     at<float>(h->ws, o_yf));
  CK(hipGetLastError());
  CK(launch_qr_lowp(st, at<float>(h->ws, o_yf), (int)d, (int)n, at<float>(h->ws, o_tm), at<double>(h->ws, o_y), R,
                    at<double>(h->ws, o_rh), Rinv, at<double>(h->ws, o_rih), sketch_prec == RL_SKETCH_BF16));
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_astream(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int32_t b,
                    const double* W, double* AW, double* G, int32_t dot2) {
  if (!h || !A || !W || !AW || !G || m < 1 || n < 1 || lda < n || b < 1) return RL_ERR_ARG;
  if (!astream_shape_ok(is_complex != 0, dot2 != 0, n, b, A, lda)) return RL_ERR_UNSUPPORTED;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  const int es = is_complex ? 2 : 1;
  Arena a;
  const size_t o_part = a.take(sizeof(double) * astream_part_doubles(m, (int)n, b, es)),
               o_tmp = a.take(sizeof(double) * astream_tmp_doubles(m, (int)n, b, es)),
               o_g3 = a.take(sizeof(double) * 3 * (size_t)n * b * es);
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  CK(launch_astream(st, is_complex != 0, b, dot2 != 0, A, lda, m, (int)n, W, AW, nullptr, nullptr, 1,
                    at<double>(h->ws, o_part), at<double>(h->ws, o_tmp), at<double>(h->ws, o_g3), nullptr));
  CK(hipMemcpyAsync(G, at<double>(h->ws, o_g3), sizeof(double) * (size_t)n * b * es, hipMemcpyDeviceToDevice, st));
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_astream_iter(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int32_t b,
                         const double* W, const double* AV, const double* AX, double* AW, double* G3, int32_t dot2) {
  if (!h || !A || !W || !AV || !AW || !G3 || m < 1 || n < 1 || lda < n || b < 1) return RL_ERR_ARG;
  if (!astream_shape_ok(is_complex != 0, dot2 != 0, n, b, A, lda)) return RL_ERR_UNSUPPORTED;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  const int es = is_complex ? 2 : 1;
  Arena a;
  const size_t o_part = a.take(sizeof(double) * astream_part_doubles(m, (int)n, b, es)),
               o_tmp = a.take(sizeof(double) * astream_tmp_doubles(m, (int)n, b, es));
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  CK(launch_astream(st, is_complex != 0, b, dot2 != 0, A, lda, m, (int)n, W, AW, AV, AX, 0,
                    at<double>(h->ws, o_part), at<double>(h->ws, o_tmp), G3, nullptr));
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_astream_iter_noalloc(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda,
                                 int32_t b, const double* W, const double* AV, const double* AX, double* AW,
                                 double* G3, int32_t dot2) {
  if (!h || !A || !W || !AV || !AW || !G3 || m < 1 || n < 1 || lda < n || b < 1) return RL_ERR_ARG;
  if (!astream_shape_ok(is_complex != 0, dot2 != 0, n, b, A, lda)) return RL_ERR_UNSUPPORTED;
  const int es = is_complex ? 2 : 1;
  Arena a;
  const size_t o_part = a.take(sizeof(double) * astream_part_doubles(m, (int)n, b, es)),
               o_tmp = a.take(sizeof(double) * astream_tmp_doubles(m, (int)n, b, es));
  if (a.off > RL_NOALLOC_SCRATCH_BYTES) return RL_ERR_SCRATCH;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  void* base = scratch_of(h->device);
  if (base == nullptr) return RL_ERR_DEVICE;
  CK(launch_astream(h->stream, is_complex != 0, b, dot2 != 0, A, lda, m, (int)n, W, AW, AV, AX, 0,
                    at<double>(base, o_part), at<double>(base, o_tmp), G3, nullptr));
  return RL_OK;
}

int rl_step_tall_svd(rl_handle h, int is_complex, int64_t m, int32_t t, const double* P, double* sigma, double* C) {
  if (!h || !P || !sigma || !C || m < 1 || t < 1 || t > 32) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  const size_t esb = is_complex ? 16 : 8;
  const int64_t g = tsqr_groups(m, t);
  Arena a;
  const size_t o_a = a.take(esb * g * t * t), o_b = a.take(esb * g * t * t), o_ctl = a.take(sizeof(Ctl));
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  CK(hipMemsetAsync(at<void>(h->ws, o_ctl), 0, sizeof(Ctl), st));
  void* Rt = nullptr;
  CK(launch_tsqr(st, is_complex != 0, P, t, nullptr, 0, nullptr, 0, m, at<void>(h->ws, o_a), at<void>(h->ws, o_b),
                 &Rt, at<Ctl>(h->ws, o_ctl), 0));
  CK(launch_rt_svd(st, is_complex != 0, t, Rt, sigma, C));
  CK(hipStreamSynchronize(st));
  return RL_OK;
}

int rl_step_orth(rl_handle h, int is_complex, int64_t n, int32_t b, const double* V, const double* X,
                 int32_t project, int32_t with_x, double* W, int32_t* degenerate) {
  if (!h || !W || !degenerate || n < 1 || n > INT32_MAX || b < 1 || b > 16) return RL_ERR_ARG;
  if (project && (!V || (with_x && !X))) return RL_ERR_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return RL_ERR_DEVICE;
  Arena a;
  const size_t o_ctl = a.take(sizeof(Ctl));
  int rc = ensure_ws(h, a.off + 256);
  if (rc != RL_OK) return rc;
  hipStream_t st = h->stream;
  Ctl* ctl = at<Ctl>(h->ws, o_ctl);
  CK(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
  CK(launch_orth(st, is_complex != 0, (int)n, b, V, project ? X : nullptr, project ? 1 : 0, (project && with_x) ? 1 : 0,
                 W, ctl, 0, 0));
  Ctl hc;
  CK(hipMemcpyAsync(&hc, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  *degenerate = hc.degenerate ? 1 : 0;
  return RL_OK;
}

int rl_server_create(rl_server_h* out, int device, size_t hbm_budget_bytes, int32_t max_inflight) {
  if (!out || max_inflight < 1 || max_inflight > 64 || hbm_budget_bytes == 0) return RL_ERR_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return RL_ERR_DEVICE;
  rl_server* s = new (std::nothrow) rl_server();
  if (!s) return RL_ERR_NOMEM;
  s->device = device;
  s->budget = (int64_t)hbm_budget_bytes;
  for (int i = 0; i < max_inflight; ++i) {
    hipStream_t st = nullptr;
    rl_handle h = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || rl_create(&h, device, st) != RL_OK) {
      if (st) (void)hipStreamDestroy(st);
      s->stopping = true;
      rl_server_destroy(s);
      return RL_ERR_DEVICE;
    }
    h->ws_async = true;
    s->lds_budget = h->lds_budget;
    s->streams.push_back(st);
    s->ctxs.push_back(h);
  }
  for (int i = 0; i < max_inflight; ++i) s->workers.emplace_back(server_worker, s, i);
  *out = s;
  return RL_OK;
}

int rl_server_submit(rl_server_h s, const rl_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return RL_ERR_ARG;
  if (!req->A || !req->sigma || !req->V) return RL_ERR_ARG;
  const bool cplx = req->is_complex != 0;
  rl_opts o;
  if (req->opts) o = *req->opts;
  else rl_default_opts(&o, req->m, req->n, req->k);
  int rc = check_opts(req->m, req->n, req->k, o);
  if (rc != RL_OK) return rc;
  if (req->lda < req->n || req->ldv < req->k || (req->U && req->ldu < req->k)) return RL_ERR_ARG;
  if (cplx && o.sketch_prec != RL_SKETCH_F64) return RL_ERR_UNSUPPORTED;
  if (!astream_shape_ok(cplx, o.dot2 != 0, req->n, o.block, req->A, req->lda)) return RL_ERR_UNSUPPORTED;
  rl_job* j = new (std::nothrow) rl_job();
  if (!j) return RL_ERR_NOMEM;
  j->cplx = cplx;
  j->m = req->m;
  j->n = req->n;
  j->k = req->k;
  j->A = req->A;
  j->lda = req->lda;
  j->sigma = req->sigma;
  j->V = req->V;
  j->ldv = req->ldv;
  j->U = req->U;
  j->ldu = req->ldu;
  j->opts = o;
  j->opts.profile = 0;
  j->bytes = planned_bytes(cplx, req->m, req->n, req->k, o, s->lds_budget);
  if (j->bytes > s->budget) {
    delete j;
    return RL_ERR_ADMISSION;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
      delete j;
      return RL_ERR_CANCELLED;
    }
    j->ticket = s->next_ticket++;
    j->t_submit = std::chrono::steady_clock::now();
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv_work.notify_all();
  return RL_OK;
}

// A finished job is reported once and then forgotten.
static int take_result(rl_server* s, std::unique_lock<std::mutex>& lk, rl_job* j, rl_info* info,
                       rl_job_times* times) {
  (void)lk;
  const int st = j->status;
  if (info) {
    // copy the scalar fields; the server does not fill caller history arrays
    double* th = info->theta_hist;
    double* rn = info->rnorm_hist;
    const int32_t cap = info->hist_cap;
    *info = j->info;
    info->theta_hist = th;
    info->rnorm_hist = rn;
    info->hist_cap = cap;
  }
  fill_times(j, times);
  s->jobs.erase(j->ticket);
  delete j;
  return st;
}

int rl_server_poll(rl_server_h s, uint64_t ticket, int32_t* done, rl_info* info, rl_job_times* times) {
  if (!s || !done) return RL_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return RL_ERR_ARG;
  if (!it->second->done) {
    *done = 0;
    return RL_PENDING;
  }
  *done = 1;
  return take_result(s, lk, it->second, info, times);
}

int rl_server_wait(rl_server_h s, uint64_t ticket, int64_t timeout_us, rl_info* info, rl_job_times* times) {
  if (!s) return RL_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return RL_ERR_ARG;
  rl_job* j = it->second;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return j->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return j->done; })) {
    return RL_PENDING;
  }
  return take_result(s, lk, j, info, times);
}

int rl_server_destroy(rl_server_h s) {
  if (!s) return RL_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;  // queued jobs still run: destroy drains
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (rl_ctx* h : s->ctxs) rl_destroy(h);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
  return RL_OK;
}

const char* rl_status_string(int code) {
  switch (code) {
    case RL_OK: return "ok";
    case RL_NOT_CONVERGED: return "max_iter reached before the stopping rule held";
    case RL_ERR_ARG: return "invalid argument";
    case RL_ERR_DEVICE: return "HIP runtime error";
    case RL_ERR_NOMEM: return "device allocation failed";
    case RL_ERR_NONFINITE: return "NaN or Inf in the sketch or in R^{-1}";
    case RL_ERR_UNSUPPORTED:
      return "shape outside the compiled kernels (b > 10, or n > 1024 unless real, even n <= 2048, plain sums, "
             "16-byte aligned rows; or a reduced-precision sketch of complex data)";
    case RL_PENDING: return "the served job has not finished";
    case RL_ERR_ADMISSION: return "the request can never fit the server's HBM budget";
    case RL_ERR_CANCELLED: return "the server is shutting down";
    case RL_ERR_SCRATCH: return "the shape needs more scratch than the allocation-free entry point holds (32 MiB)";
    default: return "unknown status";
  }
}

}  // extern "C"
