// Launchers of the HIP kernels (host side); one definition per .hip file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace rl {

// sketch.hip
int sketch_plan_ct(int d, int64_t lds_budget, int acc_bytes);
int64_t sketch_partial_doubles(int64_t m, int64_t ncols_d, int d, int64_t lds_budget, int* nchunk_out,
                               int64_t* rows_out, int acc_bytes);
hipError_t launch_sketch(hipStream_t st, const double* A, int64_t lda_d, int64_t m, int64_t ncols_d, int es, int d,
                         int zeta, uint64_t seed, double scale, void* part, void* Ycol, Ctl* ctl,
                         int64_t lds_budget, bool fp32);

// qr.hip
// r_ready (optional) is recorded on st once R is complete (in Y and Rrow),
// before the inverses are formed.
hipError_t launch_qr_lowp(hipStream_t st, float* Yf, int d, int n, float* Tmf, double* Y, double* Rrow, double* RH,
                          double* Rinv, double* RinvH, bool bf16, hipEvent_t r_ready = nullptr);
// elements of the T workspace launch_qr and launch_qr_lowp take (the panel's
// T factor and, for sketches over 4096 rows, its leaves')
constexpr int QR_TM_ELEMS = 32 * 32 * 22;
hipError_t launch_qr(hipStream_t st, bool cplx, void* Y, int d, int n, void* Tm, void* Rrow, void* RH, void* Rinv,
                     void* RinvH, hipEvent_t r_ready = nullptr);

// astream.hip
int astream_ns(int n);
int64_t astream_blocks(int64_t m, int n, int B, int es_d);
int64_t astream_part_doubles(int64_t m, int n, int B, int es_d);
int64_t astream_tmp_doubles(int64_t m, int n, int B, int es_d);
int64_t astream_r2_blocks(int64_t m);
int astream_ccs_waves(int n);
bool astream_c2_fits(int B, int n, bool aligned);
bool astream_rm_fits(int B, int n, bool aligned, int64_t lds_max);
bool dispatch_astream_rm(int init, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart, int n_cu,
                         const Ctl* ctl, hipEvent_t mid);
bool dispatch_zm_aw_only(bool cplx, int B, hipStream_t st, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, int n_cu, const Ctl* ctl);
bool dispatch_zm_gram(bool cplx, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                      const void* P0, double* Gpart, const Ctl* ctl);
bool astream_late_residual(bool cplx, bool dot2, int n, int B, const void* A, int64_t lda);
hipError_t launch_astream_aw(hipStream_t st, bool cplx, int B, const void* A, int64_t lda, int64_t m, int n,
                             const void* W, void* AW, const Ctl* ctl);
hipError_t launch_astream_gram(hipStream_t st, bool cplx, int B, const void* A, int64_t lda, int64_t m, int n,
                               const void* P0, double* Gpart, const Ctl* ctl, int64_t* np_out);
bool astream_shape_ok(bool cplx, bool dot2, int64_t n, int B, const void* A, int64_t lda);
bool astream_zm_fits(int B, int n, bool aligned, int64_t lds_max);
bool dispatch_astream_zm(int init, int B, hipStream_t st, int64_t nrr, const void* A, int64_t lda, int64_t m, int n,
                         const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart, int n_cu,
                         const Ctl* ctl, hipEvent_t mid = nullptr);
int device_cu_count();
int64_t device_lds_max();
int64_t astream_c2_ranges(int64_t m, int n, int B);
bool dispatch_astream_c2(bool dot2, int init, int B, hipStream_t st, int64_t nrb, const void* A, int64_t lda,
                         int64_t m, int n, const void* W, void* AW, const void* AVp, const void* AXp, double* Gpart,
                         const Ctl* ctl);
bool astream_ccs_fits(int B, int n, bool aligned);
void astream_ccs_groups(int B, bool dot2, int* ng, int* bs);
int64_t astream_ccs_ranges(int64_t m, int n, int B, bool dot2);
bool dispatch_astream_ccs(bool dot2, int init, int B, hipStream_t st, int64_t nrb, const void* A, int64_t lda,
                          int64_t m, int n, const void* W, void* AW, const void* AVp, const void* AXp,
                          double* Gpart, const Ctl* ctl);
int astream_cs_waves(int n);
bool astream_cs_fits(int B, int n, bool aligned);
int64_t astream_cs_blocks(int64_t m, int n);
bool dispatch_astream_cs(bool dot2, int init, int B, hipStream_t st, int64_t nb, const double* A, int64_t lda,
                         int64_t m, int n, const double* W, double* AW, const double* AVp, const double* AXp,
                         double* Gpart, const Ctl* ctl);
bool astream_r2_fits(int B, int n, bool aligned, int64_t m, int64_t lda);
bool dispatch_astream_r2(bool dot2, int init, int B, hipStream_t st, int64_t nb, const double* A, int64_t lda,
                         int64_t m, int n, const double* W, double* AW, const double* AVp, const double* AXp,
                         double* Gpart, const Ctl* ctl);
bool dispatch_astream_gd(bool dot2, int ns, int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m,
                         int n, const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                         const Ctl* ctl);
bool dispatch_astream_gc(bool dot2, int ns, int B, hipStream_t st, int64_t nb, const void* A, int64_t lda, int64_t m,
                         int n, const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                         const Ctl* ctl);
hipError_t launch_astream_pass(hipStream_t st, bool cplx, int B, bool dot2, const void* A, int64_t lda, int64_t m,
                               int n, const void* W, void* AW, const void* AVp, const void* AXp, int init,
                               double* Gpart, const Ctl* ctl, int64_t* np_out, hipEvent_t mid = nullptr,
                               bool* mid_recorded = nullptr);
hipError_t launch_astream_reduce(hipStream_t st, bool cplx, int B, int n, int64_t np, const double* Gpart,
                                 double* tmp, double* G3, const Ctl* ctl, bool first_only = false);
// One level of that reduction (k_colsum2): grid gx x gy of 256 threads.
struct ColsumJob {
  const double* in_s;
  const double* in_e;
  int64_t stride, elen, nparts, len;
  double* out_s;
  double* out_e;
  double* fin;
  const Ctl* ctl;
  int gx, gy;
};
int astream_reduce_plan(bool cplx, int B, int n, int64_t np, const double* Gpart, double* tmp, double* G3,
                        const Ctl* ctl, ColsumJob* lev, int maxlev, bool first_only = false);
hipError_t launch_colsum_job(hipStream_t st, const ColsumJob& J);
hipError_t launch_astream(hipStream_t st, bool cplx, int B, bool dot2, const void* A, int64_t lda, int64_t m, int n,
                          const void* W, void* AW, const void* AVp, const void* AXp, int init, double* Gpart,
                          double* tmp, double* G3, const Ctl* ctl, hipEvent_t pass_done = nullptr);
// pmode 0: A_V and A_X in place; 1: AVout <- A_T C_V only; 2: A_X only
hipError_t launch_panel(hipStream_t st, bool cplx, void* AV, void* AX, const void* AW, int64_t m, int B,
                        const void* CV, const void* CX, const Ctl* ctl, int pmode = 0, void* AVout = nullptr);
hipError_t launch_refresh_out(hipStream_t st, bool cplx, int n, int64_t m, int B, int k, const void* V,
                              const void* AVf, const void* C, const double* s, double* sigma, void* Vout,
                              int64_t ldv, void* U, int64_t ldu, Ctl* ctl);
hipError_t launch_final_u(hipStream_t st, bool cplx, const void* AV, const void* AX, const void* AW, int64_t m, int B,
                          int k, const void* CV, const double* thb, void* U, int64_t ldu, const Ctl* ctl);

// precond.hip
int64_t colnorm_groups(int64_t m);
hipError_t launch_colnorm_scale(hipStream_t st, bool cplx, const double* A, int64_t lda_d, int64_t m, int n,
                                double* part, double* dscale);
hipError_t launch_prec_apply(hipStream_t st, bool cplx, int n, int B, const double* dscale, const void* R, void* W,
                             const Ctl* ctl);

// tsqr.hip
int64_t tsqr_groups(int64_t m, int t);
// side (optional): one level of the partial-sum reduction, run as extra
// workgroups of the first TSQR launch (t <= 8) or launched just before it.
hipError_t launch_tsqr(hipStream_t st, bool cplx, const void* P0, int b0, const void* P1, int b1, const void* P2,
                       int b2, int64_t m, void* bufA, void* bufB, void** Rfinal, Ctl* ctl, int check_done,
                       const ColsumJob* side = nullptr);

// Copies the control block between device memory and the handle's mapped
// host block (either direction) with vector stores.
hipError_t launch_publish(hipStream_t st, const Ctl* src, Ctl* dst);

// nside.hip
hipError_t launch_trmv(hipStream_t st, bool cplx, int B, const void* M, int n, int lower, const void* X, void* Y,
                       const Ctl* ctl, int check_done);
hipError_t launch_orth_svqb(hipStream_t st, bool cplx, int n, int B, const void* V, const void* X, int project,
                            int with_x, void* W, Ctl* ctl, int check_done);
// masked = 1: with locking on (ctl->lock), the locked columns of W are set
// to zero instead of orthonormalised
// The register-resident Orth (k_orth_reg) when n and B fit it (n <= 2048
// real, n <= 1024 complex, B <= 10); false when they do not (nothing launched).
bool launch_orth_reg_d(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x, void* W,
                       Ctl* ctl, int check_done, int masked);
bool launch_orth_reg_c(hipStream_t st, int n, int B, const void* V, const void* X, int project, int with_x, void* W,
                       Ctl* ctl, int check_done, int masked);
hipError_t launch_orth(hipStream_t st, bool cplx, int n, int B, const void* V, const void* X, int project, int with_x,
                       void* W, Ctl* ctl, int check_done, int masked = 0);
// phase 0: the whole Rayleigh-Ritz step; 1: Rayleigh-Ritz and V_new (into
// Vn) only, C, Theta and padding flags saved to Cst (RR_CST_DOUBLES); 2: the
// residual from G3's first block (A^* A_{V_new}), the stopping rule, the
// lock update, X and V <- V_new
constexpr int RR_CST_DOUBLES = 32 * 32 * 2 + 2 * 32;
hipError_t launch_rr(hipStream_t st, bool cplx, int n, int B, int init_mode, int with_x, const void* Rt, void* V,
                     void* X, const void* W, const void* G3, void* Vn, void* Rres, void* CV, void* CX, double* thb,
                     double* ht, double* hr, Ctl* ctl, int phase = 0, double* Cst = nullptr);
hipError_t launch_randblk(hipStream_t st, bool cplx, void* Wb, int64_t count, uint64_t seed);
hipError_t launch_lanczos(hipStream_t st, bool cplx, int n, const void* Ycol, int ld, const void* Rrow, void* Ub,
                          void* Vb, int KL, uint64_t seed, Ctl* ctl);
hipError_t launch_final_n(hipStream_t st, bool cplx, int n, int B, int k, const void* V, const double* thb,
                          double* sigma, void* Vout, int64_t ldv, Ctl* ctl);
hipError_t launch_max_colnorm(hipStream_t st, bool cplx, int n, int B, const void* Z, double* out);
hipError_t launch_rt_svd(hipStream_t st, bool cplx, int t, const void* Rt, double* sigma, void* C);

}  // namespace rl
