/* rlobpcg.h -- C-ABI of the MI355X (gfx950) RLOBPCG library.
 *
 * RLOBPCG (Epperly, Park, Nakatsukasa, "Fast, high-accuracy, randomized
 * nullspace computations for tall matrices") returns a few of the smallest
 * singular triplets of a tall A in C^{m x n}, m >> n (Sec. 1): a SparseStack
 * sketch S*A (Sec. 2.2) gives a preconditioner P with P P^* = ((S A)^* S A)^{-1}
 * and a sketch-and-solve start; LOBPCG on A^* A with that preconditioner then
 * refines the block (Alg. rlopcg for b = 1, Alg. rlobpcg for b > 1) until the
 * tolerance rule (eq:est_conv_criterion) and the stagnation checks
 * (eq:stagnation-check) hold.
 *
 * Conventions for every call:
 *   - Matrices are row-major.  A has leading dimension lda >= n (elements).
 *     Complex data (the _z calls) are interleaved (re, im) doubles, the layout
 *     of C99 double _Complex and of torch.complex128; sigma stays real.
 *   - Pointers named "device" are HIP device pointers that the caller
 *     allocated and owns; the library never frees or retains them past the
 *     call.  Pointers named "host" are ordinary host memory.
 *   - Work is enqueued on the handle's stream.  A solve call returns after its
 *     results are in the caller's buffers (it synchronises on its stream).
 *   - Every call returns an int status; no exception crosses the ABI.
 */
#ifndef RLOBPCG_H
#define RLOBPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define RL_OK 0
#define RL_NOT_CONVERGED 1    /* max_iter reached; outputs hold the last iterate (after the loop of Alg. rlopcg) */
#define RL_ERR_ARG (-1)       /* k < 1, b < k, 3b > n, n > m, d < n, zeta < 1 or > d, bad lda/ldv/ldu, null pointer */
#define RL_ERR_DEVICE (-2)    /* a HIP call failed */
#define RL_ERR_NOMEM (-3)     /* device workspace allocation failed */
#define RL_ERR_NONFINITE (-4) /* NaN/Inf in S*A or in R^{-1} (S*A numerically rank deficient) */
#define RL_ERR_UNSUPPORTED (-7) /* a shape outside the compiled kernels: b > 10, or n > 1024 unless A is
                                   real, n even and <= 2048, dot2 = 0 and rows 16-byte aligned (lda even);
                                   or a reduced-precision sketch of complex data */
#define RL_PENDING 2             /* served job not finished (rl_server_poll / rl_server_wait time-out) */
#define RL_ERR_ADMISSION (-5)    /* a served request whose workspace can never fit the server's budget */
#define RL_ERR_CANCELLED (-6)    /* a request submitted to a server that is shutting down */
#define RL_ERR_SCRATCH (-8)      /* rl_step_astream_iter_noalloc: the shape needs more than its 32 MiB of scratch */

/* Stopping rules (oracle.termination documents the same three). */
#define RL_STOP_PAPER 0 /* at i = 0 mod check_every: tolerance and both stagnation checks, every column */
#define RL_STOP_TOL 1   /* the tolerance alone, every iteration (Alg. rlobpcg as typeset) */
#define RL_STOP_NONE 2  /* run max_iter iterations */

/* Precision of the sketch and of its QR factorization.  Everything after
 * them (R^{-1}, the A products, residuals, Rayleigh-Ritz, orthonormalisation)
 * is FP64; the preconditioner only needs to be approximate (Sec. 2.2), but a
 * reduced-precision R loses the directions of A below about u_low ||A||, so
 * the number of iterations can grow when cond(A) u_low is not small. */
#define RL_SKETCH_F64 0  /* FP64 sketch and Householder QR */
#define RL_SKETCH_F32 1  /* FP32 sketch (A rounded once per entry) and FP32 QR; R promoted to FP64 */
#define RL_SKETCH_BF16 2 /* FP32 sketch; QR trailing updates with bfloat16 inputs and FP32 accumulation */

/* Preconditioner of the LOBPCG loop (rl_opts.loop_precond).  The start block
 * and Sigma~(1,1) always come from the sketch; the two alternatives are the
 * comparison methods of Sec. 1.1 (illustrative example):
 * RL_PREC_DIAG uses P = diag(||A(:, i)||^{-1}), so W = diag(||A(:, i)||^{-2}) R
 * (a zero column keeps P(i, i) = 1); RL_PREC_NONE uses W = R. */
#define RL_PREC_SKETCH 0 /* P = R^{-1} from the QR of S*A (the method) */
#define RL_PREC_DIAG 1
#define RL_PREC_NONE 2

/* Orth of the new search block W in the loop (rl_opts.orth), after its two
 * block projections on [V X] (Sec. 2.1: CGS2; SVQB is the faster, less stable
 * alternative the paper names).  RL_ORTH_SVQB forms G = W^* W, scales it to a
 * unit diagonal D G D, takes its eigenvectors Z and eigenvalues Lambda (raised
 * to eps * max where smaller) and sets W <- W D Z Lambda^{-1/2}. */
#define RL_ORTH_CGS2 0
#define RL_ORTH_SVQB 1

typedef struct rl_ctx* rl_handle;

/* Options.  rl_default_opts fills the paper's defaults. */
typedef struct {
  int64_t d;          /* sketch rows; default 4n (Alg. rlopcg uses 4n; Sec. 2.2 recommends 2n..4n) */
  int32_t zeta;       /* nonzeros per column of S; default 8 */
  int32_t block;      /* block size b >= k; default k */
  uint64_t seed;      /* SparseStack counter seed */
  double tau;         /* tolerance; default 2 sqrt(n) 2^-52 (Sec. 2.1) */
  int32_t max_iter;   /* default 200 for b = 1, 100 for b > 1 (Alg. rlopcg, Alg. rlobpcg) */
  int32_t check_every;/* stagnation-check cadence; default 5 (Alg. rlopcg) */
  int32_t stop_rule;  /* RL_STOP_*; default RL_STOP_PAPER */
  int32_t dot2;       /* 1: row products of A accumulated as Dot2 (real and complex); default 1 for
                         n <= 1024, else 0 (real 1024 < n <= 2048 runs plain FP64 sums on the matrix cores) */
  int32_t init_iters; /* inverse-subspace-iteration steps for the start block; default 10 */
  int32_t lanczos_steps; /* Golub-Kahan steps for Sigma~(1,1); default min(n, 64) */
  int32_t profile;    /* 1: time the pass kernels of every A-stream launch with HIP events (rl_info.t_astream_us) */
  int32_t sketch_prec; /* RL_SKETCH_*: precision of the sketch S*A and its QR (real A only); default FP64 */
  int32_t loop_precond; /* RL_PREC_*: preconditioner of the LOBPCG loop; default RL_PREC_SKETCH */
  int32_t orth;       /* RL_ORTH_*: Orth of W in the loop after the block projections; default RL_ORTH_CGS2 */
  int32_t refresh;    /* 1 (default): after the loop, A V-hat afresh (one more pass over A) and its thin SVD
                         rotate (V-hat, sigma, U-hat), so the outputs carry no drift of the products the loop
                         maintains by recurrence; 0: the last Rayleigh-Ritz's triplets, U-hat = A_V / theta */
  int32_t prec_guard; /* 1 (default): with a reduced-precision sketch_prec, estimate kappa(R) =
                         ||R||_2 ||R^{-1}||_2 from the Lanczos estimate and the start block and, when
                         kappa u_low sqrt(n) > 0.1 (u_low = 2^-24 for FP32, 2^-8 for bfloat16), redo
                         the sketch and QR in FP64 before the start pass (rl_info.sketch_prec_used) */
  int32_t lock;       /* 1: locking of converged columns (Sec. 2.3): once column j's residual meets
                         ||r_j|| <= Sigma~(1,1)^2 tau it is locked for good; it stays in V and in every
                         Rayleigh-Ritz step but gets no search direction (its columns of W and X are
                         zero), and the loop ends once every column is locked.  Default 0; not with
                         RL_ORTH_SVQB (RL_ERR_UNSUPPORTED) */
} rl_opts;

/* Per-solve report (host).  theta_hist / rnorm_hist are optional host arrays
 * of hist_cap*b doubles that receive theta_j and ||r_j(:, c)|| for iterates
 * j = 0 .. iters (row j, column c; theta_0 = +inf when b = 1). */
typedef struct {
  int32_t status;      /* RL_OK or RL_NOT_CONVERGED */
  int32_t iters;       /* loop iterations executed */
  int32_t a_passes;    /* full passes over A (sketch + start + one per iteration, + 1 with refresh) */
  int32_t degenerate;  /* a Normalize/Orth met a zero vector */
  int32_t zero_theta;  /* some returned sigma is exactly 0 (its U column is 0) */
  int32_t block;       /* b used */
  double sigma1;       /* Sigma~(1,1) estimate used in the tolerance */
  double t_setup_us;   /* sketch, QR, R^{-1}, Sigma~(1,1), start block, first Rayleigh-Ritz */
  double t_iter_us;    /* the LOBPCG loop */
  double t_final_us;   /* outputs */
  int64_t bytes_a;     /* bytes of A read by the solve (a_passes * m * n * element size) */
  int32_t hist_cap;    /* capacity (rows) of the history arrays below; 0 = none */
  int32_t n_astream;   /* A-stream launches timed (opts.profile) */
  double t_astream_us; /* summed duration of their pass kernels (the reduction of the partial sums excluded) */
  double* theta_hist;  /* host, may be NULL */
  double* rnorm_hist;  /* host, may be NULL */
  int32_t n_pass_g;    /* timed launches made of two kernels (A W, then the Gram contraction A^* [A_V A_X A_W]) */
  int32_t sketch_prec_used; /* RL_SKETCH_* of the R the loop used (RL_SKETCH_F64 after a guard fallback) */
  double t_pass_g_us;  /* summed duration of their second kernel (opts.profile) */
  double kappa_est;    /* the guard's estimate of kappa(R) for a reduced-precision sketch, else 0 */
  int32_t n_locked;    /* columns locked when the loop ended (opts.lock), else 0 */
  int32_t act_mask;    /* bit j set: column j of the block still active at the end (all b bits without lock) */
} rl_info;

/* Handle: one per (device, stream).  stream may be NULL (the null stream). */
int rl_create(rl_handle* h, int device, void* hip_stream);
int rl_destroy(rl_handle h);
int rl_set_stream(rl_handle h, void* hip_stream);

/* Fill defaults for an m x n problem with k wanted triplets (host only). */
int rl_default_opts(rl_opts* o, int64_t m, int64_t n, int32_t k);

/* The k smallest singular triplets of A: a few (1 to 10 in the paper's use)
 * of its smallest singular values with their vectors (Sec. 1; Alg. rlopcg /
 * Alg. rlobpcg).
 *   A      device, m x n, row-major, leading dimension lda
 *   sigma  device, k doubles, ascending
 *   V      device, n x k (ldv >= k): right singular vectors, column j <-> sigma[j]
 *   U      device, m x k (ldu >= k) or NULL: U(:, j) = A V(:, j) / sigma[j], from the
 *          refreshed product A V (opts.refresh) or the final Rayleigh-Ritz basis
 *   opts   host, may be NULL (defaults); info host, may be NULL
 * Vectors are defined up to a unit phase per column, and inside a cluster of
 * equal sigma only their span is defined. */
int rl_svds_smallest_d(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int32_t k,
                       const rl_opts* opts, double* sigma, double* V, int64_t ldv, double* U, int64_t ldu,
                       rl_info* info);
int rl_svds_smallest_z(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int32_t k,
                       const rl_opts* opts, double* sigma, double* V, int64_t ldv, double* U, int64_t ldu,
                       rl_info* info);

/* ---- Step entry points: one step of the path, for checking it in isolation.
 * is_complex selects real FP64 (0) or interleaved complex FP64 (1) data. */

/* Y = S*A for the SparseStack S of (d, zeta, seed) (Sec. 2.2).
 *   A device m x n (lda); Y device d x n row-major (ldy >= n). */
int rl_step_sketch(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int64_t d,
                   int32_t zeta, uint64_t seed, double* Y, int64_t ldy);

/* R from the Householder QR of Y (d x n, row-major, ldy) and R^{-1}
 * (Sec. 1 footnote: QR of the sketch).  R and Rinv are device n x n row-major
 * (upper triangular; R has a real diagonal). */
int rl_step_qr(rl_handle h, int is_complex, int64_t d, int64_t n, const double* Y, int64_t ldy, double* R,
               double* Rinv);

/* The reduced-precision sketch (RL_SKETCH_F32 and RL_SKETCH_BF16 use it):
 * Y = S*A accumulated in FP32, each entry of A rounded to FP32 once (Sec. 2.2
 * embedding, real A).  A device m x n FP64 (lda); Y device d x n FP32
 * row-major (ldy >= n). */
int rl_step_sketch_f32(rl_handle h, int64_t m, int64_t n, const double* A, int64_t lda, int64_t d, int32_t zeta,
                       uint64_t seed, float* Y, int64_t ldy);

/* R from the reduced-precision QR of the FP32 sketch Y (d x n row-major,
 * ldy): sketch_prec RL_SKETCH_F32 (FP32 Householder QR) or RL_SKETCH_BF16
 * (trailing updates with bfloat16 inputs, FP32 accumulation).  R is promoted
 * to FP64; R and R^{-1} (computed in FP64 from the promoted R) are device
 * n x n FP64 row-major.  RL_ERR_ARG for another sketch_prec. */
int rl_step_qr_lowp(rl_handle h, int64_t d, int64_t n, const float* Y, int64_t ldy, int32_t sketch_prec, double* R,
                    double* Rinv);

/* One pass over A (Alg. rlopcg, the product with the trial space, and the
 * residual's A^*): AW = A W and G = A^* AW.  W device n x b, AW device m x b,
 * G device n x b (all row-major, dense).  dot2 = 1 accumulates the row
 * products of A W as Dot2 (real and imaginary parts separately). */
int rl_step_astream(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int32_t b,
                    const double* W, double* AW, double* G, int32_t dot2);

/* The same pass in the form every LOBPCG iteration after the first uses
 * (Alg. rlopcg, Sec. 3.3: one read of A gives A W and the Gram data
 * A^* [A_V A_X A_W] of the Rayleigh-Ritz step): AW = A W and
 * G3 = [A^* AV | A^* AX | A^* AW].  W device n x b; AV, AX, AW device m x b;
 * G3 device 3 x n x b, the three n x b blocks one after the other (all
 * row-major, dense).  AX may be NULL (no previous direction yet): then the
 * middle block is zero.  dot2 = 1 accumulates A W and A^* AV as Dot2 sums.
 * RL_ERR_ARG on a NULL required pointer or bad size, RL_ERR_UNSUPPORTED for
 * a shape no pass kernel takes (as for RL_ERR_UNSUPPORTED above). */
int rl_step_astream_iter(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda, int32_t b,
                         const double* W, const double* AV, const double* AX, double* AW, double* G3, int32_t dot2);

/* rl_step_astream_iter without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results
 * (bit for bit) as rl_step_astream_iter; the caller still passes every input
 * and output.  The pass's partial sums live in a static scratch area of
 * 32 MiB per device, held from module load until the process ends; shapes
 * whose partial records need more return RL_ERR_SCRATCH before anything is
 * enqueued (every real shape with n <= 200 and b = 1, for instance, fits at
 * any m).  The call only enqueues on the handle's stream and returns: the
 * results are ready when that stream's work is done.  All calls on one GPU
 * share that GPU's scratch, so calls that overlap on one GPU (other streams,
 * other threads, other handles) race; serialise them. */
int rl_step_astream_iter_noalloc(rl_handle h, int is_complex, int64_t m, int64_t n, const double* A, int64_t lda,
                                 int32_t b, const double* W, const double* AV, const double* AX, double* AW,
                                 double* G3, int32_t dot2);

/* Rayleigh-Ritz data of a tall m x t block P (row-major, dense, t <= 32):
 * singular values (descending, device t doubles) and right singular vectors
 * C (device t x t row-major, column j <-> sigma[j]) via TSQR + one-sided Jacobi
 * (Alg. rlopcg, svd of A_T). */
int rl_step_tall_svd(rl_handle h, int is_complex, int64_t m, int32_t t, const double* P, double* sigma, double* C);

/* The search block's orthonormalisation (Alg. rlobpcg, the two block
 * projections of eq:search-direction's block against span[V X], then Orth;
 * b = 1: Normalize, Alg. rlopcg).  V and X are device n x b row-major blocks
 * with orthonormal columns (X may be NULL when with_x = 0; both are ignored
 * when project = 0); W (device, n x b row-major) is overwritten in place with
 * the orthonormal basis: W <- Orth((I - Y Y^*)^2 W), Y = [V X], computed by
 * classical Gram-Schmidt (two block passes against Y, then CGS2 column by
 * column).  A column that vanishes is replaced by the first unit vector that
 * keeps norm above 1/2 after the same projections, and *degenerate (host) is
 * set to 1; else 0.  Requires 1 <= b <= 16, 1 <= n; synchronises the stream.
 * Errors: RL_ERR_ARG on a bad size or NULL pointer. */
int rl_step_orth(rl_handle h, int is_complex, int64_t n, int32_t b, const double* V, const double* X,
                 int32_t project, int32_t with_x, double* W, int32_t* degenerate);

/* ---- Served form: continuous batching of solves of different shapes.
 *
 * Callers that stream many solves (different m, n, k) hand them to a server
 * instead of solving one at a time.  Each request is queued; a request is
 * admitted as soon as a slot is free and the workspaces of the solves in
 * flight plus its own fit hbm_budget_bytes (the caller's A and outputs are not
 * counted).  Admitted solves run concurrently, one stream per slot, so their
 * kernels overlap on the device.  A solve's results are the same as when it
 * runs alone (same kernels, same launch configuration).
 *
 * Ownership: A and the outputs are the caller's device memory and must stay
 * valid and untouched until rl_server_poll or rl_server_wait reports the job
 * done.  The server copies *req and *req->opts at submit.  A finished job is
 * reported once; afterwards its ticket is unknown (RL_ERR_ARG). */
typedef struct rl_server* rl_server_h;

typedef struct {
  int32_t is_complex; /* 0: FP64 A, V, U; 1: interleaved complex FP64 */
  int32_t k;          /* number of smallest triplets */
  int64_t m, n;
  const double* A;    /* device, m x n row-major, leading dimension lda */
  int64_t lda;
  const rl_opts* opts;/* host, may be NULL (defaults); copied at submit */
  double* sigma;      /* device, k doubles (ascending) */
  double* V;          /* device, n x k row-major (ldv) */
  int64_t ldv;
  double* U;          /* device, m x k row-major (ldu), or NULL */
  int64_t ldu;
} rl_request;

typedef struct {
  double queued_us;        /* submit -> admitted */
  double run_us;           /* admitted -> results in the caller's buffers */
  double latency_us;       /* submit -> results in the caller's buffers */
  int64_t workspace_bytes; /* device workspace the solve was admitted with */
} rl_job_times;

/* max_inflight slots (1..64), each with its own stream and worker thread. */
int rl_server_create(rl_server_h* s, int device, size_t hbm_budget_bytes, int32_t max_inflight);
/* Queue a solve; *ticket identifies it.  Argument errors as rl_svds_smallest_*,
 * RL_ERR_ADMISSION if its workspace exceeds the budget, RL_ERR_CANCELLED while
 * the server shuts down.  Never blocks on device work. */
int rl_server_submit(rl_server_h s, const rl_request* req, uint64_t* ticket);
/* *done = 0 and RL_PENDING while the job runs or waits; otherwise *done = 1
 * and the job's status (as rl_svds_smallest_*), with info (scalar fields; the
 * history arrays are not filled) and times when non-NULL. */
int rl_server_poll(rl_server_h s, uint64_t ticket, int32_t* done, rl_info* info, rl_job_times* times);
/* Block until the job is done (timeout_us < 0: no limit); RL_PENDING if the
 * time-out expires first, else as rl_server_poll with done = 1. */
int rl_server_wait(rl_server_h s, uint64_t ticket, int64_t timeout_us, rl_info* info, rl_job_times* times);
/* Stop accepting, run every queued job to the end, release the slots. */
int rl_server_destroy(rl_server_h s);

const char* rl_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* RLOBPCG_H */
