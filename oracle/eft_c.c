/* Compensated products of the oracle in plain C (test infrastructure only).
 *
 * The same arithmetic, operation for operation, as the numpy forms in
 * oracle/eft.py, so the results are bit for bit the same (checked by
 * tests/test_oracle_eft.py):
 *   Split       Veltkamp/Dekker with the factor 2^27 + 1
 *   TwoProduct  Dekker (no fused multiply-add)
 *   TwoSum      Knuth
 *   Dot2        Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26(6), 2005,
 *               Alg. 5.3), sequentially along each row, for A W
 *   Dot2 tree   TwoSum on pairs along the rows inside chunks of rows, the
 *               chunk results accumulated by TwoSum with their errors, for
 *               A^* Y
 * Complex data are interleaved (re, im).  A row of a complex product A W is
 * the real sequence [Re a, Im a] against [Re w, -Im w] (real part) and
 * [Im w, Re w] (imaginary part); a column of A^* Y is the sum over the
 * stacked rows [Re A; Im A] against [Re y; Im y] (real part) and
 * [Re A; -Im A] against [Im y; Re y] (imaginary part).
 *
 * Build (oracle/build.py): gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 * Contraction into FMA must stay off: the transformations rely on every
 * product and sum being rounded on its own.  Each output element is computed
 * by one thread in a fixed order, so the thread count does not change it. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double SPLITTER = 134217729.0; /* 2^27 + 1 */

static inline void split(double a, double* hi, double* lo) {
  const double c = SPLITTER * a;
  const double h = c - (c - a);
  *hi = h;
  *lo = a - h;
}

/* error of the product p = fl(a b) from the split halves of a and b */
static inline double prod_err(double p, double ah, double al, double bh, double bl) {
  return al * bl - (((p - ah * bh) - al * bh) - ah * bl);
}

static inline void two_sum(double a, double b, double* s, double* e) {
  const double ss = a + b;
  const double z = ss - a;
  *e = (a - (ss - z)) + (b - z);
  *s = ss;
}

void eft_set_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}

int eft_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Dot2 of x (stride sx) with the presplit y (yh, yl), length L >= 1. */
static double dot2_seq(const double* x, int64_t sx, const double* y, const double* yh, const double* yl,
                       int64_t L) {
  double xh, xl;
  split(x[0], &xh, &xl);
  double p = x[0] * y[0];
  double s = prod_err(p, xh, xl, yh[0], yl[0]);
  for (int64_t i = 1; i < L; ++i) {
    const double xi = x[i * sx];
    split(xi, &xh, &xl);
    const double h = xi * y[i];
    const double r = prod_err(h, xh, xl, yh[i], yl[i]);
    double q;
    two_sum(p, h, &p, &q);
    s = s + (q + r);
  }
  return p + s;
}

/* out (m x b, row stride ldo, elements) = A W with Dot2 rows.  Real: A m x n
 * (lda), W n x b (ldw).  Complex (cplx = 1): the same shapes in interleaved
 * complex elements (lda, ldw, ldo count complex elements). */
void eft_matmul(const double* A, int64_t m, int64_t n, int64_t lda, const double* W, int64_t b, int64_t ldw,
                int cplx, double* out, int64_t ldo) {
  if (m <= 0 || b <= 0) return;
  if (n == 0) {
    for (int64_t i = 0; i < m; ++i)
      memset(out + i * ldo * (cplx ? 2 : 1), 0, sizeof(double) * (size_t)b * (cplx ? 2 : 1));
    return;
  }
  if (!cplx) {
    /* y_j = W(:, j) presplit */
    double* ys = (double*)malloc(sizeof(double) * (size_t)(3 * n * b));
    for (int64_t j = 0; j < b; ++j)
      for (int64_t l = 0; l < n; ++l) {
        const double w = W[l * ldw + j];
        ys[j * 3 * n + l] = w;
        split(w, &ys[j * 3 * n + n + l], &ys[j * 3 * n + 2 * n + l]);
      }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < b; ++j) {
        const double* y = ys + j * 3 * n;
        out[i * ldo + j] = dot2_seq(A + i * lda, 1, y, y + n, y + 2 * n, n);
      }
    free(ys);
    return;
  }
  const int64_t L = 2 * n;
  /* per column j: the real-part sequence [Re w, -Im w] and the imaginary-part
   * sequence [Im w, Re w], each with its split halves */
  double* ys = (double*)malloc(sizeof(double) * (size_t)(6 * L * b));
  for (int64_t j = 0; j < b; ++j) {
    double* yr = ys + j * 6 * L;
    double* yi = yr + 3 * L;
    for (int64_t l = 0; l < n; ++l) {
      const double wr = W[2 * (l * ldw + j)], wi = W[2 * (l * ldw + j) + 1];
      yr[l] = wr;
      yr[n + l] = -wi;
      yi[l] = wi;
      yi[n + l] = wr;
    }
    for (int64_t l = 0; l < L; ++l) {
      split(yr[l], &yr[L + l], &yr[2 * L + l]);
      split(yi[l], &yi[L + l], &yi[2 * L + l]);
    }
  }
#pragma omp parallel
  {
    double* x = (double*)malloc(sizeof(double) * (size_t)L);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
      const double* a = A + 2 * i * lda;
      for (int64_t l = 0; l < n; ++l) {
        x[l] = a[2 * l];
        x[n + l] = a[2 * l + 1];
      }
      for (int64_t j = 0; j < b; ++j) {
        const double* yr = ys + j * 6 * L;
        const double* yi = yr + 3 * L;
        out[2 * (i * ldo + j)] = dot2_seq(x, 1, yr, yr + L, yr + 2 * L, L);
        out[2 * (i * ldo + j) + 1] = dot2_seq(x, 1, yi, yi + L, yi + 2 * L, L);
      }
    }
    free(x);
  }
  free(ys);
}

/* Value of stacked row r (0 <= r < 2m for complex, < m for real) in column c:
 * real: A(r, c); complex, part 0: [Re A; Im A]; part 1: [Re A; -Im A]. */
static inline double stacked(const double* A, int64_t m, int64_t lda, int cplx, int part, int64_t r, int64_t c) {
  if (!cplx) return A[r * lda + c];
  if (r < m) return A[2 * (r * lda + c)];
  const double v = A[2 * ((r - m) * lda + c) + 1];
  return part ? -v : v;
}

/* The matching stacked entry of y: real: y(r); complex part 0: [Re y; Im y];
 * part 1: [Im y; Re y]. */
static inline double stacked_y(const double* Y, int64_t m, int64_t ldy, int64_t j, int cplx, int part, int64_t r) {
  if (!cplx) return Y[r * ldy + j];
  if (r < m) return part ? Y[2 * (r * ldy + j) + 1] : Y[2 * (r * ldy + j)];
  return part ? Y[2 * ((r - m) * ldy + j)] : Y[2 * ((r - m) * ldy + j) + 1];
}

/* out (n x b, row stride ldo) = A^* Y, each entry a Dot2-class tree sum over
 * the (stacked) rows in chunks of row_chunk rows.  A m x n (lda), Y m x b
 * (ldy); complex counts in complex elements. */
void eft_matmul_h(const double* A, int64_t m, int64_t n, int64_t lda, const double* Y, int64_t b, int64_t ldy,
                  int cplx, int64_t row_chunk, double* out, int64_t ldo) {
  if (n <= 0 || b <= 0) return;
  const int64_t total = cplx ? 2 * m : m;
  const int nparts = cplx ? 2 : 1;
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  /* column ranges per thread: every output column's arithmetic is the same
   * whatever range holds it */
  const int64_t cw = (n + nt - 1) / nt;
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    const int64_t c0 = (int64_t)t * cw, c1 = c0 + cw < n ? c0 + cw : n;
    const int64_t w = c1 - c0;
    if (w > 0) {
      double* P = (double*)malloc(sizeof(double) * (size_t)(row_chunk * w));
      double* E = (double*)malloc(sizeof(double) * (size_t)(row_chunk * w));
      double* acc_s = (double*)malloc(sizeof(double) * (size_t)w);
      double* acc_e = (double*)malloc(sizeof(double) * (size_t)w);
      for (int64_t j = 0; j < b; ++j)
        for (int part = 0; part < nparts; ++part) {
          for (int64_t c = 0; c < w; ++c) acc_s[c] = acc_e[c] = 0.0;
          for (int64_t r0 = 0; r0 < total; r0 += row_chunk) {
            int64_t len = total - r0 < row_chunk ? total - r0 : row_chunk;
            /* P, E = TwoProduct of the chunk's entries with y */
            for (int64_t r = 0; r < len; ++r) {
              const double y = stacked_y(Y, m, ldy, j, cplx, part, r0 + r);
              double yh, yl;
              split(y, &yh, &yl);
              for (int64_t c = 0; c < w; ++c) {
                const double a = stacked(A, m, lda, cplx, part, r0 + r, c0 + c);
                double ah, al;
                split(a, &ah, &al);
                const double p = a * y;
                P[r * w + c] = p;
                E[r * w + c] = prod_err(p, ah, al, yh, yl);
              }
            }
            /* pairwise TwoSum tree; an odd level is padded with a zero row */
            while (len > 1) {
              const int64_t half = (len + 1) / 2;
              for (int64_t q = 0; q < half; ++q) {
                const int64_t r1 = 2 * q, r2 = 2 * q + 1;
                for (int64_t c = 0; c < w; ++c) {
                  const double pa = P[r1 * w + c], ea = E[r1 * w + c];
                  const double pb = r2 < len ? P[r2 * w + c] : 0.0;
                  const double eb = r2 < len ? E[r2 * w + c] : 0.0;
                  double s, tt;
                  two_sum(pa, pb, &s, &tt);
                  E[q * w + c] = (ea + eb) + tt;
                  P[q * w + c] = s;
                }
              }
              len = half;
            }
            for (int64_t c = 0; c < w; ++c) {
              double s, tt;
              two_sum(acc_s[c], P[c], &s, &tt);
              acc_s[c] = s;
              acc_e[c] = (acc_e[c] + E[c]) + tt;
            }
          }
          for (int64_t c = 0; c < w; ++c) {
            const double v = acc_s[c] + acc_e[c];
            if (cplx)
              out[2 * ((c0 + c) * ldo + j) + part] = v;
            else
              out[(c0 + c) * ldo + j] = v;
          }
        }
      free(P);
      free(E);
      free(acc_s);
      free(acc_e);
    }
  }
}
