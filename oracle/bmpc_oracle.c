/*
 * bmpc_oracle.c -- plain FP64 CPU oracle for the root-coupled branch system.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this file's library; the product path never does.  It
 * shares no code, header or table with the GPU path.
 *
 * What it computes.  x = K^{-1} b for the SPD matrix K of eq. (root_coupled_matrix)
 * whose tails K_s have the block-tridiagonal form of eq. (tail_block_tridiagonal),
 * with the unknowns and right-hand side partitioned as in Section III-B (all tails
 * in forward stage order, the root block last).  The paper's method reaches exactly
 * this x (it is a reordered Cholesky factorization, Section IV), so the oracle is the
 * plain definition solved by a different route:
 *
 *   1. each tail is stored as a scalar lower band of half-bandwidth p = 2n-1 plus a
 *      dense border of the n root rows;
 *   2. a scalar, column-oriented band Cholesky runs over the tail columns in their
 *      natural order (textbook band Cholesky, Golub & Van Loan, Matrix Computations,
 *      Sec. 4.3); every column also updates the border, which therefore fills in
 *      densely along the tail -- the fill of the forward ordering that Section IV-A
 *      describes for ordering (a) of Fig. 2;
 *   3. the root block receives R - sum_s W_s W_s^T (W_s = the tail's border rows of
 *      the factor), summed in scenario order, and is factored by a dense Cholesky;
 *   4. forward and backward substitution with the whole factor.
 *
 * Block layouts (row-major n x n blocks, 0-based stages; stage k here is the paper's
 * stage k+1):
 *   D[S][N][n][n]    diagonal blocks, only the lower triangle is read
 *   E[S][N-1][n][n]  E[s][k] sits at block (k+1, k) of tail s, E^T at (k, k+1)
 *   C[S][n][n]       C[s] sits at block (root, stage 0), C^T at (stage 0, root)
 *   R[n][n]          root block, only the lower triangle is read
 *   b, x [nrhs][(S*N+1)*n]  each right-hand side in the order above
 *
 * info (LAPACK convention): 0 on success, else the 1-based natural row index of
 * the first non-positive pivot met in this natural elimination order (the smallest
 * over tails if several fail; root rows follow all tail rows).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double now_s(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* Band storage of one tail: AB[j*(p+1) + d] = K_s[j+d][j], 0 <= d <= p. */
static void assemble_tail(int N, int n, const double* D, const double* E,
                          const double* C, double* AB, double* W) {
  const int p = 2 * n - 1;
  const int64_t Nn = (int64_t)N * n;
  memset(AB, 0, sizeof(double) * (size_t)(p + 1) * (size_t)Nn);
  memset(W, 0, sizeof(double) * (size_t)n * (size_t)Nn);
  for (int k = 0; k < N; ++k) {
    const double* Dk = D + (size_t)k * n * n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j)
        AB[((int64_t)k * n + j) * (p + 1) + (i - j)] = Dk[i * n + j];
    if (k + 1 < N) {
      const double* Ek = E + (size_t)k * n * n;  /* block (k+1, k) */
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          AB[((int64_t)k * n + j) * (p + 1) + (n + i - j)] = Ek[i * n + j];
    }
  }
  /* Root rows: K[root r][stage 0, column j] = C[r][j]; zero elsewhere. */
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) W[(int64_t)r * Nn + j] = C[r * n + j];
}

/* Band Cholesky of one tail with its border, in place.  Returns 0 or the 1-based
 * tail-local row of the first non-positive pivot. */
static int64_t factor_tail(int N, int n, double* AB, double* W) {
  const int p = 2 * n - 1;
  const int64_t Nn = (int64_t)N * n;
  for (int64_t j = 0; j < Nn; ++j) {
    double* colj = AB + j * (p + 1);
    const double piv = colj[0];
    if (!(piv > 0.0)) return j + 1;
    const double ljj = sqrt(piv);
    colj[0] = ljj;
    const int64_t last = (j + p < Nn - 1) ? j + p : Nn - 1;
    for (int64_t i = j + 1; i <= last; ++i) colj[i - j] /= ljj;
    for (int r = 0; r < n; ++r) W[r * Nn + j] /= ljj;
    for (int64_t c = j + 1; c <= last; ++c) {
      const double lcj = colj[c - j];
      double* colc = AB + c * (p + 1);
      for (int64_t i = c; i <= last; ++i) colc[i - c] -= colj[i - j] * lcj;
      for (int r = 0; r < n; ++r) W[r * Nn + c] -= W[r * Nn + j] * lcj;
    }
  }
  return 0;
}

/* Dense lower Cholesky of an n x n row-major matrix in place (upper part zeroed). */
static int64_t dense_chol(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0.0)) return j + 1;
    const double ljj = sqrt(s);
    A[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / ljj;
    }
    for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
  }
  return 0;
}

typedef struct {
  int S, N, n;
  int64_t Nn;
  int p;
  double* AB; /* S * (p+1) * Nn */
  double* W;  /* S * n * Nn */
  double* U;  /* S * n * n : W_s W_s^T */
  double* LR; /* n * n */
  int64_t info;
} factor_t;

static int do_factor(factor_t* f, const double* D, const double* E,
                     const double* C, const double* R, int nthreads) {
  const int S = f->S, N = f->N, n = f->n, p = f->p;
  const int64_t Nn = f->Nn;
  int64_t* tinfo = (int64_t*)calloc((size_t)S, sizeof(int64_t));
  if (!tinfo) return -1;
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int s = 0; s < S; ++s) {
    double* AB = f->AB + (size_t)s * (p + 1) * Nn;
    double* W = f->W + (size_t)s * n * Nn;
    assemble_tail(N, n, D + (size_t)s * N * n * n,
                  E + (size_t)s * (N > 1 ? N - 1 : 0) * n * n,
                  C + (size_t)s * n * n, AB, W);
    tinfo[s] = factor_tail(N, n, AB, W);
    double* U = f->U + (size_t)s * n * n;
    for (int r1 = 0; r1 < n; ++r1)
      for (int r2 = 0; r2 <= r1; ++r2) {
        double acc = 0.0;
        for (int64_t j = 0; j < Nn; ++j) acc += W[r1 * Nn + j] * W[r2 * Nn + j];
        U[r1 * n + r2] = acc;
        U[r2 * n + r1] = acc;
      }
  }
  f->info = 0;
  for (int s = 0; s < S; ++s)
    if (tinfo[s] != 0) {
      f->info = (int64_t)s * Nn + tinfo[s];
      break;
    }
  free(tinfo);
  /* Root Schur complement R - sum_s W_s W_s^T, scenario order; then Cholesky. */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double rij = (i >= j) ? R[i * n + j] : R[j * n + i];
      double acc = 0.0;
      for (int s = 0; s < S; ++s) acc += f->U[(size_t)s * n * n + i * n + j];
      f->LR[i * n + j] = rij - acc;
    }
  const int64_t rinfo = dense_chol(n, f->LR);
  if (f->info == 0 && rinfo != 0) f->info = (int64_t)S * Nn + rinfo;
  return 0;
}

static void do_solve(const factor_t* f, int nrhs, const double* b, double* x,
                     int nthreads) {
  const int S = f->S, n = f->n, p = f->p;
  const int64_t Nn = f->Nn;
  const int64_t len = (int64_t)S * Nn + n;
  double* z = (double*)calloc((size_t)S * n, sizeof(double));
  double* x0 = (double*)calloc((size_t)n, sizeof(double));
  (void)nthreads;
  for (int q = 0; q < nrhs; ++q) {
    const double* bq = b + (size_t)q * len;
    double* xq = x + (size_t)q * len;
    /* forward: y_s = L_s^{-1} b_s ; z_s = W_s y_s */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int s = 0; s < S; ++s) {
      const double* AB = f->AB + (size_t)s * (p + 1) * Nn;
      const double* W = f->W + (size_t)s * n * Nn;
      double* y = xq + (size_t)s * Nn;
      memcpy(y, bq + (size_t)s * Nn, sizeof(double) * (size_t)Nn);
      for (int64_t j = 0; j < Nn; ++j) {
        const double* colj = AB + j * (p + 1);
        y[j] /= colj[0];
        const int64_t last = (j + p < Nn - 1) ? j + p : Nn - 1;
        for (int64_t i = j + 1; i <= last; ++i) y[i] -= colj[i - j] * y[j];
      }
      for (int r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int64_t j = 0; j < Nn; ++j) acc += W[r * Nn + j] * y[j];
        z[(size_t)s * n + r] = acc;
      }
    }
    /* root: L_R y_0 = b_0 - sum_s z_s ; L_R^T x_0 = y_0 */
    for (int r = 0; r < n; ++r) {
      double acc = bq[(size_t)S * Nn + r];
      for (int s = 0; s < S; ++s) acc -= z[(size_t)s * n + r];
      x0[r] = acc;
    }
    for (int i = 0; i < n; ++i) {
      double t = x0[i];
      for (int k = 0; k < i; ++k) t -= f->LR[i * n + k] * x0[k];
      x0[i] = t / f->LR[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = x0[i];
      for (int k = i + 1; k < n; ++k) t -= f->LR[k * n + i] * x0[k];
      x0[i] = t / f->LR[i * n + i];
    }
    for (int r = 0; r < n; ++r) xq[(size_t)S * Nn + r] = x0[r];
    /* backward: x_s = L_s^{-T} (y_s - W_s^T x_0) */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int s = 0; s < S; ++s) {
      const double* AB = f->AB + (size_t)s * (p + 1) * Nn;
      const double* W = f->W + (size_t)s * n * Nn;
      double* y = xq + (size_t)s * Nn;
      for (int64_t j = 0; j < Nn; ++j) {
        double acc = 0.0;
        for (int r = 0; r < n; ++r) acc += W[r * Nn + j] * x0[r];
        y[j] -= acc;
      }
      for (int64_t j = Nn - 1; j >= 0; --j) {
        const double* colj = AB + j * (p + 1);
        const int64_t last = (j + p < Nn - 1) ? j + p : Nn - 1;
        double t = y[j];
        for (int64_t i = j + 1; i <= last; ++i) t -= colj[i - j] * y[i];
        y[j] = t / colj[0];
      }
    }
  }
  free(z);
  free(x0);
}

static int alloc_factor(factor_t* f, int S, int N, int n) {
  f->S = S;
  f->N = N;
  f->n = n;
  f->p = 2 * n - 1;
  f->Nn = (int64_t)N * n;
  f->AB = (double*)malloc(sizeof(double) * (size_t)S * (f->p + 1) * (size_t)f->Nn);
  f->W = (double*)malloc(sizeof(double) * (size_t)S * n * (size_t)f->Nn);
  f->U = (double*)malloc(sizeof(double) * (size_t)S * n * n);
  f->LR = (double*)malloc(sizeof(double) * (size_t)n * n);
  f->info = 0;
  if (!f->AB || !f->W || !f->U || !f->LR) return -1;
  return 0;
}

static void free_factor(factor_t* f) {
  free(f->AB);
  free(f->W);
  free(f->U);
  free(f->LR);
}

/* Number of OpenMP threads a parallel region would use with this request. */
int oracle_threads(int nthreads) {
#ifdef _OPENMP
  int got = 1;
#pragma omp parallel num_threads(nthreads)
  {
#pragma omp single
    got = omp_get_num_threads();
  }
  return got;
#else
  (void)nthreads;
  return 1;
#endif
}

/* Factor and solve.  Returns 0, or -1 on bad arguments / allocation failure.
 * times (optional, may be NULL): times[0] = factor seconds, times[1] = solve s. */
int oracle_solve(int S, int N, int n, int nrhs, const double* D, const double* E,
                 const double* C, const double* R, const double* b, double* x,
                 int nthreads, double* times, int64_t* info) {
  if (S < 1 || N < 1 || n < 1 || nrhs < 1 || nthreads < 1) return -1;
  factor_t f;
  if (alloc_factor(&f, S, N, n) != 0) {
    free_factor(&f);
    return -1;
  }
  const double t0 = now_s();
  if (do_factor(&f, D, E, C, R, nthreads) != 0) {
    free_factor(&f);
    return -1;
  }
  const double t1 = now_s();
  if (f.info == 0) do_solve(&f, nrhs, b, x, nthreads);
  const double t2 = now_s();
  if (times) {
    times[0] = t1 - t0;
    times[1] = t2 - t1;
  }
  if (info) *info = f.info;
  free_factor(&f);
  return 0;
}

/* Export the natural-order factor for small reconstruction checks:
 * AB[S][Nn][p+1] band columns, W[S][n][Nn] border rows, LR[n][n]. */
int oracle_factor_export(int S, int N, int n, const double* D, const double* E,
                         const double* C, const double* R, double* AB, double* W,
                         double* LR, int64_t* info) {
  if (S < 1 || N < 1 || n < 1) return -1;
  factor_t f;
  if (alloc_factor(&f, S, N, n) != 0) {
    free_factor(&f);
    return -1;
  }
  do_factor(&f, D, E, C, R, 1);
  memcpy(AB, f.AB, sizeof(double) * (size_t)S * (f.p + 1) * (size_t)f.Nn);
  memcpy(W, f.W, sizeof(double) * (size_t)S * n * (size_t)f.Nn);
  memcpy(LR, f.LR, sizeof(double) * (size_t)n * n);
  if (info) *info = f.info;
  free_factor(&f);
  return 0;
}
