/*
 * Driver for running the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure; built with gcc by tests/test_sanitizers.py, never on a GPU).
 *
 * It draws small block-diagonally dominant systems with a fixed linear congruential
 * generator, solves them with one and with two OpenMP threads, and checks the normwise
 * backward error of the solutions, the bitwise agreement of the two thread counts, the
 * factor export, a non-SPD input (info set) and rejected arguments.  Exit status 0 means
 * every check passed and the sanitizers reported nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_solve(int S, int N, int n, int nrhs, const double* D, const double* E,
                 const double* C, const double* R, const double* b, double* x,
                 int nthreads, double* times, int64_t* info);
int oracle_factor_export(int S, int N, int n, const double* D, const double* E,
                         const double* C, const double* R, double* AB, double* W,
                         double* LR, int64_t* info);

static uint64_t state = 88172645463325252ull;
static double unif(void) { /* in [-1, 1) */
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

/* y = K x for one right-hand side (blocks as the oracle reads them). */
static void kmul(int S, int N, int n, const double* D, const double* E, const double* C,
                 const double* R, const double* x, double* y, double* knorm) {
  const int64_t len = ((int64_t)S * N + 1) * n;
  double* rowabs = calloc((size_t)len, sizeof(double));
  memset(y, 0, sizeof(double) * (size_t)len);
  const double* x0 = x + (int64_t)S * N * n;
  double* y0 = y + (int64_t)S * N * n;
  for (int s = 0; s < S; ++s) {
    for (int k = 0; k < N; ++k) {
      const double* d = D + (((int64_t)s * N + k) * n) * n;
      const int64_t o = ((int64_t)s * N + k) * n;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const double v = i >= j ? d[i * n + j] : d[j * n + i];
          y[o + i] += v * x[o + j];
          rowabs[o + i] += fabs(v);
        }
      if (k + 1 < N) {
        const double* e = E + (((int64_t)s * (N - 1) + k) * n) * n;  /* block (k+1, k) */
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            y[o + n + i] += e[i * n + j] * x[o + j];
            y[o + j] += e[i * n + j] * x[o + n + i];
            rowabs[o + n + i] += fabs(e[i * n + j]);
            rowabs[o + j] += fabs(e[i * n + j]);
          }
      }
    }
    const double* c = C + (int64_t)s * n * n;  /* block (root, stage 0) */
    const int64_t o = (int64_t)s * N * n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        y0[i] += c[i * n + j] * x[o + j];
        y[o + j] += c[i * n + j] * x0[i];
        rowabs[(int64_t)S * N * n + i] += fabs(c[i * n + j]);
        rowabs[o + j] += fabs(c[i * n + j]);
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double v = i >= j ? R[i * n + j] : R[j * n + i];
      y0[i] += v * x0[j];
      rowabs[(int64_t)S * N * n + i] += fabs(v);
    }
  *knorm = 0.0;
  for (int64_t i = 0; i < len; ++i) *knorm = fmax(*knorm, rowabs[i]);
  free(rowabs);
}

static int run(int S, int N, int n, int nrhs, double shift) {
  const int64_t nn = (int64_t)n * n, len = ((int64_t)S * N + 1) * n;
  double* D = malloc(sizeof(double) * (size_t)(S * N * nn));
  double* E = malloc(sizeof(double) * (size_t)(S * (N > 1 ? N - 1 : 1) * nn));
  double* C = malloc(sizeof(double) * (size_t)(S * nn));
  double* R = malloc(sizeof(double) * (size_t)nn);
  double* b = malloc(sizeof(double) * (size_t)(nrhs * len));
  double* x1 = malloc(sizeof(double) * (size_t)(nrhs * len));
  double* x2 = malloc(sizeof(double) * (size_t)(nrhs * len));
  double* y = malloc(sizeof(double) * (size_t)len);
  for (int64_t i = 0; i < S * (N > 1 ? N - 1 : 1) * nn; ++i) E[i] = 0.3 * unif() / n;
  for (int64_t i = 0; i < S * nn; ++i) C[i] = 0.3 * unif() / n;
  for (int64_t blk = 0; blk < (int64_t)S * N; ++blk)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) D[blk * nn + i * n + j] = (i == j) ? 2.0 + unif() * 0.1 : 0.1 * unif() / n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) R[i * n + j] = (i == j) ? 1.0 + 0.3 * S : 0.1 * unif() / n;
  D[0] -= shift;  /* shift < 0 leaves the system SPD; a large positive one breaks it */
  for (int64_t i = 0; i < nrhs * len; ++i) b[i] = unif();
  int64_t info1 = -7, info2 = -7;
  double times[2];
  int bad = 0;
  if (oracle_solve(S, N, n, nrhs, D, E, C, R, b, x1, 1, times, &info1) != 0) bad = 1;
  if (oracle_solve(S, N, n, nrhs, D, E, C, R, b, x2, 2, times, &info2) != 0) bad = 1;
  if (shift > 0.0) {
    if (info1 != 1 || info2 != 1) { fprintf(stderr, "info %lld %lld\n", (long long)info1, (long long)info2); bad = 1; }
  } else {
    if (info1 != 0 || info2 != 0) bad = 1;
    if (memcmp(x1, x2, sizeof(double) * (size_t)(nrhs * len)) != 0) { fprintf(stderr, "threads differ\n"); bad = 1; }
    for (int q = 0; q < nrhs && !bad; ++q) {
      double knorm, rmax = 0, xmax = 0, bmax = 0;
      kmul(S, N, n, D, E, C, R, x1 + q * len, y, &knorm);
      for (int64_t i = 0; i < len; ++i) {
        rmax = fmax(rmax, fabs(b[q * len + i] - y[i]));
        xmax = fmax(xmax, fabs(x1[q * len + i]));
        bmax = fmax(bmax, fabs(b[q * len + i]));
      }
      const double be = rmax / (knorm * xmax + bmax);
      if (!(be <= 10 * 2.220446049250313e-16)) { fprintf(stderr, "backward error %g\n", be); bad = 1; }
    }
    const int p = 2 * n - 1;
    const int64_t Nn = (int64_t)N * n;
    double* AB = malloc(sizeof(double) * (size_t)(S * (p + 1) * Nn));
    double* W = malloc(sizeof(double) * (size_t)(S * n * Nn));
    double* LR = malloc(sizeof(double) * (size_t)nn);
    int64_t info3 = -7;
    if (oracle_factor_export(S, N, n, D, E, C, R, AB, W, LR, &info3) != 0 || info3 != 0) bad = 1;
    for (int i = 0; i < n && !bad; ++i)
      if (!(LR[i * n + i] > 0.0)) bad = 1;
    free(AB); free(W); free(LR);
  }
  free(D); free(E); free(C); free(R); free(b); free(x1); free(x2); free(y);
  return bad;
}

int main(void) {
  int bad = 0;
  const int shapes[][4] = {{1, 1, 1, 1}, {3, 1, 5, 2}, {2, 2, 3, 1}, {3, 9, 4, 2},
                           {2, 17, 8, 1}, {4, 33, 3, 3}, {2, 16, 16, 1}};
  for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i) {
    const int* sh = shapes[i];
    if (run(sh[0], sh[1], sh[2], sh[3], -0.0)) { fprintf(stderr, "case %zu failed\n", i); bad = 1; }
  }
  if (run(2, 5, 3, 1, 50.0)) { fprintf(stderr, "non-SPD case failed\n"); bad = 1; }
  double z = 0;
  int64_t info;
  if (oracle_solve(0, 4, 3, 1, &z, &z, &z, &z, &z, &z, 1, NULL, &info) != -1) bad = 1;
  if (oracle_solve(2, 4, 3, 0, &z, &z, &z, &z, &z, &z, 1, NULL, &info) != -1) bad = 1;
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
