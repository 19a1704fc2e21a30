/* CPU FP64 oracle for the GWAS GLS grid: TEST INFRASTRUCTURE ONLY.
 * See oracle.h for the definition it evaluates and who may call it.
 * Plain, unblocked code: correctness by inspection, not speed. */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(int threads) {
#ifdef _OPENMP
  return threads > 0 ? threads : omp_get_max_threads();
#else
  (void)threads;
  return 1;
#endif
}

static double dot(const double* a, const double* b, int64_t len) {
  double s = 0.0;
  for (int64_t k = 0; k < len; ++k) s += a[k] * b[k];
  return s;
}

/* In-place Cholesky A = L L^T of a symmetric n x n matrix held row-major in
 * L (row i at L + i*n; entries k <= i used, the rest ignored).  Column by
 * column: L[j][j] = sqrt(A[j][j] - sum_k<j L[j][k]^2), then every L[i][j],
 * i > j, = (A[i][j] - sum_k<j L[i][k] L[j][k]) / L[j][j].
 * Returns -1 on success, else the index of the first non-positive pivot. */
static int64_t chol_rows(double* L, int64_t n, int nthr) {
  for (int64_t j = 0; j < n; ++j) {
    double* Lj = L + j * n;
    double d = Lj[j] - dot(Lj, Lj, j);
    if (!(d > 0.0)) return j;
    Lj[j] = sqrt(d);
    const double piv = Lj[j];
#pragma omp parallel for num_threads(nthr) schedule(static) if (n - j > 256)
    for (int64_t i = j + 1; i < n; ++i) {
      double* Li = L + i * n;
      Li[j] = (Li[j] - dot(Li, Lj, j)) / piv;
    }
  }
  return -1;
}

/* Forward substitution L x = v, L row-major lower (as left by chol_rows). */
static void fwd_rows(const double* L, int64_t n, double* x) {
  for (int64_t i = 0; i < n; ++i) {
    const double* Li = L + i * n;
    x[i] = (x[i] - dot(Li, x, i)) / Li[i];
  }
}

static int cmp_cells(const void* a, const void* b, void* ctx) {
  const int64_t* tr = (const int64_t*)ctx;
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  if (tr[x] != tr[y]) return tr[x] < tr[y] ? -1 : 1;
  return x < y ? -1 : (x > y);
}

/* One cell: X' = [XLp | gp] (n x p, column-major), y'.  Solves the p x p
 * normal equations by Cholesky; writes b, var (unscaled S^{-1}); returns flag. */
static int32_t solve_cell(int64_t n, int64_t p, const double* Xp, const double* yp,
                          double* b, double* var) {
  double S[32 * 32], r[32], Ls[32 * 32];
  for (int64_t k = 0; k < p; ++k) {
    r[k] = dot(Xp + k * n, yp, n);
    for (int64_t l = 0; l <= k; ++l) S[k * p + l] = S[l * p + k] = dot(Xp + k * n, Xp + l * n, n);
  }
  /* Cholesky of S, row-major lower in Ls, with the relative pivot test. */
  for (int64_t j = 0; j < p; ++j) {
    for (int64_t i = j; i < p; ++i) {
      double s = S[i * p + j];
      for (int64_t k = 0; k < j; ++k) s -= Ls[i * p + k] * Ls[j * p + k];
      if (i == j) {
        if (!(s > ORACLE_DEGEN_TOL * S[j * p + j])) return j == p - 1 ? ORACLE_SNP_DEGENERATE : ORACLE_COV_SINGULAR;
        Ls[j * p + j] = sqrt(s);
      } else {
        Ls[i * p + j] = s / Ls[j * p + j];
      }
    }
  }
  /* b = S^{-1} r: L z = r, then L^T b = z. */
  double z[32];
  for (int64_t i = 0; i < p; ++i) {
    double s = r[i];
    for (int64_t k = 0; k < i; ++k) s -= Ls[i * p + k] * z[k];
    z[i] = s / Ls[i * p + i];
  }
  for (int64_t i = p - 1; i >= 0; --i) {
    double s = z[i];
    for (int64_t k = i + 1; k < p; ++k) s -= Ls[k * p + i] * b[k];
    b[i] = s / Ls[i * p + i];
  }
  /* S^{-1}: the same two solves for every unit vector. */
  for (int64_t c = 0; c < p; ++c) {
    double e[32], w[32];
    for (int64_t i = 0; i < p; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) s -= Ls[i * p + k] * e[k];
      e[i] = s / Ls[i * p + i];
    }
    for (int64_t i = p - 1; i >= 0; --i) {
      double s = e[i];
      for (int64_t k = i + 1; k < p; ++k) s -= Ls[k * p + i] * w[k];
      w[i] = s / Ls[i * p + i];
    }
    for (int64_t i = 0; i < p; ++i) var[i + c * p] = w[i];
  }
  return ORACLE_OK;
}

int oracle_gls(int64_t n, int64_t pL, const double* Phi, int64_t ldphi,
               const double* XL, int64_t ldxl, const double* G, int64_t ldg,
               const double* Y, int64_t ldy, const double* h2, const double* s2,
               int64_t n_cells, const int64_t* snp, const int64_t* trait,
               int var_conv, double* b, double* var, int32_t* flag, int threads) {
  const int64_t p = pL + 1;
  if (n < 1 || pL < 0 || p > 32 || n_cells < 0 || ldphi < n || ldxl < n || ldg < n || ldy < n)
    return -1;
  if (n_cells == 0) return 0;
  if (!Phi || !G || !Y || !h2 || !s2 || !snp || !trait || !b || !var || !flag || (pL > 0 && !XL))
    return -1;
  for (int64_t c = 0; c < n_cells; ++c)
    if (snp[c] < 0 || trait[c] < 0) return -1;
  const int nthr = oracle_threads(threads);
  const double nan = NAN;

  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * n_cells);
  for (int64_t c = 0; c < n_cells; ++c) order[c] = c;
  qsort_r(order, n_cells, sizeof(int64_t), cmp_cells, (void*)trait);

  double* L = (double*)malloc(sizeof(double) * n * n);
  double* XLp = (double*)malloc(sizeof(double) * n * (p + 1)); /* [X_L' | y'] */

  for (int64_t c0 = 0; c0 < n_cells;) {
    const int64_t j = trait[order[c0]];
    int64_t c1 = c0;
    while (c1 < n_cells && trait[order[c1]] == j) ++c1;

    /* M_j = s2 (h2 Phi + (1 - h2) I), row-major lower copy (M is symmetric). */
    const double sj = s2[j], hj = h2[j];
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k <= i; ++k)
        L[i * n + k] = sj * (hj * Phi[i + k * ldphi] + (i == k ? 1.0 - hj : 0.0));
    const int spd = chol_rows(L, n, nthr) < 0;

    if (spd) {
      /* X_L' = L^{-1} X_L and y' = L^{-1} y_j, shared by the trait's cells. */
#pragma omp parallel for num_threads(nthr)
      for (int64_t k = 0; k <= pL; ++k) {
        double* x = XLp + k * n;
        const double* src = (k < pL) ? XL + k * ldxl : Y + j * ldy;
        memcpy(x, src, sizeof(double) * n);
        fwd_rows(L, n, x);
      }
    }

#pragma omp parallel num_threads(nthr)
    {
      double* Xp = (double*)malloc(sizeof(double) * n * p);
#pragma omp for schedule(dynamic, 4)
      for (int64_t q = c0; q < c1; ++q) {
        const int64_t c = order[q];
        double* bc = b + c * p;
        double* vc = var + c * p * p;
        int32_t f = ORACLE_M_NOT_SPD;
        if (spd) {
          if (pL > 0) memcpy(Xp, XLp, sizeof(double) * n * pL);
          double* gp = Xp + pL * n;
          memcpy(gp, G + snp[c] * ldg, sizeof(double) * n);
          fwd_rows(L, n, gp);
          f = solve_cell(n, p, Xp, XLp + pL * n, bc, vc);
        }
        flag[c] = f;
        if (f != ORACLE_OK) {
          for (int64_t k = 0; k < p; ++k) bc[k] = nan;
          for (int64_t k = 0; k < p * p; ++k) vc[k] = nan;
        } else if (var_conv == 1) {
          for (int64_t k = 0; k < p * p; ++k) vc[k] *= sj;
        }
      }
      free(Xp);
    }
    c0 = c1;
  }
  free(L);
  free(XLp);
  free(order);
  return 0;
}
