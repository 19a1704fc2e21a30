/* CPU FP64 oracle for the GWAS grid of generalised least-squares problems.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
 * baseline call it; the GPU library never links, loads or calls it, and it
 * shares no code with that library.
 *
 * It evaluates the problem statement of the supplementary notes (the "probDef"
 * equation, with the GLS estimator and its variance of section 1) by the
 * plain Cholesky route of the single-instance CLAK-Chol algorithm (section 2),
 * once per (SNP, trait) cell:
 *   M_j  = s2_j (h2_j Phi + (1 - h2_j) I)
 *   L_j L_j^T = M_j
 *   X'   = L_j^{-1} [X_L | g_i],  y' = L_j^{-1} y_j
 *   S    = X'^T X',  r = X'^T y'
 *   b_ij = S^{-1} r,  Var(b_ij) = S^{-1}      (var_conv = 0, model-consistent)
 *                     Var(b_ij) = s2_j S^{-1}  (var_conv = 1, as printed)
 * All matrices are column-major with explicit leading dimensions.
 */
#ifndef CLAK_ORACLE_H
#define CLAK_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Relative pivot test of chol(S): a pivot is degenerate when pivot^2 <=
 * ORACLE_DEGEN_TOL * S_jj.  For the SNP's (last) pivot, pivot^2 / S_pp is the
 * share of the SNP's M_j^{-1}-weighted squared norm left after projecting it
 * on the covariates.  Overridable at compile time only so that a test can
 * build a deliberately wrong oracle and check that the pins notice. */
#ifndef ORACLE_DEGEN_TOL
#define ORACLE_DEGEN_TOL 1e-10
#endif

/* Per-cell flags written by oracle_gls. */
#define ORACLE_OK 0
#define ORACLE_SNP_DEGENERATE 1   /* last pivot of chol(S): pivot^2 <= ORACLE_DEGEN_TOL * S_pp */
#define ORACLE_M_NOT_SPD 2        /* chol(M_j) failed */
#define ORACLE_COV_SINGULAR 3     /* a covariate pivot of chol(S) failed */

/* n individuals, pL covariate columns, p = pL + 1.
 * Phi  n x n (ldphi), XL n x pL (ldxl), G n x (#SNP columns) (ldg),
 * Y n x (#traits) (ldy), h2[], s2[] per trait.
 * Cell c is (SNP column snp[c] of G, trait trait[c]).
 * Outputs: b[c*p + k], var[c*p*p + k + l*p] (column-major p x p), flag[c].
 * Cells whose flag is not ORACLE_OK get NaN in b and var.
 * threads <= 0 uses every available thread.
 * Returns 0, or -1 on a bad argument (nothing written). */
int oracle_gls(int64_t n, int64_t pL, const double* Phi, int64_t ldphi,
               const double* XL, int64_t ldxl, const double* G, int64_t ldg,
               const double* Y, int64_t ldy, const double* h2, const double* s2,
               int64_t n_cells, const int64_t* snp, const int64_t* trait,
               int var_conv, double* b, double* var, int32_t* flag, int threads);

/* Number of threads oracle_gls uses for a given request. */
int oracle_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
