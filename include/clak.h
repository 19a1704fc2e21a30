/* clak.h — C ABI of the MI355X CLAK-Eig library (libclak.so).
 *
 * The library solves the two-dimensional grid of generalised least-squares
 * problems of the supplementary notes (section 1, equation probDef): for every
 * SNP i and trait j
 *
 *     b_ij   = (X_i^T M_j^{-1} X_i)^{-1} X_i^T M_j^{-1} y_j,
 *     M_j    = s2_j (h2_j Phi + (1 - h2_j) I),   X_i = [X_L | g_i],
 *
 * by the multi-trait CLAK-Eig algorithm (section 3, the CLAK-Eig listing for
 * multi-trait analysis): Phi = Z W Z^T is eigendecomposed once, X_L, the SNP
 * columns and Y are rotated by Z^T, and every (SNP, trait) cell reduces to
 * diagonal-weighted sums over the n individuals plus a Schur-complement solve
 * of the partitioned p x p system S b = [b_T ; W_R^T Y_j] (p = p_L + 1).
 *
 * Conventions
 *   - Every pointer argument named d_* is a DEVICE pointer on the device that
 *     was current when the plan was created, or a pointer to pinned host
 *     memory that the device sees at the same address (hipHostMalloc); a
 *     genotype block there is read over PCIe by the ingest kernel.  Any other
 *     pointer (pageable host memory, another device's memory) is refused with
 *     CLAK_E_ARG before any device work.  All matrices are column-major with
 *     an explicit leading dimension; all sizes are int64_t.
 *   - The caller owns every buffer it passes in (inputs, outputs and the
 *     workspace).  The library owns only the opaque plan (host memory plus a
 *     rocBLAS handle), released by clak_plan_destroy.  It never frees caller
 *     memory.
 *   - No C++ exception and no abort crosses the ABI: every entry point returns
 *     a clak_status and, on failure, sets a thread-local message readable with
 *     clak_last_error().
 *   - Host-side argument checks (sizes, leading dimensions, null pointers,
 *     call order) run before any device work.  Checks that need device data
 *     (h2 range, s2 > 0, positive definiteness) run on the device inside the
 *     synchronous set-up calls, which report them through their status.
 *   - clak_run_block is asynchronous on the plan's stream.  A device fault
 *     surfaces at the next synchronising call.
 *
 * Call order for one cohort
 *   clak_plan_create -> clak_plan_workspace_size -> clak_plan_set_workspace
 *   [-> clak_plan_set_stream] -> clak_set_kinship | clak_set_eigen
 *   -> clak_set_covariates -> clak_set_traits -> clak_run_block (any number of
 *   times) -> clak_plan_destroy.
 *   clak_set_traits may be repeated (new phenotypes, same kinship and
 *   covariates); clak_set_covariates may be repeated (it invalidates the
 *   traits); clak_set_kinship/clak_set_eigen may be repeated (it invalidates
 *   covariates and traits).  Any other order returns CLAK_E_STATE.
 */
#ifndef CLAK_H
#define CLAK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum clak_status {
  CLAK_OK = 0,
  CLAK_E_ARG = 1,           /* bad size, leading dimension, null pointer, NaN/Inf, h2 outside [0,1], s2 <= 0 */
  CLAK_E_STATE = 2,         /* call out of order */
  CLAK_E_NOT_SPD = 3,       /* some h2_j w_k + 1 - h2_j <= 0: M_j not positive definite */
  CLAK_E_COV_SINGULAR = 4,  /* X_L rank deficient, or X_L^T M_j^{-1} X_L not positive definite */
  CLAK_E_EIG = 5,           /* the eigensolver did not converge */
  CLAK_E_WORKSPACE = 6,     /* workspace missing, too small or misaligned */
  CLAK_E_DEVICE = 7,        /* HIP or rocSOLVER failure */
  CLAK_E_UNSUPPORTED = 8    /* size beyond what the chosen precision supports */
} clak_status;

/* Arithmetic of the per-block path (set-up is FP64 in both).
 *   CLAK_PREC_FP64  : rotation and grid sums on FP64 MFMA.
 *   CLAK_PREC_MIXED : Z^T split into four int8 digit planes per eigenvector,
 *                     rotation by int8 MFMA with exact int32 accumulation,
 *                     rotated SNPs and the per-trait operand re-encoded as
 *                     four int8 digit planes, grid sums by int8 MFMA with
 *                     exact int32 accumulation (digit products of total
 *                     weight 256^-4 and below dropped); FP64 Schur solve. */
typedef enum clak_precision { CLAK_PREC_FP64 = 0, CLAK_PREC_MIXED = 1 } clak_precision;

/* Plan flags (bitwise or). */
#define CLAK_VAR_MODEL 0u   /* Var(b) = (X^T M^{-1} X)^{-1}                       */
#define CLAK_VAR_PAPER 1u   /* Var(b) = s2_j (X^T M^{-1} X)^{-1}, as printed        */
#define CLAK_OUT_SNP 0u     /* write the SNP effect b_ij[p-1] only                 */
#define CLAK_OUT_FULL 2u    /* write all p components of b_ij                      */
#define CLAK_STAGE_GENOTYPES 4u /* reserve a staging buffer per workspace slot: every
                                   genotype block is first copied there by the copy
                                   engine on the ingest stream (over PCIe from pinned
                                   host memory, within HBM from device memory) into
                                   16-byte-aligned rows, then ingested.  Without the
                                   flag the ingest kernel reads the caller's block,
                                   also a pinned host block over PCIe.            */
#define CLAK_CHOL 8u        /* single trait (t = 1) by CLAK-Chol (section 2): no
                               eigendecomposition.  clak_set_kinship keeps Phi;
                               clak_set_traits factors H = h2 Phi + (1 - h2) I =
                               U^T U (FP64 Cholesky) and rotates by U^-T, a lower-
                               triangular matrix, in place of Z^T, with unit
                               weights (M^-1 = U^-1 U^-T / s2), so the SNP rotation
                               skips the zero half of the matrix.  clak_set_eigen
                               and clak_estimate_vc need eigenpairs and return
                               CLAK_E_UNSUPPORTED for such a plan.              */

/* Genotype element types accepted by clak_run_block (values 0, 1, 2).
 *   CLAK_G_U8 : one byte per individual; ldg in elements.
 *   CLAK_G_F16: one half per individual; ldg in elements.
 *   CLAK_G_P2 : the SNP-major 2-bit codes of the PLINK 1 binary genotype
 *               format, four individuals per byte, individual i in bits
 *               2 (i % 4) and 2 (i % 4) + 1 of byte i / 4 of its SNP row;
 *               codes 00, 10, 11 are 2, 1, 0 copies of the first allele and
 *               01 is missing (the SNP is flagged CLAK_CELL_BAD_GENOTYPE);
 *               ldg in bytes, at least (n + 3) / 4. */
#define CLAK_G_U8 0
#define CLAK_G_F16 1
#define CLAK_G_P2 2
/* Output element types. */
#define CLAK_OUT_F32 0
#define CLAK_OUT_F64 1

/* Per-cell flag values written by clak_run_block. */
#define CLAK_CELL_OK 0
#define CLAK_CELL_DEGENERATE 1  /* g_i in span(X_L) (or numerically so): b and SE are NaN */
#define CLAK_CELL_BAD_GENOTYPE 2 /* a genotype of the SNP is not 0, 1 or 2 (or is missing): b and SE are NaN */

typedef struct clak_plan_s* clak_plan_t;

/* Creates a plan for n individuals, p_L covariate columns (X_L, normally the
 * intercept first), t traits and SNP blocks of at most max_block columns.
 * Allocates host memory and a rocBLAS handle only; no device memory.
 * Requires 1 <= p_L <= 16, n > p_L, t >= 1, max_block >= 1; MIXED requires
 * p_L <= 8 and n <= 32000 (int32 accumulation bound).  Errors: CLAK_E_ARG, CLAK_E_UNSUPPORTED,
 * CLAK_E_DEVICE. */
clak_status clak_plan_create(clak_plan_t* plan, int64_t n, int64_t p_L, int64_t t,
                             int64_t max_block, int precision, uint32_t flags);

/* Bytes of device workspace the plan needs (every buffer of the path: Z and
 * its digit planes, rotated covariates and traits, per-trait operands and one
 * SNP block's staging).  Always a multiple of 256. */
clak_status clak_plan_workspace_size(clak_plan_t plan, size_t* bytes);

/* Hands the plan a caller-owned device buffer of at least
 * clak_plan_workspace_size bytes, 256-byte aligned.  It must stay allocated
 * until the plan is destroyed or given another workspace (which resets the
 * plan to the "no kinship" state).  Errors: CLAK_E_WORKSPACE. */
clak_status clak_plan_set_workspace(clak_plan_t plan, void* d_ws, size_t bytes);

/* HIP stream (hipStream_t, may be NULL for the default stream) on which every
 * kernel of the plan is enqueued. */
clak_status clak_plan_set_stream(clak_plan_t plan, void* hip_stream);

/* The eigendecomposition that opens CLAK-Eig (section 3): Phi = Z W Z^T by the
 * FP64 rocSOLVER divide and conquer eigensolver, then the int8 digit planes of Z^T (MIXED).
 * d_Phi: n x n symmetric, leading dimension ld >= n; only its lower triangle
 * is read; it is not modified.  Synchronous.  Errors: CLAK_E_ARG, CLAK_E_STATE,
 * CLAK_E_EIG, CLAK_E_DEVICE. */
clak_status clak_set_kinship(clak_plan_t plan, const double* d_Phi, int64_t ld);

/* Alternative to clak_set_kinship: supplies Z (n x n orthonormal columns,
 * leading dimension ldz) and w (n eigenvalues) of Phi directly.  Any
 * orthonormal eigenbasis gives the same results.  Synchronous. */
clak_status clak_set_eigen(clak_plan_t plan, const double* d_Z, int64_t ldz, const double* d_w);

/* The rotation of the covariates (X_L := Z^T X_L, section 3) plus the per-SNP
 * centring basis: X_L = Q_L R (FP64 Gram-Schmidt, twice), Z^T X_L and Z^T Q_L.  d_XL: n x p_L,
 * leading dimension ld >= n.  Synchronous.  Errors: CLAK_E_ARG, CLAK_E_STATE,
 * CLAK_E_COV_SINGULAR (rank-deficient X_L), CLAK_E_DEVICE. */
clak_status clak_set_covariates(clak_plan_t plan, const double* d_XL, int64_t ld);

/* The rotation of the phenotypes (Y := Z^T Y, section 3) and the per-trait
 * part of the loop over traits: D_j = (s2_j (h2_j W + (1 - h2_j) I))^{-1}, S_TL,j = X_L^T D_j X_L (rotated
 * X_L), b_T,j, its Cholesky factor, and the per-trait operand of the grid
 * contraction.  d_Y: n x t, leading dimension ldy >= n; d_h2, d_s2: t values.
 * Synchronous.  Errors: CLAK_E_ARG (h2 outside [0,1], s2 <= 0, non-finite
 * values), CLAK_E_STATE, CLAK_E_NOT_SPD, CLAK_E_COV_SINGULAR, CLAK_E_DEVICE. */
clak_status clak_set_traits(clak_plan_t plan, const double* d_Y, int64_t ldy,
                            const double* d_h2, const double* d_s2);

/* Variance components of the reduced model y_j ~ N(X_L beta_j, s2_j (h2_j Phi
 * + (1 - h2_j) I)) for every trait: the first step of the two-step analysis
 * (section 1), by maximum likelihood or restricted maximum likelihood (the
 * parameter estimation discussed in section 4).  beta_j and s2_j are profiled
 * out in closed form; h2_j maximises the profile log-likelihood over [0, 1]
 * (101 evenly spaced points, then a golden-section search on the bracket
 * around the best of them down to a width of 1e-7).  Each evaluation costs
 * O(n p_L^2) through the eigendecomposition of Phi (eigenvalues h2 w_k + 1 - h2).
 *   method   : CLAK_VC_ML or CLAK_VC_REML.
 *   d_Y      : n x t phenotypes (t of the plan), leading dimension ldy >= n.
 *   d_h2, d_s2: t estimates each, written by the call (device memory).
 *   d_loglik : t maximised log-likelihoods (NULL allowed).
 * Needs set_covariates; the traits need not be set, and set traits stay valid
 * (the call rotates d_Y into the workspace's phenotype buffer, which run_block
 * does not read).  The outputs feed clak_set_traits directly.  Synchronous.
 * Errors: CLAK_E_ARG (non-finite y: that trait's outputs are NaN),
 * CLAK_E_STATE, CLAK_E_COV_SINGULAR, CLAK_E_DEVICE. */
#define CLAK_VC_ML 0
#define CLAK_VC_REML 1
clak_status clak_estimate_vc(clak_plan_t plan, const double* d_Y, int64_t ldy, int method, double* d_h2,
                             double* d_s2, double* d_loglik);

/* The rotation of one block of SNPs (X_R := Z^T X_R, section 3) and the inner
 * loop over (SNP, trait) cells of that block: W_R^T W_L, W_R^T W_R, W_R^T Y_j
 * as contractions over n, then b_ij := S^{-1} b_ij, optionally with the
 * p-value of the SNP effect (the estimates come with their p-values in the
 * problem statement of section 1).  Asynchronous.
 *   d_G     : n x m_blk genotypes (column = one SNP), element type g_dtype,
 *             leading dimension ldg (one row of n genotypes at least).
 *   d_b     : SNP effects; with CLAK_OUT_SNP element (i, j) at d_b[i + j*ldo],
 *             with CLAK_OUT_FULL component c at d_b[(i + j*ldo)*p + c].
 *   d_se    : standard error of the SNP effect, element (i, j) at d_se[i + j*ldo].
 *   out_dtype: CLAK_OUT_F32 or CLAK_OUT_F64 for d_b, d_se and d_pval.
 *   ldo     : >= m_blk.
 *   d_flags : optional (NULL allowed) per-cell flags at d_flags[i + j*ldo].
 *   d_pval  : optional (NULL allowed) two-sided p-value of the Wald statistic
 *             z = b_snp / SE at d_pval[i + j*ldo]: P(|N(0,1)| > |z|) =
 *             erfc(|z| / sqrt 2), equal to the chi-square(1) tail at z^2;
 *             computed in FP64 (F32 output underflows to 0 below about
 *             1e-45, F64 below about 1e-308, |z| > 37.5); NaN on a flagged cell.
 * 1 <= m_blk <= max_block.  Errors: CLAK_E_ARG, CLAK_E_STATE, CLAK_E_DEVICE. */
clak_status clak_run_block(clak_plan_t plan, int64_t m_blk, const void* d_G, int g_dtype,
                           int64_t ldg, void* d_b, void* d_se, int out_dtype, int64_t ldo,
                           uint8_t* d_flags, void* d_pval);

/* For callers that cannot allocate device memory around a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * clak_run_block_static is clak_run_block with the block's scratch buffers
 * (genotype panel, per-SNP statistics, partial sums, rotated SNPs and their
 * digit planes) in a device array of the library, one per GPU, of
 * CLAK_STATIC_SCRATCH_BYTES, instead of the plan's workspace slot.  It calls
 * no hipMalloc, hipFree or other allocating routine (the plan, its workspace
 * and every set-up call still have to come first).  The array keeps the last
 * call's contents; calls on one GPU share it, so calls that overlap on one
 * GPU (several streams, several plans) race.  Same arguments, outputs and
 * asynchrony as clak_run_block.  Errors: as clak_run_block; CLAK_E_UNSUPPORTED
 * when the plan's block scratch (clak_plan_block_scratch_size) exceeds the
 * array or the plan has CLAK_STAGE_GENOTYPES; CLAK_E_STATE while the stage
 * profiler is on; CLAK_E_DEVICE when the plan's device is not current. */
#define CLAK_STATIC_SCRATCH_BYTES (64u << 20)
clak_status clak_run_block_static(clak_plan_t plan, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg,
                                  void* d_b, void* d_se, int out_dtype, int64_t ldo, uint8_t* d_flags,
                                  void* d_pval);

/* Bytes of scratch one SNP block of the plan needs (the size of one
 * workspace slot): clak_run_block_static accepts the plan when this is at
 * most CLAK_STATIC_SCRATCH_BYTES.  Errors: CLAK_E_ARG (null argument). */
clak_status clak_plan_block_scratch_size(clak_plan_t plan, size_t* bytes);

/* One SNP block of a pipeline or batch: the arguments of clak_run_block. */
typedef struct clak_block {
  int64_t m_blk;    /* SNPs in the block, 1 <= m_blk <= max_block        */
  const void* G;    /* n x m_blk genotypes, leading dimension ldg        */
  int64_t ldg;
  void* b;          /* outputs as for clak_run_block, leading dimension ldo */
  void* se;
  int64_t ldo;
  uint8_t* flags;   /* nullable */
  void* pval;       /* nullable */
} clak_block;

typedef struct clak_pipeline_s* clak_pipeline_t;
typedef struct clak_batch_s* clak_batch_t;

/* A reusable schedule of the per-block pipeline of `plan` over n_blocks
 * blocks (the same arithmetic as n_blocks calls of clak_run_block).  Blocks
 * go round three workspace slots so that the ingest of blocks b+1 and b+2
 * runs on a side stream while block b is rotated and reduced; consecutive
 * blocks alternate between two compute streams.
 * The block arguments are validated and copied at creation; the buffers they
 * point to must stay valid, and the plan must keep its workspace, while the
 * pipeline is launched.  New traits (clak_set_traits) or covariates are picked
 * up by later launches.  Creates three streams and a few events; no device work.
 * Errors: as clak_run_block, CLAK_E_DEVICE. */
clak_status clak_pipeline_create(clak_pipeline_t* pipe, clak_plan_t plan, int64_t n_blocks,
                                 const clak_block* blocks, int g_dtype, int out_dtype);

/* Enqueues the pipeline: forked from the plan's stream and joined back to it,
 * so work later enqueued on the plan's stream runs after it (asynchronous). */
clak_status clak_pipeline_launch(clak_pipeline_t pipe);

/* Waits for the pipeline's streams and destroys them; frees no caller memory. */
clak_status clak_pipeline_destroy(clak_pipeline_t pipe);

/* Several cohorts in one submission: plans[k] (distinct plans, each READY, on
 * the same device) runs its n_blocks[k] blocks, taken consecutively from
 * `blocks`.  The batch runs on three streams of its own (an ingest stream and
 * two compute streams), whatever the number of plans, in rounds: round r
 * takes block r of every plan that has one, ordered by the work of one of
 * its blocks (n (2 n + 10 (p_L + 2) t) per SNP, largest first).  When the
 * plans' kernels agree (mixed precision, several traits, the same p_L <= 3
 * and output form, at most 16 plans) each round is one launch per kernel
 * (ingest, rotation, digit encoding, grid contraction) whose grid holds every
 * plan's work-groups in that order; otherwise the plans' per-block launches
 * run in that order on the same streams.  Same lifetime rules as a pipeline. */
clak_status clak_batch_create(clak_batch_t* batch, int n_plans, const clak_plan_t* plans, const int64_t* n_blocks,
                              const clak_block* blocks, int g_dtype, int out_dtype);

/* Enqueues the batch, forked from and joined back to hip_stream (may be NULL). */
clak_status clak_batch_launch(clak_batch_t batch, void* hip_stream);

/* How the batch runs: *batched = 1 when every round is one launch per kernel
 * over all its plans, *rounds the number of rounds, *streams the streams it
 * uses (3).  Null outputs skipped.  Errors: CLAK_E_ARG (null batch). */
clak_status clak_batch_get_info(clak_batch_t batch, int* batched, int64_t* rounds, int* streams);

/* Waits for the batch's streams and destroys them; frees no caller memory. */
clak_status clak_batch_destroy(clak_batch_t batch);

/* Launch parameters of the mixed path's kernels, all of which leave every
 * result bitwise unchanged (they only change how work maps to work-groups):
 *   rot_cfg : the rotation's tile configuration: 1 to 9, 64-row tiles of 64,
 *             128 or 256 SNPs with two, four or eight waves (6 to 9 stage
 *             their operands by direct global-to-LDS loads into a ring of
 *             three or four K slices, 1 to 5 through registers, one slice
 *             ahead); 10, the Z-resident kernel (a 32-row slice of Z^T's digit
 *             planes held in LDS per work-group, genotypes streamed into
 *             registers; n_pad <= 1024, p_L <= 4, not CLAK_CHOL, else the
 *             built-in tiles);
 *   rot_rg  : the rotation's XCD row groups (1, 2, 4, 8; the 8 XCDs split into
 *             rot_rg groups of Z^T rows x 8 / rot_rg groups of SNP tiles);
 *   grid_tt : the grid contraction's kernel: 0 the ring kernel (p_L <= 3;
 *             128 SNPs x 32 traits per work-group), 32 or 64 the two-stage
 *             kernel with that many traits per work-group;
 *   grid_xt : with grid_tt = 0, the SNP tiles of an XCD walked together over
 *             all trait groups (1, 2, 4, 8; built-in 4); with 32 or 64, the
 *             XCD trait groups (1, 2, 4, 8).
 * 0 selects the built-in choice: for the rotation, 64 x 256 tiles
 * (configuration 6) in single-trait plans whose blocks hold at least 8192
 * SNPs (slower per launch alone, faster in the block pipeline), with one XCD
 * row group under CLAK_CHOL and two otherwise, else 64 x 128 tiles and two
 * row groups; for the grid, the ring kernel for p_L <= 3.
 * Errors: CLAK_E_ARG for other values. */
clak_status clak_plan_set_tuning(clak_plan_t plan, int rot_cfg, int rot_rg, int grid_tt, int grid_xt);

/* The sizes and options the plan was created with (n, p_L, t, max_block,
 * precision, flags of clak_plan_create); null outputs are skipped.  Lets a
 * binding check the shapes of the tensors it passes against the plan before
 * any call that reads or writes them.  Errors: CLAK_E_ARG (null plan). */
clak_status clak_plan_get_shape(clak_plan_t plan, int64_t* n, int64_t* p_L, int64_t* t, int64_t* max_block,
                                int* precision, uint32_t* flags);

/* The launch parameters in effect (0: built-in choice); null outputs skipped. */
clak_status clak_plan_get_tuning(clak_plan_t plan, int* rot_cfg, int* rot_rg, int* grid_tt, int* grid_xt);

/* clak_run_block that first picks the launch parameters for this plan and
 * block: clak_autotune_pipeline over this one block (timed alone, so the
 * choice suits blocks run one at a time; pipelines should be tuned with
 * clak_autotune_pipeline over a few of their blocks).  Without p-values.
 * Synchronous.  Errors: as clak_run_block, CLAK_E_DEVICE. */
clak_status clak_autotune(clak_plan_t plan, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, void* d_b,
                          void* d_se, int out_dtype, int64_t ldo, uint8_t* d_flags, const char* cache_path);

/* Picks the launch parameters of clak_plan_set_tuning for this plan by timing
 * the block pipeline (as clak_pipeline_launch runs it) over the given blocks,
 * which should be a few (3 to 6) blocks of the size the plan will stream:
 * first every rotation configuration and XCD row grouping (with the grid at
 * its built-in choice), then, with several traits, every grid kernel and
 * XCD grouping (none for the full vector with p_L > 3).  Each candidate gets
 * one warm-up pass and the best of three timed passes; the built-in choice and
 * the three fastest others are then timed again in three interleaved rounds.
 * The fastest of these is taken if it is more than 2 % faster than the
 * built-in choice, in favour of the first candidate (in the order above)
 * within 1 % of it, so that near-equal candidates do not alternate from run
 * to run.  The choice stays in the
 * plan; with cache_path (nullable) a line "<shape> rot_cfg=C rot_rg=R
 * grid_tt=T grid_xt=X" is appended, the shape being the device architecture,
 * n_pad, p_L, t, the first block's size, the number of blocks and the plan's
 * flags, and a later call with a line for the same shape takes it without
 * timing.  The blocks' outputs are computed (the last pass runs with the
 * choice; every candidate computes the same bits).  The FP64 path has nothing
 * to tune and runs the blocks.  Synchronous.  Errors: as
 * clak_pipeline_create, CLAK_E_DEVICE. */
clak_status clak_autotune_pipeline(clak_plan_t plan, int64_t n_blocks, const clak_block* blocks, int g_dtype,
                                   int out_dtype, const char* cache_path);

/* Out-of-core genotype input.  A SNP-major PLINK 1 binary genotype file (the
 * bytes 0x6c 0x1b 0x01, then m rows of (n + 3) / 4 bytes in the CLAK_G_P2
 * coding) is read block by block by a host thread into `depth` (2 to 16)
 * pinned host buffers of `block` rows; clak_bed_scan streams the blocks
 * through the plan's block pipeline as they arrive (the ingest reads each
 * block from pinned memory over PCIe, or through the copy engine with
 * CLAK_STAGE_GENOTYPES), so disk reads, transfers and kernels overlap; a
 * buffer is refilled once the ingest that read it has completed.  The blocks
 * of X_R come from disk while earlier ones are processed, as in the
 * streaming of section 3.
 *   clak_bed_open : checks the magic bytes and the size 3 + m (n + 3) / 4,
 *                   allocates the buffers and starts the reader.  Errors:
 *                   CLAK_E_ARG (missing file, wrong magic or size, depth),
 *                   CLAK_E_DEVICE.
 *   clak_bed_scan : every SNP of the file through `plan` (n of the plan, block
 *                   <= max_block, READY); outputs as for clak_run_block with SNP
 *                   i of the file at index i (ldo >= m), d_flags and d_pval
 *                   nullable.  Synchronous (returns when the plan's stream has
 *                   finished).  A finished scan rewinds the reader, so scans
 *                   can be repeated; after a failed one the reader must be
 *                   closed (CLAK_E_STATE).  Errors: CLAK_E_ARG (read failure,
 *                   sizes), CLAK_E_STATE, CLAK_E_DEVICE.
 *   clak_bed_close: stops the reader, frees the buffers, closes the file. */
typedef struct clak_bed_s* clak_bed_t;
clak_status clak_bed_open(clak_bed_t* bed, const char* path, int64_t n, int64_t m, int64_t block, int depth);
clak_status clak_bed_scan(clak_bed_t bed, clak_plan_t plan, void* d_b, void* d_se, int out_dtype, int64_t ldo,
                          uint8_t* d_flags, void* d_pval);
clak_status clak_bed_close(clak_bed_t bed);

/* Stages of clak_run_block timed by the profiler. */
#define CLAK_STAGE_INGEST 0  /* genotype block -> int8 panel, per-SNP centring statistics */
#define CLAK_STAGE_ROTATE 1  /* X~ = Z^T G (single trait: plus the fused cell sums)     */
#define CLAK_STAGE_ENCODE 2  /* digit encoding of X~ for the grid (mixed, several traits) */
#define CLAK_STAGE_GRID 3    /* grid contraction + Schur solve, or the single-trait finish */
#define CLAK_STAGE_COUNT 4

/* Stage profiler modes. */
#define CLAK_PROFILE_OFF 0
#define CLAK_PROFILE_SERIAL 1     /* every kernel alone: its own duration      */
#define CLAK_PROFILE_PIPELINED 2  /* kernels as the pipeline overlaps them     */

/* Turns per-stage timing on in the given mode (CLAK_PROFILE_SERIAL or
 * CLAK_PROFILE_PIPELINED) or off (CLAK_PROFILE_OFF) and clears the
 * accumulators.  While on, clak_run_block brackets each stage's kernel with
 * HIP events on the stream it runs on (a little host overhead per launch).
 * SERIAL: pipelines, batches and file scans run every kernel of consecutive
 * blocks, the ingest included, on one stream, so that no two of them overlap
 * and each bracketed time is that kernel's own.  PIPELINED: they keep their
 * streams, so each bracketed time is the launch's duration as the pipeline
 * runs it (overlapping the ingest and the other compute stream's kernels).
 * Errors: CLAK_E_ARG (null plan, unknown mode), CLAK_E_DEVICE. */
clak_status clak_plan_set_profiling(clak_plan_t plan, int mode);

/* Waits for the device, then returns per stage the summed kernel time in
 * milliseconds (ms[CLAK_STAGE_COUNT]) and the number of launches timed
 * (launches[CLAK_STAGE_COUNT]) since profiling was last enabled.  Either
 * array may be NULL. */
clak_status clak_plan_get_profile(clak_plan_t plan, double* ms, int64_t* launches);

/* Waits for the device, then returns per stage (busy[CLAK_STAGE_COUNT]) the
 * time in milliseconds during which at least one of the stage's timed launches
 * ran since profiling was last enabled: the length of the union of their
 * intervals, which never exceeds the wall time of the work timed (unlike the
 * sum of overlapping launches).  Errors: CLAK_E_ARG, CLAK_E_DEVICE. */
clak_status clak_plan_get_busy(clak_plan_t plan, double* busy);

/* Destroys the plan (host memory, rocBLAS handle).  Never frees the workspace. */
clak_status clak_plan_destroy(clak_plan_t plan);

/* Message of the last failing call on this thread ("" if none). */
const char* clak_last_error(void);

/* Library version string. */
const char* clak_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CLAK_H */
