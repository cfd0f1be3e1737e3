/*
 * prrp.h -- C ABI of the MI355X (gfx950) LU_PRRP / CALU_PRRP library.
 *
 * The library factors a dense square matrix as A = Pi L U with panel rank
 * revealing pivoting (Khabou, Demmel, Grigori, Gu, "LU factorization with
 * panel rank revealing pivoting and its communication avoiding version"):
 * every b-column panel chooses its b pivot rows by a strong rank revealing QR
 * of the panel's transpose (Section 2.1, Algorithm "LU_PRRP factorization";
 * Appendix A, Algorithm "Strong RRQR"), or, for CALU_PRRP, by a tournament of
 * strong RRQRs over row tiles of the panel (Section 3.1).
 *
 * Conventions shared by every entry point
 *   - All matrix/vector pointers are DEVICE pointers.  Matrices are row-major
 *     with a leading dimension (elements between consecutive rows) >= columns.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL is
 *     the default stream).  Argument errors are detected on the host before
 *     anything is enqueued and returned synchronously.
 *   - A factorization with n > 2b runs its panels ahead of the trailing
 *     update on streams of the library's own (created once per process on
 *     the current device; the panel chain's stream is confined to
 *     PRRP_RESERVE_CUS CUs, default 96, the far update's to the others).  It
 *     starts after the work already enqueued on `stream`, and `stream` waits
 *     for all of it, so to the caller it is one operation on `stream`.
 *     Factorizations issued from several host threads are enqueued one at a
 *     time on those streams.
 *   - The caller owns every buffer.  Factor and solve calls allocate no device
 *     memory: scratch space comes from a caller-provided `workspace` whose
 *     size is returned by the matching *_workspace_size query (a pure host
 *     function that needs no GPU).
 *   - Return value: 0 = enqueued; -k = argument k invalid (1-based); -1000 - e
 *     = HIP runtime error e while enqueueing.  Numerical status (singular
 *     pivot, non-finite data, exchange loop cap) is written by the kernels to
 *     the device `prrp_stats` record (field `info`).
 *   - Pivot ties (equal or nearly equal candidates) are broken
 *     deterministically: magnitudes are compared on their binary64 encoding
 *     with the 19 low mantissa bits dropped, and the lowest current row index
 *     wins among equals (for an exchange: lowest row, then lowest slot).
 *   - Supported sizes: 1 <= n <= 2^19 - 2, 1 <= b <= 128, b <= n, and, for
 *     LU_PRRP, n small enough that one panel's strong-RRQR workgroups fit
 *     the device at once (prrp_panel_cus; about 65536 on MI355X).
 *
 * Factor output (in place, LAPACK convention): on exit A holds U on and above
 * the diagonal and the unit-lower L strictly below it (diagonal implied), and
 * perm[i] is the input row now in position i, i.e. A_in[perm[i], :] =
 * (L U)[i, :] (the problem statement A = Pi L U of the introduction).
 */
#ifndef PRRP_H
#define PRRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reduction tree of the CALU_PRRP tournament (Section 3.1: binary tree; the
 * flat tree is the sequential variant discussed with its growth bound). */
typedef enum { PRRP_TREE_BINARY = 0, PRRP_TREE_FLAT = 1 } prrp_tree_kind;

/* Arithmetic of the Schur-complement update A22 -= L21 U12.  The panel, the
 * pivot selection and the triangular solves are FP64 in every mode; the
 * trailing matrix stays FP64.  FP32 / BF16 round L21 and U12 to that type and
 * accumulate their product in FP32 before it is subtracted in FP64. */
typedef enum { PRRP_FP64 = 0, PRRP_SCHUR_FP32 = 1, PRRP_SCHUR_BF16 = 2 } prrp_precision;

/* Device-resident status and growth record written by a factorization.
 * g_W = max_abs_W / max_abs_A (growth over all intermediate active matrices
 * and U, Section 2.2), g_U = max_abs_U / max_abs_A.
 * info: 0 ok; j > 0: first panel step that met an exactly zero residual or
 * zero pivot, as a 1-based column (the factors past that column are not
 * meaningful); -1 non-finite value met; -2 a kernel's bounded wait expired;
 * -3 the strong RRQR exchange loop reached its cap without meeting tau. */
typedef struct prrp_stats {
  double max_abs_A;
  double max_abs_W;
  double max_abs_U;
  double max_block_L;   /* max |(R11^-1 R12)_ij| of the final panel selections */
  int64_t swaps;        /* strong RRQR interchanges, all panels and tree nodes */
  int32_t info;
  int32_t tree_height;  /* CALU_PRRP: height of the tallest tournament */
  int32_t panels;
  int32_t reserved[3];
} prrp_stats;

/* Compute units that the largest strong-RRQR tile of a factorization
 * (method 0: LU_PRRP, whose tile is the whole panel; method 1: CALU_PRRP with
 * `tree` and `tile_rows`) occupies with all its workgroups resident, at
 * blocks_per_cu workgroups per CU (0: the device's occupancy for each kernel
 * instance, which needs a GPU; > 0: that value, a pure host computation).
 * Factor calls reject sizes whose figure exceeds the device's CUs.  Returns 0
 * or -k for an invalid argument k. */
int prrp_panel_cus(int method, int64_t n, int b, int tree, int64_t tile_rows, int blocks_per_cu,
                   int64_t* cus);

/* Workspace bytes for prrp_factor / prrp_factor_mixed (method 0) or
 * calu_prrp_factor (method 1, tile_rows as passed there) on an n x n matrix
 * with panel width b.  Host-only; returns 0 or -k for an invalid argument. */
int prrp_workspace_size(int64_t n, int b, int method, int64_t tile_rows, size_t* bytes);

/* LU_PRRP (Section 2.1, Algorithm "LU_PRRP factorization"): in-place factor
 * of the n x n matrix A (leading dimension lda), panel width b, strong RRQR
 * threshold tau > 1 (Appendix A).  perm: device int64[n] (output).
 * stats: device prrp_stats (output, required).  Every workgroup of one
 * panel's strong RRQR waits on the others, so they must all be resident at
 * once: an n whose first panel the device cannot hold (prrp_panel_cus above
 * its compute units; on MI355X beyond about 65536) returns -2 before anything
 * is enqueued. */
int prrp_factor(double* A, int64_t n, int64_t lda, int b, double tau, int64_t* perm,
                prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream);

/* As prrp_factor with the Schur update in `schur` precision (see
 * prrp_precision).  Pivots may differ from the FP64 factorization. */
int prrp_factor_mixed(double* A, int64_t n, int64_t lda, int b, double tau, int64_t* perm,
                      prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream,
                      int schur);

/* CALU_PRRP (Section 3.1): tournament pivoting over row tiles of tile_rows
 * rows (>= b + 1; a last remainder of <= b rows joins the previous tile),
 * reduced by strong RRQR along a binary or flat tree (`tree`, a
 * prrp_tree_kind); then the panel is factored with the winners as pivots and
 * the step continues as in LU_PRRP.  `schur` as in prrp_factor_mixed.  A
 * tile (or tree node) whose strong-RRQR workgroups the device cannot hold at
 * once returns -7 before anything is enqueued. */
int calu_prrp_factor(double* A, int64_t n, int64_t lda, int b, double tau, int tree,
                     int64_t tile_rows, int64_t* perm, prrp_stats* stats, void* workspace,
                     size_t ws_bytes, void* stream, int schur);

/* Block parallel (tree PRRP_TREE_BINARY) and block pairwise (PRRP_TREE_FLAT)
 * LU_PRRP (Section 5, Appendix E).  Each panel's active rows are cut into
 * tiles as in calu_prrp_factor, except that tile_rows may equal b (the
 * pairwise tree of height n / b: a b-row leaf keeps its rows); at every node of the reduction tree strong
 * RRQR of the node's rows selects b of them and every other row r of the node
 * is eliminated against them at once: with d_r its row of
 * (R11^-1 R12)^T, row r's columns right of the panel become
 * row r - d_r [selected rows], and d_r is stored in row r's panel columns.
 * The root's rows move to the top, the diagonal block is factored by GEPP
 * (interchanges on entire rows) and U12 = L11^-1 Pi11^T A12; no further
 * update follows (every row was updated once, at its node).
 *
 * On exit A holds U on and above the diagonal, each diagonal block's L11
 * below its diagonal, and every eliminated row's d_r below the diagonal
 * blocks, rows in final order; perm[p] (device int64[n]) is the original row
 * at final position p.  nodes (device int32[node_entries], output) records
 * the elimination order the solve needs, by final position:
 *   nodes[0] = P (panels), nodes[1] = MN (nodes per panel, at most),
 *   nodes[2 + j] = panel j's node count (leaves first, up to the root),
 *   sel  = nodes + 2 + P:           sel[(j MN + v) b + s] = final position of
 *                                   node v's s-th selected row (slot order,
 *                                   the order of d_r's entries), -1 if unused,
 *   elim = sel + P MN b:            elim[j n + p] = the node of panel j that
 *                                   eliminated the row at p, -1 if none.
 * stats: device prrp_stats (output; max_block_L = max |d_r|, max_abs_W the
 * largest magnitude any updated row or U reached).  Tiles whose strong-RRQR
 * workgroups the device cannot hold at once return -7.  Sizes from
 * prrp_block_sizes; returns -10 if node_entries is short, -13 if ws_bytes is. */
int prrp_block_sizes(int64_t n, int b, int tree, int64_t tile_rows, size_t* ws_bytes,
                     int64_t* node_entries);
int prrp_block_factor(double* A, int64_t n, int64_t lda, int b, double tau, int tree,
                      int64_t tile_rows, int64_t* perm, int32_t* nodes, int64_t node_entries,
                      prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream);

/* Solve A X = B with the factors of prrp_block_factor: B[perm] swept by every
 * panel's node eliminations (each a function of the panel's starting values)
 * and L11^-1 of its pivot rows, then X = U^-1 of the result.  B, X: n x nrhs
 * row-major (ldb, ldx >= nrhs), distinct or equal.  Workspace as
 * prrp_solve_workspace_size(n, nrhs). */
int prrp_block_solve(const double* LU, int64_t n, int64_t lda, int b, const int64_t* perm,
                     const int32_t* nodes, const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes for prrp_solve / prrp_refine with nrhs right-hand sides. */
int prrp_solve_workspace_size(int64_t n, int64_t nrhs, size_t* bytes);

/* Solve A X = B with the factors of prrp_factor (introduction: A = Pi L U):
 * X = U^-1 L^-1 B[perm].  B: n x nrhs row-major (ldb >= nrhs), overwritten by
 * X.  LU, perm as returned by a factor call. */
int prrp_solve(const double* LU, int64_t n, int64_t lda, const int64_t* perm, double* B,
               int64_t nrhs, int64_t ldb, void* workspace, size_t ws_bytes, void* stream);

/* R = B - A X evaluated as if in twice the working precision and rounded
 * once (error-free TwoProduct by FMA and TwoSum, accumulated as in Ogita,
 * Rump and Oishi's Dot2).  A: n x n (lda); X, B, R: n x nrhs (ldx). */
int prrp_residual(const double* A, int64_t n, int64_t lda, const double* X, const double* B,
                  double* R, int64_t nrhs, int64_t ldx, void* stream);

/* Outcome of a refinement run (the `status` outputs below).  A run that did
 * not converge still returns 0 (its launches succeeded); the status says why
 * it stopped:
 *   PRRP_IR_CONVERGED  the last correction was at most tol max|X|;
 *   PRRP_IR_STAGNATED  the last correction did not halve (or was NaN); it has
 *                      been applied, and X is only as accurate as the last
 *                      ratio says (final_rel);
 *   PRRP_IR_CAP        max_iter corrections were taken without either. */
enum { PRRP_IR_CONVERGED = 0, PRRP_IR_STAGNATED = 1, PRRP_IR_CAP = 2 };

/* Iterative refinement of the solution of A X = B (used with the paper's
 * linear-solver experiments): X = solve(B); repeat R = prrp_residual; D =
 * solve(R); X += D, until max|D| <= tol max|X| per right-hand side, the
 * correction stops halving, or max_iter corrections.  This call synchronizes
 * `stream` once per iteration to test convergence.  iters (host, may be
 * NULL) receives the number of corrections; final_rel (host, may be NULL) the
 * last max|D|/max|X|; status (host, may be NULL) a PRRP_IR_* value. */
int prrp_refine(const double* A, const double* LU, int64_t n, int64_t lda, const int64_t* perm,
                const double* B, double* X, int64_t nrhs, int64_t ldx, double tol, int max_iter,
                int* iters, double* final_rel, int* status, void* workspace, size_t ws_bytes,
                void* stream);

/* prrp_refine with the whole loop enqueued on `stream` and no host
 * synchronisation: the stopping test runs on the device and the kernels of
 * later iterations return at once once it is met, so the call can be
 * captured in a HIP graph.  At most max_iter (<= 1000) corrections.  iters
 * (device int32, may be NULL) receives the number of corrections, final_rel
 * (device double, may be NULL) the last max|D|/max|X|, status (device int32,
 * may be NULL) a PRRP_IR_* value.  Results are identical to prrp_refine's for
 * the same arguments. */
int prrp_refine_async(const double* A, const double* LU, int64_t n, int64_t lda,
                      const int64_t* perm, const double* B, double* X, int64_t nrhs, int64_t ldx,
                      double tol, int max_iter, int32_t* iters, double* final_rel,
                      int32_t* status, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * prrp_refine_async with its scratch taken from a fixed device array inside
 * the library (prrp_static_scratch_bytes() bytes, 16 MiB, one copy per GPU,
 * held until the process ends) instead of a workspace argument.  The scratch
 * holds what prrp_solve_workspace_size(n, nrhs) counts; an n x nrhs beyond it
 * returns -8 before anything is enqueued.  It allocates nothing and calls no
 * allocating routine; its first call on a device looks up that device's copy
 * of the array.  Every call on one GPU shares that GPU's array, which keeps
 * the last call's contents (each call initialises what it reads first), so
 * calls that overlap on one GPU race: serialise them (one stream, or events).
 * Other arguments, results and status as prrp_refine_async. */
size_t prrp_static_scratch_bytes(void);
int prrp_refine_async_static(const double* A, const double* LU, int64_t n, int64_t lda,
                             const int64_t* perm, const double* B, double* X, int64_t nrhs,
                             int64_t ldx, double tol, int max_iter, int32_t* iters,
                             double* final_rel, int32_t* status, void* stream);

/* Workspace bytes for prrp_refine_gmres with at most max_inner (1..128)
 * Krylov vectors per correction.  Host-only. */
int prrp_gmres_workspace_size(int64_t n, int max_inner, size_t* bytes);

/* GMRES-based refinement of the solution of A x = b (one right-hand side):
 * each correction solves A d = r by GMRES preconditioned on the left by the
 * LU factors (Carson and Higham, SIAM J. Sci. Comput. 40, 2018) instead of
 * by one triangular solve -- the refinement for factors whose Schur updates
 * ran in low precision.  r = b - A x is formed as if in twice the working
 * precision (prrp_residual); the Arnoldi basis is orthogonalised by
 * classical Gram-Schmidt applied twice; GMRES stops when its residual
 * estimate falls below gmres_tol times its start, or after max_inner steps.
 * Outer stopping test:
 *   tol > 0: the correction's size, as prrp_refine (max|d| <= tol max|x|
 *            converged, a correction that fails to halve stagnated) -- the
 *            measure a forward-error target needs;
 *   tol = 0: the componentwise backward error w of equation "comp", as in
 *            the paper's linear-solver experiments (Section 3.3, Tables
 *            "bcaluprrp_gepp", "fcaluprrp_gepp"): w <= 2^-53 converged, a
 *            step that fails to halve w stagnated.
 * max_outer steps at most (PRRP_IR_CAP).  b, x: device n-vectors (x output).
 * outer, inner (GMRES steps in all), w_before (w of the unrefined solution),
 * w_final, final_rel (last max|d|/max|x|), status: host outputs, each may be
 * NULL.  The call synchronizes `stream` once per Arnoldi step.  Returns 0 or
 * -k for an invalid argument k. */
int prrp_refine_gmres(const double* A, const double* LU, int64_t n, int64_t lda,
                      const int64_t* perm, const double* b, double* x, double tol,
                      double gmres_tol, int max_inner, int max_outer, int* outer, int* inner,
                      double* w_before, double* w_final, double* final_rel, int* status,
                      void* workspace, size_t ws_bytes, void* stream);

/* Batched LU_PRRP of `count` independent systems of uneven sizes (the
 * algorithm of Section 2.1 on each).  A plan fixes the problems: A[i] (device,
 * n[i] x n[i], row-major, lda[i]), panel width b[i], perm[i] (device, n[i]
 * int64), stats + i (device array of count records), tau, the Schur
 * precision and the rows per panel workgroup (64 or 128: fewer, fuller
 * workgroups per strong RRQR step; the results are the same).  With A0
 * non-NULL each system is also refined after its factorization (as
 * prrp_refine_async, tolerance tol, at most max_iter corrections): A0[i] the
 * original matrix (lda[i]), B[i] and X[i] n[i] x nrhs[i] row-major.
 *
 * All device memory of the plan (work lists and per-problem workspaces) is
 * the caller's workspace of at least prrp_batch_plan_workspace_size bytes
 * (nrhs NULL when there is no refinement), which must stay allocated and
 * untouched until the plan is destroyed.  Creation uploads the work lists
 * with an asynchronous copy on `stream` and returns 0, or -k for an invalid
 * argument k (-17 no workspace, -18 workspace too small).
 *
 * Running a plan enqueues on `stream` one launch per kernel per panel step
 * over all problems still active; each system ends with exactly the factors,
 * permutation and statistics prrp_factor_mixed gives it alone.  With
 * use_graph the sequence is captured into a HIP graph on the first run and
 * replayed afterwards.  The refinement of all systems runs as one launch per
 * refinement sub-step over the batch, each system stopping on its own test.
 * Runs of one plan must not overlap. */
int prrp_batch_plan_workspace_size(int64_t count, const int64_t* n, const int* b,
                                   const int64_t* nrhs, int rows_per_wg, size_t* bytes);
int prrp_batch_plan_create(int64_t count, double* const* A, const int64_t* n, const int64_t* lda,
                           const int* b, int64_t* const* perm, prrp_stats* stats, double tau,
                           int schur, int rows_per_wg, const double* const* A0,
                           const double* const* B, double* const* X, const int64_t* nrhs,
                           double tol, int max_iter, void* workspace, size_t ws_bytes,
                           void* stream, void** plan);
int prrp_batch_plan_run(void* plan, void* stream, int use_graph);
/* Copies the refinement iteration counts, last ratios and PRRP_IR_* status
 * values (count each; any pointer may be NULL to skip it) to the host with
 * copies on `stream`, and waits for that stream. */
int prrp_batch_plan_results(void* plan, int32_t* iters, double* rels, int32_t* status,
                            void* stream);
/* Releases the plan's host state (graph, events); the workspace is the
 * caller's.  Work the plan enqueued must have completed. */
int prrp_batch_plan_destroy(void* plan);
/* C = alpha A B + beta C for row-major FP64 matrices (M x K, K x N, M x N),
 * computed by the MFMA kernel of the Schur-complement update (equation
 * "update", Section 2.1).  prec: a prrp_precision; with FP32 / BF16 the
 * operands are rounded to that type and their products accumulated in FP32,
 * C stays FP64.  beta == 0 does not read C. */
int prrp_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int prec,
              void* stream);

/* Per-phase device timing of factor calls (HIP events around every launch on
 * the factor's stream).  prrp_profile_enable(1) clears the counters and starts
 * recording; while enabled each factor call keeps its events until
 * prrp_profile_read, which waits for them and returns, per phase, the summed
 * milliseconds and the number of launches (arrays of PRRP_PHASES entries;
 * either may be NULL).  Phases: 0 strong RRQR / tournament, 1 diagonal GEPP,
 * 2 row moves, 3 L21 product, 4 U12 product, 5 Schur update, 6 start-up. */
#define PRRP_PHASES 7
int prrp_profile_enable(int on);
int prrp_profile_read(double* ms, int64_t* launches);

/* Human-readable text for a return code or an info value. */
const char* prrp_status_string(int code);

/* Library version string. */
const char* prrp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PRRP_H */
