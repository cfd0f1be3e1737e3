// Launch interfaces of the gfx950 kernels (host side of the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prrp.h"

namespace prrp {

constexpr int kPostW = 4 + 128;   // words per posted candidate: key, slot, row, alpha, beta
constexpr int kMaxGroups = 256;   // tiles per srrqr launch

// ------------------------------------------------------------ strong RRQR
// One problem of a batched launch (group g of the grid is problem g): its
// panel, outputs and slot sets.  Panel rows are the m rows below k0.
struct SrrqrProblem {
  const double* A;
  int64_t lda;
  int64_t k0;
  int m;
  int pad0;
  double* Y;                  // nullable
  int64_t ldy;
  int32_t* sel_out;           // [kMaxB]
  uint64_t* slots;            // this launch's slot set of the problem
  int32_t* rounds_out;        // [1]
  uint64_t* clear_base;       // the problem's previous slot set (nullable)
  int clear_G, clear_bw;
  const int32_t* clear_rounds;
  prrp_stats* stats;
};

struct SrrqrArgs {
  const double* A;
  int64_t lda;
  int64_t k0;                 // panel = A[k0 + r, k0 + c], c < bw
  int bw;
  int ngroups;                // independent tiles in this launch
  int G;                      // workgroups per tile
  int rpw;                    // tile rows per workgroup
  int32_t tile_start[kMaxGroups];  // first panel row, or offset into row_list
  int32_t tile_len[kMaxGroups];
  const int32_t* row_list;    // nullable: tile rows are row_list[tile_start + t]
  uint64_t tau_bits;          // truncated encoding of tau
  int report_rank;            // write rank deficiency into stats->info
  int record_block_L;         // record max |M| into stats->max_block_L
  int32_t* sel_out;           // [ngroups][kMaxB] selected panel rows, slot order
  double* Y;                  // nullable: M^T rows of unselected panel rows
  int64_t ldy;
  uint64_t* slots;            // this launch's slot set
  size_t group_stride;        // words between groups' slot areas
  int32_t* rounds_out;        // [ngroups] rounds used (for the next launch's clear)
  uint64_t* clear_base;       // slot set of the previous launch (nullable)
  size_t clear_group_stride;
  int clear_ngroups, clear_G, clear_bw;
  const int32_t* clear_rounds;
  prrp_stats* stats;
  uint32_t* abort_flag;
  const SrrqrProblem* probs;  // nullable: batched launch, one problem per group
  // Panel rows read from `panel` (row r at panel + r * ldp) instead of A.
  const double* panel;        // nullable
  int64_t ldp;
  // Final selection of a single whole-panel tile (ngroups 1, no row_list):
  // the kernel also forms the row moves of Pi_j (dst [0, 2 kMaxB), src
  // [2 kMaxB, 4 kMaxB), count at [4 kMaxB]), writes the rows of M^T at their
  // positions after the moves, and srcmap[r - bw] = the panel row that lands
  // at position r >= bw.
  int32_t* plan_mv;           // nullable
  int32_t* srcmap;
  // Block order: 0 puts a tile's workgroups together (block g * G + w), 1
  // interleaves the tiles (block w * ngroups + g), so that with ngroups a
  // multiple of 8 a tile's workgroups share an XCD.  Interleaving needs the
  // whole launch to fit the device at once: otherwise every tile could hold
  // some of its workgroups resident while waiting on ones never placed.
  int interleave;
};
hipError_t launch_srrqr(const SrrqrArgs& a, hipStream_t stream);
// LDS of one workgroup of nt threads (256 or 1024) for a panel of width bw.
size_t srrqr_smem_bytes(int bw, int nt);
// Most rows one workgroup holds (a workgroup holding more than 128 rows runs
// with 1024 threads).
int srrqr_max_rpw();
hipError_t srrqr_prepare();   // raise the dynamic LDS limit of every instance
// Workgroups of the instance for (bw, rows per workgroup, workgroups per
// tile) one CU holds at once (after srrqr_prepare).  Every workgroup of a
// tile must be resident together.
hipError_t srrqr_blocks_per_cu(int bw, int rpw, int G, int* blocks);

// ----------------------------------------------- diagonal block and moves
struct GeppArgs {
  double* A;
  int64_t lda;
  int64_t k0;
  int bw;
  int m;                      // panel rows
  const int32_t* sel;         // [bw] selected panel rows in slot order
  double* PL;                 // [bw][bw]  Pi11 L11 (row p11[j] = row j of L11)
  int32_t* mv_dst;            // [2 kMaxB] row moves of Pi_j: panel position <- panel row
  int32_t* mv_src;
  int32_t* n_moves;
  prrp_stats* stats;
  int32_t* p11;               // [bw] GEPP output: slot of the row at each final position
  const double* panel;        // nullable: panel rows read from here (row r at panel + r * ldp)
  int64_t ldp;
};
// Moves of Pi_j^T from the selection (sel, bw -> mv_dst, mv_src, n_moves).
hipError_t launch_plan(const GeppArgs& a, hipStream_t stream);
hipError_t launch_plan_batched(const GeppArgs* list, int count, hipStream_t stream);

// Pi11 on the top bw rows of the panel at k0: columns left of the panel and perm.
struct PermTopArgs {
  double* A;
  int64_t lda;
  int64_t k0;
  int bw;
  int64_t* perm;
  const int32_t* p11;
};
hipError_t launch_perm_top(const PermTopArgs& a, hipStream_t stream);
hipError_t launch_perm_top_batched(const PermTopArgs* list, int count, int64_t max_k0,
                                   hipStream_t stream);
hipError_t launch_gepp(const GeppArgs& a, hipStream_t stream);
// CALU_PRRP root, one launch of two workgroups: sel <- winners, the moves of
// Pi_j (as launch_plan) and srcmap[t - bw] = the panel row that lands at
// position t >= bw; and W = A11^-1 (bw x bw, row-major, ld bw) of the
// winners' panel block (slot order), Gauss-Jordan with partial pivoting.
hipError_t launch_root(const GeppArgs& a, const int32_t* winners, int32_t* sel, int32_t* srcmap,
                       double* W, hipStream_t stream);
// U12 = L11^-1 Pi11^T A12 in place (p11 nullable: identity).
hipError_t launch_trsm_u12(double* A, int64_t lda, int64_t k0, int bw, int64_t nr, double* amax1,
                           double* amax2, const int32_t* p11, hipStream_t stream);

struct MoveArgs {
  double* A;
  int64_t lda;
  int64_t n;
  int64_t k0;
  int bw;
  const int32_t* mv_dst;
  const int32_t* mv_src;
  const int32_t* n_moves;
  int64_t* perm;              // nullable: perm entries move too
  double* Y;                  // rows of Y follow displaced rows (nullable)
  int64_t ldy;
  int64_t c_begin, c_end;     // columns moved: [c_begin, c_end) except the
  int64_t skip_lo;            //   skip_w columns from skip_lo
  int skip_w;
  int top_only;               // only the moves into the top bw positions
};
hipError_t launch_moves(const MoveArgs& a, hipStream_t stream);

// U12 = L11^-1 A12 of the panel at k0 (nr columns right of the panel).
struct TrsmArgs {
  double* A;
  int64_t lda;
  int64_t k0;
  int bw;
  int64_t nr;
  double* amax1;              // nullable: max |U12| recorded here
  double* amax2;              // nullable: and here
  const int32_t* p11;         // nullable: rows of A12 taken in this order (Pi11^T A12)
};

// Batched forms: one problem per entry of a device-resident list; the grid
// covers the largest problem and surplus workgroups exit.
hipError_t launch_gepp_batched(const GeppArgs* list, int count, int bw, hipStream_t stream);
hipError_t launch_moves_batched(const MoveArgs* list, int count, int64_t max_outside,
                                hipStream_t stream);
hipError_t launch_trsm_u12_batched(const TrsmArgs* list, int count, int bw, int64_t max_nr,
                                   hipStream_t stream);
// Raises the dynamic LDS limit of the batched kernels (before graph capture).
hipError_t prepare_batched_kernels();

// -------------------------------------------------------------- GEMMs
// C = alpha * A * B + beta * C, row-major, FP64 operands; the Schur variants
// round A and B to `prec` and accumulate in FP32 (prec != PRRP_FP64).
// amax (nullable): max |C_new| recorded into *amax.
struct GemmArgs {
  int M, N, K;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  double alpha, beta;
  double* amax;               // nullable: max |C_new| recorded here
  double* amax2;              // nullable: and here
  int prec;
  const int32_t* b_rows;      // nullable: row k of B is B + b_rows[k] * ldb
  // nullable: C_new = alpha A B + beta C_in written to C, row r of C_in at
  // Cin + c_rows[r] * ldcin (gathered rows; C_in and C never overlap)
  const double* Cin;
  int64_t ldcin;
  const int32_t* c_rows;
  int gather_rows;            // gathered row indices are clamped into [0, gather_rows)
  const int32_t* a_rows;      // nullable: row i of A is A + a_rows[i] * lda (clamped too)
  // With c_rows: 1 writes row r of C_new at C + c_rows[r] * ldc (C may then be
  // C_in itself: each element is read and written by one thread).
  int c_scatter;
};
hipError_t launch_gemm(const GemmArgs& a, hipStream_t stream);
hipError_t launch_gemm_batched(const GemmArgs* list, int count, int max_m, int max_n, int prec,
                               hipStream_t stream);

// ------------------------------- block parallel / block pairwise LU_PRRP
// After a tree level's strong RRQR (launch args `s`, which wrote each left-out
// row's d_r into its panel columns): per node g, its left-out rows in node
// order at elim + g * elim_stride, the records (node_sel[(node0 + g) kMaxB +
// slot] = original row of the selected row, elim_node[original row] = node0
// + g, *count = node0 + ngroups), and list[g] = the GEMM updating those rows'
// trailing columns in place.
struct BlockNodeArgs {
  double* A;
  int64_t lda, k0, n;
  int m;                      // panel rows (n - k0)
  int node0;                  // index of the level's first node within the panel
  int32_t* elim;
  int elim_stride;
  const int64_t* perm;
  int32_t* node_sel;          // this panel's [max nodes][kMaxB]
  int32_t* elim_node;         // this panel's [n], by original row
  int32_t* count;             // this panel's node count
  GemmArgs* list;             // [ngroups]
  double* amax;
};
hipError_t launch_block_nodes(const SrrqrArgs& s, const BlockNodeArgs& b, hipStream_t stream);
// p[i] = v + step i
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, int32_t step, hipStream_t stream);

// The caller's node records (final positions) from the ones kept by
// original row: out = [panels, max_nodes, counts[panels],
// sel[panels][max_nodes][b] (-1 where unused), elim[panels][n] (-1: not
// eliminated in that panel)]; inv (n entries) is scratch.
struct BlockRecordArgs {
  const int64_t* perm;
  int64_t n;
  int panels, max_nodes, b;
  const int32_t* counts;
  const int32_t* node_sel;    // [panels][max_nodes][kMaxB]
  const int32_t* elim_node;   // [panels][n]
  int32_t* inv;
  int32_t* out;
};
hipError_t launch_block_records(const BlockRecordArgs& a, hipStream_t stream);

// One panel of the block factorization's forward sweep (Y in final row order).
struct BlockForwardArgs {
  const double* LU;
  int64_t lda, n;
  int b, j;
  const int32_t* nodes;       // the records above
  const double* ycur;
  double* ynext;
  int64_t ldy, nrhs;
};
hipError_t launch_block_forward(const BlockForwardArgs& a, hipStream_t stream);
hipError_t launch_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                            int64_t nrhs, hipStream_t stream);

// -------------------------------------------------------------- misc
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s);
hipError_t launch_init_factor(const double* A, int64_t n, int64_t lda, int64_t* perm,
                              prrp_stats* stats, uint32_t* abort_flag, int tree_height, int panels,
                              hipStream_t s);

// -------------------------------------------------------------- solves
// X = B[perm]; fills Y (nullable) with the sentinel and zeroes tickets[0..1].
hipError_t launch_gather_rows(const double* B, int64_t ldb, const int64_t* perm, double* X,
                              int64_t ldx, int64_t n, int64_t nrhs, double* Y, int64_t ldy,
                              uint32_t* tickets, const uint32_t* skip, hipStream_t s);
// Blocked triangular solve; Yout must hold the sentinel on entry and *ticket
// must be 0.  Fill (nullable) receives the sentinel, block by block, once a
// block's rows of Bin have been consumed.
hipError_t launch_trsv_blocked(const double* LU, int64_t n, int64_t lda, const double* Bin,
                               int64_t ldb, double* Yout, int64_t ld, int64_t nrhs, int lower,
                               uint32_t* ticket, double* Fill, int64_t ldf, const uint32_t* skip,
                               hipStream_t s);
hipError_t launch_residual(const double* A, int64_t n, int64_t lda, const double* X, int64_t ldx,
                           const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs,
                           const uint32_t* skip, hipStream_t s);
// R = B - A X as launch_residual, and wout[r] = the componentwise backward
// error max_i |R_i| / (|A| |X| + |B|)_i of right-hand side r (wout zeroed by
// the caller).
hipError_t launch_residual_w(const double* A, int64_t n, int64_t lda, const double* X,
                             int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                             int64_t nrhs, double* wout, hipStream_t s);
// Krylov vectors (k contiguous n-vectors V[i], k <= 128): out[i] = V[i] . w
// (fixed reduction order; part: 256 x 128 doubles of scratch; accumulate adds
// to out), w (or dst) = w + sign sum_i c[i] V[i] [/ *inv_of], and the 2-norm.
hipError_t launch_dots(const double* V, int64_t n, int k, const double* w, double* part,
                       double* out, int accumulate, hipStream_t s);
hipError_t launch_combine(const double* V, int64_t n, int k, const double* c, double sign,
                          double* w, const double* inv_of, double* dst, hipStream_t s);
hipError_t launch_nrm2(const double* w, int64_t n, double* part, double* out, hipStream_t s);
hipError_t launch_axpy_maxrel(double* X, int64_t ldx, const double* D, int64_t ldd, int64_t n,
                              int64_t nrhs, double* out2, const uint32_t* skip, hipStream_t s);

// Device-resident state of a refinement loop (see ir_check_kernel).
struct IrState {
  uint32_t done;
  uint32_t iter;
  double prev;
};
hipError_t launch_ir_init(IrState* st, double* mx, int64_t nrhs, int32_t* iters_out,
                          double* rel_out, int32_t* status_out, hipStream_t s);
hipError_t launch_ir_check(IrState* st, double* mx, int64_t nrhs, double tol, int max_iter,
                           int32_t* iters_out, double* rel_out, int32_t* status_out,
                           hipStream_t s);

// One system of a batched refinement (right-hand sides with ld = nrhs; the
// buffers are the system's solve workspace).
struct IrArgs {
  const double* A;            // original matrix
  int64_t n, lda;
  const double* LU;           // factors (lda)
  const int64_t* perm;
  const double* B;
  double* X;
  int64_t nrhs;
  double *t1, *t2, *r, *mx;
  uint32_t* ticket;           // [2]
  IrState* st;
  int32_t* iters_out;
  double* rel_out;
  int32_t* status_out;        // PRRP_IR_* of the last stopping test
};
// The whole refinement loop of prrp_refine_async for every system of a list,
// one launch per sub-step over all systems.
hipError_t launch_refine_batched(const IrArgs* list, int count, int64_t max_n, int64_t max_nrhs,
                                 double tol, int max_iter, hipStream_t s);
hipError_t launch_build_lists(const int32_t* child_sel, int nchild, int bw, int32_t* lists,
                              int32_t* promoted_out, int npairs, int flat_tile_start,
                              int flat_tile_len, hipStream_t s);

}  // namespace prrp
