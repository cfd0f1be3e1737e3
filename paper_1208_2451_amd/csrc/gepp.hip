// Diagonal-block GEPP and row interchanges of one LU_PRRP panel step.
//
// Algorithm "LU_PRRP factorization", Section 2.1: Pi_j^T applied to the
// entire matrix, the b x b diagonal block factored with partial pivoting
// (A_jj = Pi_jj L_jj U_jj), and the point form of L and U12.
//
// plan_kernel (one wave): Pi_j^T as the transpositions "row k0+i <-> current
//   position of the i-th selected row" (i = 0..bw-1), reduced to a list of
//   whole-row moves (destination position <- source row).
// moves_kernel: applies the moves to a range of columns (outside the panel),
//   optionally to perm, and to the rows of M^T that belong to displaced rows.
// gepp_kernel (one workgroup): gathers the selected rows' panel block (in
//   slot order, from their positions before the moves) and factors it with
//   the tie rule, blocked by 8 columns: one wave factors each 8-column
//   sub-panel in registers (rows keep their slots; only their position labels
//   move), the block's interchanges and U block are applied column-parallel,
//   and a rank-8 update follows.  Outputs: L11\U11 in A's diagonal block,
//   PL = Pi11 L11 (so that L21 = M^T PL, the point form of the block
//   L = (R11^-1 R12)^T), and p11 (the slot at each final position).
// perm_top_kernel: applies Pi11 to the top bw rows in the columns left of the
//   panel and to perm.
// trsm_u12_kernel: U12 = L11^-1 Pi11^T A12, column-parallel (A12 rows read in
//   Pi11 order, written back in place).
#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {
constexpr int kGeppThreads = 256;
}

// Register "arrays" of a wave, two entries per lane (index e -> lane e & 63,
// slot e >> 6), read with readlane and written by a lane select, always with
// wave-uniform indices (no LDS round trips in the sequential plan).
struct LaneArr {
  int lo, hi;
  __device__ __forceinline__ int get(int e) const {
    return (e < 64) ? __builtin_amdgcn_readlane(lo, e) : __builtin_amdgcn_readlane(hi, e - 64);
  }
  __device__ __forceinline__ void set(int e, int v, int lane) {
    if (e < 64) lo = (lane == e) ? v : lo;
    else hi = (lane == e - 64) ? v : hi;
  }
};

__device__ __forceinline__ void gepp_body(const GeppArgs& a) {
  extern __shared__ double sm[];
  const int bw = a.bw;
  const int ld = bw + 1;
  double* D = sm;                               // [bw][ld]
  int* ssel = reinterpret_cast<int*>(D + bw * ld);   // [kMaxB] selection, slot order
  int* p11 = ssel + kMaxB;                      // [kMaxB] slot at each final position
  int* ipivb = p11 + kMaxB;                     // [8] interchanges of the current block
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  if (tid < kMaxB) {
    p11[tid] = tid;
    if (tid < bw) ssel[tid] = a.sel[tid];
  }
  __syncthreads();
  // gather the selected rows (panel part) in slot order; loads before stores
  {
    const int ty = tid >> 4, tx = tid & 15;
    double v[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = ty + 16 * u;
      const int64_t sr = i < bw ? min(max(ssel[i], 0), a.m - 1) : 0;
      const double* src = a.panel ? a.panel + sr * a.ldp : a.A + (a.k0 + sr) * a.lda + a.k0;
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int c = tx + 16 * w;
        v[u][w] = (i < bw && c < bw) ? src[c] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int i = ty + 16 * u, c = tx + 16 * w;
        if (i < bw && c < bw) D[i * ld + c] = v[u][w];
      }
  }
  __syncthreads();

  // ------------------------------------------------ blocked GEPP (8 columns)
  for (int J = 0; J < bw; J += 8) {
    const int jb = min(8, bw - J);
    if (wave == 0) {
      // (a) sub-panel rows J.. in registers: lane holds rows J+lane, J+lane+64
      double p[2][8];
      int ps[2];                          // current position of each held row
      bool hv[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int r = J + lane + 64 * s;
        hv[s] = r < bw;
        ps[s] = r;
        const int rr = hv[s] ? r : J;
#pragma unroll
        for (int c = 0; c < 8; ++c) p[s][c] = D[rr * ld + J + (c < jb ? c : 0)];
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        if (jj >= jb) break;
        const int col = J + jj;
        uint64_t best = 0;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const uint64_t k = (hv[s] && ps[s] >= col) ? make_key(fabs(p[s][jj]), (uint32_t)ps[s]) : 0ull;
          best = umax(best, k);
        }
        const uint64_t kk = wave_max_key(best);
        const int piv = (int)key_index(kk);
        if (lane == 0) {
          if ((kk >> kDropBits) == 0 && a.stats) set_info(a.stats, (int32_t)(a.k0 + col + 1));
          if (key_nonfinite(kk) && a.stats) set_info(a.stats, -1);
          ipivb[jj] = piv;
          const int t = p11[col]; p11[col] = p11[piv]; p11[piv] = t;
        }
        // the row holding position piv becomes position col and vice versa
        const bool w0 = hv[0] && ps[0] == piv, w1 = hv[1] && ps[1] == piv;
        const uint64_t bal0 = __ballot(w0), bal1 = __ballot(w1);
        const int wl = bal0 ? (int)__builtin_ctzll(bal0) : (int)__builtin_ctzll(bal1);
        const int wslot = bal0 ? 0 : 1;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          if (hv[s] && ps[s] == col) ps[s] = piv;
          else if (hv[s] && ps[s] == piv) ps[s] = col;
        }
        // pivot row values (uniform)
        double u[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) u[c] = readlane_d(wslot ? p[1][c] : p[0][c], wl);
        const double pv = u[jj];
        if (pv != 0.0) {
          const double inv = 1.0 / pv;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            if (hv[s] && ps[s] > col) {
              const double l = p[s][jj] * inv;
              p[s][jj] = l;
#pragma unroll
              for (int c = jj + 1; c < 8; ++c) p[s][c] = fma(-l, u[c], p[s][c]);
            }
          }
        }
      }
      // write the sub-panel back at the rows' final positions
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (hv[s]) {
#pragma unroll
          for (int c = 0; c < 8; ++c)
            if (c < jb) D[ps[s] * ld + J + c] = p[s][c];
        }
      }
    }
    __syncthreads();
    // (b) the block's interchanges on the other columns, then (c) the U block
    //     U(J:J+jb, J+jb:) = L(J:J+jb, J:J+jb)^-1 (...), one thread per column
    for (int c = tid; c < bw; c += kGeppThreads) {
      if (c >= J && c < J + jb) continue;
      for (int jj = 0; jj < jb; ++jj) {
        const int pj = ipivb[jj];
        if (pj != J + jj) {
          const double t0 = D[(J + jj) * ld + c];
          D[(J + jj) * ld + c] = D[pj * ld + c];
          D[pj * ld + c] = t0;
        }
      }
      if (c >= J + jb) {
        double x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = (i < jb) ? D[(J + i) * ld + c] : 0.0;
#pragma unroll
        for (int i = 1; i < 8; ++i) {
          if (i < jb) {
            double acc = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) acc = fma(-D[(J + i) * ld + J + k], x[k], acc);
            x[i] = acc;
            D[(J + i) * ld + c] = acc;
          }
        }
      }
    }
    __syncthreads();
    // (d) rank-jb update of the trailing block
    const int t0 = J + jb;
    if (t0 < bw) {
      const int ty = tid >> 4, tx = tid & 15;
      for (int i0 = t0 + ty; i0 < bw; i0 += 64) {
        double lv[4][8];
        int ii[4];
#pragma unroll
        for (int a4 = 0; a4 < 4; ++a4) {
          ii[a4] = i0 + 16 * a4;
          const int ic = min(ii[a4], bw - 1);
#pragma unroll
          for (int k = 0; k < 8; ++k) lv[a4][k] = (k < jb) ? D[ic * ld + J + k] : 0.0;
        }
        for (int c0 = t0 + tx; c0 < bw; c0 += 16) {
          double uv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) uv[k] = (k < jb) ? D[(J + k) * ld + c0] : 0.0;
          double cv[4];
#pragma unroll
          for (int a4 = 0; a4 < 4; ++a4) cv[a4] = D[min(ii[a4], bw - 1) * ld + c0];
#pragma unroll
          for (int a4 = 0; a4 < 4; ++a4) {
#pragma unroll
            for (int k = 0; k < 8; ++k) cv[a4] = fma(-lv[a4][k], uv[k], cv[a4]);
            if (ii[a4] < bw) D[ii[a4] * ld + c0] = cv[a4];
          }
        }
      }
    }
    __syncthreads();
  }

  // ------------------------------------------- outputs: LU11, PL, moves
  double umax = 0.0;
  for (int i = tid >> 4; i < bw; i += 16) {
    for (int c = tid & 15; c < bw; c += 16) {
      const double v = D[i * ld + c];
      a.A[(a.k0 + i) * a.lda + a.k0 + c] = v;
      if (c >= i) umax = fmax(umax, fabs(v));
      // PL: row p11[i] of PL holds row i of L11 (unit diagonal)
      a.PL[p11[i] * bw + c] = (c < i) ? v : (c == i ? 1.0 : 0.0);
    }
  }
  if (tid < bw) a.p11[tid] = p11[tid];
  if (a.stats) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) umax = fmax(umax, __shfl_xor(umax, o, 64));
    if (lane == 0) {
      atomic_max_pos(&a.stats->max_abs_U, umax);
      atomic_max_pos(&a.stats->max_abs_W, umax);
    }
  }
}

// Moves of Pi_j^T (one wave; plan in registers).
// Lane-array helpers without branches (e is wave-uniform).
__device__ __forceinline__ int la_get(const LaneArr& A, int e) {
  return __builtin_amdgcn_readlane(e < 64 ? A.lo : A.hi, e & 63);
}
__device__ __forceinline__ void la_set(LaneArr& A, bool c, int e, int v, int lane) {
  A.lo = (c && lane == e) ? v : A.lo;
  A.hi = (c && lane + 64 == e) ? v : A.hi;
}

__device__ __forceinline__ void plan_body(const GeppArgs& a) {
  const int bw = a.bw;
  const int lane = threadIdx.x;
  // the selection in registers (two entries per lane), read by lane
  const LaneArr ssel{lane < bw ? a.sel[lane] : 0, lane + 64 < bw ? a.sel[lane + 64] : 0};
  LaneArr top{lane, lane + 64}, pos{lane, lane + 64}, rec{0, 0}, dq{0, 0}, ds{0, 0};
  int nd = 0;
  for (int i = 0; i < bw; ++i) {
    const int r = la_get(ssel, i);
    const bool rin = r < bw;                       // the selected row starts in the top block
    const int pr = la_get(pos, rin ? r : 0);
    const int q = rin ? pr : r;                    // its current position
    if (q == i) continue;
    const int d = la_get(top, i);                  // the row it displaces
    la_set(top, true, i, r, lane);
    la_set(pos, rin, r, i, lane);
    const bool qin = q < bw;
    // q inside the top block: a plain transposition there
    la_set(top, qin, q, d, lane);
    // q outside: d leaves the block for position q, recorded as a move
    const int kr = la_get(rec, rin ? r : 0);
    const int k = rin ? kr : nd;
    la_set(dq, !qin && !rin, k, q, lane);
    la_set(ds, !qin, k, d, lane);
    la_set(rec, !qin, d, k, lane);
    la_set(pos, true, d, q, lane);
    nd += (!qin && !rin) ? 1 : 0;
  }
  // top positions take the selected rows in slot order
  if (lane < bw) { a.mv_dst[lane] = lane; a.mv_src[lane] = top.lo; }
  if (lane + 64 < bw) { a.mv_dst[lane + 64] = lane + 64; a.mv_src[lane + 64] = top.hi; }
  if (lane < nd) { a.mv_dst[bw + lane] = dq.lo; a.mv_src[bw + lane] = ds.lo; }
  if (lane + 64 < nd) { a.mv_dst[bw + lane + 64] = dq.hi; a.mv_src[bw + lane + 64] = ds.hi; }
  if (lane == 0) *a.n_moves = bw + nd;
}

__global__ __launch_bounds__(64) void plan_kernel(GeppArgs a) { plan_body(a); }

__global__ __launch_bounds__(64) void plan_batched_kernel(const GeppArgs* list) {
  const GeppArgs a = list[blockIdx.x];
  plan_body(a);
}

hipError_t launch_plan(const GeppArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_plan_batched(const GeppArgs* list, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(plan_batched_kernel, dim3(count), dim3(64), 0, stream, list);
  return hipGetLastError();
}

// ------------------------------------------- CALU_PRRP tournament root
// After the tournament the panel's winners are known; the step continues as
// in LU_PRRP with the block L_2j = A21 A11^-1 (Section 3.1: the QR without
// pivoting of the panel transpose with the winners first gives
// (R11^-1 R12)^T, which is the same matrix).  The root does it without a
// cross-workgroup step: root_prep forms the moves of Pi_j and the source-row
// map while block_inverse forms W = A11^-1 (two workgroups of one launch,
// independent of each other), and one gathered GEMM writes the rows of
// Y = A21 W at their positions after the moves.

// sel <- the winners (slot order); the moves of Pi_j as plan_kernel forms
// them; srcmap[t - bw] = the panel row that lands at position t >= bw.
__device__ __forceinline__ void root_prep_body(const GeppArgs& a, const int32_t* winners,
                                               int32_t* sel, int32_t* srcmap) {
  const int tid = threadIdx.x;
  if (tid < a.bw) sel[tid] = winners[tid];
  __syncthreads();              // plan_body reads a.sel == sel
  if (tid < 64) plan_body(a);
  for (int t = a.bw + tid; t < a.m; t += 256) srcmap[t - a.bw] = t;
  __syncthreads();
  const int nm = *a.n_moves;
  for (int e = a.bw + tid; e < nm; e += 256) {
    const int d = a.mv_dst[e];
    if (d >= a.bw && d < a.m) srcmap[d - a.bw] = a.mv_src[e];
  }
}


// W = A11^-1 for the bw x bw block of the selected rows (slot order), by
// Gauss-Jordan elimination with partial pivoting, in place, in registers.
// Thread (ty, tx) of a 16 x 16 grid holds rows 8 ty .. 8 ty + 7 and columns
// 8 tx .. 8 tx + 7.  Step k pivots column k on the unused row p_k with the
// largest |entry| (tie rule), scales that row by 1 / pivot, and eliminates
// column k from every other row, storing column p_k of the accumulated
// inverse transform in place of column k; so at the end
// S[i][j] = (A11^-1)[q_i][p_j], q the inverse of p.  An exactly zero pivot
// sets info (the column).
//
// Blocked by 8 columns (the same pivots and the same result up to rounding
// order as one column at a time):
//  (1) the owners of the block's columns post them to LDS (all rows);
//  (2) wave 0 runs the block's 8 steps on those columns alone, in registers
//      with no barrier and no branch (lane l holds rows l and l + 64): a row
//      i != p takes v -= g_i r with g_i = v_ik / pivot and r the pivot row, so
//      the reciprocal feeds the FMAs directly; the block's columns then hold
//      X, the columns p_k of the block's accumulated transform;
//  (3) the holders of the block's pivot rows post those rows as they were
//      before the block;
//  (4) every other column takes S[i][j] = [i not a pivot row of the block]
//      S[i][j] + sum_k X[i][k] S_old[p_k][j], a rank-8 update, and the
//      block's columns take X.
// Three barriers per 8 columns; the LDS buffers alternate between blocks.
// A last block of fewer than 8 columns runs its surplus steps as no-ops:
// every row is used by then, so the winning key is 0 and the reciprocal 0.
constexpr int kInvThreads = 256;

__device__ __forceinline__ void block_inverse_body(const GeppArgs& a, double* W) {
  // lbuf: pan[2] (block columns: column c, row i at c kMaxB + i), then
  // prw[2] (old pivot rows: step kc, column j at kc kMaxB + j); at the end
  // the staging of 32 rows of W
  __shared__ double lbuf[4 * 8 * kMaxB];
  __shared__ int pivrow[kMaxB];           // p_k
  __shared__ int slotof[kMaxB];           // q: the step whose pivot row is i (-1: none yet)
  const int bw = a.bw;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  // T[c][r] = entry (8 ty + r, 8 tx + c); the row indices are loaded first
  typedef double col8 __attribute__((ext_vector_type(8)));
  col8 T[8];
  // (every load in bounds and unconditional, so that all of them are in
  // flight together; padding entries are replaced by 0 afterwards)
  int srow[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) srow[r] = a.sel[min(8 * ty + r, bw - 1)];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t sr = min(max(srow[r], 0), a.m - 1);
    const double* src = a.panel ? a.panel + sr * a.ldp : a.A + (a.k0 + sr) * a.lda + a.k0;
#pragma unroll
    for (int c = 0; c < 8; ++c) T[c][r] = src[min(8 * tx + c, bw - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) T[c][r] = (8 * ty + r < bw && 8 * tx + c < bw) ? T[c][r] : 0.0;
  if (tid < kMaxB) slotof[tid] = -1;
  // the pivot rows of surplus steps are never posted: keep their terms finite
  for (int e = tid; e < 2 * 8 * kMaxB; e += kInvThreads) lbuf[2 * 8 * kMaxB + e] = 0.0;
  // wave 0's rows lane and lane + 64 (padding rows never pivot)
  bool used0 = lane >= bw, used1 = lane + 64 >= bw;
  const int nkt = (bw + 7) >> 3;
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    const int nk = min(8, bw - 8 * kt);          // steps in this block
    double* const pan = lbuf + buf * 8 * kMaxB;
    double* const prw = lbuf + (2 + buf) * 8 * kMaxB;
    // (1) the block's columns, all rows
    if (tx == kt) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int r = 0; r < 8; ++r) pan[c * kMaxB + 8 * ty + r] = T[c][r];
    }
    __syncthreads();
    // (2) the block's steps on its own columns
    if (wave == 0) {
      double v0[8], v1[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        v0[c] = pan[c * kMaxB + lane];
        v1[c] = pan[c * kMaxB + lane + 64];
      }
      int pk[8];
      int ev = 0;                                // first info event of the block
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const uint64_t k0v = used0 ? 0ull : make_key(fabs(v0[kc]), (uint32_t)lane);
        const uint64_t k1v = used1 ? 0ull : make_key(fabs(v1[kc]), (uint32_t)(lane + 64));
        const uint64_t kk = wave_max_key(umax(k0v, k1v));
        const int p = __builtin_amdgcn_readfirstlane((int)key_index(kk));
        const bool zero = (kk >> kDropBits) == 0;
        const int evk = zero ? (int)(a.k0 + 8 * kt + kc + 1) : (key_nonfinite(kk) ? -1 : 0);
        ev = (ev == 0 && kc < nk) ? evk : ev;
        pk[kc] = p;
        const bool hi = p >= 64;
        const int pl = p & 63;
        double rv[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) rv[c] = readlane_d(hi ? v1[c] : v0[c], pl);
        const double pinv = zero ? 0.0 : 1.0 / rv[kc];
        // rows other than p: v -= g r, column kc becomes -g; row p becomes
        // r / pivot with 1 / pivot in column kc (g = -1 / pivot)
        const bool isp0 = lane == p, isp1 = lane + 64 == p;
        const double g0 = (isp0 ? -1.0 : v0[kc]) * pinv;
        const double g1 = (isp1 ? -1.0 : v1[kc]) * pinv;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (c == kc) {
            v0[c] = -g0;
            v1[c] = -g1;
          } else {
            v0[c] = fma(-g0, rv[c], isp0 ? 0.0 : v0[c]);
            v1[c] = fma(-g1, rv[c], isp1 ? 0.0 : v1[c]);
          }
        }
        used0 = used0 || isp0;
        used1 = used1 || isp1;
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        pan[c * kMaxB + lane] = v0[c];
        pan[c * kMaxB + lane + 64] = v1[c];
      }
      int pme = pk[0];
#pragma unroll
      for (int kc = 1; kc < 8; ++kc) pme = (lane == kc) ? pk[kc] : pme;
      if (lane < nk) {
        pivrow[8 * kt + lane] = pme;
        slotof[pme] = 8 * kt + lane;
      }
      if (lane == 0 && ev != 0 && a.stats) set_info(a.stats, ev);
    }
    __syncthreads();
    // (3) the block's pivot rows as they were before it; pm marks this
    // thread's rows among them
    unsigned pm = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int kc = slotof[8 * ty + r] - 8 * kt;
      if (kc >= 0 && kc < nk) {
        pm |= 1u << r;
#pragma unroll
        for (int c = 0; c < 8; ++c) prw[kc * kMaxB + 8 * tx + c] = T[c][r];
      }
    }
    __syncthreads();
    // (4) the update (surplus steps of a short last block add 0 x finite)
    if (tx == kt) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int r = 0; r < 8; ++r) T[c][r] = pan[c * kMaxB + 8 * ty + r];
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) T[c][r] = ((pm >> r) & 1u) ? 0.0 : T[c][r];
      // step kc + 1's operands are read while step kc's FMAs run
      double f[2][8], rp[2][8];
#pragma unroll
      for (int r = 0; r < 8; ++r) f[0][r] = pan[8 * ty + r];
#pragma unroll
      for (int c = 0; c < 8; ++c) rp[0][c] = prw[8 * tx + c];
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const int cb = kc & 1;
        if (kc + 1 < 8) {
#pragma unroll
          for (int r = 0; r < 8; ++r) f[cb ^ 1][r] = pan[(kc + 1) * kMaxB + 8 * ty + r];
#pragma unroll
          for (int c = 0; c < 8; ++c) rp[cb ^ 1][c] = prw[(kc + 1) * kMaxB + 8 * tx + c];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int c = 0; c < 8; ++c) T[c][r] = fma(f[cb][r], rp[cb][c], T[c][r]);
      }
    }
  }
  // entry (i, j) = W[q_i][p_j]: one wave's 32 rows at a time are put in
  // place in LDS, then written as whole rows of W
  int pc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) pc[c] = 8 * tx + c < bw ? pivrow[8 * tx + c] : 0;
  for (int w = 0; w < kInvThreads / 64; ++w) {
    __syncthreads();
    if (32 * w >= bw) break;
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (8 * tx + c < bw) lbuf[(8 * ty + r - 32 * w) * kMaxB + pc[c]] = T[c][r];
    }
    __syncthreads();
    // this thread's column of rows 32 w + (tid >> 7) + 2 u: all reads first
    constexpr int kU = 32 * kMaxB / kInvThreads;
    const int col = tid % kMaxB, rr0 = tid / kMaxB;
    double sv[kU];
    int wr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      sv[u] = lbuf[(rr0 + 2 * u) * kMaxB + col];
      wr[u] = slotof[32 * w + rr0 + 2 * u];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (32 * w + rr0 + 2 * u < bw && col < bw) W[(int64_t)wr[u] * bw + col] = sv[u];
  }
}

// The root's two parts in one launch: workgroup 0 inverts the winners' block
// (reading the winners directly), workgroup 1 writes sel, the moves and the
// source-row map.  Neither reads what the other writes.
__global__ __launch_bounds__(kInvThreads) void root_kernel(GeppArgs a, const int32_t* winners,
                                                          int32_t* sel, int32_t* srcmap,
                                                          double* W) {
  if (blockIdx.x == 0) {
    GeppArgs b = a;
    b.sel = winners;
    block_inverse_body(b, W);
  } else {
    root_prep_body(a, winners, sel, srcmap);
  }
}

hipError_t launch_root(const GeppArgs& a, const int32_t* winners, int32_t* sel, int32_t* srcmap,
                       double* W, hipStream_t stream) {
  hipLaunchKernelGGL(root_kernel, dim3(2), dim3(kInvThreads), 0, stream, a, winners, sel, srcmap,
                     W);
  return hipGetLastError();
}

// Pi11 on the top bw rows: row k0+i takes row k0+p11[i] in the columns left
// of the panel (32-column strips per workgroup) and in perm (workgroup 0).
__device__ __forceinline__ void perm_top_body(const PermTopArgs& a, int bx) {
  __shared__ double buf[kMaxB][33];
  __shared__ int64_t pbuf[kMaxB];
  const int tid = threadIdx.x;
  const int bw = a.bw;
  const int cc = tid & 31, r8 = tid >> 5;      // 8 rows per pass
  const int64_t col = (int64_t)bx * 32 + cc;
  const bool cv = col < a.k0;
  for (int i = r8; i < bw; i += 8)
    buf[i][cc] = cv ? a.A[(a.k0 + a.p11[i]) * a.lda + col] : 0.0;
  if (bx == 0 && tid < bw) pbuf[tid] = a.perm[a.k0 + a.p11[tid]];
  __syncthreads();
  if (cv)
    for (int i = r8; i < bw; i += 8) a.A[(a.k0 + i) * a.lda + col] = buf[i][cc];
  if (bx == 0 && tid < bw) a.perm[a.k0 + tid] = pbuf[tid];
}

__global__ __launch_bounds__(256) void perm_top_kernel(PermTopArgs a) { perm_top_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void perm_top_batched_kernel(const PermTopArgs* list) {
  const PermTopArgs a = list[blockIdx.y];
  if (blockIdx.x > 0 && (int64_t)blockIdx.x * 32 >= a.k0) return;
  perm_top_body(a, blockIdx.x);
}

hipError_t launch_perm_top(const PermTopArgs& a, hipStream_t stream) {
  const int64_t grid = std::max<int64_t>(1, (a.k0 + 31) / 32);
  hipLaunchKernelGGL(perm_top_kernel, dim3((unsigned)grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_perm_top_batched(const PermTopArgs* list, int count, int64_t max_k0,
                                   hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int64_t grid = std::max<int64_t>(1, (max_k0 + 31) / 32);
  hipLaunchKernelGGL(perm_top_batched_kernel, dim3((unsigned)grid, (unsigned)count), dim3(256), 0,
                     stream, list);
  return hipGetLastError();
}

__global__ __launch_bounds__(kGeppThreads) void gepp_kernel(GeppArgs a) { gepp_body(a); }

// Batched form: problem blockIdx.x of `list`.
__global__ __launch_bounds__(kGeppThreads) void gepp_batched_kernel(const GeppArgs* list) {
  const GeppArgs a = list[blockIdx.x];
  gepp_body(a);
}

size_t gepp_smem_bytes(int bw) {
  return sizeof(double) * (size_t)(bw * (bw + 1)) + sizeof(int) * (2 * kMaxB + 8);
}

hipError_t launch_gepp(const GeppArgs& a, hipStream_t stream) {
  const size_t smem = gepp_smem_bytes(a.bw);
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)gepp_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)gepp_smem_bytes(kMaxB));
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  hipLaunchKernelGGL(gepp_kernel, dim3(1), dim3(kGeppThreads), smem, stream, a);
  return hipGetLastError();
}

hipError_t launch_gepp_batched(const GeppArgs* list, int count, int bw, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)gepp_batched_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)gepp_smem_bytes(kMaxB));
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  hipLaunchKernelGGL(gepp_batched_kernel, dim3(count), dim3(kGeppThreads), gepp_smem_bytes(bw),
                     stream, list);
  return hipGetLastError();
}

// --------------------------------------------------------------- moves
// Each workgroup moves a 32-column strip of every moved row through LDS;
// columns [k0, k0 + bw) are skipped (overwritten by L11\U11 and L21).
// Workgroup 0 also moves perm and the rows of Y of displaced rows.
namespace {
constexpr int kMoveThreads = 256;
constexpr int kStrip = 32;
}

__device__ __forceinline__ void moves_body(const MoveArgs& a, int bx, int nbx) {
  __shared__ double buf[2 * kMaxB][kStrip];
  __shared__ int64_t pbuf[2 * kMaxB];
  const int nm = min(a.top_only ? min(*a.n_moves, a.bw) : *a.n_moves, 2 * kMaxB);
  const int lim = (int)(a.n - a.k0 - 1);       // entries are panel rows: clamp into the panel
  const int tid = threadIdx.x;
  const int64_t span = (a.c_end - a.c_begin) - a.skip_w;   // columns to move
  const int64_t c0 = (int64_t)bx * kStrip;
  const int cc = tid & (kStrip - 1);
  const int r8 = tid / kStrip;                 // 8 rows per pass
  const bool cvalid = c0 + cc < span;
  int64_t col = a.c_begin + c0 + cc;
  if (col >= a.skip_lo) col += a.skip_w;
  for (int t0 = r8; t0 < nm; t0 += 8 * (kMoveThreads / kStrip)) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * (kMoveThreads / kStrip);
      v[u] = (cvalid && t < nm) ? a.A[(a.k0 + min(max(a.mv_src[t], 0), lim)) * a.lda + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * (kMoveThreads / kStrip);
      if (t < nm) buf[t][cc] = v[u];
    }
  }
  if (bx == 0 && a.perm) {
    for (int t = tid; t < nm; t += kMoveThreads) pbuf[t] = a.perm[a.k0 + min(max(a.mv_src[t], 0), lim)];
  }
  __syncthreads();
  for (int t = r8; t < nm; t += kMoveThreads / kStrip)
    if (cvalid && a.mv_dst[t] != a.mv_src[t])
      a.A[(a.k0 + min(max(a.mv_dst[t], 0), lim)) * a.lda + col] = buf[t][cc];
  if (bx == 0 && a.perm) {
    for (int t = tid; t < nm; t += kMoveThreads) a.perm[a.k0 + min(max(a.mv_dst[t], 0), lim)] = pbuf[t];
  }
  // Y rows: displaced rows (moves past the top block) carry their M columns;
  // spread over the workgroups, loads of a batch issued before its stores
  if (a.Y) {
    const int nd = nm - a.bw;
    const int64_t total = (int64_t)nd * a.bw;
    const int64_t stride = (int64_t)nbx * kMoveThreads;
    for (int64_t e0 = bx * (int64_t)kMoveThreads + tid; e0 < total; e0 += 8 * stride) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + u * stride;
        const int t = a.bw + (int)(e / a.bw), c = (int)(e % a.bw);
        v[u] = (e < total) ? a.Y[(int64_t)min(max(a.mv_src[t], 0), lim) * a.ldy + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + u * stride;
        const int t = a.bw + (int)(e / a.bw), c = (int)(e % a.bw);
        if (e < total) a.Y[(int64_t)min(max(a.mv_dst[t], 0), lim) * a.ldy + c] = v[u];
      }
    }
  }
}

__global__ __launch_bounds__(kMoveThreads) void moves_kernel(MoveArgs a) {
  moves_body(a, blockIdx.x, gridDim.x);
}

// Batched form: problem blockIdx.y of `list`, strips blockIdx.x.
__global__ __launch_bounds__(kMoveThreads) void moves_batched_kernel(const MoveArgs* list) {
  const MoveArgs a = list[blockIdx.y];
  moves_body(a, blockIdx.x, gridDim.x);
}

// U12 = L11^-1 A12: 32 columns per workgroup, 8 lanes per column, lane l8 of a
// column holding rows l8, l8 + 8, ...; L11 (strict lower, packed by rows) in LDS.
namespace {
constexpr int kTrsmCols = 32;
}

__device__ __forceinline__ void trsm_u12_body(const TrsmArgs& t, int bx) {
  extern __shared__ double Lp[];            // L(i,k), k < i, at i(i-1)/2 + k
  double* A = t.A;
  const int64_t lda = t.lda, k0 = t.k0, nr = t.nr;
  const int bw = t.bw;
  double* amax1 = t.amax1;
  double* amax2 = t.amax2;
  const int tid = threadIdx.x;
  const int l8 = tid & 7;
  const int lane = tid & 63;
  const int64_t c = (int64_t)bx * kTrsmCols + (tid >> 3);
  {
    // rows i = (tid >> 5) + 8u, columns k = (tid & 31) + 32w; loads first
    double v[16][4];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = (tid >> 5) + 8 * u;
      const double* row = A + (k0 + (i < bw ? i : 0)) * lda + k0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int k = (tid & 31) + 32 * w;
        v[u][w] = (i < bw && k < i) ? row[k] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int i = (tid >> 5) + 8 * u, k = (tid & 31) + 32 * w;
        if (i < bw && k < i) Lp[i * (i - 1) / 2 + k] = v[u][w];
      }
  }
  const bool cv = c < nr;
  double x[16];
  double* col = A + k0 * lda + k0 + bw + c;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = l8 + 8 * k;
    const int rs = (r < bw && t.p11) ? t.p11[r] : r;     // Pi11^T A12
    x[k] = (cv && r < bw) ? col[(int64_t)rs * lda] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
    for (int li = 0; li < 8; ++li) {
      const int i = 8 * kk + li;
      if (i >= bw) break;
      const double xi = __shfl(x[kk], (lane & ~7) | li, 64);
      double lv[16];
      // L(r, i) for r > i; unguarded reads stay inside the packed array
#pragma unroll
      for (int k = kk; k < 16; ++k) {
        const int r = l8 + 8 * k;
        lv[k] = Lp[r * (r - 1) / 2 + i];
      }
#pragma unroll
      for (int k = kk; k < 16; ++k) {
        const int r = l8 + 8 * k;
        if (r > i && r < bw) x[k] = fma(-lv[k], xi, x[k]);
      }
    }
  }
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = l8 + 8 * k;
    if (cv && r < bw) {
      col[(int64_t)r * lda] = x[k];
      m = fmax(m, fabs(x[k]));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (lane == 0 && amax1) {
    atomic_max_pos(amax1, m);
    if (amax2) atomic_max_pos(amax2, m);
  }
}

__global__ __launch_bounds__(256) void trsm_u12_kernel(TrsmArgs t) { trsm_u12_body(t, blockIdx.x); }

// Batched form: problem blockIdx.y of `list`; column blocks past a problem's
// columns exit.
__global__ __launch_bounds__(256) void trsm_u12_batched_kernel(const TrsmArgs* list) {
  const TrsmArgs t = list[blockIdx.y];
  if ((int64_t)blockIdx.x * kTrsmCols >= t.nr) return;
  trsm_u12_body(t, blockIdx.x);
}

hipError_t launch_trsm_u12(double* A, int64_t lda, int64_t k0, int bw, int64_t nr, double* amax1,
                           double* amax2, const int32_t* p11, hipStream_t stream) {
  if (nr <= 0) return hipSuccess;
  static bool attr_done = false;
  const size_t smem = sizeof(double) * (size_t)(kMaxB * (kMaxB - 1) / 2 + 1);
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)trsm_u12_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  const int64_t grid = (nr + kTrsmCols - 1) / kTrsmCols;
  TrsmArgs t{A, lda, k0, bw, nr, amax1, amax2, p11};
  hipLaunchKernelGGL(trsm_u12_kernel, dim3((unsigned)grid), dim3(256),
                     sizeof(double) * (size_t)(bw * (bw - 1) / 2 + 1), stream, t);
  return hipGetLastError();
}

hipError_t prepare_batched_kernels() {
  hipError_t e = hipFuncSetAttribute((const void*)gepp_batched_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)gepp_smem_bytes(kMaxB));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)trsm_u12_batched_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * (size_t)(kMaxB * (kMaxB - 1) / 2 + 1)));
}

hipError_t launch_trsm_u12_batched(const TrsmArgs* list, int count, int bw, int64_t max_nr,
                                   hipStream_t stream) {
  if (count <= 0 || max_nr <= 0) return hipSuccess;
  static bool attr_done = false;
  const size_t smem = sizeof(double) * (size_t)(kMaxB * (kMaxB - 1) / 2 + 1);
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)trsm_u12_batched_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  const int64_t grid = (max_nr + kTrsmCols - 1) / kTrsmCols;
  hipLaunchKernelGGL(trsm_u12_batched_kernel, dim3((unsigned)grid, (unsigned)count), dim3(256),
                     sizeof(double) * (size_t)(bw * (bw - 1) / 2 + 1), stream, list);
  return hipGetLastError();
}

hipError_t launch_moves(const MoveArgs& a, hipStream_t stream) {
  const int64_t span = (a.c_end - a.c_begin) - a.skip_w;
  const int64_t grid = std::max<int64_t>(1, (span + kStrip - 1) / kStrip);
  hipLaunchKernelGGL(moves_kernel, dim3((unsigned)grid), dim3(kMoveThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_moves_batched(const MoveArgs* list, int count, int64_t max_outside,
                                hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int64_t grid = std::max<int64_t>(1, (max_outside + kStrip - 1) / kStrip);
  hipLaunchKernelGGL(moves_batched_kernel, dim3((unsigned)grid, (unsigned)count),
                     dim3(kMoveThreads), 0, stream, list);
  return hipGetLastError();
}

}  // namespace prrp
