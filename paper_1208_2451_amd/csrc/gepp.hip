// Diagonal-block GEPP and row interchanges of one LU_PRRP panel step.
//
// Algorithm "LU_PRRP factorization", lines applying Pi_j^T to the entire
// matrix and factoring the b x b diagonal block with partial pivoting
// (A_jj = Pi_jj L_jj U_jj), Section 2.1.
//
// gepp_kernel (one workgroup):
//   1. plan: Pi_j^T as the transpositions "row k0+i <-> current position of
//      the i-th selected row" (i = 0..bw-1), reduced to a list of whole-row
//      moves (destination position <- source row);
//   2. GEPP of the gathered block (selected rows in slot order) with the tie
//      rule; its interchanges are folded into the moves of the top bw rows;
//   3. outputs: L11\U11 written into A's diagonal block, PL = Pi11 L11 (so
//      that L21 = M^T PL, the point form of the block L = (R11^-1 R12)^T), and
//      L11^-1 (so that U12 = L11^-1 A12 is a GEMM).
// moves_kernel: applies the moves to the columns outside the panel, to perm,
// and to the rows of M^T that belong to displaced rows.
#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {
constexpr int kGeppThreads = 256;
}

__global__ __launch_bounds__(kGeppThreads) void gepp_kernel(GeppArgs a) {
  extern __shared__ double sm[];
  const int bw = a.bw;
  const int ld = bw + 1;
  double* D = sm;                          // [bw][ld]
  double* lcol = D + bw * ld;              // [kMaxB]
  double* xcol = lcol + kMaxB;             // [kMaxB]
  uint64_t* red = reinterpret_cast<uint64_t*>(xcol + kMaxB);   // [8]
  int* topAt = reinterpret_cast<int*>(red + 8);   // [kMaxB]
  int* posTop = topAt + kMaxB;             // [kMaxB]
  int* recIdx = posTop + kMaxB;            // [kMaxB]
  int* dstq = recIdx + kMaxB;              // [kMaxB]
  int* dsrc = dstq + kMaxB;                // [kMaxB]
  int* p11 = dsrc + kMaxB;                 // [kMaxB]
  int* misc = p11 + kMaxB;                 // [8]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  // gather the selected rows (panel part) in slot order
  for (int e = tid; e < bw * bw; e += kGeppThreads) {
    const int i = e / bw, c = e - i * bw;
    D[i * ld + c] = a.A[(a.k0 + a.sel[i]) * a.lda + a.k0 + c];
  }
  if (tid < kMaxB) { p11[tid] = tid; }
  // transposition plan (sequential; one lane)
  if (tid == 0) {
    for (int i = 0; i < bw; ++i) { topAt[i] = i; posTop[i] = i; }
    int nd = 0;
    for (int i = 0; i < bw; ++i) {
      const int r = a.sel[i];
      const int q = (r < bw) ? posTop[r] : r;
      if (q == i) continue;
      const int d = topAt[i];
      topAt[i] = r;
      if (r < bw) posTop[r] = i;
      if (q < bw) {
        topAt[q] = d;
        posTop[d] = q;
      } else {
        int k;
        if (r < bw) {
          k = recIdx[r];
        } else {
          k = nd++;
          dstq[k] = q;
        }
        dsrc[k] = d;
        recIdx[d] = k;
        posTop[d] = q;
      }
    }
    misc[0] = nd;
  }
  __syncthreads();

  // ------------------------------------------------------------- GEPP
  double umax = 0.0;
  for (int j = 0; j < bw; ++j) {
    if (wave == 0) {
      const int i0 = j + lane, i1 = j + lane + 64;
      uint64_t k0 = (i0 < bw) ? make_key(fabs(D[i0 * ld + j]), (uint32_t)i0) : 0ull;
      uint64_t k1 = (i1 < bw) ? make_key(fabs(D[i1 * ld + j]), (uint32_t)i1) : 0ull;
      uint64_t kk = wave_max_u64(k0 > k1 ? k0 : k1);
      if (lane == 0) {
        const int piv = (int)key_index(kk);
        misc[1] = piv;
        a.stats ? (void)0 : (void)0;
        if ((kk >> kDropBits) == 0) {
          if (a.stats) set_info(a.stats, (int32_t)(a.k0 + j + 1));
        }
        if (key_nonfinite(kk) && a.stats) set_info(a.stats, -1);
        const int t = p11[j]; p11[j] = p11[piv]; p11[piv] = t;
      }
    }
    __syncthreads();
    const int piv = misc[1];
    if (piv != j && tid < bw) {
      const double t = D[j * ld + tid];
      D[j * ld + tid] = D[piv * ld + tid];
      D[piv * ld + tid] = t;
    }
    __syncthreads();
    const double pv = D[j * ld + j];
    const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
    if (tid > j && tid < bw) lcol[tid] = D[tid * ld + j] * inv;
    __syncthreads();
    const int nr = bw - j - 1;
    if (pv != 0.0) {
      for (int e = tid; e < nr * (nr + 1); e += kGeppThreads) {
        const int i = j + 1 + e / (nr + 1);
        const int c = j + e % (nr + 1);
        if (c == j) D[i * ld + j] = lcol[i];
        else D[i * ld + c] = fma(-lcol[i], D[j * ld + c], D[i * ld + c]);
      }
    }
    __syncthreads();
  }

  // ------------------------------------------- outputs: LU11, PL, moves
  for (int e = tid; e < bw * bw; e += kGeppThreads) {
    const int i = e / bw, c = e - i * bw;
    const double v = D[i * ld + c];
    a.A[(a.k0 + i) * a.lda + a.k0 + c] = v;
    if (c >= i) umax = fmax(umax, fabs(v));
    // PL: row p11[i] of PL holds row i of L11 (unit diagonal)
    a.PL[p11[i] * bw + c] = (c < i) ? v : (c == i ? 1.0 : 0.0);
  }
  if (tid < bw) {
    a.mv_dst[tid] = tid;
    a.mv_src[tid] = topAt[p11[tid]];
  }
  const int nd = misc[0];
  if (tid < nd) {
    a.mv_dst[bw + tid] = dstq[tid];
    a.mv_src[bw + tid] = dsrc[tid];
  }
  if (tid == 0) *a.n_moves = bw + nd;
  if (a.stats) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) umax = fmax(umax, __shfl_xor(umax, o, 64));
    if (lane == 0) {
      atomic_max_pos(&a.stats->max_abs_U, umax);
      atomic_max_pos(&a.stats->max_abs_W, umax);
    }
  }

  // ------------------------------------------ L11^-1 in place (unit lower)
  // Column j of the inverse below the diagonal: -Linv(j+1:, j+1:) L(j+1:, j),
  // from the right-most column leftwards.  Two threads per row split the sum.
  for (int j = bw - 2; j >= 0; --j) {
    if (tid > j && tid < bw) xcol[tid] = D[tid * ld + j];
    __syncthreads();
    const int i = j + 1 + (tid >> 1);
    double acc = 0.0;
    if (i < bw) {
      for (int k = j + 1 + (tid & 1); k < i; k += 2) acc = fma(D[i * ld + k], xcol[k], acc);
    }
    acc += __shfl_xor(acc, 1, 64);
    __syncthreads();
    if (i < bw && (tid & 1) == 0) D[i * ld + j] = -(xcol[i] + acc);
    __syncthreads();
  }
  for (int e = tid; e < bw * bw; e += kGeppThreads) {
    const int i = e / bw, c = e - i * bw;
    a.Linv[i * bw + c] = (c < i) ? D[i * ld + c] : (c == i ? 1.0 : 0.0);
  }
}

size_t gepp_smem_bytes(int bw) {
  return sizeof(double) * (size_t)(bw * (bw + 1) + 2 * kMaxB) + sizeof(uint64_t) * 8 +
         sizeof(int) * (6 * kMaxB + 8);
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

// --------------------------------------------------------------- moves
// Each workgroup moves a 32-column strip of every moved row through LDS;
// columns [k0, k0 + bw) are skipped (overwritten by L11\U11 and L21).
// Workgroup 0 also moves perm and the rows of Y of displaced rows.
namespace {
constexpr int kMoveThreads = 256;
constexpr int kStrip = 32;
}

__global__ __launch_bounds__(kMoveThreads) void moves_kernel(MoveArgs a) {
  __shared__ double buf[2 * kMaxB][kStrip];
  __shared__ int64_t pbuf[2 * kMaxB];
  const int nm = *a.n_moves;
  const int tid = threadIdx.x;
  const int64_t outside = a.n - a.bw;          // columns outside the panel
  const int64_t c0 = (int64_t)blockIdx.x * kStrip;
  const int cc = tid & (kStrip - 1);
  const int r8 = tid / kStrip;                 // 8 rows per pass
  int64_t col = c0 + cc;
  const bool cvalid = col < outside;
  if (col >= a.k0) col += a.bw;
  for (int t = r8; t < nm; t += kMoveThreads / kStrip)
    buf[t][cc] = cvalid ? a.A[(a.k0 + a.mv_src[t]) * a.lda + col] : 0.0;
  if (blockIdx.x == 0) {
    for (int t = tid; t < nm; t += kMoveThreads) pbuf[t] = a.perm[a.k0 + a.mv_src[t]];
  }
  __syncthreads();
  for (int t = r8; t < nm; t += kMoveThreads / kStrip)
    if (cvalid && a.mv_dst[t] != a.mv_src[t]) a.A[(a.k0 + a.mv_dst[t]) * a.lda + col] = buf[t][cc];
  if (blockIdx.x == 0) {
    for (int t = tid; t < nm; t += kMoveThreads) a.perm[a.k0 + a.mv_dst[t]] = pbuf[t];
    // Y rows: displaced rows (moves past the top block) carry their M columns
    if (a.Y) {
      for (int t = a.bw; t < nm; ++t) {
        for (int c = tid; c < a.bw; c += kMoveThreads)
          a.Y[(int64_t)a.mv_dst[t] * a.ldy + c] = a.Y[(int64_t)a.mv_src[t] * a.ldy + c];
      }
    }
  }
}

hipError_t launch_moves(const MoveArgs& a, hipStream_t stream) {
  const int64_t outside = a.n - a.bw;
  const int64_t grid = std::max<int64_t>(1, (outside + kStrip - 1) / kStrip);
  hipLaunchKernelGGL(moves_kernel, dim3((unsigned)grid), dim3(kMoveThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace prrp
