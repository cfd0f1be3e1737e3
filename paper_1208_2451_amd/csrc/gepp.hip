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
//   3. outputs: L11\U11 written into A's diagonal block and PL = Pi11 L11 (so
//      that L21 = M^T PL, the point form of the block L = (R11^-1 R12)^T).
// moves_kernel: applies the moves to the columns outside the panel, to perm,
// and to the rows of M^T that belong to displaced rows.
// trsm_u12_kernel: U12 = L11^-1 A12 (after the moves), column-parallel.
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
  int* ssel = p11 + kMaxB;                 // [kMaxB] selection (slot order)
  int* misc = ssel + kMaxB;                // [8]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  if (tid < kMaxB) {
    p11[tid] = tid;
    if (tid < bw) ssel[tid] = a.sel[tid];
  }
  __syncthreads();
  // gather the selected rows (panel part) in slot order; all loads of a
  // thread are issued before the first LDS store
  {
    const int ty = tid >> 4, tx = tid & 15;
    double v[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = ty + 16 * u;
      const double* src = a.A + (a.k0 + (i < bw ? ssel[i] : 0)) * a.lda + a.k0;
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
  // transposition plan (sequential; one lane)
  if (tid == 0) {
    for (int i = 0; i < bw; ++i) { topAt[i] = i; posTop[i] = i; }
    int nd = 0;
    for (int i = 0; i < bw; ++i) {
      const int r = ssel[i];
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
      const double d0 = D[min(i0, bw - 1) * ld + j], d1 = D[min(i1, bw - 1) * ld + j];
      uint64_t k0 = (i0 < bw) ? make_key(fabs(d0), (uint32_t)i0) : 0ull;
      uint64_t k1 = (i1 < bw) ? make_key(fabs(d1), (uint32_t)i1) : 0ull;
      uint64_t kk = wave_max_key(k0 > k1 ? k0 : k1);
      if (lane == 0) {
        const int piv = (int)key_index(kk);
        misc[1] = piv;
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
    if (pv != 0.0) {
      // each wave sweeps whole row segments (contiguous LDS); four rows per
      // batch with every read issued before the first write
      const int c0 = j + lane, c1 = j + 64 + lane;
      const bool in0 = c0 < bw, in1 = c1 < bw;
      const int c0c = in0 ? c0 : 0, c1c = in1 ? c1 : 0;
      const double u0 = D[j * ld + c0c], u1 = D[j * ld + c1c];
      for (int i0 = j + 1 + wave; i0 < bw; i0 += 16) {
        double l[4], a0[4], a1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int ic = min(i0 + 4 * t, bw - 1);
          l[t] = lcol[ic];
          a0[t] = D[ic * ld + c0c];
          a1[t] = D[ic * ld + c1c];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = i0 + 4 * t;
          if (i < bw) {
            if (in0) D[i * ld + c0] = (c0 == j) ? l[t] : fma(-l[t], u0, a0[t]);
            if (in1) D[i * ld + c1] = fma(-l[t], u1, a1[t]);
          }
        }
      }
    }
    __syncthreads();
  }

  // ------------------------------------------- outputs: LU11, PL, moves
  for (int i = tid >> 4; i < bw; i += 16) {
    for (int c = tid & 15; c < bw; c += 16) {
      const double v = D[i * ld + c];
      a.A[(a.k0 + i) * a.lda + a.k0 + c] = v;
      if (c >= i) umax = fmax(umax, fabs(v));
      // PL: row p11[i] of PL holds row i of L11 (unit diagonal)
      a.PL[p11[i] * bw + c] = (c < i) ? v : (c == i ? 1.0 : 0.0);
    }
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

}

size_t gepp_smem_bytes(int bw) {
  return sizeof(double) * (size_t)(bw * (bw + 1) + 2 * kMaxB) + sizeof(uint64_t) * 8 +
         sizeof(int) * (7 * kMaxB + 8);
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
  for (int t0 = r8; t0 < nm; t0 += 8 * (kMoveThreads / kStrip)) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * (kMoveThreads / kStrip);
      v[u] = (cvalid && t < nm) ? a.A[(a.k0 + a.mv_src[t]) * a.lda + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * (kMoveThreads / kStrip);
      if (t < nm) buf[t][cc] = v[u];
    }
  }
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

// U12 = L11^-1 A12: 32 columns per workgroup, 8 lanes per column, lane l8 of a
// column holding rows l8, l8 + 8, ...; L11 (strict lower, packed by rows) in LDS.
namespace {
constexpr int kTrsmCols = 32;
}

__global__ __launch_bounds__(256) void trsm_u12_kernel(double* A, int64_t lda, int64_t k0, int bw,
                                                       int64_t nr, double* amax1, double* amax2) {
  extern __shared__ double Lp[];            // L(i,k), k < i, at i(i-1)/2 + k
  const int tid = threadIdx.x;
  const int l8 = tid & 7;
  const int lane = tid & 63;
  const int64_t c = (int64_t)blockIdx.x * kTrsmCols + (tid >> 3);
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
    x[k] = (cv && r < bw) ? col[(int64_t)r * lda] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
    for (int li = 0; li < 8; ++li) {
      const int i = 8 * kk + li;
      if (i >= bw) break;
      const double xi = __shfl(x[kk], (lane & ~7) | li, 64);
#pragma unroll
      for (int k = kk; k < 16; ++k) {
        const int r = l8 + 8 * k;
        if (r > i && r < bw) x[k] = fma(-Lp[r * (r - 1) / 2 + i], xi, x[k]);
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

hipError_t launch_trsm_u12(double* A, int64_t lda, int64_t k0, int bw, int64_t nr, double* amax1,
                           double* amax2, hipStream_t stream) {
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
  hipLaunchKernelGGL(trsm_u12_kernel, dim3((unsigned)grid), dim3(256),
                     sizeof(double) * (size_t)(bw * (bw - 1) / 2 + 1), stream, A, lda, k0, bw, nr,
                     amax1, amax2);
  return hipGetLastError();
}

hipError_t launch_moves(const MoveArgs& a, hipStream_t stream) {
  const int64_t outside = a.n - a.bw;
  const int64_t grid = std::max<int64_t>(1, (outside + kStrip - 1) / kStrip);
  hipLaunchKernelGGL(moves_kernel, dim3((unsigned)grid), dim3(kMoveThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace prrp
