// Block parallel and block pairwise LU_PRRP on gfx950 (Section 5,
// Appendix E): the bookkeeping between a tree level's strong RRQR and the
// update of the rows it eliminated, the node records the solve replays, and
// the solve's forward step.
//
// A level's strong RRQR launch writes, for every row a node leaves out, its
// multipliers d_r (the row of (R11^-1 R12)^T) into the row's panel columns.
// block_nodes_kernel then lists each node's eliminated rows in node order,
// records the node (selected rows in slot order, and for every eliminated
// row the node's index), and fills one GEMM per node: the eliminated rows'
// trailing columns minus d_r times the selected rows' trailing columns,
// gathered by row lists and written back in place.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {
constexpr int kNodeThreads = 256;
}

__global__ __launch_bounds__(kNodeThreads) void block_nodes_kernel(SrrqrArgs s, BlockNodeArgs b) {
  __shared__ int32_t sel_sh[kMaxB];
  __shared__ int wave_cnt[kNodeThreads / 64];
  __shared__ int base_sh;
  const int g = blockIdx.x;
  const int bw = s.bw;
  const int len = s.tile_len[g];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t* sel = s.sel_out + (size_t)g * kMaxB;
  if (tid < bw) sel_sh[tid] = sel[tid];
  if (tid == 0) base_sh = 0;
  __syncthreads();
  int32_t* el = b.elim + (size_t)g * b.elim_stride;
  for (int i0 = 0; i0 < len; i0 += kNodeThreads) {
    const int i = i0 + tid;
    int r = 0;
    bool out = false;
    if (i < len) {
      r = s.row_list ? s.row_list[s.tile_start[g] + i] : s.tile_start[g] + i;
      bool chosen = false;
      for (int t = 0; t < bw; ++t) chosen = chosen || sel_sh[t] == r;
      out = !chosen;
    }
    // order-preserving compaction of the rows left out
    const uint64_t mask = __ballot(out);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(mask);
    __syncthreads();
    int off = base_sh;
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    if (out && off + before < b.elim_stride) {
      el[off + before] = r;
      b.elim_node[b.perm[b.k0 + r]] = b.node0 + g;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int w = 0; w < kNodeThreads / 64; ++w) t += wave_cnt[w];
      base_sh += t;
    }
    __syncthreads();
  }
  if (tid < bw) b.node_sel[(size_t)(b.node0 + g) * kMaxB + tid] = (int32_t)b.perm[b.k0 + sel_sh[tid]];
  if (tid == 0) {
    if (g == 0) *b.count = b.node0 + s.ngroups;
    GemmArgs ga;
    ga.M = len - bw;
    ga.N = (int)(b.n - b.k0 - bw);
    ga.K = bw;
    ga.A = b.A + b.k0 * b.lda + b.k0;              // d_r in the panel columns
    ga.lda = b.lda;
    double* trail = b.A + b.k0 * b.lda + b.k0 + bw;
    ga.B = trail;
    ga.ldb = b.lda;
    ga.C = trail;
    ga.ldc = b.lda;
    ga.alpha = -1.0;
    ga.beta = 1.0;
    ga.amax = b.amax;
    ga.amax2 = nullptr;
    ga.prec = PRRP_FP64;
    ga.b_rows = sel;
    ga.Cin = trail;
    ga.ldcin = b.lda;
    ga.c_rows = el;
    ga.gather_rows = b.m;
    ga.a_rows = el;
    ga.c_scatter = 1;
    b.list[g] = ga;
  }
}

hipError_t launch_block_nodes(const SrrqrArgs& s, const BlockNodeArgs& b, hipStream_t stream) {
  hipLaunchKernelGGL(block_nodes_kernel, dim3(s.ngroups), dim3(kNodeThreads), 0, stream, s, b);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t v, int32_t step) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v + step * (int32_t)i;
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, int32_t step, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 2048);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, count, v,
                     step);
  return hipGetLastError();
}

__global__ void inverse_perm_kernel(const int64_t* perm, int64_t n, int32_t* inv) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = perm[p];
    if (r >= 0 && r < n) inv[r] = (int32_t)p;
  }
}

// Records by original row number -> the caller's records by final position.
__global__ void block_records_kernel(BlockRecordArgs a) {
  const int64_t n = a.n;
  const int P = a.panels, MN = a.max_nodes, b = a.b;
  int32_t* counts = a.out + 2;
  int32_t* sel = counts + P;
  int32_t* elim = sel + (size_t)P * MN * b;
  const int64_t nsel = (int64_t)P * MN * b;
  const int64_t total = 2 + P + nsel + (int64_t)P * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < 2) {
      a.out[e] = e == 0 ? P : MN;
    } else if (e < 2 + P) {
      counts[e - 2] = a.counts[e - 2];
    } else if (e < 2 + P + nsel) {
      const int64_t q = e - 2 - P;              // (j * MN + v) * b + t
      const int64_t jv = q / b;
      const int t = (int)(q - jv * b);
      const int32_t id = a.node_sel[jv * kMaxB + t];
      sel[q] = (id >= 0 && id < n) ? a.inv[id] : -1;
    } else {
      const int64_t q = e - 2 - P - nsel;       // j * n + p
      const int64_t j = q / n, p = q - j * n;
      const int64_t id = a.perm[p];
      elim[q] = (id >= 0 && id < n) ? a.elim_node[j * n + id] : -1;
    }
  }
}

hipError_t launch_block_records(const BlockRecordArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(inverse_perm_kernel, dim3((unsigned)std::min<int64_t>((a.n + 255) / 256, 2048)),
                     dim3(256), 0, stream, a.perm, a.n, a.inv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = 2 + a.panels + (int64_t)a.panels * a.max_nodes * a.b +
                        (int64_t)a.panels * a.n;
  hipLaunchKernelGGL(block_records_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)),
                     dim3(256), 0, stream, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ solve
// One panel j of the forward sweep, Y (final row order, n x nrhs) from Ycur
// to Ynext: rows above the panel are final (copied); every row eliminated at
// a node of panel j becomes y_r - d_r . y[node's selected rows], all from
// Ycur -- a node reads only rows no node of the panel has changed yet, so
// the nodes are independent given the panel's starting values; the panel's
// pivot rows (never eliminated) take L11^-1, one wave per right-hand side in
// the last workgroup.
__global__ __launch_bounds__(256) void block_forward_kernel(BlockForwardArgs a) {
  const int64_t n = a.n;
  const int64_t k0 = (int64_t)a.j * a.b;
  const int bw = (int)min<int64_t>(a.b, n - k0);
  const int P = a.nodes[0], MN = a.nodes[1];
  const int32_t* sel = a.nodes + 2 + P;
  const int32_t* elim = sel + (size_t)P * MN * a.b + (size_t)a.j * n;
  const int64_t nrhs = a.nrhs;
  if ((int)blockIdx.x == (int)gridDim.x - 1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t r = wave; r < nrhs; r += 4) {
      double y0 = lane < bw ? a.ycur[(k0 + lane) * a.ldy + r] : 0.0;
      double y1 = lane + 64 < bw ? a.ycur[(k0 + lane + 64) * a.ldy + r] : 0.0;
      for (int i = 0; i < bw; ++i) {
        const double yi = i < 64 ? __shfl(y0, i, 64) : __shfl(y1, i - 64, 64);
        if (lane > i && lane < bw) y0 = fma(-a.LU[(k0 + lane) * a.lda + k0 + i], yi, y0);
        if (lane + 64 > i && lane + 64 < bw)
          y1 = fma(-a.LU[(k0 + lane + 64) * a.lda + k0 + i], yi, y1);
      }
      if (lane < bw) a.ynext[(k0 + lane) * a.ldy + r] = y0;
      if (lane + 64 < bw) a.ynext[(k0 + lane + 64) * a.ldy + r] = y1;
    }
    return;
  }
  const int64_t total = n * nrhs;
  const int64_t nthr = (int64_t)(gridDim.x - 1) * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += nthr) {
    const int64_t p = e / nrhs, r = e - p * nrhs;
    if (p >= k0 && p < k0 + bw) continue;             // pivot rows: the last workgroup
    double y = a.ycur[p * a.ldy + r];
    const int v = p >= k0 + bw ? elim[p] : -1;
    if (v >= 0 && v < MN) {
      const int32_t* s = sel + ((size_t)a.j * MN + v) * a.b;
      const double* d = a.LU + p * a.lda + k0;
      for (int c = 0; c < bw; ++c) {
        const int32_t q = s[c];
        if (q >= 0 && q < n) y = fma(-d[c], a.ycur[(int64_t)q * a.ldy + r], y);
      }
    }
    a.ynext[p * a.ldy + r] = y;
  }
}

hipError_t launch_block_forward(const BlockForwardArgs& a, hipStream_t stream) {
  const int64_t blocks = std::min<int64_t>((a.n * a.nrhs + 255) / 256, 1024) + 1;
  hipLaunchKernelGGL(block_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

__global__ void copy_rows_kernel(const double* src, int64_t lds, double* dst, int64_t ldd,
                                 int64_t n, int64_t nrhs) {
  const int64_t total = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / nrhs, r = e - p * nrhs;
    dst[p * ldd + r] = src[p * lds + r];
  }
}

hipError_t launch_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                            int64_t nrhs, hipStream_t stream) {
  const int64_t blocks = std::min<int64_t>((n * nrhs + 255) / 256, 2048);
  hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src, lds, dst,
                     ldd, n, nrhs);
  return hipGetLastError();
}

}  // namespace prrp
