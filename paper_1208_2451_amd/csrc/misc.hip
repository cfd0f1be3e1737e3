// Small helper kernels: fills, factorization start-up (identity permutation,
// stats record, max |A| for the growth factor's denominator).
#include "common.h"
#include "kernels.h"

namespace prrp {

__global__ void fill_u64_kernel(uint64_t* p, size_t n, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void init_stats_kernel(prrp_stats* st, uint32_t* abort_flag, int tree_height, int panels) {
  if (threadIdx.x == 0) {
    st->max_abs_A = 0.0;
    st->max_abs_W = 0.0;
    st->max_abs_U = 0.0;
    st->max_block_L = 0.0;
    st->swaps = 0;
    st->info = 0;
    st->tree_height = tree_height;
    st->panels = panels;
    *abort_flag = 0u;
  }
}

// perm = identity; max |A| into max_abs_A and max_abs_W (nonfinite -> info -1).
// Rows are strided over the workgroups and each row is read by the whole
// workgroup, two doubles per lane per load.
__global__ __launch_bounds__(256) void init_factor_kernel(const double* A, int64_t n, int64_t lda,
                                                          int64_t* perm, prrp_stats* st) {
  double m = 0.0;
  bool bad = false;
  const bool pairs = (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const double* row = A + i * lda;
    if (pairs) {
      const double2* r2 = reinterpret_cast<const double2*>(row);
      const int64_t h = n / 2;
      // four loads in flight per lane before they are reduced
      int64_t j = threadIdx.x;
      for (; j + 768 < h; j += 1024) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = r2[j + 256 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double a = fabs(v[u].x), c = fabs(v[u].y);
          bad = bad || !(a <= 1.7976931348623157e308) || !(c <= 1.7976931348623157e308);
          m = fmax(m, fmax(a, c));
        }
      }
      for (; j < h; j += 256) {
        const double2 v = r2[j];
        const double a = fabs(v.x), c = fabs(v.y);
        bad = bad || !(a <= 1.7976931348623157e308) || !(c <= 1.7976931348623157e308);
        m = fmax(m, fmax(a, c));
      }
      if ((n & 1) && threadIdx.x == 0) {
        const double a = fabs(row[n - 1]);
        bad = bad || !(a <= 1.7976931348623157e308);
        m = fmax(m, a);
      }
    } else {
      for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double a = fabs(row[j]);
        bad = bad || !(a <= 1.7976931348623157e308);
        m = fmax(m, a);
      }
    }
  }
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) perm[i] = i;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) {
    atomic_max_pos(&st->max_abs_A, m);
    atomic_max_pos(&st->max_abs_W, m);
  }
  if (bad) set_info(st, -1);
}

hipError_t launch_init_factor(const double* A, int64_t n, int64_t lda, int64_t* perm,
                              prrp_stats* stats, uint32_t* abort_flag, int tree_height, int panels,
                              hipStream_t s) {
  hipLaunchKernelGGL(init_stats_kernel, dim3(1), dim3(64), 0, s, stats, abort_flag, tree_height,
                     panels);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = n < 2048 ? n : 2048;
  hipLaunchKernelGGL(init_factor_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, n, lda, perm,
                     stats);
  return hipGetLastError();
}

// Candidate lists of a tournament level.  Binary tree (flat_tile_start < 0):
// pair p stacks child 2p's candidates over child 2p+1's, each in increasing
// row order; an odd last child is copied to promoted_out[npairs].  Flat tree:
// the running candidates (increasing) over the rows of the next tile.
__global__ __launch_bounds__(256) void build_lists_kernel(const int32_t* child, int nchild, int bw,
                                                          int32_t* lists, int32_t* promoted_out,
                                                          int npairs, int flat_start, int flat_len) {
  __shared__ int32_t v[2 * kMaxB];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  if (flat_start >= 0) {
    if (tid < bw) v[tid] = child[tid];
    __syncthreads();
    if (tid < bw) {
      const int32_t x = v[tid];
      int rank = 0;
      for (int j = 0; j < bw; ++j) rank += v[j] < x;
      lists[rank] = x;
    }
    for (int t = tid; t < flat_len; t += 256) lists[bw + t] = flat_start + t;
    return;
  }
  if (p < npairs) {
    if (tid < 2 * bw) v[tid] = child[(2 * p + tid / bw) * kMaxB + tid % bw];
    __syncthreads();
    if (tid < 2 * bw) {
      const int half = tid / bw;
      const int32_t x = v[tid];
      int rank = 0;
      for (int j = 0; j < bw; ++j) rank += v[half * bw + j] < x;
      lists[p * 2 * bw + half * bw + rank] = x;
    }
  } else if ((nchild & 1) && tid < bw) {
    promoted_out[npairs * kMaxB + tid] = child[(nchild - 1) * kMaxB + tid];
  }
}

hipError_t launch_build_lists(const int32_t* child_sel, int nchild, int bw, int32_t* lists,
                              int32_t* promoted_out, int npairs, int flat_tile_start,
                              int flat_tile_len, hipStream_t s) {
  const int blocks = (flat_tile_start >= 0) ? 1 : npairs + (nchild & 1);
  hipLaunchKernelGGL(build_lists_kernel, dim3(blocks), dim3(256), 0, s, child_sel, nchild, bw,
                     lists, promoted_out, npairs, flat_tile_start, flat_tile_len);
  return hipGetLastError();
}

}  // namespace prrp
