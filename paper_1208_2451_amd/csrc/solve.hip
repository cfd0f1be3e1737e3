// Solves with the in-place factors of A[perm] = L U, the extended-precision
// residual of iterative refinement, and the refinement update.
//
// trsv_kernel: blocked triangular solve with many right-hand sides in one
// launch.  Workgroups take 64-row blocks in dependency order from a ticket
// counter; a block accumulates the products with already solved blocks
// (oldest first) as their values appear -- the output starts out holding a
// sentinel and each value is written once with a device-scope store, so no
// fences are needed -- then solves its diagonal block, one wave per
// right-hand side, with the block's rows held in registers.
//
// residual_kernel: r = b - A x with the error-free transformations TwoProduct
// (by FMA) and TwoSum, accumulated per lane as in Ogita, Rump and Oishi's Dot2
// and combined across the wave by error-free pairwise sums, rounded once.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {
constexpr int NB = 64;
constexpr int RC = 8;    // right-hand sides per pass
}

// X = B[perm] (row gather); also resets the solve's tickets and fills the
// first solve's output Y with the sentinel.
__device__ __forceinline__ void gather_rows_body(const double* B, int64_t ldb, const int64_t* perm,
                                                 double* X, int64_t ldx, int64_t n, int64_t nrhs,
                                                 double* Y, int64_t ldy, uint32_t* tickets,
                                                 const uint32_t* skip, int bx, int nbx) {
  if (skip && *skip) return;
  const int64_t total = n * nrhs;
  if (bx == 0 && threadIdx.x < 2 && tickets) tickets[threadIdx.x] = 0u;
  for (int64_t e = bx * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)nbx * blockDim.x) {
    const int64_t i = e / nrhs, r = e - i * nrhs;
    X[i * ldx + r] = B[perm[i] * ldb + r];
    if (Y) reinterpret_cast<uint64_t*>(Y)[i * ldy + r] = kKeySent;
  }
}

__global__ void gather_rows_kernel(const double* B, int64_t ldb, const int64_t* perm, double* X,
                                   int64_t ldx, int64_t n, int64_t nrhs, double* Y, int64_t ldy,
                                   uint32_t* tickets, const uint32_t* skip) {
  gather_rows_body(B, ldb, perm, X, ldx, n, nrhs, Y, ldy, tickets, skip, blockIdx.x, gridDim.x);
}

hipError_t launch_gather_rows(const double* B, int64_t ldb, const int64_t* perm, double* X,
                              int64_t ldx, int64_t n, int64_t nrhs, double* Y, int64_t ldy,
                              uint32_t* tickets, const uint32_t* skip, hipStream_t s) {
  int64_t blocks = (n * nrhs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, B, ldb, perm, X,
                     ldx, n, nrhs, Y, ldy, tickets, skip);
  return hipGetLastError();
}

template <bool LOWER, int RCT>
__device__ __forceinline__ void trsv_body(const double* LU, int64_t n, int64_t lda,
                                          const double* Bin, int64_t ldb, double* Yout, int64_t ld,
                                          int64_t nrhs, uint32_t* ticket, double* Fill, int64_t ldf,
                                          const uint32_t* skip) {
  if (skip && *skip) return;
  // Yout starts out holding the sentinel; every solution value is written
  // exactly once, so dependent blocks poll the values they need.
  __shared__ double D[NB][NB + 1];
  __shared__ double yj[NB][RCT];
  __shared__ double part[4][NB][RCT];
  __shared__ int blk_s;
  __shared__ int bad_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    blk_s = (int)atomicAdd(ticket, 1u);
    bad_s = 0;
  }
  __syncthreads();
  const int nb = (int)((n + NB - 1) / NB);
  const int t = blk_s;
  if (t >= nb) return;
  const int k = LOWER ? t : nb - 1 - t;
  const int64_t r0 = (int64_t)k * NB;
  const int rows = (int)min<int64_t>(NB, n - r0);
  {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = (tid >> 6) + 4 * u, c = tid & 63;
      v[u] = (i < rows && c < rows) ? LU[(r0 + i) * lda + r0 + c] : 0.0;
    }
    // stored as the substitution uses it: only the entries that act on other
    // rows' values (strictly below the diagonal for L, strictly above for
    // U), so that a step is one FMA on every lane; the diagonal itself in the
    // padding column
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = (tid >> 6) + 4 * u, c = tid & 63;
      D[i][c] = (LOWER ? i > c : i < c) ? v[u] : 0.0;
      if (i == c) D[i][NB] = v[u];
    }
  }
  __syncthreads();
  const int ri = tid & 63, q = tid >> 6;      // row, column quarter
  const int nd = LOWER ? k : nb - 1 - k;      // blocks this one depends on
  // What the diagonal solve needs besides the solution values, loaded before
  // the wait for them: this lane's row of the block (in registers), its
  // right-hand sides, and (upper) the reciprocal of its diagonal entry.
  double drow[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) drow[i] = D[lane][i];
  const double dself = (lane < rows) ? D[lane][NB] : 1.0;
  const double rinv = 1.0 / dself;
  constexpr int RPW = (RCT + 3) / 4;          // right-hand sides per wave and pass
  for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RCT) {
    const int nr = (int)min<int64_t>(RCT, nrhs - rc0);
    double bin[RPW];
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int r = wave + 4 * t;
      bin[t] = (r < nr && lane < rows) ? Bin[(r0 + lane) * ldb + rc0 + r] : 0.0;
    }
    double acc[RCT];
#pragma unroll
    for (int r = 0; r < RCT; ++r) acc[r] = 0.0;
    // dependencies oldest (earliest solved) first; the L tile of a dependency
    // is loaded before its solution values are waited for
    for (int d = 0; d < nd; ++d) {
      const int j = LOWER ? d : nb - 1 - d;
      const int64_t c0 = (int64_t)j * NB;
      const int cols = (int)min<int64_t>(NB, n - c0);
      double l[16];
      {
        const double* lrow = LU + (r0 + (ri < rows ? ri : 0)) * lda + c0;
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (ri < rows && q * 16 + u < cols) ? lrow[q * 16 + u] : 0.0;
      }
      int bad = 0;
      for (int e = tid; e < NB * RCT; e += 256) {
        const int c = e / RCT, r = e % RCT;
        double v = 0.0;
        if (c < cols && r < nr) {
          const uint64_t* p = reinterpret_cast<const uint64_t*>(Yout + (c0 + c) * ld + rc0 + r);
          uint64_t w = ld_dev(p);
          unsigned it = 0;
          while (w == kKeySent) {
            __builtin_amdgcn_s_sleep(1);
            w = ld_dev(p);
            if (++it > kSpinLimit) { bad = 1; break; }
          }
          v = __longlong_as_double((long long)w);
        }
        yj[c][r] = v;
      }
      if (bad) bad_s = 1;
      __syncthreads();
      if (bad_s) return;
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int r = 0; r < RCT; ++r) acc[r] = fma(l[u], yj[q * 16 + u][r], acc[r]);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RCT; ++r) part[q][ri][r] = acc[r];
    __syncthreads();
    // One wave per right-hand side solves the diagonal block.  Each lane keeps
    // its row of the block in registers and takes the solved values by
    // readlane, so a substitution step is one lane read and one FMA (the
    // row holds zeros where it must not act).
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int r = wave + 4 * t;
      if (r >= nr) break;
      double bv = 0.0;
      if (lane < rows)
        bv = bin[t] - (part[0][lane][r] + part[1][lane][r] + part[2][lane][r] + part[3][lane][r]);
      if (LOWER) {
        // rows past the block's end hold zeros, so their steps change nothing
#pragma unroll
        for (int i = 0; i < NB; ++i) bv = fma(-drow[i], readlane_d(bv, i), bv);
      } else {
        // quotient b_i / u_ii from the reciprocal and one exact-remainder
        // correction (the remainder b - u y is exact under FMA).  Lane i keeps
        // b_i minus the later rows' terms; its quotient is formed for the
        // substitution and again, identically, for every lane at the end
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
          const double bi = readlane_d(bv, i);
          const double di = readlane_d(dself, i), rr = readlane_d(rinv, i);
          double y = bi * rr;
          y = fma(rr, fma(-di, y, bi), y);
          bv = fma(-drow[i], y, bv);
        }
        const double y = bv * rinv;
        bv = fma(rinv, fma(-dself, y, bv), y);
      }
      if (lane < rows)
        st_dev(reinterpret_cast<uint64_t*>(Yout + (r0 + lane) * ld + rc0 + r),
               (uint64_t)__double_as_longlong(bv));
    }
    __syncthreads();
  }
  // the next solve's output starts out holding the sentinel (this block's rows)
  if (Fill) {
    for (int e = tid; e < rows * nrhs; e += 256) {
      const int i = e / (int)nrhs, r = e - i * (int)nrhs;
      reinterpret_cast<uint64_t*>(Fill)[(r0 + i) * ldf + r] = kKeySent;
    }
  }
}

template <bool LOWER, int RCT>
__global__ __launch_bounds__(256) void trsv_kernel(const double* LU, int64_t n, int64_t lda,
                                                   const double* Bin, int64_t ldb, double* Yout,
                                                   int64_t ld, int64_t nrhs, uint32_t* ticket,
                                                   double* Fill, int64_t ldf,
                                                   const uint32_t* skip) {
  trsv_body<LOWER, RCT>(LU, n, lda, Bin, ldb, Yout, ld, nrhs, ticket, Fill, ldf, skip);
}

hipError_t launch_trsv_blocked(const double* LU, int64_t n, int64_t lda, const double* Bin,
                               int64_t ldb, double* Yout, int64_t ld, int64_t nrhs, int lower,
                               uint32_t* ticket, double* Fill, int64_t ldf, const uint32_t* skip,
                               hipStream_t s) {
  const int nb = (int)((n + NB - 1) / NB);
#define PRRP_TRSV(LO, R)                                                                       \
  hipLaunchKernelGGL((trsv_kernel<LO, R>), dim3(nb), dim3(256), 0, s, LU, n, lda, Bin, ldb, Yout, \
                     ld, nrhs, ticket, Fill, ldf, skip)
  if (nrhs == 1) {
    if (lower) PRRP_TRSV(true, 1); else PRRP_TRSV(false, 1);
  } else {
    if (lower) PRRP_TRSV(true, RC); else PRRP_TRSV(false, RC);
  }
#undef PRRP_TRSV
  return hipGetLastError();
}

// ------------------------------------------------------------ residual
// The error-free transformations below must not be contracted into FMAs.
#pragma clang fp contract(off)
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// With wout non-null it also forms the componentwise backward error of
// equation "comp": wout[r] = max_i |R_i| / (|A| |X| + |B|)_i over the rows
// (device maximum; the caller zeroes wout; a zero denominator with a non-zero
// residual gives +inf).
__device__ __forceinline__ void residual_body(const double* A, int64_t n, int64_t lda,
                                              const double* X, int64_t ldx, const double* B,
                                              int64_t ldb, double* R, int64_t ldr, int64_t nrhs,
                                              const uint32_t* skip, int bx,
                                              double* wout = nullptr) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)bx * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* arow = A + row * lda;
  for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RC) {
    const int nr = (int)min<int64_t>(RC, nrhs - rc0);
    double p[RC], s[RC], den[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      p[r] = (lane == 0 && r < nr) ? B[row * ldb + rc0 + r] : 0.0;
      s[r] = 0.0;
      den[r] = fabs(p[r]);
    }
    if (nr == 1) {
      // one right-hand side: eight columns' loads in flight per lane ahead of
      // their (unchanged, sequential) Dot2 steps; one load at a time left the
      // kernel latency-bound at about a third of the HBM rate
      double p0 = p[0], s0 = s[0], d0 = den[0];
      const double* xc = X + rc0;
      auto step = [&](double a, double x) __attribute__((always_inline)) {
        const double h = a * x;
        const double e = fma(a, x, -h);
        double t, q;
        two_sum(p0, -h, t, q);
        p0 = t;
        s0 += q - e;
        if (wout) d0 = fma(fabs(a), fabs(x), d0);
      };
      int64_t c = lane;
      for (; c + 64 * 7 < n; c += 64 * 8) {
        double av[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          av[u] = arow[c + 64 * u];
          xv[u] = xc[(c + 64 * u) * ldx];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) step(av[u], xv[u]);
      }
      for (; c < n; c += 64) step(arow[c], xc[c * ldx]);
      p[0] = p0;
      s[0] = s0;
      den[0] = d0;
    } else {
      for (int64_t c = lane; c < n; c += 64) {
        const double a = arow[c];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          if (r < nr) {
            const double x = X[c * ldx + rc0 + r];
            const double h = a * x;
            const double e = fma(a, x, -h);
            double t, q;
            two_sum(p[r], -h, t, q);
            p[r] = t;
            s[r] += q - e;
            if (wout) den[r] = fma(fabs(a), fabs(x), den[r]);
          }
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const double po = __shfl_xor(p[r], o, 64);
        const double so = __shfl_xor(s[r], o, 64);
        double t, q;
        two_sum(p[r], po, t, q);
        p[r] = t;
        s[r] = s[r] + so + q;
      }
    }
    if (wout) {
#pragma unroll
      for (int r = 0; r < RC; ++r) den[r] = wave_sum(den[r]);
    }
    if (lane == 0) {
      for (int r = 0; r < nr; ++r) {
        const double res = p[r] + s[r];
        R[row * ldr + rc0 + r] = res;
        if (wout) {
          const double num = fabs(res);
          const double q = den[r] > 0.0 ? num / den[r]
                                        : (num > 0.0 ? __longlong_as_double(0x7FF0000000000000ll)
                                                     : 0.0);
          atomic_max_pos(&wout[rc0 + r], q);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void residual_kernel(const double* A, int64_t n, int64_t lda,
                                                       const double* X, int64_t ldx, const double* B,
                                                       int64_t ldb, double* R, int64_t ldr,
                                                       int64_t nrhs, const uint32_t* skip) {
  residual_body(A, n, lda, X, ldx, B, ldb, R, ldr, nrhs, skip, blockIdx.x);
}

__global__ __launch_bounds__(256) void residual_w_kernel(const double* A, int64_t n, int64_t lda,
                                                         const double* X, int64_t ldx,
                                                         const double* B, int64_t ldb, double* R,
                                                         int64_t ldr, int64_t nrhs, double* wout) {
  residual_body(A, n, lda, X, ldx, B, ldb, R, ldr, nrhs, nullptr, blockIdx.x, wout);
}

hipError_t launch_residual_w(const double* A, int64_t n, int64_t lda, const double* X,
                             int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                             int64_t nrhs, double* wout, hipStream_t s) {
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(residual_w_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, n, lda, X,
                     ldx, B, ldb, R, ldr, nrhs, wout);
  return hipGetLastError();
}

// ------------------------------------------------- Krylov vector kernels
// The GMRES corrections keep their basis as k contiguous n-vectors V[i].
// dots: out[i] = V[i] . w for i < k, reduced in a fixed order (partial sums
// per block, then one pass over the blocks), so results are reproducible.
constexpr int kDotBlocks = 256;
constexpr int kMaxKrylov = 128;

__global__ __launch_bounds__(256) void dots_partial_kernel(const double* V, int64_t n, int k,
                                                           const double* w, double* part) {
  __shared__ double red[4][kMaxKrylov];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = (n + kDotBlocks - 1) / kDotBlocks;
  const int64_t r0 = blockIdx.x * chunk, r1 = min<int64_t>(n, r0 + chunk);
  for (int i = 0; i < k; ++i) {
    double acc = 0.0;
    for (int64_t r = r0 + tid; r < r1; r += 256) acc = fma(V[(int64_t)i * n + r], w[r], acc);
    acc = wave_sum_fixed(acc);
    if (lane == 0) red[wave][i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < k; i += 256)
    part[(int64_t)blockIdx.x * kMaxKrylov + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
}

__global__ __launch_bounds__(256) void dots_final_kernel(const double* part, int k, double* out,
                                                         int accumulate) {
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x & 63; b < kDotBlocks; b += 64) acc += part[(int64_t)b * kMaxKrylov + i];
  acc = wave_sum_fixed(acc);
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + acc : acc;
}

hipError_t launch_dots(const double* V, int64_t n, int k, const double* w, double* part,
                       double* out, int accumulate, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (k > kMaxKrylov) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dots_partial_kernel, dim3(kDotBlocks), dim3(256), 0, s, V, n, k, w, part);
  hipLaunchKernelGGL(dots_final_kernel, dim3(k), dim3(64), 0, s, part, k, out, accumulate);
  return hipGetLastError();
}

// w += sign * sum_i c[i] V[i] (c on the device); with inv_of non-null the
// result is then divided by *inv_of (zero stays zero); written to dst, or in
// place when dst is null.
__global__ __launch_bounds__(256) void combine_kernel(const double* V, int64_t n, int k,
                                                      const double* c, double sign, double* w,
                                                      const double* inv_of, double* dst) {
  __shared__ double cs[kMaxKrylov];
  for (int i = threadIdx.x; i < k; i += 256) cs[i] = sign * c[i];
  __syncthreads();
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r >= n) return;
  double acc = w ? w[r] : 0.0;
  for (int i = 0; i < k; ++i) acc = fma(cs[i], V[(int64_t)i * n + r], acc);
  if (inv_of) {
    const double d = *inv_of;
    acc = d != 0.0 ? acc / d : 0.0;
  }
  (dst ? dst : w)[r] = acc;
}

hipError_t launch_combine(const double* V, int64_t n, int k, const double* c, double sign,
                          double* w, const double* inv_of, double* dst, hipStream_t s) {
  if (k > kMaxKrylov) return hipErrorInvalidValue;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, V, n, k, c, sign, w,
                     inv_of, dst);
  return hipGetLastError();
}

// out = sqrt(part-reduced w . w)
__global__ void sqrt_kernel(double* x) {
  if (threadIdx.x == 0) *x = sqrt(*x);
}
hipError_t launch_nrm2(const double* w, int64_t n, double* part, double* out, hipStream_t s) {
  hipError_t e = launch_dots(w, n, 1, w, part, out, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

hipError_t launch_residual(const double* A, int64_t n, int64_t lda, const double* X, int64_t ldx,
                           const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs,
                           const uint32_t* skip, hipStream_t s) {
  const int64_t blocks = (n + 3) / 4;
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, n, lda, X, ldx,
                     B, ldb, R, ldr, nrhs, skip);
  return hipGetLastError();
}

// X += D; out[2r] = max|D(:,r)|, out[2r+1] = max|X(:,r)| (out zeroed by the caller).
// One thread per row; maxima reduced per wave before the device-scope max.
__device__ __forceinline__ void axpy_maxrel_body(double* X, int64_t ldx, const double* D,
                                                 int64_t ldd, int64_t n, int64_t nrhs, double* out,
                                                 const uint32_t* skip, int bx) {
  if (skip && *skip) return;
  const int64_t i = bx * (int64_t)256 + threadIdx.x;
  for (int64_t r = 0; r < nrhs; ++r) {
    double dm = 0.0, xm = 0.0;
    if (i < n) {
      const double d = D[i * ldd + r];
      const double x = X[i * ldx + r] + d;
      X[i * ldx + r] = x;
      dm = fabs(d);
      xm = fabs(x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dm = fmax(dm, __shfl_xor(dm, o, 64));
      xm = fmax(xm, __shfl_xor(xm, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomic_max_pos(&out[2 * r], dm);
      atomic_max_pos(&out[2 * r + 1], xm);
    }
  }
}

__global__ __launch_bounds__(256) void axpy_maxrel_kernel(double* X, int64_t ldx, const double* D,
                                                          int64_t ldd, int64_t n, int64_t nrhs,
                                                          double* out, const uint32_t* skip) {
  axpy_maxrel_body(X, ldx, D, ldd, n, nrhs, out, skip, blockIdx.x);
}

hipError_t launch_axpy_maxrel(double* X, int64_t ldx, const double* D, int64_t ldd, int64_t n,
                              int64_t nrhs, double* out, const uint32_t* skip, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(axpy_maxrel_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, ldx, D, ldd,
                     n, nrhs, out, skip);
  return hipGetLastError();
}

// ---------------------------------------------- device-side refinement loop
// State of a refinement run kept on the device so that the whole loop can be
// enqueued (or captured in a graph) without host round trips: the stopping
// test runs in ir_check_kernel and later iterations' kernels see `done` and
// return at once.
__device__ __forceinline__ void ir_init_body(IrState* st, double* mx, int64_t nrhs,
                                             int32_t* iters_out, double* rel_out,
                                             int32_t* status_out) {
  const int t = threadIdx.x;
  if (t == 0) {
    st->done = 0u;
    st->iter = 0u;
    st->prev = __longlong_as_double(0x7FF0000000000000ll);   // +inf
    if (iters_out) *iters_out = 0;
    if (rel_out) *rel_out = 0.0;
    if (status_out) *status_out = PRRP_IR_CAP;   // no correction taken yet
  }
  for (int64_t i = t; i < 2 * nrhs; i += blockDim.x) mx[i] = 0.0;
}

// Same stopping test as the host-driven loop: stop when the correction is at
// most tol times the solution (per right-hand side, worst case), or when it
// no longer halves, or after max_iter corrections.  The status says which
// (PRRP_IR_CONVERGED, PRRP_IR_STAGNATED, PRRP_IR_CAP); a NaN correction
// counts as stagnation.
__device__ __forceinline__ void ir_check_body(IrState* st, double* mx, int64_t nrhs, double tol,
                                              int max_iter, int32_t* iters_out, double* rel_out,
                                              int32_t* status_out) {
  if (threadIdx.x != 0 || st->done) return;
  double rel = 0.0;
  for (int64_t r = 0; r < nrhs; ++r) {
    const double xm = mx[2 * r + 1] > 0.0 ? mx[2 * r + 1] : 1.0;
    rel = fmax(rel, mx[2 * r] / xm);
    mx[2 * r] = 0.0;
    mx[2 * r + 1] = 0.0;
  }
  const unsigned it = st->iter + 1u;
  st->iter = it;
  int32_t status = PRRP_IR_CAP;
  if (rel <= tol) status = PRRP_IR_CONVERGED;
  else if (!(rel <= 0.5 * st->prev)) status = PRRP_IR_STAGNATED;
  if (status != PRRP_IR_CAP || (int)it >= max_iter) st->done = 1u;
  st->prev = rel;
  if (iters_out) *iters_out = (int32_t)it;
  if (rel_out) *rel_out = rel;
  if (status_out) *status_out = status;
}

__global__ void ir_init_kernel(IrState* st, double* mx, int64_t nrhs, int32_t* iters_out,
                               double* rel_out, int32_t* status_out) {
  ir_init_body(st, mx, nrhs, iters_out, rel_out, status_out);
}
__global__ void ir_check_kernel(IrState* st, double* mx, int64_t nrhs, double tol, int max_iter,
                                int32_t* iters_out, double* rel_out, int32_t* status_out) {
  ir_check_body(st, mx, nrhs, tol, max_iter, iters_out, rel_out, status_out);
}

hipError_t launch_ir_init(IrState* st, double* mx, int64_t nrhs, int32_t* iters_out,
                          double* rel_out, int32_t* status_out, hipStream_t s) {
  hipLaunchKernelGGL(ir_init_kernel, dim3(1), dim3(64), 0, s, st, mx, nrhs, iters_out, rel_out,
                     status_out);
  return hipGetLastError();
}

hipError_t launch_ir_check(IrState* st, double* mx, int64_t nrhs, double tol, int max_iter,
                           int32_t* iters_out, double* rel_out, int32_t* status_out,
                           hipStream_t s) {
  hipLaunchKernelGGL(ir_check_kernel, dim3(1), dim3(64), 0, s, st, mx, nrhs, tol, max_iter,
                     iters_out, rel_out, status_out);
  return hipGetLastError();
}


// ----------------------------------------- refinement of a batch of systems
// One launch per refinement sub-step over all systems of a batch (system
// blockIdx.y of the list); surplus workgroups of smaller systems exit, and a
// system that has met its stopping test skips its remaining work.  phase 0:
// the first solve of B into X; phase 1: the correction solve of R in place.
__global__ void ir_init_batched_kernel(const IrArgs* list) {
  const IrArgs a = list[blockIdx.x];
  ir_init_body(a.st, a.mx, a.nrhs, a.iters_out, a.rel_out, a.status_out);
}

__global__ void gather_batched_kernel(const IrArgs* list, int phase) {
  const IrArgs a = list[blockIdx.y];
  const int64_t nb = (a.n * a.nrhs + 255) / 256;
  if ((int64_t)blockIdx.x >= nb) return;
  gather_rows_body(phase ? a.r : a.B, a.nrhs, a.perm, a.t1, a.nrhs, a.n, a.nrhs, a.t2, a.nrhs,
                   a.ticket, phase ? &a.st->done : nullptr, blockIdx.x, (int)nb);
}

template <bool LOWER>
__global__ __launch_bounds__(256) void trsv_batched_kernel(const IrArgs* list, int phase) {
  const IrArgs a = list[blockIdx.y];
  double* out = phase ? a.r : a.X;
  if (LOWER)
    trsv_body<true, RC>(a.LU, a.n, a.lda, a.t1, a.nrhs, a.t2, a.nrhs, a.nrhs, a.ticket, out,
                        a.nrhs, phase ? &a.st->done : nullptr);
  else
    trsv_body<false, RC>(a.LU, a.n, a.lda, a.t2, a.nrhs, out, a.nrhs, a.nrhs, a.ticket + 1,
                         nullptr, 0, phase ? &a.st->done : nullptr);
}

__global__ __launch_bounds__(256) void residual_batched_kernel(const IrArgs* list) {
  const IrArgs a = list[blockIdx.y];
  residual_body(a.A, a.n, a.lda, a.X, a.nrhs, a.B, a.nrhs, a.r, a.nrhs, a.nrhs, &a.st->done,
                blockIdx.x);
}

__global__ __launch_bounds__(256) void axpy_batched_kernel(const IrArgs* list) {
  const IrArgs a = list[blockIdx.y];
  axpy_maxrel_body(a.X, a.nrhs, a.r, a.nrhs, a.n, a.nrhs, a.mx, &a.st->done, blockIdx.x);
}

__global__ void ir_check_batched_kernel(const IrArgs* list, double tol, int max_iter) {
  const IrArgs a = list[blockIdx.x];
  ir_check_body(a.st, a.mx, a.nrhs, tol, max_iter, a.iters_out, a.rel_out, a.status_out);
}

hipError_t launch_refine_batched(const IrArgs* list, int count, int64_t max_n, int64_t max_nrhs,
                                 double tol, int max_iter, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned gb = (unsigned)std::max<int64_t>(1, (max_n * max_nrhs + 255) / 256);
  const unsigned tb = (unsigned)((max_n + NB - 1) / NB);
  const unsigned rb = (unsigned)((max_n + 3) / 4);
  const unsigned ab = (unsigned)((max_n + 255) / 256);
  const unsigned c = (unsigned)count;
  hipLaunchKernelGGL(ir_init_batched_kernel, dim3(c), dim3(64), 0, s, list);
  hipLaunchKernelGGL(gather_batched_kernel, dim3(gb, c), dim3(256), 0, s, list, 0);
  hipLaunchKernelGGL((trsv_batched_kernel<true>), dim3(tb, c), dim3(256), 0, s, list, 0);
  hipLaunchKernelGGL((trsv_batched_kernel<false>), dim3(tb, c), dim3(256), 0, s, list, 0);
  for (int it = 1; it <= max_iter; ++it) {
    hipLaunchKernelGGL(residual_batched_kernel, dim3(rb, c), dim3(256), 0, s, list);
    hipLaunchKernelGGL(gather_batched_kernel, dim3(gb, c), dim3(256), 0, s, list, 1);
    hipLaunchKernelGGL((trsv_batched_kernel<true>), dim3(tb, c), dim3(256), 0, s, list, 1);
    hipLaunchKernelGGL((trsv_batched_kernel<false>), dim3(tb, c), dim3(256), 0, s, list, 1);
    hipLaunchKernelGGL(axpy_batched_kernel, dim3(ab, c), dim3(256), 0, s, list);
    hipLaunchKernelGGL(ir_check_batched_kernel, dim3(c), dim3(64), 0, s, list, tol, max_iter);
  }
  return hipGetLastError();
}

}  // namespace prrp
