// Tiled MFMA GEMM for gfx950: C = alpha * A * B + beta * C (row-major).
//
// Used for the Schur-complement update A22 -= L21 U12 (equation "update" of
// Section 2.1, which carries nearly all of the 2n^3/3 flops, Appendix C) and
// for the two triangular solves of a panel step, written as products with
// explicitly formed b x b factors (L21 = M^T (Pi11 L11), U12 = L11^-1 A12).
//
// Tile BM x BN (128 x 128, or 64 x 64 for small or skinny products) per
// workgroup of WM x WN waves, K staged through LDS 16 deep (32 for BF16)
// with the next K-slab prefetched into registers while the current one is
// multiplied.  FP64 uses v_mfma_f64_16x16x4f64; the reduced
// precision Schur variants round the FP64 operands to FP32 or BF16 on their
// way into LDS and use v_mfma_f32_16x16x4f32 / v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation; C stays FP64.
//
// The update of the next panel's columns gathers: rows of B through a row
// list (the selected rows, before the moves of Pi_j) and rows of C_in through
// another (the rows that land at each position), writing C out of place.
// The CALU_PRRP root gathers the rows of A (the panel rows that land at each
// position) for Y = A21 A11^-1.  B's row indices are staged in LDS once per
// workgroup (K <= 256), so no K-slab waits for an index load.
//
// The epilogue issues its loads in groups: all output-row indices, then per
// 16-row block all input values, all results, all stores.  On gfx950 the
// vector-memory counter covers stores as well as loads, so a wait for a load
// issued after a store also waits for the store; one output at a time (load,
// wait, store) cost two memory latencies per output.
//
// MFMA 16x16 operand layout (wave64): A operand lane l holds A[l%16][k-group
// l/16], B operand lane l holds B[k-group l/16][l%16].  The 4 accumulator
// values of lane l are D[4*(l/16) + v][l%16] for the FP32-accumulating
// instructions but D[l/16 + 4*v][l%16] for v_mfma_f64_16x16x4f64 (measured
// with a one-wave probe on gfx950).
#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {
constexpr int BK = 16;
constexpr int kGemmThreads = 256;
constexpr int APAD = 4;   // LDS row padding (elements)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <typename T> struct Lds;
template <> struct Lds<double> { typedef double type; };
template <> struct Lds<float> { typedef float type; };
template <> struct Lds<unsigned short> { typedef unsigned short type; };

template <typename T> __device__ __forceinline__ T conv(double v);
template <> __device__ __forceinline__ double conv<double>(double v) { return v; }
template <> __device__ __forceinline__ float conv<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ unsigned short conv<unsigned short>(double v) {
  return f2bf((float)v);
}
}  // namespace

// T: LDS/operand element type (double, float, bf16 as unsigned short).
template <typename T, int BM, int BN, int WM = 2, int WN = 2, int KSD = BK>
__device__ __forceinline__ void gemm_body(const GemmArgs& g, int bx, int by) {
  constexpr int NT = 64 * WM * WN;                  // threads
  constexpr int WI = BM / (16 * WM), WJ = BN / (16 * WN);   // 16x16 blocks per wave
  // bf16 needs K multiples of 32 per MFMA; stage 32-deep slabs for it
  constexpr int KS = (sizeof(T) == 2) ? 32 : KSD;
  __shared__ T As[2][KS][BM + APAD];
  __shared__ T Bs[2][KS][BN + APAD];
  __shared__ double red[WM * WN];
  // the gathered B rows' indices, staged once (a per-slab index load would
  // put a dependent load latency, and a wait for every load in flight, into
  // each K-slab)
  constexpr int kSelK = 256;
  __shared__ int bsel[kSelK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int m0 = by * BM;
  const int n0 = bx * BN;
  const int M = g.M, N = g.N, K = g.K;

  // global -> register staging: each thread holds KS*BM/NT A and KS*BN/NT B values
  constexpr int AV = KS * BM / NT;
  constexpr int BV = KS * BN / NT;
  double ra[AV], rb[BV];
  const int a_row = tid / (KS / AV), a_k = (tid % (KS / AV)) * AV;
  const int b_k = tid / (BN / BV), b_n = (tid % (BN / BV)) * BV;

  const int gr = m0 + a_row;
  const int64_t arow =
      (gr < M) ? (g.a_rows ? (int64_t)min(max(g.a_rows[gr], 0), g.gather_rows - 1) : (int64_t)gr)
               : 0;
  const bool bsel_lds = g.b_rows != nullptr && K <= kSelK;
  if (bsel_lds) {
    for (int k = tid; k < K; k += NT) bsel[k] = min(max(g.b_rows[k], 0), g.gather_rows - 1);
  }
  __syncthreads();
  auto load_slab = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int gk = k0 + a_k + v;
      ra[v] = (gr < M && gk < K) ? g.A[arow * g.lda + gk] : 0.0;
    }
    const int gk = k0 + b_k;
    int64_t brow = 0;
    if (gk < K) {
      if (bsel_lds) brow = bsel[gk];
      else brow = g.b_rows ? (int64_t)min(max(g.b_rows[gk], 0), g.gather_rows - 1) : (int64_t)gk;
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int gc = n0 + b_n + v;
      rb[v] = (gk < K && gc < N) ? g.B[brow * g.ldb + gc] : 0.0;
    }
  };
  auto store_slab = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < AV; ++v) As[buf][a_k + v][a_row] = conv<T>(ra[v]);
#pragma unroll
    for (int v = 0; v < BV; ++v) Bs[buf][b_k][b_n + v] = conv<T>(rb[v]);
  };

  d4 accd[WI][WJ];
  f4 accf[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      accd[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accf[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  const int nslab = (K + KS - 1) / KS;
  const int li = lane & 15, lk = lane >> 4;
  auto compute = [&](int cur) __attribute__((always_inline)) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int kq = 0; kq < KS / 4; ++kq) {
        double av[WI], bv[WJ];
#pragma unroll
        for (int i = 0; i < WI; ++i) av[i] = As[cur][kq * 4 + lk][wm * (BM / WM) + i * 16 + li];
#pragma unroll
        for (int j = 0; j < WJ; ++j) bv[j] = Bs[cur][kq * 4 + lk][wn * (BN / WN) + j * 16 + li];
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
          for (int j = 0; j < WJ; ++j)
            accd[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], accd[i][j], 0, 0, 0);
      }
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int kq = 0; kq < KS / 4; ++kq) {
        float av[WI], bv[WJ];
#pragma unroll
        for (int i = 0; i < WI; ++i) av[i] = As[cur][kq * 4 + lk][wm * (BM / WM) + i * 16 + li];
#pragma unroll
        for (int j = 0; j < WJ; ++j) bv[j] = Bs[cur][kq * 4 + lk][wn * (BN / WN) + j * 16 + li];
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
          for (int j = 0; j < WJ; ++j)
            accf[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], accf[i][j], 0, 0, 0);
      }
    } else {
      // bf16: one 16x16x32 MFMA per 32-deep slab; lane holds 8 consecutive k
      s8 av[WI], bv[WJ];
#pragma unroll
      for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          av[i][t] = (short)As[cur][lk * 8 + t][wm * (BM / WM) + i * 16 + li];
        }
#pragma unroll
      for (int j = 0; j < WJ; ++j)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          bv[j][t] = (short)Bs[cur][lk * 8 + t][wn * (BN / WN) + j * 16 + li];
        }
#pragma unroll
      for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j)
          accf[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], accf[i][j], 0, 0, 0);
    }
  };
  load_slab(0);
  store_slab(0);
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int cur = sl & 1;
    if (sl + 1 < nslab) load_slab((sl + 1) * KS);
    compute(cur);
    if (sl + 1 < nslab) store_slab(cur ^ 1);
    __syncthreads();
  }

  // epilogue, in passes so that the loads of a pass are all in flight
  // together (a load, its wait and a store per output would serialize them,
  // since C may alias Cin): first the output rows' indices.  Every output
  // element is a distinct memory element read and written by this thread
  // only.
  constexpr int RV = 4;                 // output rows per 16 x 16 block and lane
  int craw[WI][RV];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int v = 0; v < RV; ++v) {
      const int r = m0 + wm * (BM / WM) + i * 16 + ((sizeof(T) == 8) ? (lk + 4 * v) : (4 * lk + v));
      // (rows past M read a valid index and are not used; no divergent branch
      // around the loads)
      craw[i][v] = g.Cin ? g.c_rows[min(r, M - 1)] : r;
    }
  // all index loads issued before the first use (the scheduler would
  // otherwise wait for each right after it)
  __builtin_amdgcn_sched_barrier(0);
  int64_t crow[WI][RV];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int v = 0; v < RV; ++v)
      crow[i][v] = g.Cin ? (int64_t)min(max(craw[i][v], 0), g.gather_rows - 1) : (int64_t)craw[i][v];
  // then, one 16-row block at a time (so that the input values held at once
  // stay few), the input values and the stores
  double amax = 0.0;
#pragma unroll
  for (int i = 0; i < WI; ++i) {
    double cinv[WJ][RV];
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int v = 0; v < RV; ++v) {
        const int r = m0 + wm * (BM / WM) + i * 16 + ((sizeof(T) == 8) ? (lk + 4 * v) : (4 * lk + v));
        const int c = n0 + wn * (BN / WN) + j * 16 + li;
        const double* cin = g.Cin ? g.Cin + crow[i][v] * g.ldcin + c
                                  : g.C + (g.c_scatter ? crow[i][v] : (int64_t)r) * g.ldc + c;
        cinv[j][v] = (r < M && c < N && g.beta != 0.0) ? *cin : 0.0;
      }
    // every value of the block formed before its first store: a wait for a
    // load while a store is pending must wait for the store too
    __builtin_amdgcn_sched_barrier(0);
    // (the maximum is taken here, unconditionally, so that the values are
    // not moved into the stores' branches)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int v = 0; v < RV; ++v) {
        const int r = m0 + wm * (BM / WM) + i * 16 + ((sizeof(T) == 8) ? (lk + 4 * v) : (4 * lk + v));
        const int c = n0 + wn * (BN / WN) + j * 16 + li;
        const double p = (sizeof(T) == 8) ? accd[i][j][v] : (double)accf[i][j][v];
        cinv[j][v] = (g.beta != 0.0) ? fma(g.alpha, p, g.beta * cinv[j][v]) : g.alpha * p;
        amax = fmax(amax, (r < M && c < N) ? fabs(cinv[j][v]) : 0.0);
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int v = 0; v < RV; ++v) {
        const int r = m0 + wm * (BM / WM) + i * 16 + ((sizeof(T) == 8) ? (lk + 4 * v) : (4 * lk + v));
        const int c = n0 + wn * (BN / WN) + j * 16 + li;
        if (r < M && c < N) g.C[(g.c_scatter ? crow[i][v] : (int64_t)r) * g.ldc + c] = cinv[j][v];
      }
  }
  if (g.amax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    if (lane == 0) red[wave] = amax;
    __syncthreads();
    if (tid == 0) {
      double mx = red[0];
#pragma unroll
      for (int w = 1; w < WM * WN; ++w) mx = fmax(mx, red[w]);
      atomic_max_pos(g.amax, mx);
      if (g.amax2) atomic_max_pos(g.amax2, mx);
    }
  }
}

template <typename T, int BM, int BN, int WM = 2, int WN = 2, int KSD = BK>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(GemmArgs g) {
  gemm_body<T, BM, BN, WM, WN, KSD>(g, blockIdx.x, blockIdx.y);
}

// Batched form: problem blockIdx.z of `list`; tiles outside a problem's C exit.
template <typename T, int BM, int BN>
__global__ __launch_bounds__(kGemmThreads) void gemm_batched_kernel(const GemmArgs* list) {
  const GemmArgs g = list[blockIdx.z];
  if ((int)blockIdx.y * BM >= g.M || (int)blockIdx.x * BN >= g.N) return;
  gemm_body<T, BM, BN>(g, blockIdx.x, blockIdx.y);
}

hipError_t launch_gemm_batched(const GemmArgs* list, int count, int max_m, int max_n, int prec,
                               hipStream_t stream) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 63) / 64, (max_m + 63) / 64, count);
  if (prec == PRRP_SCHUR_FP32)
    hipLaunchKernelGGL((gemm_batched_kernel<float, 64, 64>), grid, dim3(kGemmThreads), 0, stream, list);
  else if (prec == PRRP_SCHUR_BF16)
    hipLaunchKernelGGL((gemm_batched_kernel<unsigned short, 64, 64>), grid, dim3(kGemmThreads), 0,
                       stream, list);
  else
    hipLaunchKernelGGL((gemm_batched_kernel<double, 64, 64>), grid, dim3(kGemmThreads), 0, stream,
                       list);
  return hipGetLastError();
}

template <int BM, int BN, int WM = 2, int WN = 2, int KSD = BK>
static hipError_t launch_tiles(const GemmArgs& a, hipStream_t stream) {
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM);
  const dim3 block(64 * WM * WN);
  if (a.prec == PRRP_SCHUR_FP32)
    hipLaunchKernelGGL((gemm_kernel<float, BM, BN, WM, WN, KSD>), grid, block, 0, stream, a);
  else if (a.prec == PRRP_SCHUR_BF16)
    hipLaunchKernelGGL((gemm_kernel<unsigned short, BM, BN, WM, WN, KSD>), grid, block, 0, stream, a);
  else
    hipLaunchKernelGGL((gemm_kernel<double, BM, BN, WM, WN, KSD>), grid, block, 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, hipStream_t stream) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  // 128 x 128 tiles when they fill the chip twice over, else 64 x 64.  The
  // large tiles run 8 waves (4 x 2, each 32 x 64) for FP64 and 16 waves
  // (4 x 4, each 32 x 32) for FP32 / BF16 operands: several waves per SIMD
  // hide the LDS and global latency between MFMA bursts (measured on MI355X:
  // FP64 16 -> 32 TFLOP/s, FP32 35 -> 52 TFLOP/s at 8064 x 7936 x 128).
  const int64_t big = (int64_t)((a.M + 127) / 128) * ((a.N + 127) / 128);
  if (big >= 512) {
    if (a.prec == PRRP_FP64) return launch_tiles<128, 128, 4, 2, 16>(a, stream);
    return launch_tiles<128, 128, 4, 4, 16>(a, stream);
  }
  return launch_tiles<64, 64>(a, stream);
}

}  // namespace prrp
