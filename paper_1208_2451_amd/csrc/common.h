// Shared device helpers of the gfx950 LU_PRRP / CALU_PRRP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prrp.h"

namespace prrp {

constexpr int kMaxB = 128;           // widest panel
constexpr int kDropBits = 19;        // tie bins: binary64 encoding >> 19
constexpr uint64_t kIdxMask = (1ull << kDropBits) - 1;
constexpr int64_t kMaxN = (1ll << kDropBits) - 2;
constexpr uint64_t kKeySent = ~0ull;                    // "not yet posted" key
constexpr uint64_t kDataSent = 0xFFF4DEADBEEF5AA5ull;   // "not yet posted" data word
constexpr int kMaxExchange = 96;     // strong RRQR interchanges per tile before giving up
constexpr unsigned kSpinLimit = 1u << 22;   // polls before a wait is declared failed

// ---------------------------------------------------------------- tie keys
// Key of a non-negative magnitude v at candidate index idx: larger keys win;
// magnitudes equal after dropping the low mantissa bits tie, and then the
// lower index wins.  Key 0 means "no candidate" (idx = kIdxMask never occurs).
__device__ __forceinline__ uint64_t mag_bits(double v) {
  return static_cast<uint64_t>(__double_as_longlong(v)) >> kDropBits;
}
__device__ __forceinline__ uint64_t make_key(double v, uint32_t idx) {
  return (mag_bits(v) << kDropBits) | (kIdxMask - idx);
}
__device__ __forceinline__ uint32_t key_index(uint64_t k) {
  return static_cast<uint32_t>(kIdxMask - (k & kIdxMask));
}
__device__ __forceinline__ bool key_nonfinite(uint64_t k) {
  return (k >> kDropBits) >= (0x7FF0000000000000ull >> kDropBits);
}

// ---------------------------------------------------- device-scope atomics
// Through global-address-space pointers: flat accesses would also count
// against the LDS wait counter, so every later LDS wait would wait for them.
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(1))) uint32_t g_u32;
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store((g_u64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
  return __hip_atomic_load((g_u64*)const_cast<uint64_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store((g_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev_u32(const uint32_t* p) {
  return __hip_atomic_load((g_u32*)const_cast<uint32_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
// Plain global loads and stores (no flat addressing).
__device__ __forceinline__ double ld_g(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}
__device__ __forceinline__ void st_g(double* p, double v) {
  *(__attribute__((address_space(1))) double*)p = v;
}

// Max of a non-negative double into a device record (bit order = value order).
__device__ __forceinline__ void atomic_max_pos(double* p, double v) {
  if (!(v >= 0.0)) v = __longlong_as_double(0x7FF8000000000000ll);  // NaN sorts last
  __hip_atomic_fetch_max(reinterpret_cast<unsigned long long*>(p),
                         static_cast<unsigned long long>(__double_as_longlong(v)),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// First non-zero info wins.
__device__ __forceinline__ void set_info(prrp_stats* st, int32_t v) {
  int32_t expect = 0;
  __hip_atomic_compare_exchange_strong(&st->info, &expect, v, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------ DPP lane permutations
// Data-parallel-primitive moves between lanes (no LDS round trip).  Controls:
// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror
// (lane i <-> 7-i within 8) = 0x141, row_mirror (i <-> 15-i within 16) = 0x140.
// Every lane's source is valid for these permutations, so the "old" operand
// is never read (bound_ctrl set): no move to initialise it.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
// Sum over each aligned group of 8 lanes (every lane gets the group sum).
__device__ __forceinline__ double sum8(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}
__device__ __forceinline__ uint64_t umax(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t max8_u64(uint64_t v) {
  v = umax(v, dpp_u64<0xB1>(v));
  v = umax(v, dpp_u64<0x4E>(v));
  v = umax(v, dpp_u64<0x141>(v));
  return v;
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
// Wave-wide max of a 64-bit key; the result is wave-uniform.
__device__ __forceinline__ uint64_t wave_max_key(uint64_t v) {
  v = max8_u64(v);
  v = umax(v, dpp_u64<0x140>(v));          // rows of 16
  return umax(umax(readlane_u64(v, 0), readlane_u64(v, 16)),
              umax(readlane_u64(v, 32), readlane_u64(v, 48)));
}
// The same when the 8 lanes of every row already hold one value (sum8 leaves
// the same bits in all 8 lanes: each butterfly level adds the same two
// operands in either order): only the 8 rows are compared.
__device__ __forceinline__ uint64_t wave_max_rows(uint64_t v) {
  v = umax(v, dpp_u64<0x140>(v));          // rows of 16
  return umax(umax(readlane_u64(v, 0), readlane_u64(v, 16)),
              umax(readlane_u64(v, 32), readlane_u64(v, 48)));
}
// Wave-wide sum in a fixed order (bitwise reproducible); wave-uniform result.
__device__ __forceinline__ double wave_sum_fixed(double v) {
  v = sum8(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// ------------------------------------------------------ wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

}  // namespace prrp
