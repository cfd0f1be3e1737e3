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
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev_u32(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
