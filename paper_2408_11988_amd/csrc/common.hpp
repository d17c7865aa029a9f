// Shared device and host helpers of the TS-SpGEMM library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "tsspgemm.h"

namespace tss {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 256;      // threads per workgroup of the row kernels (4 wavefronts)
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxDenseD = 1024; // dense (SPA) accumulator limit, Sec. III-C: SPA for d <= 1024

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of `m` held by lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src_lane) {
  return (uint32_t)__shfl((int)v, src_lane, kWave);
}

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int mask) {
  return (uint32_t)__shfl_xor((int)v, mask, kWave);
}

// Sum over the wavefront (all 64 lanes get the result).
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele with cross-lane reads).
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

// ---------------------------------------------------------------- host helpers

// Words per bitmap row for width d: ceil(d/32) rounded up to a power of two.
inline int bitmap_words(int64_t d) {
  int w = (int)((d + 31) / 32);
  int p = 1;
  while (p < w) p <<= 1;
  return p;
}

void set_error(const std::string& msg);
const std::string& get_error();

#define TSS_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ::tss::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                    \
      return TSSPGEMM_ERR_HIP;                                                                 \
    }                                                                                          \
  } while (0)

#define TSS_CHECK_LAUNCH()                                                                     \
  do {                                                                                         \
    hipError_t e_ = hipGetLastError();                                                         \
    if (e_ != hipSuccess) {                                                                    \
      ::tss::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));               \
      return TSSPGEMM_ERR_HIP;                                                                 \
    }                                                                                          \
  } while (0)

inline unsigned grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace tss
