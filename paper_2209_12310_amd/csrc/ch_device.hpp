// Device helpers shared by the filter, hull and batch kernels.
#pragma once

#include "ch_internal.hpp"

namespace chk {

__device__ __forceinline__ double cross3(int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t cx,
                                         int32_t cy) {
  const double t = (double)(by - ay) * (double)(cx - ax);
  return __builtin_fma((double)(bx - ax), (double)(cy - ay), -t);
}

// True when the turn a -> b -> c disqualifies b: not strictly left for the
// lower chain, not strictly right for the upper chain (both left to right).
template <bool LOWER>
__device__ __forceinline__ bool bad_turn(int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t cx,
                                         int32_t cy) {
  const double c = cross3(ax, ay, bx, by, cx, cy);
  return LOWER ? (c <= 0.0) : (c >= 0.0);
}

// Wave-wide maximum of a 64-bit value with DPP lane moves (VALU only):
// neighbours, quads, half rows, rows; then the four row results through
// readlane. All 64 lanes must be active; the result is wave-uniform.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_max_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, 0xF, 0xF, false);
  const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, 0xF, 0xF, false);
  const uint64_t o = ((uint64_t)ohi << 32) | olo;
  return o > v ? o : v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = dpp_max_u64<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_max_u64<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_max_u64<0x141>(v);  // row_half_mirror
  v = dpp_max_u64<0x140>(v);  // row_mirror
  uint64_t r = 0;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, row * 16);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), row * 16);
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    r = x > r ? x : r;
  }
  return r;
}

// Orders this wave's LDS accesses before and after the call (the waves of a
// workgroup are not synchronised).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ascending bitonic sort of key[0..P2), P2 a power of two >= kBlock. Wave w
// owns elements [w*P2/4, (w+1)*P2/4): stages whose partner distance keeps
// pairs inside that range need only a wave-level sync; the others (the last
// two or three distances of the largest merges) use workgroup barriers.
__device__ inline void bitonic_sort(uint64_t* key, uint32_t P2) {
  const uint32_t R = P2 / kWaves;
  const uint32_t lane = threadIdx.x & 63, base = (threadIdx.x >> 6) * R;
  bool block_mode = false;  // the previous stage used block-wide pairs
  for (uint32_t k = 2; k <= P2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (2 * j <= R) {
        if (block_mode) { __syncthreads(); block_mode = false; }
        for (uint32_t i = lane; i < R / 2; i += 64) {
          const uint32_t a = base + (((i & ~(j - 1)) << 1) | (i & (j - 1)));
          const uint32_t b = a + j;
          const uint64_t ka = key[a], kb = key[b];
          if ((ka > kb) == ((a & k) == 0)) { key[a] = kb; key[b] = ka; }
        }
        wave_sync();
      } else {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < P2 / 2; i += kBlock) {
          const uint32_t a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
          const uint32_t b = a | j;
          const uint64_t ka = key[a], kb = key[b];
          if ((ka > kb) == ((a & k) == 0)) { key[a] = kb; key[b] = ka; }
        }
        block_mode = true;
      }
    }
  }
  __syncthreads();
}

// Block-wide exclusive scan of one value per thread (all threads call it).
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t s_w[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(incl, d);
    if (lane >= d) incl += u;
  }
  if (lane == 63) s_w[w] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = s_w[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

}  // namespace chk
