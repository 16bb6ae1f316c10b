// Device helpers shared by the filter, hull and batch kernels.
#pragma once

#include "ch_internal.hpp"

namespace chk {

static constexpr float kGridF = 1048576.0f;  // 2^20: float units -> grid units

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

__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

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

// Sample-polygon tests (see SamplePoly). in_disc: a point of the disc is
// strictly inside the polygon. dx, dy are exact (both operands are multiples
// of 2^-20 in [0, 1)); the fp32 sum of squares is at least (1 - 2^-23) times
// the exact one, and r2 carries a larger margin, so the test never accepts a
// point outside the exact disc.
__device__ __forceinline__ bool in_disc(float x, float y, float cx, float cy, float r2) {
  const float dx = x - cx, dy = y - cy;
  return __builtin_fmaf(dx, dx, dy * dy) < r2;
}

// The inner region of the polygon: its disc, or its octagon |dx| < os,
// |dy| < os, |dx| + |dy| < ot about the same centre (also inside it; |dx|,
// |dy| and their sum are exact for grid values, os and ot are verified
// exactly). A point in either is strictly inside the polygon. Every
// comparison is false for a NaN coordinate, so such a point is never inside.
__device__ __forceinline__ bool in_inner(float x, float y, float cx, float cy, float r2, float os,
                                         float ot) {
  const float dx = __builtin_fabsf(x - cx), dy = __builtin_fabsf(y - cy);
  return (__builtin_fmaf(dx, dx, dy * dy) < r2) | ((dx < os) & (dy < os) & (dx + dy < ot));
}

// Exact: p strictly inside the counter-clockwise strictly convex polygon
// v[0..nv) (nv >= 3). p must lie strictly left of v0->v1 and strictly right
// of v0->v[nv-1]; a binary search over the fan at v0 finds the wedge
// v0, v_lo, v_lo+1 holding p, and p is inside when strictly left of that
// wedge's outer side.
__device__ __forceinline__ bool poly_strict_inside(const int32_t* vx, const int32_t* vy, uint32_t nv,
                                                   int32_t px, int32_t py) {
  const int32_t ax = vx[0], ay = vy[0];
  if (!(cross3(ax, ay, vx[1], vy[1], px, py) > 0.0)) return false;
  if (!(cross3(ax, ay, vx[nv - 1], vy[nv - 1], px, py) < 0.0)) return false;
  uint32_t lo = 1, hi = nv - 1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cross3(ax, ay, vx[mid], vy[mid], px, py) >= 0.0) lo = mid;
    else hi = mid;
  }
  return cross3(vx[lo], vy[lo], vx[hi], vy[hi], px, py) > 0.0;
}

// A 32- or 64-bit lane move through DPP (all 64 lanes active).
template <int CTRL, class T>
__device__ __forceinline__ T dpp_mov(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    const int x = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, ((uint64_t)b << 32) | a);
  }
}

template <class T>
__device__ __forceinline__ T read_lane(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(T, ((uint64_t)b << 32) | a);
  }
}

// Wave-wide reduction with an associative, commutative op: neighbour and
// quad swaps, then the half-row and row mirrors leave every lane of a row
// with the row's result; the four rows combine through readlane. All 64
// lanes must be active; the result is wave-uniform.
template <class T, class Op>
__device__ __forceinline__ T wave_allreduce(T v, Op op) {
  v = op(v, dpp_mov<0xB1>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_mov<0x4E>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_mov<0x141>(v));  // row_half_mirror
  v = op(v, dpp_mov<0x140>(v));  // row_mirror
  return op(op(read_lane(v, 0), read_lane(v, 16)), op(read_lane(v, 32), read_lane(v, 48)));
}

// Inclusive scan over the wave with DPP (VALU only): Hillis-Steele within
// each row of 16 lanes (row shifts by 1, 2, 4, 8; lanes without a source add
// 0), then each row adds the running total of the rows before it through the
// row broadcasts of lanes 15 and 31. All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1, 3
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2, 3
  return v;
}

// Block-wide exclusive scan of one value per thread (all threads call it).
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t s_w[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
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
