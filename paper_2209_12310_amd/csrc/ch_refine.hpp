// Refined filter of the hull path (ch_hull and ch_hull_batch; ch_filter keeps
// the octagon test alone, so its survivor list is exactly the paper's).
//
// The octagon of Sec. III discards little when many points lie close to the
// hull -- points near a circle keep ~99% of the input. The remedy is the same
// rule with a finer polygon: take a strided sample of the input, find its
// extreme points in many directions, and use the convex polygon they span.
// Its vertices are input points, so a point strictly inside it is a convex
// combination of other input points and cannot be a strict hull vertex; the
// hull is unchanged, only fewer candidates reach the hull pass.
//
// Directions: d = 0 .. D-1 counter-clockwise, (a, b) = round(1024 (cos, sin)
// of 2 pi d / D). Their angles are strictly increasing (the rounding moves an
// angle by < 1e-3 rad, the spacing is > 1e-2 rad), so the extreme points,
// taken in direction order, run counter-clockwise around the sample's hull.
// Dot products a x + b y of grid points stay below 1449 * 2^20 < 2^31.
//
// The polygon is checked before use (strictly convex, one turn around an
// inner grid point); any doubt disables it, which only costs time. Sample
// values outside the domain are clamped into the grid: such an input fails
// pass 1 with a domain error, and pass 2 never uses its polygon.
#pragma once

#include "ch_device.hpp"

namespace chk {

__device__ __forceinline__ void direction(uint32_t d, uint32_t D, int32_t& a, int32_t& b) {
  const double t = 6.283185307179586 * (double)d / (double)D;
  a = (int32_t)__builtin_rint(1024.0 * cos(t));
  b = (int32_t)__builtin_rint(1024.0 * sin(t));
}

// Grid coordinates of a point, clamped into the grid (see above).
__device__ __forceinline__ int2 grid_point(const float* __restrict__ xy, size_t i) {
  const float tx = xy[2 * i] * kGridF, ty = xy[2 * i + 1] * kGridF;
  int2 p;
  p.x = (int32_t)__builtin_fminf(__builtin_fmaxf(tx, 0.f), kGridF - 1.f);
  p.y = (int32_t)__builtin_fminf(__builtin_fmaxf(ty, 0.f), kGridF - 1.f);
  return p;
}

__device__ __forceinline__ int64_t orient64(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                                            int64_t cx, int64_t cy) {
  return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Whole workgroup. px/py[0..m0) (LDS) hold the extreme points in direction
// order; writes the SamplePoly. Steps: drop repeats of the previous point
// (cyclically), drop points where the boundary does not turn left, then
// verify and measure in wave 0: every turn strictly left, the rounded vertex
// mean c strictly left of every side, exactly one side crossing the line
// y = c.y upwards (one turn around c), and r2 = the squared distance from c
// to the nearest side line, rounded down with a relative margin of 2^-19.
__device__ inline void build_poly(int32_t* px, int32_t* py, uint32_t m0, SamplePoly* __restrict__ out) {
  __shared__ int32_t qx[kPolyMax], qy[kPolyMax];
  __shared__ uint32_t s_ok;
  const uint32_t E = (m0 + kBlock - 1) / kBlock;
  const uint32_t j0 = threadIdx.x * E;
  // 1. repeats
  uint32_t keep = 0, nk = 0;
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t j = j0 + e;
    if (j < m0) {
      const uint32_t p = j ? j - 1 : m0 - 1;
      if (px[j] != px[p] || py[j] != py[p]) { keep |= 1u << e; ++nk; }
    }
  }
  uint32_t m1;
  uint32_t pos = block_excl_scan(nk, m1);
  for (uint32_t e = 0; e < E; ++e)
    if (keep & (1u << e)) { qx[pos] = px[j0 + e]; qy[pos] = py[j0 + e]; ++pos; }
  __syncthreads();
  // 2. collinear or reflex points
  const uint32_t E1 = (m1 + kBlock - 1) / kBlock;
  const uint32_t i0 = threadIdx.x * E1;
  keep = 0; nk = 0;
  for (uint32_t e = 0; e < E1 && m1 >= 3; ++e) {
    const uint32_t i = i0 + e;
    if (i < m1) {
      const uint32_t p = i ? i - 1 : m1 - 1, q = i + 1 < m1 ? i + 1 : 0;
      if (orient64(qx[p], qy[p], qx[i], qy[i], qx[q], qy[q]) > 0) { keep |= 1u << e; ++nk; }
    }
  }
  uint32_t m;
  pos = block_excl_scan(nk, m);
  for (uint32_t e = 0; e < E1; ++e)
    if (keep & (1u << e)) { px[pos] = qx[i0 + e]; py[pos] = qy[i0 + e]; ++pos; }
  __syncthreads();
  // 3. verify, centre, disc. The centre is the polygon's area centroid
  //    (interior for a convex polygon; computed in fp64 relative to vertex
  //    0, rounded to the grid), else the vertex mean; exact tests decide.
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double sa = 0.0, scx = 0.0, scy = 0.0;
    int64_t sx = 0, sy = 0;
    const int64_t ox = m ? px[0] : 0, oy = m ? py[0] : 0;
    for (uint32_t j = lane; j < m; j += 64) {
      const uint32_t k = j + 1 < m ? j + 1 : 0;
      const double x0 = (double)(px[j] - ox), y0 = (double)(py[j] - oy);
      const double x1 = (double)(px[k] - ox), y1 = (double)(py[k] - oy);
      const double cr = x0 * y1 - x1 * y0;
      sa += cr; scx += (x0 + x1) * cr; scy += (y0 + y1) * cr;
      sx += px[j]; sy += py[j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sa += __shfl_xor(sa, o); scx += __shfl_xor(scx, o); scy += __shfl_xor(scy, o);
      sx += __shfl_xor(sx, o); sy += __shfl_xor(sy, o);
    }
    bool good = false;
    int64_t cx = 0, cy = 0;
    double r2 = 0.0;
    for (int cand = 0; cand < 2 && !good && m >= 3; ++cand) {
      if (cand == 0) {
        if (!(sa > 0.0)) continue;
        cx = ox + (int64_t)__builtin_rint(scx / (3.0 * sa));
        cy = oy + (int64_t)__builtin_rint(scy / (3.0 * sa));
      } else {
        cx = (int64_t)__builtin_rint((double)sx / (double)m);
        cy = (int64_t)__builtin_rint((double)sy / (double)m);
      }
      bool ok = true;
      uint32_t ups = 0;
      r2 = __builtin_inf();
      for (uint32_t j = lane; j < m; j += 64) {
        const uint32_t p = j ? j - 1 : m - 1, k = j + 1 < m ? j + 1 : 0;
        ok = ok && orient64(px[p], py[p], px[j], py[j], px[k], py[k]) > 0;
        const int64_t o = orient64(px[j], py[j], px[k], py[k], cx, cy);
        ok = ok && o > 0;
        ups += (py[j] <= cy && py[k] > cy) ? 1u : 0u;
        const int64_t ex = (int64_t)px[k] - px[j], ey = (int64_t)py[k] - py[j];
        const double od = (double)o;
        r2 = __builtin_fmin(r2, od * od / (double)(ex * ex + ey * ey));
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        ups += __shfl_xor(ups, o);
        r2 = __builtin_fmin(r2, __shfl_xor(r2, o));
      }
      good = __ballot(!ok) == 0 && ups == 1;
    }
    if (lane == 0) {
      s_ok = good ? 1u : 0u;
      out->nv = good ? m : 0u;
      out->cx = (int32_t)cx;
      out->cy = (int32_t)cy;
      // grid units^2 -> float units^2 (2^-40), then the margin.
      out->r2 = good ? (float)(r2 * 0x1p-40 * (1.0 - 0x1p-19)) : 0.0f;
    }
  }
  __syncthreads();
  if (s_ok)
    for (uint32_t j = threadIdx.x; j < m; j += kBlock) { out->vx[j] = px[j]; out->vy[j] = py[j]; }
}

// Order-preserving key of a direction maximum: the dot product (biased to
// unsigned; never 0 here) above the sample number.
__device__ __forceinline__ uint64_t dir_key(int32_t dot, uint32_t tag) {
  return ((uint64_t)((uint32_t)dot ^ 0x80000000u) << 32) | tag;
}

// Largest dot product over the sample points sp[0..cnt) (LDS) in the
// directions (a0, b0) and (a1, b1), with the position of its first
// occurrence. Every lane reads the same point (an LDS broadcast); the dot
// products use 24-bit multiplies (|a|, |b| <= 1024, coordinates < 2^20).
__device__ __forceinline__ void dir_max2(const int2* __restrict__ sp, uint32_t cnt, int32_t a0,
                                         int32_t b0, int32_t a1, int32_t b1, int32_t& d0,
                                         uint32_t& q0, int32_t& d1, uint32_t& q1) {
  d0 = d1 = INT32_MIN;
  q0 = q1 = 0;
#pragma unroll 8
  for (uint32_t q = 0; q < cnt; ++q) {
    const int2 p = sp[q];
    const int32_t e0 = __mul24(a0, p.x) + __mul24(b0, p.y);
    const int32_t e1 = __mul24(a1, p.x) + __mul24(b1, p.y);
    if (e0 > d0) { d0 = e0; q0 = q; }
    if (e1 > d1) { d1 = e1; q1 = q; }
  }
}

// Single set: the direction maxima live in the workspace and are cleared
// first (sample_dirs_clear). Then each workgroup takes sample points
// b*kSamplePer .. +kSamplePer-1 of kSampleN spread evenly over [0, n) (point
// floor(k n / kSampleN)) -- all of them, or with an octagon `oct` only those
// strictly outside it (any input points span a safe polygon) -- folds their
// maximum per direction into the shared maxima (64-bit atomic max of the
// biased dot product above the sample number), and the last one to arrive
// builds the polygon from them, or leaves it out when some direction got no
// point (sample_dirs_block).
struct SampleDirs {
  uint64_t key[kPolyMax];
  uint32_t arrive;
  uint32_t cand;       // candidate records written by the fused pass
  uint32_t pad[62];
};
static_assert(sizeof(SampleDirs) <= size_t(kPolyMax) * 8 + 256, "workspace slot of the maxima");

__device__ __forceinline__ void sample_dirs_clear(SampleDirs* __restrict__ sd) {
  for (uint32_t d = threadIdx.x; d < (uint32_t)kPolyMax; d += kBlock) sd->key[d] = 0ull;
  if (threadIdx.x == 0) {
    sd->arrive = 0;
    sd->cand = 0;
  }
}

__device__ inline void sample_dirs_block(const float* __restrict__ xy, uint32_t n,
                                         const Octagon* __restrict__ oct,
                                         SampleDirs* __restrict__ sd, SamplePoly* __restrict__ poly,
                                         uint32_t blk, uint32_t nblk) {
  static_assert(kPolyMax == 2 * kBlock, "two directions per thread");
  static_assert(kSamplePer == (uint32_t)kBlock, "one sample point per thread");
  __shared__ int2 sp[kSamplePer];
  __shared__ uint32_t sq[kSamplePer];
  __shared__ int32_t px[kPolyMax], py[kPolyMax];
  __shared__ uint32_t s_last, s_miss;
  // This thread's sample point; kept when strictly outside the octagon.
  const uint32_t k = blk * kSamplePer + threadIdx.x;
  const int2 p = grid_point(xy, (size_t)((uint64_t(k) * n) / kSampleN));
  bool out = oct == nullptr;
  if (oct && oct->status == 0) {
    const double x = (double)p.x * 0x1p-20, y = (double)p.y * 0x1p-20;
    double mn = __builtin_inf();
#pragma unroll
    for (int i = 0; i < 8; ++i)
      mn = __builtin_fmin(mn, __builtin_fma(oct->A[i], x, __builtin_fma(oct->B[i], y, oct->C[i])));
    out = mn < 0.0;
  }
  uint32_t m;
  const uint32_t pos = block_excl_scan(out ? 1u : 0u, m);
  if (out) { sp[pos] = p; sq[pos] = k; }
  __syncthreads();
  if (m) {
    const uint32_t d = threadIdx.x;
    int32_t a0, b0, a1, b1;
    direction(d, kPolyMax, a0, b0);
    direction(d + kBlock, kPolyMax, a1, b1);
    int32_t e0, e1;
    uint32_t q0, q1;
    dir_max2(sp, m, a0, b0, a1, b1, e0, q0, e1, q1);
    atomicMax((unsigned long long*)&sd->key[d], (unsigned long long)dir_key(e0, sq[q0]));
    atomicMax((unsigned long long*)&sd->key[d + kBlock], (unsigned long long)dir_key(e1, sq[q1]));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&sd->arrive, 1u) == nblk - 1 ? 1u : 0u;
    s_miss = 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  uint64_t key[kPolyMax / kBlock];
#pragma unroll
  for (int e = 0; e < kPolyMax / kBlock; ++e) {
    key[e] = __hip_atomic_load(&sd->key[threadIdx.x + e * kBlock], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    if (!key[e]) s_miss = 1;  // a direction without a sample point outside the octagon
  }
  __syncthreads();
  if (s_miss) {
    if (threadIdx.x == 0) poly->nv = 0;
    return;
  }
#pragma unroll
  for (int e = 0; e < kPolyMax / kBlock; ++e) {
    const int2 v = grid_point(xy, (size_t)((uint64_t((uint32_t)key[e]) * n) / kSampleN));
    px[threadIdx.x + e * kBlock] = v.x;
    py[threadIdx.x + e * kBlock] = v.y;
  }
  __syncthreads();
  build_poly(px, py, kPolyMax, poly);
}

}  // namespace chk
