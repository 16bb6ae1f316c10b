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
// of 2 pi d / D) for d < D/2 and the negation of direction d - D/2 after
// that (so one dot product serves a direction and its opposite). Their angles are strictly increasing (the rounding moves an
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
  // Directions D/2 .. D-1 are the negations of 0 .. D/2-1, exactly.
  const uint32_t h = d < D / 2 ? d : d - D / 2;
  double sn, cs;
  sincos(6.283185307179586 * (double)h / (double)D, &sn, &cs);
  a = (int32_t)__builtin_rint(1024.0 * cs);
  b = (int32_t)__builtin_rint(1024.0 * sn);
  if (d >= D / 2) { a = -a; b = -b; }
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

// Largest and smallest dot product over the sample points sp[0..cnt) (LDS)
// in direction (a, b), with the positions of their first occurrences: the
// maxima in the direction and in its opposite (whose dot product is the
// negation). Every lane reads the same point (an LDS broadcast); the dot
// products use 24-bit multiplies (|a|, |b| <= 1024, coordinates < 2^20).
__device__ __forceinline__ void dir_minmax(const int2* __restrict__ sp, uint32_t cnt, int32_t a,
                                           int32_t b, int32_t& dmax, uint32_t& qmax,
                                           int32_t& dmin, uint32_t& qmin) {
  dmax = INT32_MIN;
  dmin = INT32_MAX;
  qmax = qmin = 0;
#pragma unroll 8
  for (uint32_t q = 0; q < cnt; ++q) {
    const int2 p = sp[q];
    const int32_t e = __mul24(a, p.x) + __mul24(b, p.y);
    if (e > dmax) { dmax = e; qmax = q; }
    if (e < dmin) { dmin = e; qmin = q; }
  }
}

// Single set, before the fused pass. k_sample_dirs: workgroup b takes sample
// points b*kSamplePer .. +kSamplePer-1 of kSampleN spread evenly over [0, n)
// (point floor(k n / kSampleN)) and writes, per direction, its largest dot
// product with that point's coordinates (one partial per workgroup and
// direction, written contiguously, no atomics). k_sample_reduce: each
// workgroup folds the partials of kReduceDirsPerBlock directions into the
// extreme point per direction, and the last to arrive builds the polygon.
struct SampleDirs {
  int32_t vx[kPolyMax], vy[kPolyMax];  // extreme sample point per direction
  uint32_t arrive;
  uint32_t cand;       // candidate records written by the fused pass
  uint32_t pad[62];
  int4 part[kSampleBlocks][kPolyMax];  // (dot product, x, y, 0)
};
constexpr uint32_t kReduceDirsPerBlock = 8;
constexpr uint32_t kSampleReduceBlocks = kPolyMax / kReduceDirsPerBlock;

}  // namespace chk
