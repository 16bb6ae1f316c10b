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

// Pseudo-angle of the direction (dx, dy) != 0: a strictly increasing function
// of its angle from the +x axis counter-clockwise, onto [0, 4) -- the sine of
// the L1-normalised vector, unrolled per quadrant (0, 1, 2, 3 at the +x, +y,
// -x, -y axes). pangle64 is exact up to one rounding of the division;
// pangle32 (for the query points) is within 4e-7 of the exact value for
// integer inputs below 2^21 in magnitude.
__device__ __forceinline__ double pangle64(double dx, double dy) {
  const double a = dy / (__builtin_fabs(dx) + __builtin_fabs(dy));
  return dx >= 0.0 ? (dy >= 0.0 ? a : 4.0 + a) : 2.0 - a;
}
__device__ __forceinline__ float pangle32(float dx, float dy) {
  const float a = dy * __builtin_amdgcn_rcpf(__builtin_fabsf(dx) + __builtin_fabsf(dy));
  return dx >= 0.f ? (dy >= 0.f ? a : 4.f + a) : 2.f - a;
}

// Wedge table of a polygon about its centre c: the vertices, in
// counter-clockwise order starting at the smallest pseudo-angle, split the
// plane around c into wedges (wedge j between vertices j and j+1, the last
// one wrapping through angle 0). Bin k of Bins (kLutBins for the sample
// polygon of one set, kRefineLut and kBatchLutBins for the second polygons)
// covers the pseudo-angles
// [k w - eps, (k+1) w + eps], w = 4 / Bins, eps = 2^-16 (far above the
// error of pangle32); its entry holds the first wedge meeting that interval
// (low 16 bits) and the number of consecutive wedges that do (high 16 bits).
constexpr double kLutEps = 0x1p-16;

// Exact: p strictly inside the polygon. A point is strictly inside exactly
// when it is strictly left of every side, and one that is not is on or right
// of the side of the wedge its direction from c falls in; the bin of its
// computed pseudo-angle lists that wedge (the error is below eps), so testing
// the listed sides decides. c itself is strictly inside.
template <uint32_t Bins = kLutBins>
__device__ __forceinline__ bool poly_lut_inside(const int32_t* vx, const int32_t* vy, uint32_t nv,
                                                const uint32_t* lut, int32_t cx, int32_t cy,
                                                int32_t px, int32_t py) {
  const float dx = (float)(px - cx), dy = (float)(py - cy);
  if (dx == 0.f && dy == 0.f) return true;
  const float th = pangle32(dx, dy);
  const uint32_t k = min((uint32_t)(th * (float)(Bins / 4)), Bins - 1);
  const uint32_t e = lut[k];
  uint32_t j = e & 0xffffu;
  bool in = true;
  for (uint32_t c = e >> 16; c > 0; --c) {
    const uint32_t jn = j + 1 < nv ? j + 1 : 0;
    in = in && cross3(vx[j], vy[j], vx[jn], vy[jn], px, py) > 0.0;
    j = jn;
  }
  return in;
}

// Whole workgroup: the inner octagon |dx| <= s, |dy| <= s, |dx| + |dy| <= t
// (s <= t <= 2s) about c of the polygon px/py[0..m) (m = 0: none), written
// as out->os, out->ot in float units. A side with o = twice the area of its
// triangle with c and M, m' = the larger and smaller of |ex|, |ey| holds the
// octagon when s (M - m') + t m' <= o (the octagon's farthest vertex from the
// side's line, scaled by |e|). s_max = min o / M; for eight candidate s
// (s_max (1 - 2^-k), k = 3..10) the largest t follows, and the largest area
// 4 s^2 - 2 (2 s - t)^2 wins. The
// float values are checked against every side in exact arithmetic (products
// of a float and an integer below 2^21 are exact in fp64); a failure drops
// the octagon. mx/my: LDS scratch of V int32 each.
template <uint32_t V>
__device__ inline void fit_octagon(const int32_t* px, const int32_t* py, uint32_t m, int32_t cx,
                                   int32_t cy, int32_t* mx, int32_t* my, SamplePolyT<V>* __restrict__ out) {
  constexpr int kCand = 8;
  __shared__ double s_o[V];
  __shared__ double s_red[kWaves][kCand];
  __shared__ double s_smax[kWaves];
  __shared__ uint32_t s_fail;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double smax = __builtin_inf();
  for (uint32_t j = threadIdx.x; j < m; j += kBlock) {
    const uint32_t k = j + 1 < m ? j + 1 : 0;
    const int64_t ex = (int64_t)px[k] - px[j], ey = (int64_t)py[k] - py[j];
    const int64_t ax = ex < 0 ? -ex : ex, ay = ey < 0 ? -ey : ey;
    s_o[j] = (double)orient64(px[j], py[j], px[k], py[k], cx, cy);
    mx[j] = (int32_t)(ax > ay ? ax : ay);
    my[j] = (int32_t)(ax > ay ? ay : ax);
    smax = __builtin_fmin(smax, s_o[j] / (double)mx[j]);
  }
  smax = wave_allreduce(smax, [](double a, double b) { return __builtin_fmin(a, b); });
  if (lane == 0) s_smax[w] = smax;
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();
  smax = s_smax[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) smax = __builtin_fmin(smax, s_smax[i]);
  // Thread: candidate c = tid % 8 (s = smax (1 - 2^-(c+3))), sides tid / 8,
  // + 32, ... (near-axis sides bound t hard when s is close to smax).
  const uint32_t c = threadIdx.x % kCand, sl = threadIdx.x / kCand;
  const double sc = smax * (1.0 - __builtin_ldexp(1.0, -(int)c - 3));
  double t = 2.0 * sc;
  for (uint32_t j = sl; j < m; j += kBlock / kCand)
    if (my[j] > 0) t = __builtin_fmin(t, (s_o[j] - sc * (double)(mx[j] - my[j])) / (double)my[j]);
#pragma unroll
  for (int o = 32; o >= kCand; o >>= 1) t = __builtin_fmin(t, __shfl_xor(t, o));
  if (lane < kCand) s_red[w][lane] = t;
  __syncthreads();
  __shared__ float s_os, s_ot;
  if (threadIdx.x < 64) {
    // Lane i < kCand scores candidate i (its area); the largest wins, the
    // first of equal ones.
    double a = -1.0, si = 0.0, ti = 0.0;
    if (lane < kCand && m >= 3) {
      ti = s_red[0][lane];
#pragma unroll
      for (int q = 1; q < kWaves; ++q) ti = __builtin_fmin(ti, s_red[q][lane]);
      si = smax * (1.0 - __builtin_ldexp(1.0, -lane - 3));
      const double ar = 4.0 * si * si - 2.0 * (2.0 * si - ti) * (2.0 * si - ti);
      if (si > 0.0 && ti >= si) a = ar;
    }
    int win = 0;
    double best = read_lane(a, 0);
#pragma unroll
    for (int i = 1; i < kCand; ++i) {
      const double ai = read_lane(a, i);
      if (ai > best) { best = ai; win = i; }
    }
    const double bs = read_lane(si, win), bt = read_lane(ti, win);
    if (lane == 0) {
      // grid units -> float units, shrunk by a relative 2^-20
      s_os = best > 0.0 ? (float)(bs * 0x1p-20 * (1.0 - 0x1p-20)) : 0.0f;
      s_ot = best > 0.0 ? (float)(bt * 0x1p-20 * (1.0 - 0x1p-20)) : 0.0f;
    }
  }
  __syncthreads();
  const double gs = (double)s_os * 0x1p20, gt = (double)s_ot * 0x1p20;  // exact
  for (uint32_t j = threadIdx.x; j < m; j += kBlock)
    if (!(gs * (double)(mx[j] - my[j]) + gt * (double)my[j] <= s_o[j])) s_fail = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool keep = m >= 3 && s_fail == 0 && s_os > 0.0f;
    out->os = keep ? s_os : 0.0f;
    out->ot = keep ? s_ot : 0.0f;
  }
  __syncthreads();
}

// Whole workgroup. px/py[0..m0) (LDS) hold the extreme points in direction
// order; writes the SamplePoly, and with lut != null its wedge table. Steps:
// drop repeats of the previous point (cyclically), drop points where the
// boundary does not turn left (for up to Passes rounds), then verify and
// measure in wave 0: every turn
// strictly left, the centre c strictly left of every side, exactly one side
// crossing the line y = c.y upwards (one turn around c); r2 = the squared
// distance from c to the nearest side line, rounded down with a relative
// margin of 2^-19; then the inner octagon (see fit_octagon). With a table
// the vertices are stored from the one of
// smallest pseudo-angle about c on; a sequence of pseudo-angles that does not
// wrap exactly once disables the polygon.
template <uint32_t Bins = kLutBins, int Passes = 1, uint32_t V = kPolyMax>
__device__ inline void build_poly(int32_t* px, int32_t* py, uint32_t m0, SamplePolyT<V>* __restrict__ out,
                                  uint32_t* __restrict__ lut = nullptr) {
  static_assert(V <= 32 * kBlock, "items per thread fit a 32-bit mask");
  __shared__ int32_t qx[V], qy[V];
  __shared__ uint32_t s_ok, s_m, s_desc, s_rot;
  __shared__ int32_t s_cx, s_cy;
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
  // 2. collinear or reflex points, for up to Passes rounds (dropping a point
  //    can make a neighbour reflex; the rounds stop once one drops none)
  uint32_t m = m1;
  for (int it = 0; it < Passes; ++it) {
    if (it) {
      if (m == m1 || m < 3) break;
      for (uint32_t j = threadIdx.x; j < m; j += kBlock) { qx[j] = px[j]; qy[j] = py[j]; }
      __syncthreads();
      m1 = m;
    }
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
    pos = block_excl_scan(nk, m);
    for (uint32_t e = 0; e < E1; ++e)
      if (keep & (1u << e)) { px[pos] = qx[i0 + e]; py[pos] = qy[i0 + e]; ++pos; }
    if (Passes > 1) __syncthreads();
  }
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
    auto add_d = [](double a, double b) { return a + b; };
    auto add_i = [](int64_t a, int64_t b) { return a + b; };
    sa = wave_allreduce(sa, add_d);
    scx = wave_allreduce(scx, add_d);
    scy = wave_allreduce(scy, add_d);
    sx = wave_allreduce(sx, add_i);
    sy = wave_allreduce(sy, add_i);
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
      ups = wave_allreduce(ups, [](uint32_t a, uint32_t b) { return a + b; });
      r2 = wave_allreduce(r2, [](double a, double b) { return __builtin_fmin(a, b); });
      good = __ballot(!ok) == 0 && ups == 1;
    }
    if (lane == 0) {
      s_ok = good ? 1u : 0u;
      s_m = m;
      s_cx = (int32_t)cx;
      s_cy = (int32_t)cy;
      s_desc = 0;
      s_rot = 0;
      out->cx = (int32_t)cx;
      out->cy = (int32_t)cy;
      // grid units^2 -> float units^2 (2^-40), then the margin.
      out->r2 = good ? (float)(r2 * 0x1p-40 * (1.0 - 0x1p-19)) : 0.0f;
    }
  }
  __syncthreads();
  const bool ok = s_ok != 0;
  fit_octagon(px, py, ok ? m : 0u, s_cx, s_cy, qx, qy, out);
  if (!lut) {
    if (ok)
      for (uint32_t j = threadIdx.x; j < m; j += kBlock) { out->vx[j] = px[j]; out->vy[j] = py[j]; }
    if (threadIdx.x == 0) out->nv = ok ? m : 0u;
    return;
  }
  // 4. wedge table: rotate to the smallest pseudo-angle, then bin.
  __shared__ double s_t[V];
  const double ccx = s_cx, ccy = s_cy;
  if (ok) {
    for (uint32_t j = threadIdx.x; j < m; j += kBlock)
      s_t[j] = pangle64((double)px[j] - ccx, (double)py[j] - ccy);
  }
  __syncthreads();
  if (ok) {
    for (uint32_t j = threadIdx.x; j < m; j += kBlock) {
      const uint32_t p = j ? j - 1 : m - 1;
      if (!(s_t[j] > s_t[p])) { atomicAdd(&s_desc, 1u); s_rot = j; }
    }
  }
  __syncthreads();
  const bool use = ok && s_desc == 1;
  if (use) {
    const uint32_t r = s_rot;
    for (uint32_t j = threadIdx.x; j < m; j += kBlock) {
      const uint32_t q = j + r < m ? j + r : j + r - m;
      qx[j] = px[q];
      qy[j] = py[q];
    }
  }
  __syncthreads();
  if (use) {
    for (uint32_t j = threadIdx.x; j < m; j += kBlock) {
      s_t[j] = pangle64((double)qx[j] - ccx, (double)qy[j] - ccy);
      out->vx[j] = qx[j];
      out->vy[j] = qy[j];
    }
  }
  __syncthreads();
  // Bin k's interval ends, looked up by a binary search over the sorted
  // vertex angles: the wedge holding an angle th is the last vertex j with
  // t_j <= th, or the wrapping wedge m-1 when th < t_0. Each thread takes
  // Bins / kBlock consecutive bins and runs their searches in lockstep
  // (independent LDS reads in flight together).
  constexpr uint32_t kQ = Bins / kBlock;
  static_assert(Bins % kBlock == 0, "whole bins per thread");
  constexpr double w = 4.0 / (double)Bins;
  if (use) {
    double th[2 * kQ];
    uint32_t pos[2 * kQ];
#pragma unroll
    for (uint32_t i = 0; i < kQ; ++i) {
      const uint32_t k = threadIdx.x * kQ + i;
      double lo = (double)k * w - kLutEps, hi = (double)(k + 1) * w + kLutEps;
      th[2 * i] = lo < 0.0 ? lo + 4.0 : lo;
      th[2 * i + 1] = hi >= 4.0 ? hi - 4.0 : hi;
    }
#pragma unroll
    for (uint32_t q = 0; q < 2 * kQ; ++q) pos[q] = 0;
    uint32_t step = 1;
    while (step * 2 <= m) step *= 2;
    for (; step > 0; step >>= 1) {
      // Loads first (clamped, unconditional), so all of them are in flight
      // together; then the updates.
      double v[2 * kQ];
#pragma unroll
      for (uint32_t q = 0; q < 2 * kQ; ++q) {
        const uint32_t c = pos[q] + step;
        v[q] = s_t[c < m ? c : m - 1];
      }
#pragma unroll
      for (uint32_t q = 0; q < 2 * kQ; ++q) {
        const uint32_t c = pos[q] + step;
        pos[q] = (c < m) & (v[q] <= th[q]) ? c : pos[q];
      }
    }
    const double t0 = s_t[0];
#pragma unroll
    for (uint32_t i = 0; i < kQ; ++i) {
      const uint32_t a = th[2 * i] < t0 ? m - 1 : pos[2 * i];
      const uint32_t b = th[2 * i + 1] < t0 ? m - 1 : pos[2 * i + 1];
      lut[threadIdx.x * kQ + i] = a | (((b >= a ? b - a : b + m - a) + 1) << 16);
    }
  }
  if (threadIdx.x == 0) out->nv = use ? m : 0u;
}

// Largest and smallest dot product over the sample points sp[0..cnt) (LDS,
// cnt <= 2048) in direction (a, b), with the positions of the points that
// attain them: the maxima in the direction and in its opposite (whose dot
// product is the negation). Every lane reads the same point (an LDS
// broadcast); the dot products use 24-bit multiplies (|a|, |b| <= 1024,
// coordinates < 2^20, |dot| < 1.5 * 2^30). The scan keeps one int32 key per
// side, the dot product with its low 11 bits replaced by the position, so a
// max and a min carry the position along: the chosen point is extreme to
// within 2^11 of its dot product (a vertex of the polygon only has to be an
// input point), and the returned dot products are the exact ones of the
// chosen points.
static_assert(kBatchSample <= 2048 && kSamplePer <= 2048, "positions fit 11 bits");
__device__ __forceinline__ void dir_minmax(const int2* __restrict__ sp, uint32_t cnt, int32_t a,
                                           int32_t b, int32_t& dmax, uint32_t& qmax,
                                           int32_t& dmin, uint32_t& qmin) {
  int32_t kmax = INT32_MIN, kmin = INT32_MAX;
#pragma unroll 8
  for (uint32_t q = 0; q < cnt; ++q) {
    const int2 p = sp[q];
    const int32_t e = __mul24(a, p.x) + __mul24(b, p.y);
    const int32_t k = (e & ~0x7FF) | (int32_t)q;
    kmax = k > kmax ? k : kmax;
    kmin = k < kmin ? k : kmin;
  }
  qmax = (uint32_t)kmax & 0x7FFu;
  qmin = (uint32_t)kmin & 0x7FFu;
  if (cnt == 0) qmax = qmin = 0;
  const int2 pM = sp[qmax < cnt ? qmax : 0], pm = sp[qmin < cnt ? qmin : 0];
  dmax = cnt ? __mul24(a, pM.x) + __mul24(b, pM.y) : INT32_MIN;
  dmin = cnt ? __mul24(a, pm.x) + __mul24(b, pm.y) : INT32_MAX;
}

// Single set, before the fused pass. k_sample_dirs: workgroup b takes sample
// points b*kSamplePer .. +kSamplePer-1 of kSampleN spread evenly over [0, n)
// (point floor(k n / kSampleN); single points, not the batch sampler's runs:
// with runs the fused pass measured slower on normal data) and writes, per direction, its largest dot
// product with that point's coordinates (one partial per workgroup and
// direction, written contiguously, no atomics). k_sample_reduce: each
// workgroup folds the partials of kReduceDirsPerBlock directions into the
// extreme point per direction, and the last to arrive builds the polygon.
struct SampleDirs {
  int32_t vx[kPolyMax], vy[kPolyMax];  // extreme sample point per direction
  uint32_t arrive;
  uint32_t cand;       // candidate records written by the fused pass
  uint32_t mode;       // how the fused pass ran (bits: polygon, octagon, whole grid)
  uint32_t pad[61];
  uint32_t lut[kLutBins];              // wedge table of the polygon (see build_poly)
  int4 part[kSampleBlocks][kPolyMax];  // (dot product, x, y, 0)
};
constexpr uint32_t kReduceDirsPerBlock = 8;

constexpr uint32_t kSampleReduceBlocks = kPolyMax / kReduceDirsPerBlock;

}  // namespace chk
