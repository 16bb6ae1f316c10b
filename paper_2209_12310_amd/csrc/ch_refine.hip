// Refined filter: the kernels that build the sample polygons (one set before
// its fused pass; one workgroup per set in batch mode).
#include "ch_refine.hpp"

namespace chk {

// Whole workgroup, one chunk of sample points: thread t holds points
// t + k kBlock (k < P) in v, and sp holds them all. Keeps the points that can
// be extreme in some direction: the extreme points E_0..E_7 of the chunk in
// the directions x, x+y, y, y-x, -x, -x-y, -y, x-y (the largest key (value,
// position), so exact maxima) lie on its convex hull in counter-clockwise
// order, so a point strictly left of every side E_d E_{d+1} of nonzero length
// is strictly inside the hull and is no direction's maximum. The others are
// compacted to the front of sp (in an order of their own); returns their
// count, at least one. Orientations in fp64 are exact (coordinates below
// 2^20). key: LDS scratch of kWaves x 8.
template <uint32_t P>
__device__ inline uint32_t octagon_sieve(const int2 (&v)[P], int2* sp, int64_t (*key)[8]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  auto val = [](int2 p, int d) -> int32_t {
    const int32_t a = d == 0 || d == 1 || d == 7 ? p.x : (d == 3 || d == 4 || d == 5 ? -p.x : 0);
    const int32_t b = d == 1 || d == 2 || d == 3 ? p.y : (d == 5 || d == 6 || d == 7 ? -p.y : 0);
    return a + b;
  };
  auto mx = [](int64_t a, int64_t b) { return a > b ? a : b; };
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    int64_t k = INT64_MIN;
#pragma unroll
    for (uint32_t i = 0; i < P; ++i)
      k = mx(k, (int64_t)((uint64_t)(int64_t)val(v[i], d) << 32 | (threadIdx.x + i * kBlock)));
    k = wave_allreduce(k, mx);
    if (lane == 0) key[w][d] = k;
  }
  __syncthreads();
  double ex[8], ey[8], ax[8], ay[8];
  bool use[8];
  int2 e[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    int64_t k = key[0][d];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) k = mx(k, key[i][d]);
    e[d] = sp[(uint32_t)k & 0xFFFFu];
  }
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int2 a = e[d], b = e[(d + 1) & 7];
    ax[d] = a.x;
    ay[d] = a.y;
    ex[d] = (double)(b.x - a.x);
    ey[d] = (double)(b.y - a.y);
    use[d] = a.x != b.x || a.y != b.y;
  }
  uint32_t keep = 0, nk = 0;
#pragma unroll
  for (uint32_t i = 0; i < P; ++i) {
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      inside = inside && (!use[d] || ex[d] * ((double)v[i].y - ay[d]) - ey[d] * ((double)v[i].x - ax[d]) > 0.0);
    if (!inside) { keep |= 1u << i; ++nk; }
  }
  uint32_t m;
  uint32_t pos = block_excl_scan(nk, m);  // its barriers: every vertex read above is done
#pragma unroll
  for (uint32_t i = 0; i < P; ++i)
    if (keep & (1u << i)) sp[pos++] = v[i];
  return m;
}

// Batch (before the single read): a workgroup per set of at least
// sample_min (and kBatchSample) points; the workgroups take the sets of the
// plan's list (longest jobs first) one at a time through a shared counter.
// Per set: batch_chunks chunks of kBatchSample sample points, kBatchDirs
// directions, the polygon in the set's SamplePoly (the plan clears the
// polygon of the other sets; the pass tests against it by a binary search,
// no wedge table: building one per set cost the sampler more than it saved
// the pass). The direction
// scans run over a chunk's points left by octagon_sieve. A chunk's points
// are runs of kSampleRun consecutive input points (one 128-byte line each)
// with the runs spread evenly over the set: a sample point per line fetched,
// where single points at a large stride would fetch a line each. Four
// workgroups per CU (at most 128 VGPRs, a few spilled) keep more sets' sample
// loads in flight than three.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_sample(const float* __restrict__ xy,
                                                         const uint64_t* __restrict__ off,
                                                         BatchHdr* __restrict__ bh,
                                                         const uint32_t* __restrict__ slist,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t sample_min) {
  // Thread t takes direction pair t % kPairs (a direction and its opposite)
  // over half t / kPairs of each chunk's sample; the halves are combined.
  constexpr uint32_t kPairs = kBatchDirs / 2;
  static_assert(2 * kPairs == (uint32_t)kBlock, "two threads per direction pair");
  constexpr uint32_t kRuns = kBatchSample / kSampleRun;  // runs per chunk
  constexpr uint32_t kPer = kBatchSample / kBlock;       // chunk points per thread
  __shared__ int2 sp[kBatchSample];
  __shared__ int64_t s_key[kWaves][8];
  __shared__ int32_t px[kBatchDirs], py[kBatchDirs];
  __shared__ int32_t s_e[2][kPairs];
  __shared__ int2 s_p[2][kPairs];
  __shared__ uint32_t s_item;
  const uint32_t nlist = bh->nsampled;
  const uint32_t pr = threadIdx.x % kPairs, half = threadIdx.x / kPairs;
  int32_t a0, b0;
  direction(pr, kBatchDirs, a0, b0);
  for (;;) {
    __syncthreads();  // the previous set is done with the shared arrays and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(&bh->sample_next, 1u);
    __syncthreads();
    if (s_item >= nlist) break;
    const uint32_t s = slist[s_item];
    const uint64_t base = off[s];
    const uint64_t n = off[s + 1] - base;
    const uint32_t nch = batch_chunks(n, sample_min);
    const uint64_t nr = uint64_t(nch) * kRuns;  // runs over the whole set
    // running extremes of this thread's direction pair over the chunks
    // (kept by the threads of half 0)
    int32_t bmax = INT32_MIN, bmin = INT32_MAX;
    int2 pmax = make_int2(0, 0), pmin = make_int2(0, 0);
    for (uint32_t c = 0; c < nch; ++c) {
      __syncthreads();  // the previous chunk or set is done with the shared arrays
      int2 v[kPer];
#pragma unroll
      for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t q = threadIdx.x + k * kBlock;
        const uint64_t r = uint64_t(c) * kRuns + q / kSampleRun;
        v[k] = grid_point(xy, base + min<uint64_t>((r * n) / nr + q % kSampleRun, n - 1));
        sp[q] = v[k];
      }
      const uint32_t m = octagon_sieve(v, sp, s_key);
      __syncthreads();
      const uint32_t h0 = half * (m / 2), h1 = half ? m : m / 2;
      int32_t emax = INT32_MIN, emin = INT32_MAX;
      uint32_t q0 = h0, q1 = h0;
      if (h1 > h0) {
        dir_minmax(sp + h0, h1 - h0, a0, b0, emax, q0, emin, q1);
        q0 += h0;
        q1 += h0;
      }
      if (half) {
        s_e[0][pr] = emax;
        s_e[1][pr] = emin;
        s_p[0][pr] = sp[q0];
        s_p[1][pr] = sp[q1];
      }
      __syncthreads();
      if (!half) {
        // the first half wins ties (the first occurrence among the chunk's
        // sieved points), and earlier chunks win ties over later ones
        int2 cmax = sp[q0], cmin = sp[q1];
        if (s_e[0][pr] > emax) { emax = s_e[0][pr]; cmax = s_p[0][pr]; }
        if (s_e[1][pr] < emin) { emin = s_e[1][pr]; cmin = s_p[1][pr]; }
        if (emax > bmax) { bmax = emax; pmax = cmax; }
        if (emin < bmin) { bmin = emin; pmin = cmin; }
      }
    }
    if (!half) {
      px[pr] = pmax.x;
      py[pr] = pmax.y;
      px[pr + kPairs] = pmin.x;
      py[pr + kPairs] = pmin.y;
    }
    __syncthreads();
    build_poly(px, py, kBatchDirs, &polys[s]);
  }
}

static_assert(sizeof(SampleDirs) <= size_t(kPolyMax) * 8 + 256 + size_t(kLutBins) * 4 +
                                         size_t(kSampleBlocks) * kPolyMax * 16,
              "workspace slot of the direction maxima");

__global__ __launch_bounds__(kBlock) void k_sample_dirs(const float* __restrict__ xy, uint32_t n,
                                                        SampleDirs* __restrict__ sd,
                                                        uint32_t* __restrict__ count0,
                                                        RefineState* __restrict__ rs) {
  static_assert(kPolyMax == 2 * kBlock, "a direction and its opposite per thread");
  static_assert(kRefineBins == 4 * kSampleBlocks, "four second-polygon bins cleared per workgroup");
  __shared__ int2 sp[kSamplePer];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sd->arrive = 0;  // for k_sample_reduce
    sd->cand = 0;    // for the fused pass
    *count0 = 0;     // survivors of the candidates' octagon test, two launches on
    rs->arrive = 0;  // for k_refine_bins
  }
  if (threadIdx.x < 4) rs->bin[4 * blockIdx.x + threadIdx.x] = 0ull;
  const uint32_t k0 = blockIdx.x * kSamplePer;
  for (uint32_t q = threadIdx.x; q < kSamplePer; q += kBlock)
    sp[q] = grid_point(xy, (size_t)((uint64_t(k0 + q) * n) / kSampleN));
  __syncthreads();
  const uint32_t d = threadIdx.x;
  int32_t a, b;
  direction(d, kPolyMax, a, b);
  int32_t emax, emin;
  uint32_t qmax, qmin;
  dir_minmax(sp, kSamplePer, a, b, emax, qmax, emin, qmin);
  sd->part[blockIdx.x][d] = make_int4(emax, sp[qmax].x, sp[qmax].y, 0);
  sd->part[blockIdx.x][d + kBlock] = make_int4(-emin, sp[qmin].x, sp[qmin].y, 0);
}

__global__ __launch_bounds__(kBlock) void k_sample_reduce(const float* __restrict__ xy, uint32_t n,
                                                          SampleDirs* __restrict__ sd,
                                                          SamplePoly* __restrict__ poly) {
  constexpr uint32_t kLanes = kBlock / kReduceDirsPerBlock;  // lanes per direction
  static_assert(kLanes == 32 && kSampleBlocks % kLanes == 0, "32 lanes per direction");
  __shared__ int32_t px[kPolyMax], py[kPolyMax];
  __shared__ uint32_t s_last;
  const uint32_t d = blockIdx.x * kReduceDirsPerBlock + threadIdx.x / kLanes;
  const uint32_t ln = threadIdx.x % kLanes;
  // Each lane of a direction reads every kLanes-th row of the partials.
  int4 best = make_int4(INT32_MIN, 0, 0, 0);
#pragma unroll 8
  for (uint32_t b = ln; b < kSampleBlocks; b += kLanes) {
    const int4 v = sd->part[b][d];
    const bool gt = v.x > best.x;  // per component: a select of the whole int4 goes through memory
    best.x = gt ? v.x : best.x;
    best.y = gt ? v.y : best.y;
    best.z = gt ? v.z : best.z;
  }
#pragma unroll
  for (uint32_t o = 1; o < kLanes; o <<= 1) {
    const int32_t ox = __shfl_xor(best.x, (int)o), oy = __shfl_xor(best.y, (int)o);
    const int32_t oz = __shfl_xor(best.z, (int)o);
    if (ox > best.x) { best.x = ox; best.y = oy; best.z = oz; }
  }
  if (ln == 0) {
    sd->vx[d] = best.y;
    sd->vy[d] = best.z;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&sd->arrive, 1u) == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (uint32_t e = threadIdx.x; e < (uint32_t)kPolyMax; e += kBlock) {
    px[e] = __hip_atomic_load(&sd->vx[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    py[e] = __hip_atomic_load(&sd->vy[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  build_poly(px, py, kPolyMax, poly, sd->lut);
}

// Single set, when the block hull finds too many survivors: a second
// polygon from the survivor records themselves. The plane around c (the
// sample polygon's centre, else the mean of the octagon's vertices) is cut
// into kRefineBins bins of pseudo-angle; per bin the record of largest dot
// product with the bin's middle direction is kept: each workgroup takes the
// maxima of (dot product, record) over its records in LDS and folds its
// non-empty bins into rs->bin with 64-bit atomic max. The last workgroup to
// arrive gathers the kept records in bin order, clears the bins and the
// counter for the next call, and builds the polygon and its wedge table with
// build_poly (repeats and reflex points dropped until none remain). Every
// vertex is an input point, so a record strictly inside it is not a hull
// vertex, whichever records were kept; a failed check leaves nv = 0. For
// points near a smooth curve the kept records are the extreme points in the
// bins' directions, and the polygon is as close to the hull as its number of
// sides allows. Clears rs->cnt for k_refine_filter.
__global__ __launch_bounds__(kBlock) void k_refine_bins(const Rec* __restrict__ in,
                                                        const uint32_t* __restrict__ count_in,
                                                        const SamplePoly* __restrict__ poly,
                                                        const Octagon* __restrict__ oct,
                                                        RefineState* __restrict__ rs) {
  constexpr uint32_t B = kRefineBins, E = B / kBlock;
  static_assert(B % kBlock == 0, "whole bins per thread");
  __shared__ uint64_t s_bin[B];
  __shared__ int32_t s_da[B], s_db[B];
  __shared__ uint32_t s_last;
  const uint32_t m = *count_in;
  int32_t cx = poly->cx, cy = poly->cy;
  if (poly->nv < 3) {
    int64_t sx = 0, sy = 0;
    for (int v = 0; v < 8; ++v) { sx += oct->vx[v]; sy += oct->vy[v]; }
    cx = (int32_t)(sx / 8);
    cy = (int32_t)(sy / 8);
  }
  // Bin k: pseudo-angles [4k, 4k + 4) / B; its middle direction as an
  // integer vector with |a| + |b| = 1024 (dot products below 2^30).
  for (uint32_t k = threadIdx.x; k < B; k += kBlock) {
    const float pa = ((float)k + 0.5f) * (4.0f / (float)B);
    const uint32_t q = (uint32_t)pa;
    const int32_t f = (int32_t)__builtin_rintf((pa - (float)q) * 1024.0f);
    const int32_t u = 1024 - f, v = f;
    s_da[k] = q == 0 ? u : (q == 1 ? -v : (q == 2 ? -u : v));
    s_db[k] = q == 0 ? v : (q == 1 ? u : (q == 2 ? -v : -u));
    s_bin[k] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rs->cnt = 0;
  __syncthreads();
  constexpr int kR = 16;  // records per thread and step, loaded together
  const uint32_t stride = gridDim.x * kBlock * kR;
  for (uint32_t i0 = blockIdx.x * kBlock * kR + threadIdx.x; i0 < m; i0 += stride) {
    Rec r[kR];
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * kBlock;
      r[j] = in[i < m ? i : m - 1];
    }
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * kBlock;
      const float dx = (float)(r[j].x - cx), dy = (float)(r[j].y - cy);
      if (i >= m || (dx == 0.f && dy == 0.f)) continue;
      const uint32_t k = min((uint32_t)(pangle32(dx, dy) * (float)(B / 4)), B - 1);
      const int32_t dot = __mul24(s_da[k], r[j].x) + __mul24(s_db[k], r[j].y) + (1 << 30);
      atomicMax(&s_bin[k], ((uint64_t)(uint32_t)dot << 32) | i);
    }
  }
  __syncthreads();
  // Only bins that beat the value seen now go to the atomic (the launcher
  // keeps the grid small: every workgroup folds up to kRefineBins bins).
  for (uint32_t k = threadIdx.x; k < B; k += kBlock) {
    const uint64_t v = s_bin[k];
    if (v && v > __hip_atomic_load(&rs->bin[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax((unsigned long long*)&rs->bin[k], (unsigned long long)v);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(&rs->arrive, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // Thread t takes bins tE .. tE + E - 1 (bin order kept by the scan).
  uint64_t key[E];
  uint32_t nk = 0;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t k = threadIdx.x * E + e;
    key[e] = __hip_atomic_load(&rs->bin[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    nk += key[e] ? 1u : 0u;
    rs->bin[k] = 0ull;
  }
  if (threadIdx.x == 0) rs->arrive = 0;
  uint32_t mp;
  uint32_t pos = block_excl_scan(nk, mp);  // its barriers: every thread is done with s_da / s_db
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    if (key[e]) {
      const Rec r = in[(uint32_t)key[e]];
      s_da[pos] = r.x;
      s_db[pos] = r.y;
      ++pos;
    }
  }
  __syncthreads();
  build_poly<kRefineLut, 16, kRefineBins>(s_da, s_db, mp, &rs->poly, rs->lut);
}

// The records not strictly inside the second polygon (all of them when it
// failed its checks), in any order, with one reservation per wave and step;
// their count in rs->cnt.
__global__ __launch_bounds__(kBlock) void k_refine_filter(const Rec* __restrict__ in,
                                                          const uint32_t* __restrict__ count_in,
                                                          RefineState* __restrict__ rs,
                                                          Rec* __restrict__ out) {
  __shared__ int32_t s_vx[kRefineBins], s_vy[kRefineBins];
  __shared__ uint32_t s_lut[kRefineLut];
  const uint32_t m = *count_in;
  const uint32_t nv = min(rs->poly.nv, kRefineBins);
  const int32_t cx = rs->poly.cx, cy = rs->poly.cy;
  if (nv >= 3) {
    for (uint32_t i = threadIdx.x; i < nv; i += kBlock) { s_vx[i] = rs->poly.vx[i]; s_vy[i] = rs->poly.vy[i]; }
    for (uint32_t i = threadIdx.x; i < kRefineLut; i += kBlock) s_lut[i] = rs->lut[i];
  }
  __syncthreads();
  __shared__ uint32_t s_w[kWaves], s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  constexpr int kR = 8;  // records per lane and step, loaded together
  // Workgroup b takes the contiguous records [b m / G, (b + 1) m / G) in
  // steps of kBlock kR, with one reservation per step.
  const uint32_t r0 = (uint32_t)((uint64_t)blockIdx.x * m / gridDim.x);
  const uint32_t r1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * m / gridDim.x);
  for (uint32_t s0 = r0; s0 < r1; s0 += kBlock * kR) {
    const uint32_t i0 = s0 + w * 64 * kR;
    Rec r[kR];
    uint64_t bk[kR];
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * 64 + lane;
      r[j] = i < r1 ? in[i] : Rec{};
    }
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * 64 + lane;
      const bool keep = i < r1 && !(nv >= 3 && poly_lut_inside<kRefineLut>(s_vx, s_vy, nv, s_lut, cx, cy,
                                                                           r[j].x, r[j].y));
      bk[j] = __ballot(keep);
      tot += popc64(bk[j]);
    }
    if (lane == 0) s_w[w] = tot;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      before += q < w ? s_w[q] : 0u;
      all += s_w[q];
    }
    if (threadIdx.x == 0 && all) s_base = atomicAdd(&rs->cnt, all);
    __syncthreads();
    uint32_t p = s_base + before;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      if ((bk[j] >> lane) & 1ull) out[p + popc64(bk[j] & lt)] = r[j];
      p += popc64(bk[j]);
    }
    __syncthreads();  // s_w and s_base are rewritten next step
  }
}

hipError_t launch_refine(const Rec* in, const uint32_t* count_in, uint32_t max_in,
                         const SamplePoly* poly, const Octagon* oct, RefineState* rs, Rec* out,
                         uint32_t max_blocks, hipStream_t st, LaunchHook* hk) {
  // Bins: a workgroup per 4096 records (one step each), at most 128 (each
  // folds its bins into the shared ones with atomics, so not many); the
  // test: a workgroup per 2048 records, at most max_blocks.
  uint32_t gb = (max_in + 4095) / 4096;
  gb = gb < 1 ? 1 : (gb > 128 ? 128 : gb);
  uint32_t g = (max_in + 2047) / 2048;
  g = g < 1 ? 1 : (g > max_blocks ? max_blocks : g);
  hooked(hk, "refine_bins", [&] {
    hipLaunchKernelGGL(k_refine_bins, dim3(gb), dim3(kBlock), 0, st, in, count_in, poly, oct, rs);
  });
  hooked(hk, "refine_filter", [&] {
    hipLaunchKernelGGL(k_refine_filter, dim3(g), dim3(kBlock), 0, st, in, count_in, rs, out);
  });
  return hipGetLastError();
}

hipError_t launch_sample_poly(const float* xy, uint32_t n, void* scratch, SamplePoly* poly,
                              uint32_t* count0, RefineState* rs, hipStream_t st) {
  SampleDirs* sd = static_cast<SampleDirs*>(scratch);
  hipLaunchKernelGGL(k_sample_dirs, dim3(kSampleBlocks), dim3(kBlock), 0, st, xy, n, sd, count0, rs);
  hipLaunchKernelGGL(k_sample_reduce, dim3(kSampleReduceBlocks), dim3(kBlock), 0, st, xy, n, sd, poly);
  return hipGetLastError();
}

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, BatchHdr* bh,
                               const uint32_t* slist, SamplePoly* polys, uint32_t sample_min,
                               uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_sample, dim3(grid), dim3(kBlock), 0, st, xy, off, bh, slist, polys,
                     sample_min);
  return hipGetLastError();
}

}  // namespace chk
