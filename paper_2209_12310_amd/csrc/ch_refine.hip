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
// directions, the polygon in the set's SamplePoly with its wedge table of
// kBatchLutBins bins in luts (the plan clears the polygon of the other
// sets). The direction
// scans run over a chunk's points left by octagon_sieve. A chunk's points
// are runs of kSampleRun consecutive input points (one 128-byte line each)
// with the runs spread evenly over the set: a sample point per line fetched,
// where single points at a large stride would fetch a line each.
__global__ __launch_bounds__(kBlock) void k_batch_sample(const float* __restrict__ xy,
                                                         const uint64_t* __restrict__ off,
                                                         BatchHdr* __restrict__ bh,
                                                         const uint32_t* __restrict__ slist,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t* __restrict__ luts,
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
    build_poly<kBatchLutBins>(px, py, kBatchDirs, &polys[s], luts + size_t(s) * kBatchLutBins);
  }
}

static_assert(sizeof(SampleDirs) <= size_t(kPolyMax) * 8 + 256 + size_t(kLutBins) * 4 +
                                         size_t(kSampleBlocks) * kPolyMax * 16,
              "workspace slot of the direction maxima");

__global__ __launch_bounds__(kBlock) void k_sample_dirs(const float* __restrict__ xy, uint32_t n,
                                                        SampleDirs* __restrict__ sd,
                                                        uint32_t* __restrict__ count0) {
  static_assert(kPolyMax == 2 * kBlock, "a direction and its opposite per thread");
  __shared__ int2 sp[kSamplePer];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sd->arrive = 0;  // for k_sample_reduce
    sd->cand = 0;    // for the fused pass
    *count0 = 0;     // survivors of the candidates' octagon test, two launches on
  }
  constexpr uint32_t kRunsAll = kSampleN / kSampleRun, kRunsPer = kSamplePer / kSampleRun;
  for (uint32_t q = threadIdx.x; q < kSamplePer; q += kBlock) {
    const uint64_t r = uint64_t(blockIdx.x) * kRunsPer + q / kSampleRun;
    sp[q] = grid_point(xy, (size_t)min<uint64_t>((r * n) / kRunsAll + q % kSampleRun, n - 1));
  }
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

hipError_t launch_sample_poly(const float* xy, uint32_t n, void* scratch, SamplePoly* poly,
                              uint32_t* count0, hipStream_t st) {
  SampleDirs* sd = static_cast<SampleDirs*>(scratch);
  hipLaunchKernelGGL(k_sample_dirs, dim3(kSampleBlocks), dim3(kBlock), 0, st, xy, n, sd, count0);
  hipLaunchKernelGGL(k_sample_reduce, dim3(kSampleReduceBlocks), dim3(kBlock), 0, st, xy, n, sd, poly);
  return hipGetLastError();
}

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, BatchHdr* bh,
                               const uint32_t* slist, SamplePoly* polys, uint32_t* luts,
                               uint32_t sample_min, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_sample, dim3(grid), dim3(kBlock), 0, st, xy, off, bh, slist, polys,
                     luts, sample_min);
  return hipGetLastError();
}

}  // namespace chk
