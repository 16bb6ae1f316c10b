// Refined filter: the kernels that build the sample polygons (one set before
// its fused pass; one workgroup per set in batch mode).
#include "ch_refine.hpp"

namespace chk {

// Batch (before the single read): one workgroup per set of at least
// sample_min (and kBatchSample) points, sets taken with a fixed stride:
// chunks of kBatchSample sample points (one chunk per kBatchChunkPoints
// points of the set, at most kBatchChunksMax, spread evenly over it),
// kBatchDirs directions, the polygon in the set's SamplePoly. Smaller sets
// get none.
__global__ __launch_bounds__(kBlock) void k_batch_sample(const float* __restrict__ xy,
                                                         const uint64_t* __restrict__ off,
                                                         uint32_t nsets,
                                                         const BatchHdr* __restrict__ bh,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t sample_min) {
  // Thread t takes direction pair t % kPairs (a direction and its opposite)
  // over half t / kPairs of each chunk's sample; the halves are combined.
  constexpr uint32_t kPairs = kBatchDirs / 2;
  static_assert(2 * kPairs == (uint32_t)kBlock, "two threads per direction pair");
  __shared__ int2 sp[kBatchSample];
  __shared__ int32_t px[kBatchDirs], py[kBatchDirs];
  __shared__ int32_t s_e[2][kPairs];
  __shared__ int2 s_p[2][kPairs];
  const bool bad_off = bh->bad_offsets != 0;
  const uint32_t pr = threadIdx.x % kPairs, half = threadIdx.x / kPairs;
  int32_t a0, b0;
  direction(pr, kBatchDirs, a0, b0);
  for (uint32_t s = blockIdx.x; s < nsets; s += gridDim.x) {
    const uint64_t base = off[s];
    const uint64_t n = bad_off ? 0 : off[s + 1] - base;
    if (n < sample_min || n < kBatchSample) {
      if (threadIdx.x == 0) polys[s].nv = 0;
      continue;
    }
    const uint32_t nch = (uint32_t)min<uint64_t>(max<uint64_t>(n / kBatchChunkPoints, 1), kBatchChunksMax);
    const uint64_t ns = uint64_t(nch) * kBatchSample;
    // running extremes of this thread's direction pair over the chunks
    // (kept by the threads of half 0)
    int32_t bmax = INT32_MIN, bmin = INT32_MAX;
    int2 pmax = make_int2(0, 0), pmin = make_int2(0, 0);
    for (uint32_t c = 0; c < nch; ++c) {
      __syncthreads();  // the previous chunk or set is done with the shared arrays
      for (uint32_t q = threadIdx.x; q < kBatchSample; q += kBlock)
        sp[q] = grid_point(xy, base + ((uint64_t(c) * kBatchSample + q) * n) / ns);
      __syncthreads();
      const uint32_t m = kBatchSample;
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
        // the first half wins ties (the first occurrence in the chunk), and
        // earlier chunks win ties over later ones
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
                                                        uint32_t* __restrict__ count0) {
  static_assert(kPolyMax == 2 * kBlock, "a direction and its opposite per thread");
  __shared__ int2 sp[kSamplePer];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sd->arrive = 0;  // for k_sample_reduce
    sd->cand = 0;    // for the fused pass
    *count0 = 0;     // survivors of the candidates' octagon test, two launches on
  }
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

hipError_t launch_sample_poly(const float* xy, uint32_t n, void* scratch, SamplePoly* poly,
                              uint32_t* count0, hipStream_t st) {
  SampleDirs* sd = static_cast<SampleDirs*>(scratch);
  hipLaunchKernelGGL(k_sample_dirs, dim3(kSampleBlocks), dim3(kBlock), 0, st, xy, n, sd, count0);
  hipLaunchKernelGGL(k_sample_reduce, dim3(kSampleReduceBlocks), dim3(kBlock), 0, st, xy, n, sd, poly);
  return hipGetLastError();
}

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, uint32_t nsets,
                               const BatchHdr* bh, SamplePoly* polys, uint32_t sample_min,
                               uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_sample, dim3(grid), dim3(kBlock), 0, st, xy, off, nsets, bh, polys,
                     sample_min);
  return hipGetLastError();
}

}  // namespace chk
