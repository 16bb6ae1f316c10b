// Refined filter, batch side: one workgroup per set builds the set's sample
// polygon (the single-set side runs inside the octagon build, ch_filter.hip).
#include "ch_refine.hpp"

namespace chk {

// Batch: one workgroup per set of at least sample_min (and kBatchSample)
// points, sets taken with a fixed stride: kBatchSample sample points,
// kBatchDirs directions, the polygon in the set's SamplePoly. Smaller sets
// get none.
__global__ __launch_bounds__(kBlock) void k_batch_sample(const float* __restrict__ xy,
                                                         const uint64_t* __restrict__ off,
                                                         uint32_t nsets,
                                                         const BatchHdr* __restrict__ bh,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t sample_min) {
  static_assert(kBatchDirs == 2 * (uint32_t)kBlock, "two directions per thread");
  __shared__ int2 sp[kBatchSample];
  __shared__ int32_t px[kBatchDirs], py[kBatchDirs];
  const bool bad_off = bh->bad_offsets != 0;
  int32_t a0, b0, a1, b1;
  direction(threadIdx.x, kBatchDirs, a0, b0);
  direction(threadIdx.x + kBlock, kBatchDirs, a1, b1);
  for (uint32_t s = blockIdx.x; s < nsets; s += gridDim.x) {
    const uint64_t base = off[s];
    const uint64_t n = bad_off ? 0 : off[s + 1] - base;
    if (n < sample_min || n < kBatchSample) {
      if (threadIdx.x == 0) polys[s].nv = 0;
      continue;
    }
    __syncthreads();  // the previous set is done with the shared arrays
    for (uint32_t q = threadIdx.x; q < kBatchSample; q += kBlock)
      sp[q] = grid_point(xy, base + (q * n) / kBatchSample);
    __syncthreads();
    int32_t e0, e1;
    uint32_t q0, q1;
    dir_max2(sp, kBatchSample, a0, b0, a1, b1, e0, q0, e1, q1);
    px[threadIdx.x] = sp[q0].x;
    py[threadIdx.x] = sp[q0].y;
    px[threadIdx.x + kBlock] = sp[q1].x;
    py[threadIdx.x + kBlock] = sp[q1].y;
    __syncthreads();
    build_poly(px, py, kBatchDirs, &polys[s]);
  }
}

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, uint32_t nsets,
                               const BatchHdr* bh, SamplePoly* polys, uint32_t sample_min,
                               uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_sample, dim3(grid), dim3(kBlock), 0, st, xy, off, nsets, bh, polys,
                     sample_min);
  return hipGetLastError();
}

}  // namespace chk
