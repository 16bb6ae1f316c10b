// Refined filter: the kernels that build the sample polygons (one set before
// its fused pass; one workgroup per set in batch mode).
#include "ch_refine.hpp"

namespace chk {

// Batch (after the per-set octagons): one workgroup per set of at least
// sample_min (and kBatchSample) points, sets taken with a fixed stride:
// kBatchSample sample points, those strictly outside the set's octagon kept,
// kBatchDirs directions, the polygon in the set's SamplePoly. Smaller sets,
// and sets whose sample lies inside the octagon, get none.
__global__ __launch_bounds__(kBlock) void k_batch_sample(const float* __restrict__ xy,
                                                         const uint64_t* __restrict__ off,
                                                         uint32_t nsets,
                                                         const BatchHdr* __restrict__ bh,
                                                         const SetState* __restrict__ sets,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t sample_min) {
  static_assert(kBatchDirs == 2 * (uint32_t)kBlock, "two directions per thread");
  constexpr uint32_t E = kBatchSample / kBlock;  // sample points per thread
  __shared__ int2 sp[kBatchSample];
  __shared__ int32_t px[kBatchDirs], py[kBatchDirs];
  const bool bad_off = bh->bad_offsets != 0;
  int32_t a0, b0, a1, b1;
  direction(threadIdx.x, kBatchDirs, a0, b0);
  direction(threadIdx.x + kBlock, kBatchDirs, a1, b1);
  for (uint32_t s = blockIdx.x; s < nsets; s += gridDim.x) {
    const uint64_t base = off[s];
    const uint64_t n = bad_off ? 0 : off[s + 1] - base;
    const Octagon* __restrict__ oct = &sets[s].oct;
    if (n < sample_min || n < kBatchSample || oct->status != 0) {
      if (threadIdx.x == 0) polys[s].nv = 0;
      continue;
    }
    // Sample points strictly outside the set's octagon, compacted.
    int2 v[E];
    uint32_t outm = 0, nout = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t q = threadIdx.x * E + e;
      v[e] = grid_point(xy, base + (q * n) / kBatchSample);
      const double x = (double)v[e].x * 0x1p-20, y = (double)v[e].y * 0x1p-20;
      double mn = __builtin_inf();
#pragma unroll
      for (int i = 0; i < 8; ++i)
        mn = __builtin_fmin(mn, __builtin_fma(oct->A[i], x, __builtin_fma(oct->B[i], y, oct->C[i])));
      if (mn < 0.0) { outm |= 1u << e; ++nout; }
    }
    __syncthreads();  // the previous set is done with the shared arrays
    uint32_t m;
    uint32_t pos = block_excl_scan(nout, m);
#pragma unroll
    for (uint32_t e = 0; e < E; ++e)
      if (outm & (1u << e)) sp[pos++] = v[e];
    __syncthreads();
    if (m == 0) {
      if (threadIdx.x == 0) polys[s].nv = 0;
      continue;
    }
    int32_t e0, e1;
    uint32_t q0, q1;
    dir_max2(sp, m, a0, b0, a1, b1, e0, q0, e1, q1);
    px[threadIdx.x] = sp[q0].x;
    py[threadIdx.x] = sp[q0].y;
    px[threadIdx.x + kBlock] = sp[q1].x;
    py[threadIdx.x + kBlock] = sp[q1].y;
    __syncthreads();
    build_poly(px, py, kBatchDirs, &polys[s]);
  }
}

// Single set, before the fused pass: clear the maxima, then kSampleBlocks
// workgroups of sample_dirs_block over all sample points.
__global__ __launch_bounds__(kBlock) void k_sample_zero(SampleDirs* __restrict__ sd) {
  sample_dirs_clear(sd);
}

__global__ __launch_bounds__(kBlock) void k_sample_dirs(const float* __restrict__ xy, uint32_t n,
                                                        SampleDirs* __restrict__ sd,
                                                        SamplePoly* __restrict__ poly) {
  sample_dirs_block(xy, n, nullptr, sd, poly, blockIdx.x, gridDim.x);
}

hipError_t launch_sample_poly(const float* xy, uint32_t n, void* scratch, SamplePoly* poly,
                              hipStream_t st) {
  SampleDirs* sd = static_cast<SampleDirs*>(scratch);
  hipLaunchKernelGGL(k_sample_zero, dim3(1), dim3(kBlock), 0, st, sd);
  hipLaunchKernelGGL(k_sample_dirs, dim3(kSampleBlocks), dim3(kBlock), 0, st, xy, n, sd, poly);
  return hipGetLastError();
}

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, uint32_t nsets,
                               const BatchHdr* bh, const SetState* sets, SamplePoly* polys,
                               uint32_t sample_min, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_sample, dim3(grid), dim3(kBlock), 0, st, xy, off, nsets, bh, sets,
                     polys, sample_min);
  return hipGetLastError();
}

}  // namespace chk
