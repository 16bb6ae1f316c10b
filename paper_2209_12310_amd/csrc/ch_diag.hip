// Diagnostics beside the method: a plain read stream that measures the read
// bandwidth this device reaches, the reference the fused pass's roofline
// fraction is read against (8 TB/s is the vendor peak, not a reachable rate).
#include "ch_internal.hpp"

namespace chk {

// Every thread reads kRows 16-byte words per step, kStride = the grid's
// thread count apart (each step of the grid covers kRows contiguous
// stretches), non-temporal, and folds them into one value so that no load
// is dead code; the value is written only in a case that never happens for
// finite data (the sum of a NaN-free buffer compared with a NaN).
template <int kRows>
__global__ __launch_bounds__(kBlock) void k_read_stream(const float4* __restrict__ p, size_t n16,
                                                        float* __restrict__ sink) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const size_t stride = (size_t)gridDim.x * kBlock;
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  float acc = 0.f;
  for (; i + (kRows - 1) * stride < n16; i += kRows * stride) {
    f4v v[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u)
      v[u] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p + i + u * stride));
#pragma unroll
    for (int u = 0; u < kRows; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n16; i += stride) {
    const float4 v = p[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc != acc && sink) sink[0] = acc;
}

hipError_t launch_read_stream(const void* d_buf, size_t bytes, uint32_t blocks, float* sink,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_read_stream<4>, dim3(blocks), dim3(kBlock), 0, st,
                     static_cast<const float4*>(d_buf), bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace chk
