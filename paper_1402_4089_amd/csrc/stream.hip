// Streaming-read kernel for bandwidth measurement (the reference the benchmark's roofline
// quotes beside the HBM spec): every byte of a buffer is read once per pass with 16-byte
// loads, four in flight per thread, and nothing but a never-taken conditional store is
// written.
#include "internal.h"

namespace hmcx {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_read(const u32x4* __restrict__ x, int64_t n16,
                                                   unsigned* __restrict__ sink) {
  unsigned acc = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const u32x4 a = x[i], b = x[i + stride], c = x[i + 2 * stride], d = x[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const u32x4 a = x[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9E3779B9u && sink) sink[blockIdx.x] = acc;
}

}  // namespace

hipError_t launch_stream_read(const void* buf, int64_t bytes, int reps, unsigned* sink, hipStream_t s) {
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(stream_read, dim3(2048), dim3(256), 0, s, static_cast<const u32x4*>(buf),
                       bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace hmcx
