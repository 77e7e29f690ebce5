// Streaming-read probe: the device's achievable HBM read bandwidth, the practical ceiling for
// the HBM-bound kernels (the one-query answer reads its database exactly once).  Each workgroup
// streams its own contiguous chunk of the buffer with nontemporal 16-byte loads, eight
// independent loads in flight per thread; a workgroup's loads of one pass cover 4 KiB.  On
// MI355X this reads faster than a grid-stride loop over the whole buffer (about 7.0 TB/s
// against 6.3 TB/s for 1 GiB).
#include "internal.h"
#include "zippir.h"

namespace zp {

__global__ __launch_bounds__(256) void read_probe_kernel(const u32x4* __restrict__ p, size_t n16,
                                                         uint32_t* __restrict__ sink) {
  constexpr int kU = 8;
  const size_t chunk = (n16 + gridDim.x - 1) / gridDim.x;
  const size_t begin = blockIdx.x * chunk;
  const size_t end = min(n16, begin + chunk);
  uint32_t acc = 0;
  for (size_t i = begin + threadIdx.x; i < end; i += 256 * kU) {
    u32x4 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const size_t j = i + (size_t)u * 256;
      v[u] = j < end ? __builtin_nontemporal_load(p + j) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  // one word per block keeps the loads alive
  __shared__ uint32_t red[4];
  for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace zp

extern "C" pir_status pir_read_probe(const void* buf, uint64_t bytes, uint32_t* sink, uint32_t blocks,
                                     void* hip_stream) {
  if (!buf || !sink || blocks == 0 || bytes < 16) return PIR_EINVAL;
  if (((uintptr_t)buf & 15) != 0) return PIR_EINVAL;
  zp::read_probe_kernel<<<blocks, 256, 0, (hipStream_t)hip_stream>>>(
      reinterpret_cast<const zp::u32x4*>(buf), bytes / 16, sink);
  return hipGetLastError() == hipSuccess ? PIR_OK : PIR_EDEVICE;
}
