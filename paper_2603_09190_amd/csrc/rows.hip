// Row gather/scatter used by database updates and by partial recomputation of H.
#include "internal.h"

namespace zp {

__global__ __launch_bounds__(256) void gather_rows_u8_kernel(const uint8_t* __restrict__ src,
                                                             int pitch,
                                                             const uint32_t* __restrict__ rows,
                                                             uint8_t* __restrict__ dst) {
  const int i = blockIdx.y;
  const u32x4* s = reinterpret_cast<const u32x4*>(src + (size_t)rows[i] * pitch);
  u32x4* d = reinterpret_cast<u32x4*>(dst + (size_t)i * pitch);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < pitch / 16; c += gridDim.x * blockDim.x)
    d[c] = s[c];
}

void launch_gather_rows_u8(const uint8_t* src, int pitch, const uint32_t* rows, int nrows,
                           uint8_t* dst, hipStream_t s) {
  if (nrows <= 0) return;
  dim3 grid(min(64, (pitch / 16 + 255) / 256), nrows);
  gather_rows_u8_kernel<<<grid, 256, 0, s>>>(src, pitch, rows, dst);
}

// dst row rows[i] (pitch dst_pitch, bytes beyond cols left zero) <- src row i (pitch src_pitch)
__global__ __launch_bounds__(256) void scatter_rows_u8_kernel(const uint8_t* __restrict__ src,
                                                              int src_pitch, int cols,
                                                              const uint32_t* __restrict__ rows,
                                                              uint8_t* __restrict__ dst,
                                                              int dst_pitch) {
  const int i = blockIdx.y;
  const uint8_t* s = src + (size_t)i * src_pitch;
  uint8_t* d = dst + (size_t)rows[i] * dst_pitch;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < dst_pitch; c += gridDim.x * blockDim.x)
    d[c] = c < cols ? s[c] : (uint8_t)0;
}

void launch_scatter_rows_u8(const uint8_t* src, int src_pitch, int cols, const uint32_t* rows,
                            int nrows, uint8_t* dst, int dst_pitch, hipStream_t s) {
  if (nrows <= 0) return;
  dim3 grid(min(64, (dst_pitch + 255) / 256), nrows);
  scatter_rows_u8_kernel<<<grid, 256, 0, s>>>(src, src_pitch, cols, rows, dst, dst_pitch);
}

__global__ void gather_rowsum_kernel(const int32_t* __restrict__ src,
                                     const uint32_t* __restrict__ rows, int nrows,
                                     int32_t* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nrows) dst[i] = src[rows[i]];
}

void launch_gather_rowsum(const int32_t* src, const uint32_t* rows, int nrows, int32_t* dst,
                          hipStream_t s) {
  if (nrows <= 0) return;
  gather_rowsum_kernel<<<(nrows + 255) / 256, 256, 0, s>>>(src, rows, nrows, dst);
}

__global__ __launch_bounds__(256) void scatter_rows_u32_kernel(const uint32_t* __restrict__ src,
                                                               int width,
                                                               const uint32_t* __restrict__ rows,
                                                               uint32_t* __restrict__ dst) {
  const int i = blockIdx.y;
  const uint32_t* s = src + (size_t)i * width;
  uint32_t* d = dst + (size_t)rows[i] * width;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < width; c += gridDim.x * blockDim.x)
    d[c] = s[c];
}

void launch_scatter_rows_u32(const uint32_t* src, int width, const uint32_t* rows, int nrows,
                             uint32_t* dst, hipStream_t s) {
  if (nrows <= 0) return;
  dim3 grid(min(64, (width + 255) / 256), nrows);
  scatter_rows_u32_kernel<<<grid, 256, 0, s>>>(src, width, rows, dst);
}

}  // namespace zp
