// Online answer for one query: b = D . qu mod 2^32 (Alg. 5, Response, first line).
//
// HBM-bound: every byte of D is read once.  The u8 x u32 product is split into the four
// bytes of the query, each handled by v_dot4_u32_u8 (four u8 x u8 products accumulated
// into a wrapping u32), so one full-rate instruction covers one byte of D:
//   D.qu = sum_b 2^(8b) * (D . qu_b)  mod 2^32,  qu_b = byte b of qu.
// Each plane sum may wrap mod 2^32; the shifted recombination is still exact mod 2^32.
#include "internal.h"

namespace zp {

__global__ __launch_bounds__(256) void pack_planes_u8_kernel(const uint32_t* __restrict__ q,
                                                             int cols, int pitch,
                                                             uint8_t* __restrict__ planes) {
  const int i4 = blockIdx.x * blockDim.x + threadIdx.x;  // one thread per 4 columns
  if (4 * i4 >= pitch) return;
  uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = 4 * i4 + t;
    const uint32_t v = (i < cols) ? q[i] : 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) w[b] |= ((v >> (8 * b)) & 0xFFu) << (8 * t);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) reinterpret_cast<uint32_t*>(planes + (size_t)b * pitch)[i4] = w[b];
}

void launch_pack_planes_u8(const uint32_t* q, int cols, int pitch, uint8_t* planes,
                           hipStream_t s) {
  const int n4 = pitch / 4;
  pack_planes_u8_kernel<<<(n4 + 255) / 256, 256, 0, s>>>(q, cols, pitch, planes);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
  return v;
}

// Each wave owns kRows consecutive rows; lanes stride over 16-byte column chunks, so
// one iteration reads kRows x 1 KiB of D, fully coalesced, and the query planes once.
template <int kRows>
__global__ __launch_bounds__(256) void matvec_kernel(const uint8_t* __restrict__ D, int rows,
                                                     int pitch,
                                                     const uint8_t* __restrict__ planes,
                                                     uint32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * 4 + wave) * kRows;
  if (row0 >= rows) return;
  const int nchunk = pitch >> 4;
  const u32x4* __restrict__ p0 = reinterpret_cast<const u32x4*>(planes);
  const u32x4* __restrict__ p1 = reinterpret_cast<const u32x4*>(planes + (size_t)pitch);
  const u32x4* __restrict__ p2 = reinterpret_cast<const u32x4*>(planes + 2 * (size_t)pitch);
  const u32x4* __restrict__ p3 = reinterpret_cast<const u32x4*>(planes + 3 * (size_t)pitch);
  const u32x4* rowp[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int row = min(row0 + r, rows - 1);
    rowp[r] = reinterpret_cast<const u32x4*>(D + (size_t)row * pitch);
  }
  uint32_t acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[r][b] = 0;

  for (int ch = lane; ch < nchunk; ch += 64) {
    const u32x4 q0 = p0[ch], q1 = p1[ch], q2 = p2[ch], q3 = p3[ch];
    u32x4 d[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) d[r] = __builtin_nontemporal_load(rowp[r] + ch);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      acc[r][0] = __builtin_amdgcn_udot4(d[r].x, q0.x, acc[r][0], false);
      acc[r][0] = __builtin_amdgcn_udot4(d[r].y, q0.y, acc[r][0], false);
      acc[r][0] = __builtin_amdgcn_udot4(d[r].z, q0.z, acc[r][0], false);
      acc[r][0] = __builtin_amdgcn_udot4(d[r].w, q0.w, acc[r][0], false);
      acc[r][1] = __builtin_amdgcn_udot4(d[r].x, q1.x, acc[r][1], false);
      acc[r][1] = __builtin_amdgcn_udot4(d[r].y, q1.y, acc[r][1], false);
      acc[r][1] = __builtin_amdgcn_udot4(d[r].z, q1.z, acc[r][1], false);
      acc[r][1] = __builtin_amdgcn_udot4(d[r].w, q1.w, acc[r][1], false);
      acc[r][2] = __builtin_amdgcn_udot4(d[r].x, q2.x, acc[r][2], false);
      acc[r][2] = __builtin_amdgcn_udot4(d[r].y, q2.y, acc[r][2], false);
      acc[r][2] = __builtin_amdgcn_udot4(d[r].z, q2.z, acc[r][2], false);
      acc[r][2] = __builtin_amdgcn_udot4(d[r].w, q2.w, acc[r][2], false);
      acc[r][3] = __builtin_amdgcn_udot4(d[r].x, q3.x, acc[r][3], false);
      acc[r][3] = __builtin_amdgcn_udot4(d[r].y, q3.y, acc[r][3], false);
      acc[r][3] = __builtin_amdgcn_udot4(d[r].z, q3.z, acc[r][3], false);
      acc[r][3] = __builtin_amdgcn_udot4(d[r].w, q3.w, acc[r][3], false);
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    uint32_t v = acc[r][0] + (acc[r][1] << 8) + (acc[r][2] << 16) + (acc[r][3] << 24);
    v = wave_sum(v);
    if (lane == 0 && row0 + r < rows) out[row0 + r] = v;
  }
}

constexpr int kMatvecRows = 8;

void launch_matvec(const uint8_t* D, int rows, int pitch, const uint8_t* planes, uint32_t* b,
                   hipStream_t s) {
  const int per_block = 4 * kMatvecRows;
  const int blocks = (rows + per_block - 1) / per_block;
  matvec_kernel<kMatvecRows><<<blocks, 256, 0, s>>>(D, rows, pitch, planes, b);
}

}  // namespace zp
