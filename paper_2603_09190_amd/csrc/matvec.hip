// Online answer for one query: b = D . qu mod 2^32 (Alg. 5, Response, first line).
//
// HBM-bound: every byte of D is read once.  The u8 x u32 product is split into the four
// bytes of the query, each handled by v_dot4_u32_u8 (four u8 x u8 products accumulated
// into a wrapping u32), so one full-rate instruction covers one byte of D:
//   D.qu = sum_b 2^(8b) * (D . qu_b)  mod 2^32,  qu_b = byte b of qu.
// Each plane sum may wrap mod 2^32; the shifted recombination is still exact mod 2^32.
#include <algorithm>

#include "internal.h"
#include "wavenum.h"

namespace zp {

// Packs the query's byte planes and clears the answer vector (the matvec adds into it).
__global__ __launch_bounds__(256) void pack_planes_u8_kernel(const uint32_t* __restrict__ q,
                                                             int cols, int pitch,
                                                             uint8_t* __restrict__ planes,
                                                             uint32_t* __restrict__ b, int rows) {
  const int i4 = blockIdx.x * blockDim.x + threadIdx.x;  // one thread per 4 columns
  for (int r = i4; r < rows; r += gridDim.x * blockDim.x) b[r] = 0u;
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

void launch_pack_planes_u8(const uint32_t* q, int cols, int pitch, uint8_t* planes, uint32_t* b,
                           int rows, hipStream_t s) {
  const int n4 = pitch / 4;
  pack_planes_u8_kernel<<<(n4 + 255) / 256, 256, 0, s>>>(q, cols, pitch, planes, b, rows);
}

// A wave owns 4096 columns of the query (64 per lane, as four
// 1 KiB-coalesced 16-byte pieces) held in registers as byte planes, and streams down
// `rows_per_wave` rows.  Per row the wave reduces its partial dot product and adds it into
// b with a 32-bit atomic add, which is exact modulo 2^32 and independent of order.
// b must be zero before the launch.
constexpr int kSegCols = 4096;

template <int kR>
__global__ __launch_bounds__(256) void matvec_seg_kernel(const uint8_t* __restrict__ D, int rows,
                                                         int pitch,
                                                         const uint8_t* __restrict__ planes,
                                                         uint32_t* __restrict__ out,
                                                         int rows_per_wave) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg0 = blockIdx.y * kSegCols;
  const int row_begin = (blockIdx.x * 4 + wave) * rows_per_wave;
  if (row_begin >= rows) return;
  const int row_end = min(rows, row_begin + rows_per_wave);
  bool valid[4];
  int off[4];
  u32x4 q[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off[k] = seg0 + 1024 * k + 16 * lane;
    valid[k] = off[k] < pitch;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      q[k][b] = valid[k] ? *reinterpret_cast<const u32x4*>(planes + (size_t)b * pitch + off[k])
                         : u32x4{0u, 0u, 0u, 0u};
  }
  for (int row = row_begin; row < row_end; row += kR) {
    u32x4 d[kR][4];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int rr = min(row + r, row_end - 1);
      const uint8_t* rp = D + (size_t)rr * pitch;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        d[r][k] = valid[k] ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rp + off[k]))
                           : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      uint32_t a[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          a[b] = __builtin_amdgcn_udot4(d[r][k].x, q[k][b].x, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].y, q[k][b].y, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].z, q[k][b].z, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].w, q[k][b].w, a[b], false);
        }
      uint32_t v = a[0] + (a[1] << 8) + (a[2] << 16) + (a[3] << 24);
      v = wave_sum64(v);
      if (lane == 0 && row + r < row_end) atomicAdd(out + row + r, v);
    }
  }
}

constexpr int kSegRowsPerWave = 32;

void launch_matvec(const uint8_t* D, int rows, int pitch, const uint8_t* planes, uint32_t* b,
                   hipStream_t s) {
  // b accumulates one atomic partial per column segment; launch_pack_planes_u8 cleared it.
  // Databases above kLaunchBytes are streamed in row chunks of at most that many bytes, so
  // work queued on other streams is dispatched between chunks instead of waiting for the
  // whole database.
  const int chunk_rows = (int)std::max<long long>(4 * kSegRowsPerWave,
                                                  (kLaunchBytes / pitch) / (4 * kSegRowsPerWave) * (4 * kSegRowsPerWave));
  for (int r0 = 0; r0 < rows; r0 += chunk_rows) {
    const int nr = std::min(chunk_rows, rows - r0);
    dim3 grid((nr + 4 * kSegRowsPerWave - 1) / (4 * kSegRowsPerWave), (pitch + kSegCols - 1) / kSegCols);
    matvec_seg_kernel<4><<<grid, 256, 0, s>>>(D + (size_t)r0 * pitch, nr, pitch, planes, b + r0,
                                              kSegRowsPerWave);
  }
}

}  // namespace zp
