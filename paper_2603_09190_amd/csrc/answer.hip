// The online step for one query and one client in two launches: the answer
// b = D . qu mod 2^32 (Alg. 5, Response, first line) and the combined response
// c_j = K_j (1 + b_j N) mod N^2 (Sec. 4.3, "Smaller responses w/ Paillier addition").
//
// Launch 1 is the matvec of matvec.hip with two changes: each wave builds its query byte
// planes from the raw uint32 query itself (no packing launch), and each (row, column segment)
// partial sum is stored to its own slot instead of being added into b (so b needs no clearing).
// Launch 2 sums a row's segment partials (mod 2^32), stores b_j, and combines it into c_j with
// the single Montgomery step of compress.hip.  Both launches together read D once and move
// 3 x 512 B per row for K', M' and c, against three launches (pack, matvec, combine) before.
#include <algorithm>

#include "internal.h"
#include "wavenum.h"

namespace zp {

constexpr int kPartSegCols = 4096;   // columns per segment: 64 per lane, 4 x 16-byte pieces
constexpr int kPartRowsPerWave = 32;

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
  return v;
}

// The 16 query entries from column c0 as four byte planes: word t of plane b holds byte b of
// entries c0 + 4t .. c0 + 4t + 3.  Entries at or beyond cols are zero.
__device__ __forceinline__ void query_planes16(const uint32_t* __restrict__ q, int cols, int c0,
                                               u32x4 (&pl)[4]) {
  uint32_t v[16];
  if (c0 + 16 <= cols) {  // q is 16-byte aligned and c0 a multiple of 16: four 16-byte loads
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const u32x4 x = *reinterpret_cast<const u32x4*>(q + c0 + 4 * t);
      v[4 * t] = x.x; v[4 * t + 1] = x.y; v[4 * t + 2] = x.z; v[4 * t + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = (c0 + i < cols) ? q[c0 + i] : 0u;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint32_t x = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) x |= ((v[4 * t + u] >> (8 * b)) & 0xFFu) << (8 * u);
      w[t] = x;
    }
    pl[b] = u32x4{w[0], w[1], w[2], w[3]};
  }
}

// grid (row groups of 4 x kPartRowsPerWave rows, column segments); part[j * nseg + s]
// receives row j's dot product over segment s (mod 2^32), so a row's partials are contiguous.
template <int kR>
__global__ __launch_bounds__(256) void matvec_part_kernel(const uint8_t* __restrict__ D, int rows,
                                                          int pitch, const uint32_t* __restrict__ q,
                                                          int cols, uint32_t* __restrict__ part,
                                                          int nseg) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = blockIdx.y;
  const int seg0 = seg * kPartSegCols;
  const int row_begin = (blockIdx.x * 4 + wave) * kPartRowsPerWave;
  if (row_begin >= rows) return;
  const int row_end = min(rows, row_begin + kPartRowsPerWave);
  bool valid[4];
  int off[4];
  u32x4 qp[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off[k] = seg0 + 1024 * k + 16 * lane;
    valid[k] = off[k] < pitch;
    query_planes16(q, cols, off[k], qp[k]);
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
          a[b] = __builtin_amdgcn_udot4(d[r][k].x, qp[k][b].x, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].y, qp[k][b].y, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].z, qp[k][b].z, a[b], false);
          a[b] = __builtin_amdgcn_udot4(d[r][k].w, qp[k][b].w, a[b], false);
        }
      const uint32_t v = wave_sum_u32(a[0] + (a[1] << 8) + (a[2] << 16) + (a[3] << 24));
      if (lane == 0 && row + r < row_end) part[(size_t)(row + r) * nseg + seg] = v;
    }
  }
}

// b_j = sum_s part[j * nseg + s] mod 2^32, then c_j = (K'_j + b_j M'_j + q N^2) / 2^32 reduced
// once (the combine of compress.hip).  Each wave takes kCombineRows consecutive rows and loads
// the next row's K', M' and partials while it reduces the current one.
constexpr int kCombineRows = 8;

template <int P>
__global__ __launch_bounds__(256) void combine_parts_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                            const uint32_t* __restrict__ Mp,
                                                            const uint32_t* __restrict__ part, int nseg,
                                                            int rows, uint32_t* __restrict__ b,
                                                            uint32_t* __restrict__ C) {
  const int wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = wave * kCombineRows;
  if (row0 >= rows) return;
  const int row1 = min(rows, row0 + kCombineRows);
  const int lane = lane_id();
  auto partial = [&](int row) {
    return lane < nseg ? part[(size_t)row * nseg + lane] : 0u;
  };
  WNum<P> M2, t, m, tn, mn;
  wn_load(M2, cd.N2);
  wn_load_n(t, Kp + (size_t)row0 * cd.L, cd.L);
  wn_load_n(m, Mp + (size_t)row0 * cd.L, cd.L);
  uint32_t pj = partial(row0), pn = 0;
  for (int row = row0; row < row1; ++row) {
    if (row + 1 < row1) {
      wn_load_n(tn, Kp + (size_t)(row + 1) * cd.L, cd.L);
      wn_load_n(mn, Mp + (size_t)(row + 1) * cd.L, cd.L);
      pn = partial(row + 1);
    }
    uint32_t sum = pj;  // lanes at or beyond nseg hold 0: log2(nseg) exchanges leave the total in lane 0
    for (int off = 1; off < nseg; off <<= 1) sum += (uint32_t)__shfl_xor((int)sum, off, 64);
    const uint32_t bj = __builtin_amdgcn_readfirstlane(sum);
    if (lane == 0) b[row] = bj;
    uint64_t c = 0;
    mont_step(t, c, bj, m, M2, cd.m2prime);
    const uint64_t ovf = wn_resolve(t, c);
    wn_cond_sub(t, ovf, M2);
    wn_store_n(C + (size_t)row * cd.L, t, cd.L);
    t = tn;
    m = mn;
    pj = pn;
  }
}

int answer_segments(int pitch) { return (pitch + kPartSegCols - 1) / kPartSegCols; }

void launch_matvec_part(const uint8_t* D, int rows, int pitch, const uint32_t* q, int cols,
                        uint32_t* part, hipStream_t s) {
  if (rows <= 0) return;
  const int nseg = answer_segments(pitch);
  // row chunks of at most kLaunchBytes of D per launch (as launch_matvec)
  const int group = 4 * kPartRowsPerWave;
  const int chunk_rows = (int)std::max<long long>(group, (kLaunchBytes / pitch) / group * group);
  for (int r0 = 0; r0 < rows; r0 += chunk_rows) {
    const int nr = std::min(chunk_rows, rows - r0);
    dim3 grid((nr + group - 1) / group, nseg);
    matvec_part_kernel<2><<<grid, 256, 0, s>>>(D + (size_t)r0 * pitch, nr, pitch, q, cols,
                                               part + (size_t)r0 * nseg, nseg);
  }
}

void launch_combine_parts(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Mp,
                          const uint32_t* part, int nseg, int rows, uint32_t* b, uint32_t* C,
                          hipStream_t s) {
  if (rows <= 0) return;
  const int waves = (rows + kCombineRows - 1) / kCombineRows;
  const int blocks = (waves + 3) / 4;
  switch (cd.P) {
    case 1: combine_parts_kernel<1><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 2: combine_parts_kernel<2><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 3: combine_parts_kernel<3><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 4: combine_parts_kernel<4><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
  }
}

}  // namespace zp
