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
#include "rownum.h"
#include "wavenum.h"

namespace zp {

constexpr int kPartSegCols = 4096;   // columns per segment: 64 per lane, 4 x 16-byte pieces
constexpr int kPartRowsPerWave = 32;

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
      const uint32_t v = wave_sum64(a[0] + (a[1] << 8) + (a[2] << 16) + (a[3] << 24));
      if (lane == 0 && row + r < row_end) part[(size_t)(row + r) * nseg + seg] = v;
    }
  }
}

// b_j = sum_s part[j * nseg + s] mod 2^32, then c_j = (K'_j + b_j M'_j + q N^2) / 2^32 reduced
// once (the combine of compress.hip).  Each wave takes kCombineRows consecutive rows and requests
// every row's K', M' and partials before it reduces the first one, so one memory latency covers
// all of them (a short last wave re-reads its last row instead of branching around loads).
constexpr int kCombineRows = 8;

// The limbs of a row for a later wn_zero_above: every lane loads, at indices clamped to the row,
// so no branch separates the loads of consecutive rows (a branch would make the wave wait for
// each row's loads before requesting the next).
template <int P>
__device__ __forceinline__ void wn_load_clamped(WNum<P>& x, const uint32_t* __restrict__ src, int nl) {
  const int base = P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = src[min(base + j, nl - 1)];
}

template <int P>
__device__ __forceinline__ void wn_zero_above(WNum<P>& x, int nl) {
  const int base = P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = base + j < nl ? x.v[j] : 0u;
}

template <int P>
__global__ __launch_bounds__(256) void combine_parts_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                            const uint32_t* __restrict__ Mp,
                                                            const uint32_t* __restrict__ part, int nseg,
                                                            int rows, uint32_t* __restrict__ b,
                                                            uint32_t* __restrict__ C) {
  const int wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = wave * kCombineRows;
  if (row0 >= rows) return;
  const int nr = min(rows - row0, kCombineRows);
  const int lane = lane_id();
  WNum<P> M2;
  wn_load(M2, cd.N2);
  WNum<P> t[kCombineRows], m[kCombineRows];
  uint32_t pj[kCombineRows];
#pragma unroll
  for (int i = 0; i < kCombineRows; ++i) {
    const int row = row0 + min(i, nr - 1);
    wn_load_clamped(t[i], Kp + (size_t)row * cd.L, cd.L);
    wn_load_clamped(m[i], Mp + (size_t)row * cd.L, cd.L);
    pj[i] = part[(size_t)row * nseg + min(lane, nseg - 1)];
  }
#pragma unroll
  for (int i = 0; i < kCombineRows; ++i) {
    if (i >= nr) break;
    // lanes at or beyond nseg count nothing: log2(nseg) exchanges leave the total in lane 0
    uint32_t sum = lane < nseg ? pj[i] : 0u;
    wn_zero_above(t[i], cd.L);
    wn_zero_above(m[i], cd.L);
    for (int off = 1; off < nseg; off <<= 1) sum += (uint32_t)__shfl_xor((int)sum, off, 64);
    const uint32_t bj = __builtin_amdgcn_readfirstlane(sum);
    if (lane == 0) b[row0 + i] = bj;
    uint64_t c = 0;
    mont_step(t[i], c, bj, m[i], M2, cd.m2prime);
    const uint64_t ovf = wn_resolve(t[i], c);
    wn_cond_sub(t[i], ovf, M2);
    wn_store_n(C + (size_t)(row0 + i) * cd.L, t[i], cd.L);
  }
}

// The same combine with four rows per wavefront, one per 16-lane row (rownum.h): each lane
// holds Q = 4P consecutive limbs of its row's K', M' and c, so a row's operands are read and
// written in 16-byte pieces when the row fills all 16 Q limbs (kFull), and the fixed work of
// the CIOS step, the carry resolution and the final subtraction is shared by four rows.  A
// lane also reads one segment partial of its row (segments 16 apart for more than 16), and an
// exchange inside the row adds them up.  A wave takes kCombineRows rows, four per pass, and
// requests every pass's operands before the first pass computes.
template <int P, bool kFull>
__global__ __launch_bounds__(256) void combine_parts_quad_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                                 const uint32_t* __restrict__ Mp,
                                                                 const uint32_t* __restrict__ part, int nseg,
                                                                 int rows, uint32_t* __restrict__ b,
                                                                 uint32_t* __restrict__ C) {
  constexpr int Q = 4 * P;
  constexpr int kPasses = kCombineRows / 4;
  const int wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = wave * kCombineRows;
  if (row0 >= rows) return;
  const int rl = row_lane();
  RNum<Q> t[kPasses], m[kPasses];
  uint32_t ps[kPasses];
#pragma unroll
  for (int i = 0; i < kPasses; ++i) {
    const int row = min(rows - 1, row0 + 4 * i + row_index());
    rn_load_row<P, kFull>(t[i], Kp + (size_t)row * cd.L, cd.L);
    rn_load_row<P, kFull>(m[i], Mp + (size_t)row * cd.L, cd.L);
    ps[i] = part[(size_t)row * nseg + min(rl, nseg - 1)];
  }
  RNum<Q> M2;
  rn_load(M2, cd.N2);
#pragma unroll
  for (int i = 0; i < kPasses; ++i) {
    if (row0 + 4 * i >= rows) break;
    const int mine = row0 + 4 * i + row_index();
    const int row = min(rows - 1, mine);
    uint32_t sum = rl < nseg ? ps[i] : 0u;
    for (int s0 = 16; s0 < nseg; s0 += 16)  // more than 16 segments (over 65536 columns)
      sum += s0 + rl < nseg ? part[(size_t)row * nseg + s0 + rl] : 0u;
    sum = row_sum16(sum);
    rn_zero_above<P, kFull>(t[i], cd.L);
    rn_zero_above<P, kFull>(m[i], cd.L);
    uint64_t c = 0;
    rn_mont_step(t[i], c, sum, m[i], M2, cd.m2prime);
    const uint64_t ovf = rn_resolve(t[i], c);
    rn_cond_sub(t[i], ovf, M2);
    if (mine < rows) {
      if (rl == 0) b[mine] = sum;
      rn_store_row<P, kFull>(C + (size_t)mine * cd.L, t[i], cd.L);
    }
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
    matvec_part_kernel<4><<<grid, 256, 0, s>>>(D + (size_t)r0 * pitch, nr, pitch, q, cols,
                                               part + (size_t)r0 * nseg, nseg);
  }
}

void launch_combine_parts(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Mp,
                          const uint32_t* part, int nseg, int rows, uint32_t* b, uint32_t* C,
                          hipStream_t s) {
  if (rows <= 0) return;
  const int waves = (rows + kCombineRows - 1) / kCombineRows;
  const int blocks = (waves + 3) / 4;
  if (rows >= kQuadItems) {  // four rows per wavefront once that still leaves several per SIMD
    // 16-byte pieces need rows that fill the lanes and 16-byte aligned arrays
    const bool full = cd.L == 64 * cd.P && ((reinterpret_cast<uintptr_t>(Kp) | reinterpret_cast<uintptr_t>(Mp) |
                                              reinterpret_cast<uintptr_t>(C)) & 15) == 0;
#define ZP_COMBINE_QUAD(PP)                                                                        \
  (full ? combine_parts_quad_kernel<PP, true><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C) \
        : combine_parts_quad_kernel<PP, false><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C))
    switch (cd.P) {
      case 1: ZP_COMBINE_QUAD(1); break;
      case 2: ZP_COMBINE_QUAD(2); break;
      case 3: ZP_COMBINE_QUAD(3); break;
      case 4: ZP_COMBINE_QUAD(4); break;
    }
#undef ZP_COMBINE_QUAD
    return;
  }
  switch (cd.P) {
    case 1: combine_parts_kernel<1><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 2: combine_parts_kernel<2><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 3: combine_parts_kernel<3><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
    case 4: combine_parts_kernel<4><<<blocks, 256, 0, s>>>(cd, Kp, Mp, part, nseg, rows, b, C); break;
  }
}

}  // namespace zp
