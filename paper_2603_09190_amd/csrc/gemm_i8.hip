// D . X mod 2^32 for a uint8 matrix D and uint32 vectors X, on signed int8 MFMA.
//
// Used for the batched online answer B = D.Q (many clients' queries at once; D and the
// answer are shared, Sec. 4.3) and for the global hint H = D.A (Alg. 5 preamble).
//
// Byte planes: with X_b = byte b of X,  D.X = sum_b 2^(8b) (D . X_b) mod 2^32.
// Shift to signed: D' = D - 128 and X_b' = X_b - 128 lie in [-128, 127] (XOR 0x80), and
//   D.X_b = D'.X_b' + 128 sum_i X_b'[i] + 128 sum_i D'[i] + 16384 cols      (exact),
// so each plane is one int8 MFMA contraction plus a per-column term (colsum, per batch)
// and a per-row term (rowsum, per database).  Everything is accumulated in wrapping
// 32-bit integers.  One launch covers at most 65536 columns of D, which keeps every MFMA
// partial sum within +-2^30; longer rows are processed in chunks added into the output.
#include "internal.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------- packing

__global__ __launch_bounds__(256) void pack_planes_s8_kernel(const uint32_t* __restrict__ x,
                                                             long long stride_c,
                                                             long long stride_i, int cols,
                                                             int pitch, int8_t* __restrict__ Xs,
                                                             int32_t* __restrict__ colsum) {
  const int c = blockIdx.y;
  const int i4 = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t part[4] = {0, 0, 0, 0};
  if (4 * i4 < pitch) {
    uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = 4 * i4 + t;
      if (i < cols) {
        const uint32_t v = x[c * stride_c + (long long)i * stride_i];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t sb = ((v >> (8 * b)) & 0xFFu) ^ 0x80u;  // two's complement of byte-128
          w[b] |= sb << (8 * t);
          part[b] += (int32_t)(int8_t)sb;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
      reinterpret_cast<uint32_t*>(Xs + ((size_t)c * 4 + b) * pitch)[i4] = w[b];
  }
  // block reduction of the four column sums
  __shared__ int32_t red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int32_t v = part[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][b] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int b = threadIdx.x;
    const int32_t v = red[0][b] + red[1][b] + red[2][b] + red[3][b];
    atomicAdd(colsum + c * 4 + b, v);
  }
}

void launch_pack_planes_s8(const uint32_t* x, long long stride_c, long long stride_i, int ncol,
                           int cols, int pitch, int8_t* Xs, int32_t* colsum, hipStream_t s) {
  (void)hipMemsetAsync(colsum, 0, sizeof(int32_t) * 4 * (size_t)ncol, s);
  dim3 grid((pitch / 4 + 255) / 256, ncol);
  pack_planes_s8_kernel<<<grid, 256, 0, s>>>(x, stride_c, stride_i, cols, pitch, Xs, colsum);
}

__global__ __launch_bounds__(64) void rowsum_kernel(const uint8_t* __restrict__ D, int cols,
                                                    int pitch, int32_t* __restrict__ rowsum) {
  const int row = blockIdx.x;
  const uint32_t* p = reinterpret_cast<const uint32_t*>(D + (size_t)row * pitch);
  uint32_t acc = 0;
  // padding bytes beyond cols are zero, so summing the whole pitch is exact
  for (int i = threadIdx.x; i < pitch / 4; i += 64) acc = __builtin_amdgcn_udot4(p[i], 0x01010101u, acc, false);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += (uint32_t)__shfl_xor((int)acc, off, 64);
  if (threadIdx.x == 0) rowsum[row] = (int32_t)acc - 128 * cols;
}

void launch_rowsum(const uint8_t* D, int rows, int cols, int pitch, int32_t* rowsum,
                   hipStream_t s) {
  rowsum_kernel<<<rows, 64, 0, s>>>(D, cols, pitch, rowsum);
}

// ----------------------------------------------------------------------------- contraction

constexpr int kBM = 128;          // rows of D per block (4 waves x 32 rows)
constexpr int kBC = 32;           // vectors per block (2 blocks of 16)
constexpr int kKB = 256;          // bytes of K per pipeline step
constexpr int kLdsStride = kKB + 16;
constexpr int kChunk = 65536;     // K bytes per launch (keeps MFMA partials within +-2^30)

// LDS holds the X tile of one K step as 128 rows (plane-major: row = b*32 + c) of 256 bytes.
// Lane (g = lane/16, r = lane%16) feeds MFMA s of the step with bytes [64g + 16s, +16) of its
// D row (A operand) and of its X row (B operand).  The same k-set feeds both operands, so
// the MFMA's internal ordering of k inside one instruction does not matter.
__global__ __launch_bounds__(256) void gemm_planes_kernel(
    const uint8_t* __restrict__ D, int rows, int cols, int pitch, const int8_t* __restrict__ Xs,
    const int32_t* __restrict__ colsum, int ncol, const int32_t* __restrict__ rowsum,
    uint32_t* __restrict__ out, int out_rowmajor, long long out_ld, int k0, int k1,
    int first_chunk) {
  __shared__ __attribute__((aligned(16))) int8_t xs[4 * kBC][kLdsStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int rowblk = blockIdx.x * kBM;
  const int cblk = blockIdx.y * kBC;

  const uint8_t* dp[2];
#pragma unroll
  for (int mr = 0; mr < 2; ++mr) {
    const int row = min(rowblk + 32 * wave + 16 * mr + r, rows - 1);
    dp[mr] = D + (size_t)row * pitch + 64 * g;
  }
  // X tile loading: thread tid fills LDS row tid/2 (plane b = row/32, vector row%32), half tid%2
  const int xrow = tid >> 1, xhalf = tid & 1;
  const int xb = xrow >> 5, xc = cblk + (xrow & 31);
  const bool xvalid = xc < ncol;
  const int8_t* xp = Xs + ((size_t)(xvalid ? xc : 0) * 4 + xb) * pitch + 128 * xhalf;

  v4i acc[2][2][4];
#pragma unroll
  for (int mr = 0; mr < 2; ++mr)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[mr][qb][b] = v4i{0, 0, 0, 0};

  u32x4 xr[8];
  u32x4 da[2][4];
  auto load_step = [&](int k) {
#pragma unroll
    for (int t = 0; t < 8; ++t)
      xr[t] = xvalid ? *reinterpret_cast<const u32x4*>(xp + k + 16 * t) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int mr = 0; mr < 2; ++mr)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        da[mr][s] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(dp[mr] + k) + s);
  };

  load_step(k0);
  for (int k = k0; k < k1; k += kKB) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t)
      *reinterpret_cast<u32x4*>(&xs[xrow][128 * xhalf + 16 * t]) = xr[t];
    __syncthreads();
    u32x4 dcur[2][4];
#pragma unroll
    for (int mr = 0; mr < 2; ++mr)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        u32x4 v = da[mr][s];
        v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
        dcur[mr][s] = v;
      }
    if (k + kKB < k1) load_step(k + kKB);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      v4i xf[2][4];
#pragma unroll
      for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          xf[qb][b] = *reinterpret_cast<const v4i*>(&xs[b * 32 + 16 * qb + r][64 * g + 16 * s]);
#pragma unroll
      for (int mr = 0; mr < 2; ++mr) {
        const u32x4 dv = dcur[mr][s];
        const v4i a = v4i{(int)dv.x, (int)dv.y, (int)dv.z, (int)dv.w};
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[mr][qb][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, xf[qb][b], acc[mr][qb][b], 0, 0, 0);
      }
    }
  }

  // epilogue: output element (row, c) sits in lane (g, r) register i with
  // row = 16 mr + 4 g + i inside the wave's 32 rows and c = 16 qb + r inside the block.
#pragma unroll
  for (int mr = 0; mr < 2; ++mr)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const int c = cblk + 16 * qb + r;
      if (c >= ncol) continue;
      uint32_t cs[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) cs[b] = first_chunk ? 128u * (uint32_t)colsum[c * 4 + b] : 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rowblk + 32 * wave + 16 * mr + 4 * g + i;
        if (row >= rows) continue;
        const uint32_t rterm = first_chunk ? 128u * (uint32_t)rowsum[row] + 16384u * (uint32_t)cols : 0u;
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          v += ((uint32_t)acc[mr][qb][b][i] + cs[b] + rterm) << (8 * b);
        uint32_t* o = out_rowmajor ? out + (size_t)row * ncol + c : out + (size_t)c * out_ld + row;
        if (first_chunk) *o = v; else *o += v;
      }
    }
}

void launch_gemm_planes(const uint8_t* D, int rows, int cols, int pitch, const int8_t* Xs,
                        const int32_t* colsum, int ncol, const int32_t* rowsum, uint32_t* out,
                        bool out_rowmajor, long long out_ld, hipStream_t s) {
  dim3 grid((rows + kBM - 1) / kBM, (ncol + kBC - 1) / kBC);
  for (int k0 = 0; k0 < pitch; k0 += kChunk) {
    const int k1 = min(pitch, k0 + kChunk);
    gemm_planes_kernel<<<grid, 256, 0, s>>>(D, rows, cols, pitch, Xs, colsum, ncol, rowsum, out,
                                            out_rowmajor ? 1 : 0, out_ld, k0, k1, k0 == 0 ? 1 : 0);
  }
}

}  // namespace zp
