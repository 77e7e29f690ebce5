// Global hint H = D.A mod 2^32 (Alg. 5 preamble; reused by every client, Sec. 4.3
// "Reusability of the offline phase") as a compute-bound int8 MFMA contraction.
//
// A's uint32 entries are split into four byte planes A_b and shifted to signed bytes (XOR 0x80),
// as for the batched answer:
//   D.A_b = D'.A_b' + 128 sum_i A_b'[i] + 128 sum_i D'[i] + 16384 cols,   H = sum_b 2^(8b) D.A_b.
// The work is 8 rows cols n int8 operations against at most 4 n pitch + rows pitch operand
// bytes, so it is bound by the MFMA rate, not by HBM, once each operand fragment is reused often
// enough from registers:
//   - a workgroup of four wavefronts takes 256 rows (MR = 4 tiles of 16 per wavefront) and 64
//     columns of A (16 tiles: four 16-column groups x four planes);
//   - a wavefront keeps 4 x 16 accumulator tiles; each A fragment (16 rows of D, read straight
//     from memory into registers) feeds 16 MFMAs and each B fragment (16 plane columns of A,
//     staged through LDS and shared by the four wavefronts) feeds 4;
//   - the four planes of one column of H sit in the same lane and register of four tiles, so the
//     epilogue adds them with shifts and no data exchange.
// The grid is XCD-aware: the 32 workgroups that one XCD runs together form a 4 x 8 super-tile
// (four row blocks, eight column blocks), so each D fragment is fetched once per XCD and served
// from its L2 to the other seven column blocks, and each A fragment to the other three row blocks.
#include <algorithm>

#include "internal.h"
#include "stage.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int kHNT = 16;      // column tiles per workgroup: 4 column groups x 4 planes
constexpr int kHCols = 64;    // columns of A per workgroup
constexpr int kHSR = 4;       // super-tile: row blocks ...
constexpr int kHSC = 8;       // ... x column blocks run together on one XCD

}  // namespace

// Apt: the signed planes of A in fragment order.  Piece (G, p) is 1 KiB at (G (pitch / 64) + p)
// KiB, G = b (npad / 16) + kg, holding plane b of A columns 16 kg .. 16 kg + 15 over K bytes
// 64 p .. 64 p + 63: lane (g, r) = 16 g + r's 16 bytes at 16 (16 g + r) are
//   (byte b of A[64 p + 16 g + u][16 kg + r]) ^ 0x80,  u < 16
// (0 for rows at or beyond cols and columns at or beyond n).  One thread per (kg, p, lane)
// reads 16 entries of A once and writes the four planes.
__global__ __launch_bounds__(256) void a_planes_kernel(const uint32_t* __restrict__ A, int cols, int n, int npad,
                                                       int pitch, long long pieces, u32x4* __restrict__ Apt) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= pieces) return;  // pieces = (npad / 16) (pitch / 64) 64
  const int l = (int)(idx & 63);
  const long long q = idx >> 6;
  const int np = pitch / 64;
  const int p = (int)(q % np);
  const int kg = (int)(q / np);
  const int g = l >> 4, r = l & 15;
  const int col = 16 * kg + r;
  const int i0 = 64 * p + 16 * g;
  uint32_t w[4][4] = {};
  if (col < n) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i0 + u;
      const uint32_t v = i < cols ? A[(size_t)i * n + col] : 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t sb = i < cols ? (((v >> (8 * b)) & 0xFFu) ^ 0x80u) : 0u;
        w[b][u >> 2] |= sb << (8 * (u & 3));
      }
    }
  }
  const long long groups = npad / 16;
#pragma unroll
  for (int b = 0; b < 4; ++b)
    Apt[((b * groups + kg) * np + p) * 64 + l] = u32x4{w[b][0], w[b][1], w[b][2], w[b][3]};
}

void launch_a_planes(const uint32_t* A, int cols, int n, int pitch, uint8_t* Apt, hipStream_t s) {
  const int npad = hgemm_npad(n);
  const long long pieces = (long long)(npad / 16) * (pitch / 64) * 64;
  a_planes_kernel<<<(unsigned)((pieces + 255) / 256), 256, 0, s>>>(A, cols, n, npad, pitch, pieces,
                                                                   reinterpret_cast<u32x4*>(Apt));
}

int hgemm_npad(int n) { return (n + kHCols - 1) / kHCols * kHCols; }

// Acolsum[k 4 + b] = sum_{i<cols} (byte b of A[i][k]) - 128 (zeroed first): 64 columns per
// workgroup (one per lane), rows dealt to its four wavefronts and to gridDim.y workgroups.
__global__ __launch_bounds__(256) void a_colsum_kernel(const uint32_t* __restrict__ A, int cols, int n,
                                                       int32_t* __restrict__ Acolsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  int32_t sum[4] = {0, 0, 0, 0};
  if (col < n)
    for (int i = blockIdx.y * 4 + wave; i < cols; i += gridDim.y * 4) {
      const uint32_t v = A[(size_t)i * n + col];
#pragma unroll
      for (int b = 0; b < 4; ++b) sum[b] += (int32_t)((v >> (8 * b)) & 0xFFu) - 128;
    }
  __shared__ int32_t red[4][64][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) red[wave][lane][b] = sum[b];
  __syncthreads();
  if (wave == 0 && col < n) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      atomicAdd(Acolsum + (size_t)col * 4 + b, red[0][lane][b] + red[1][lane][b] + red[2][lane][b] + red[3][lane][b]);
  }
}

__global__ void a_colsum_zero_kernel(int32_t* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

void launch_a_colsum(const uint32_t* A, int cols, int n, int32_t* Acolsum, hipStream_t s) {
  a_colsum_zero_kernel<<<(4 * n + 255) / 256, 256, 0, s>>>(Acolsum, 4 * n);
  dim3 grid((n + 63) / 64, std::min(64, (cols + 1023) / 1024));
  a_colsum_kernel<<<grid, 256, 0, s>>>(A, cols, n, Acolsum);
}

// kTiled: D is the tiled copy (16-row groups contiguous, 16-row x 64-byte pieces); otherwise
// row-major with the given pitch (the rows of a partial refresh).  Rows of the last 16-row group
// past `rows` are read (they exist in both layouts as padding or repeat the last row) and never
// stored.  A workgroup takes 64 MR rows (MR tiles per wavefront) and 64 columns of A.  Both
// operands pass through LDS in NS stages of one 64-byte K slice, by direct global-to-LDS loads
// (stage.h), so the only wait per slice is for that slice's loads; one barrier per slice.  In
// LDS, lane 4 r + g of an A kilobyte holds row r, bytes 16 g .. 16 g + 15 (the tiled copy's own
// order), which the MFMA's lane (g, r) reads back; B kilobytes are in fragment order already.
template <int MR, int NS, bool kTiled>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, MR <= 2 ? 2 : 1)))
void hgemm_kernel(const uint8_t* __restrict__ D, int rows, int cols, int pitch, const uint8_t* __restrict__ Apt,
                  int n, int npad, const int32_t* __restrict__ Acolsum, const int32_t* __restrict__ rowsum,
                  uint32_t* __restrict__ H, int nrb, int ncb) {
  constexpr int kAChunks = 4 * MR;
  constexpr int kChunks = kAChunks + kHNT;
  constexpr int kStage = kChunks * 1024;
  constexpr int kEpi = 4 * kHNT * 64 * 16;  // the epilogue's 16 KiB per wavefront
  constexpr int kLds = NS * kStage > kEpi ? NS * kStage : kEpi;
  constexpr int kPerWave = MR + kHNT / 4;
  __shared__ __attribute__((aligned(1024))) uint8_t lds[kLds];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, r = lane & 15;
  // XCD-aware placement: workgroup L runs on XCD L mod 8; its slot on that XCD picks a
  // super-tile and a place in it
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int round = slot / (kHSR * kHSC), loc = slot % (kHSR * kHSC);
  const int st = round * 8 + xcd;
  const int nsc = (ncb + kHSC - 1) / kHSC;
  const int rb = (st / nsc) * kHSR + loc / kHSC;
  const int cb = (st % nsc) * kHSC + loc % kHSC;
  if (rb >= nrb || cb >= ncb) return;
  const int S = pitch / 64;
  const int last_group = (rows - 1) >> 4;

  // loads of this wavefront per slice: its own MR A kilobytes, then B tiles wave + 4 q
  const uint8_t* src[kPerWave];
  int dst[kPerWave];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int T = min((rb * 4 + wave) * MR + i, last_group);
    // lane l carries row l / 4, bytes 16 (l mod 4) of the 16-row x 64-byte piece
    if constexpr (kTiled) src[i] = D + (size_t)T * 16 * pitch + lane * 16;
    else src[i] = D + (size_t)min(16 * T + (lane >> 2), rows - 1) * pitch + (lane & 3) * 16;
    dst[i] = (wave * MR + i) * 1024;
  }
  const long long groups = npad / 16;
#pragma unroll
  for (int q = 0; q < kHNT / 4; ++q) {
    const int t = wave + 4 * q;  // tile t = 4 cgrp + b: plane b of columns 16 (4 cb + cgrp) + r
    const long long G = (t & 3) * groups + 4 * cb + (t >> 2);
    src[MR + q] = Apt + (size_t)G * S * 1024 + lane * 16;
    dst[MR + q] = (kAChunks + t) * 1024;
  }
  auto issue = [&](int p) {
    const int pc = min(p, S - 1);
    uint8_t* base = lds + (p % NS) * kStage;
#pragma unroll
    for (int j = 0; j < kPerWave; ++j) {
      const size_t adv = j < MR ? (kTiled ? (size_t)pc * 1024 : (size_t)pc * 64) : (size_t)pc * 1024;
      g2l16(src[j] + adv, base + dst[j]);
    }
  };

  v4i acc[MR][kHNT];
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int t = 0; t < kHNT; ++t) acc[i][t] = v4i{0, 0, 0, 0};

#pragma unroll
  for (int p = 0; p < NS - 1; ++p) issue(p);
  const int aread = (r * 4 + g) * 16;  // where the MFMA's lane (g, r) finds row r, bytes 16 g
  for (int p = 0; p < S; ++p) {
    wait_vmcnt<(NS - 2) * kPerWave>();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    issue(p + NS - 1);
    const uint8_t* base = lds + (p % NS) * kStage;
    v4i bf[kHNT];
#pragma unroll
    for (int t = 0; t < kHNT; ++t) bf[t] = *reinterpret_cast<const v4i*>(base + (kAChunks + t) * 1024 + lane * 16);
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      u32x4 v = *reinterpret_cast<const u32x4*>(base + (wave * MR + i) * 1024 + aread);
      v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
      const v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
      for (int t = 0; t < kHNT; ++t) acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[t], acc[i][t], 0, 0, 0);
    }
  }
  wait_vmcnt<0>();  // the surplus loads past the last slice write LDS the epilogue reuses
  lds_barrier_sync();

  // epilogue: H[row][col] = sum_b (acc_b + 128 colsum_b + 128 rowsum + 16384 cols) 2^(8b).  Each
  // wavefront parks one row tile of raw accumulators in its own 16 KiB of LDS (tile t, lane,
  // element), then lane c builds column c of the 64 for each of the tile's 16 rows, so every
  // store writes 256 contiguous bytes of a row of H.
  uint32_t* wl = reinterpret_cast<uint32_t*>(lds) + wave * (kHNT * 64 * 4);
  const uint32_t kterm = 16384u * (uint32_t)cols;
  const int c = lane;  // column within the block's 64
  const int col = kHCols * cb + c;
  const int cgrp = c >> 4, cr = c & 15;
  uint32_t ct[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) ct[b] = col < n ? 128u * (uint32_t)Acolsum[col * 4 + b] : 0u;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
#pragma unroll
    for (int t = 0; t < kHNT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) wl[(t * 64 + lane) * 4 + e] = (uint32_t)acc[i][t][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const int row0 = ((rb * 4 + wave) * MR + i) * 16;
#pragma unroll 4
    for (int rho = 0; rho < 16; ++rho) {
      const int row = row0 + rho;
      if (row >= rows) break;
      const uint32_t rterm = 128u * (uint32_t)rowsum[row] + kterm;
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        v += (wl[((cgrp * 4 + b) * 64 + (rho >> 2) * 16 + cr) * 4 + (rho & 3)] + ct[b] + rterm) << (8 * b);
      if (col < n) H[(size_t)row * n + col] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }
}

// The same contraction with eight wavefronts (two per SIMD): wavefront (wr, wc) = (w mod 4, w / 4)
// takes four row tiles of the workgroup's 256 rows and the eight column tiles of column half wc
// (two 16-column groups x four planes), 4 x 8 accumulator tiles that fit the architectural VGPRs.
// Each slice stages 16 A and 16 B kilobytes as before, four loads per wavefront; the epilogue
// parks one row tile at a time in the wavefront's 8 KiB of LDS and lanes 32 h + c build column c
// of the half's 32 for rows h, h + 2, ..., so every store writes 128 contiguous bytes of a row.
// kPair: the slice loop software-pipelined over two register sets (NS = 4), described at the
// loop.
template <int NS, bool kTiled, bool kPair = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void hgemm_w8_kernel(const uint8_t* __restrict__ D, int rows, int cols, int pitch, const uint8_t* __restrict__ Apt,
                     int n, int npad, const int32_t* __restrict__ Acolsum, const int32_t* __restrict__ rowsum,
                     uint32_t* __restrict__ H, int nrb, int ncb) {
  constexpr int kAChunks = 16;                  // row tiles of the workgroup's 256 rows
  constexpr int kChunks = kAChunks + kHNT;
  constexpr int kStage = kChunks * 1024;
  constexpr int kEpi = 8 * 8 * 64 * 16;         // the epilogue's 8 KiB per wavefront
  constexpr int kLds = NS * kStage > kEpi ? NS * kStage : kEpi;
  constexpr int kPerWave = kChunks / 8;
  __shared__ __attribute__((aligned(1024))) uint8_t lds[kLds];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 3, wc = wave >> 2;
  const int g = lane >> 4, r = lane & 15;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int round = slot / (kHSR * kHSC), loc = slot % (kHSR * kHSC);
  const int st = round * 8 + xcd;
  const int nsc = (ncb + kHSC - 1) / kHSC;
  const int rb = (st / nsc) * kHSR + loc / kHSC;
  const int cb = (st % nsc) * kHSC + loc % kHSC;
  if (rb >= nrb || cb >= ncb) return;
  const int S = pitch / 64;
  const int last_group = (rows - 1) >> 4;

  // loads of this wavefront per slice: pieces wave, wave + 8, wave + 16, wave + 24 (A row tiles,
  // then B tiles t = 4 cgrp + b)
  const uint8_t* src[kPerWave];
  int dst[kPerWave];
  bool isa[kPerWave];
  const long long groups = npad / 16;
#pragma unroll
  for (int j = 0; j < kPerWave; ++j) {
    const int c = wave + 8 * j;
    dst[j] = c * 1024;
    isa[j] = c < kAChunks;
    if (c < kAChunks) {
      const int T = min(rb * kAChunks + c, last_group);
      if constexpr (kTiled) src[j] = D + (size_t)T * 16 * pitch + lane * 16;
      else src[j] = D + (size_t)min(16 * T + (lane >> 2), rows - 1) * pitch + (lane & 3) * 16;
    } else {
      const int t = c - kAChunks;
      const long long G = (t & 3) * groups + 4 * cb + (t >> 2);
      src[j] = Apt + (size_t)G * S * 1024 + lane * 16;
    }
  }
  auto issue = [&](int p) {
    const int pc = min(p, S - 1);
    uint8_t* base = lds + (p % NS) * kStage;
#pragma unroll
    for (int j = 0; j < kPerWave; ++j) {
      const size_t adv = isa[j] ? (kTiled ? (size_t)pc * 1024 : (size_t)pc * 64) : (size_t)pc * 1024;
      g2l16(src[j] + adv, base + dst[j]);
    }
  };

  v4i acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[i][t] = v4i{0, 0, 0, 0};

  const int aread = (r * 4 + g) * 16;  // where the MFMA's lane (g, r) finds row r, bytes 16 g
  auto compute = [&](int p) {
    const uint8_t* base = lds + (p % NS) * kStage;
    v4i bf[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      bf[t] = *reinterpret_cast<const v4i*>(base + (kAChunks + 8 * wc + t) * 1024 + lane * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u32x4 v = *reinterpret_cast<const u32x4*>(base + (wr * 4 + i) * 1024 + aread);
      v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
      const v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[t], acc[i][t], 0, 0, 0);
    }
  };
  if constexpr (kPair) {
    // Operands of slice p + 1 are read from LDS into a second register set while the MFMAs of
    // slice p run, so that a wavefront's LDS reads overlap its own products; the barrier of a
    // slice therefore comes one slice earlier (slice p + 1 must have landed before its reads),
    // and four buffers keep the one being overwritten (slice p - 1) consumed.
    static_assert(NS == 4, "the pipelined loop uses four buffers");
    v4i b0[8], b1[8];
    u32x4 a0[4], a1[4];
    auto load_regs = [&](int p, v4i (&bf)[8], u32x4 (&af)[4]) {
      const uint8_t* base = lds + (p % NS) * kStage;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        bf[t] = *reinterpret_cast<const v4i*>(base + (kAChunks + 8 * wc + t) * 1024 + lane * 16);
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const u32x4*>(base + (wr * 4 + i) * 1024 + aread);
    };
    auto mfma_regs = [&](const v4i (&bf)[8], const u32x4 (&af)[4]) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const u32x4 v = af[i] ^ 0x80808080u;
        const v4i a = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bf[t], acc[i][t], 0, 0, 0);
      }
    };
    auto sync_slice = [&]() {
      wait_vmcnt<kPerWave>();
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    };
    issue(0);
    issue(1);
    issue(2);
    wait_vmcnt<2 * kPerWave>();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    load_regs(0, b0, a0);
    for (int p = 0; p < S; p += 2) {
      sync_slice();  // slice p + 1 landed; slice p - 1's buffer consumed by every wavefront
      issue(p + 3);
      load_regs(p + 1, b1, a1);
      mfma_regs(b0, a0);
      if (p + 1 < S) {
        sync_slice();
        issue(p + 4);
        load_regs(p + 2, b0, a0);
        mfma_regs(b1, a1);
      }
    }
  } else {
#pragma unroll
    for (int p = 0; p < NS - 1; ++p) issue(p);
    for (int p = 0; p < S; ++p) {
      wait_vmcnt<(NS - 2) * kPerWave>();
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      issue(p + NS - 1);
      compute(p);
    }
  }
  wait_vmcnt<0>();  // the surplus loads past the last slice write LDS the epilogue reuses
  lds_barrier_sync();

  // epilogue: H[row][col] = sum_b (acc_b + 128 colsum_b + 128 rowsum + 16384 cols) 2^(8b)
  uint32_t* wl = reinterpret_cast<uint32_t*>(lds) + wave * (8 * 64 * 4);
  const uint32_t kterm = 16384u * (uint32_t)cols;
  const int c = lane & 31, half = lane >> 5;  // column within the half's 32, row parity
  const int col = kHCols * cb + 32 * wc + c;
  const int cgrp = c >> 4, cr = c & 15;
  uint32_t ct[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) ct[b] = col < n ? 128u * (uint32_t)Acolsum[col * 4 + b] : 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) wl[(t * 64 + lane) * 4 + e] = (uint32_t)acc[i][t][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const int row0 = (rb * kAChunks + wr * 4 + i) * 16;
#pragma unroll 4
    for (int k = 0; k < 8; ++k) {
      const int rho = 2 * k + half;
      const int row = row0 + rho;
      if (row < rows) {
        const uint32_t rterm = 128u * (uint32_t)rowsum[row] + kterm;
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          v += (wl[((cgrp * 4 + b) * 64 + (rho >> 2) * 16 + cr) * 4 + (rho & 3)] + ct[b] + rterm) << (8 * b);
        if (col < n) H[(size_t)row * n + col] = v;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }
}

struct HVariant {
  int mr, ns;  // mr 0: the eight-wavefront kernel; mr 1: the same with its LDS reads pipelined
};
static const HVariant kHVariants[] = {{4, 4}, {4, 3}, {2, 4}, {2, 3}, {0, 3}, {0, 4}, {1, 4}};

int hgemm_variants() { return (int)(sizeof(kHVariants) / sizeof(kHVariants[0])); }

template <int MR, int NS>
static void launch_hgemm_t(const uint8_t* D, bool tiled, int rows, int cols, int pitch, const uint8_t* Apt, int n,
                           const int32_t* Acolsum, const int32_t* rowsum, uint32_t* H, hipStream_t s) {
  const int npad = hgemm_npad(n);
  const int nrb = (rows + 64 * MR - 1) / (64 * MR);
  const int ncb = npad / kHCols;
  const int nsr = (nrb + kHSR - 1) / kHSR, nsc = (ncb + kHSC - 1) / kHSC;
  // super-tiles are dealt to the XCDs round by round: 8 per round
  const long long rounds = ((long long)nsr * nsc + 7) / 8;
  const long long nblocks = rounds * 8 * kHSR * kHSC;
  if (tiled)
    hgemm_kernel<MR, NS, true><<<(unsigned)nblocks, 256, 0, s>>>(D, rows, cols, pitch, Apt, n, npad, Acolsum, rowsum, H, nrb, ncb);
  else
    hgemm_kernel<MR, NS, false><<<(unsigned)nblocks, 256, 0, s>>>(D, rows, cols, pitch, Apt, n, npad, Acolsum, rowsum, H, nrb, ncb);
}

void launch_hgemm(const uint8_t* D, bool tiled, int rows, int cols, int pitch, const uint8_t* Apt, int n,
                  const int32_t* Acolsum, const int32_t* rowsum, uint32_t* H, int variant, hipStream_t s) {
  if (rows <= 0 || n <= 0) return;
  const HVariant v = kHVariants[(variant >= 0 && variant < hgemm_variants()) ? variant : 0];
  if (v.mr == 0 || v.mr == 1) {
    const int npad = hgemm_npad(n);
    const int nrb = (rows + 255) / 256;
    const int ncb = npad / kHCols;
    const int nsr = (nrb + kHSR - 1) / kHSR, nsc = (ncb + kHSC - 1) / kHSC;
    const long long rounds = ((long long)nsr * nsc + 7) / 8;
    const unsigned nblocks = (unsigned)(rounds * 8 * kHSR * kHSC);
#define ZP_H8(N, T) hgemm_w8_kernel<N, T><<<nblocks, 512, 0, s>>>(D, rows, cols, pitch, Apt, n, npad, Acolsum, rowsum, H, nrb, ncb)
    if (v.mr == 1) {
      if (tiled)
        hgemm_w8_kernel<4, true, true><<<nblocks, 512, 0, s>>>(D, rows, cols, pitch, Apt, n, npad, Acolsum, rowsum, H, nrb, ncb);
      else
        hgemm_w8_kernel<4, false, true><<<nblocks, 512, 0, s>>>(D, rows, cols, pitch, Apt, n, npad, Acolsum, rowsum, H, nrb, ncb);
    } else if (v.ns == 3) {
      if (tiled) ZP_H8(3, true); else ZP_H8(3, false);
    } else {
      if (tiled) ZP_H8(4, true); else ZP_H8(4, false);
    }
#undef ZP_H8
    return;
  }
  if (v.mr == 4 && v.ns == 4) launch_hgemm_t<4, 4>(D, tiled, rows, cols, pitch, Apt, n, Acolsum, rowsum, H, s);
  else if (v.mr == 4) launch_hgemm_t<4, 3>(D, tiled, rows, cols, pitch, Apt, n, Acolsum, rowsum, H, s);
  else if (v.ns == 4) launch_hgemm_t<2, 4>(D, tiled, rows, cols, pitch, Apt, n, Acolsum, rowsum, H, s);
  else launch_hgemm_t<2, 3>(D, tiled, rows, cols, pitch, Apt, n, Acolsum, rowsum, H, s);
}

}  // namespace zp
