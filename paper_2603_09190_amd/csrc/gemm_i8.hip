// D . X mod 2^32 for a uint8 matrix D and uint32 vectors X, on signed int8 MFMA; with one
// plane, D . X for uint8 vectors X (exact 32-bit sums, used by the offset answer).
//
// Used for the batched online answer B = D.Q (many clients' queries at once; D is shared
// by all clients, Sec. 4.3) and for the global hint H = D.A (Alg. 5 preamble).
//
// Byte planes: with X_b = byte b of X,  D.X = sum_b 2^(8b) (D . X_b) mod 2^32.
// Shift to signed: D' = D - 128 and X_b' = X_b - 128 lie in [-128, 127] (XOR 0x80), and
//   D.X_b = D'.X_b' + 128 sum_i X_b'[i] + 128 sum_i D'[i] + 16384 cols      (exact),
// so each plane is one int8 MFMA contraction plus a per-column term (colsum, per batch)
// and a per-row term (rowsum, per database).  Everything is accumulated in wrapping
// 32-bit integers.
#include <algorithm>

#include "internal.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits for every
// outstanding global load, which would drain the D prefetch ring at each K step.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ----------------------------------------------------------------------------- packing

__global__ __launch_bounds__(256) void pack_planes_s8_kernel(const uint32_t* __restrict__ x,
                                                             long long stride_c,
                                                             long long stride_i, int cols,
                                                             int pitch, int8_t* __restrict__ Xs,
                                                             int32_t* __restrict__ colsum) {
  const int c = blockIdx.x;
  const int i4 = blockIdx.y * blockDim.x + threadIdx.x;
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
  // vectors on x (up to 2^31 blocks), 1024-column pieces on y (at most 2^14 for pitch <= 2^24)
  dim3 grid(ncol, (pitch / 4 + 255) / 256);
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

constexpr int kBC = 32;           // vectors per block (2 blocks of 16)
constexpr int kMaxBlockK = 65536; // K bytes per block (keeps MFMA partials within +-2^30)

// A wave computes 16 kMR rows x 32 vectors x kPl planes (4 for uint32 vectors, 1 for uint8
// vectors) with v_mfma_i32_16x16x64_i8: in slice s of a kKB-byte K step, lane (g = lane/16,
// r = lane%16) supplies bytes [64s + 16g, +16) of its D row (A operand) and of its X row
// (B operand), so each load instruction reads 64 contiguous bytes of each of 16 rows.  The
// same k-set feeds both operands, so the MFMA's internal ordering of k does not matter.  The
// plane results of one output sit in the same lane and register, so the epilogue combines
// them without data exchange.
// A block of kW waves covers 16 kMR kW rows and one K range of at most 64 KiB (split-K,
// which keeps every MFMA partial within +-2^30); each wave keeps kDepth K steps of D in
// flight, the X tile (kPl groups x 32 vectors x kKB bytes) is double-buffered in LDS with one
// barrier per step, and partial results are added into the zeroed output with 32-bit atomic
// adds (exact modulo 2^32 in any order).
// kWide: X holds uint8 vectors (one plane) and the kPl accumulator groups are kPl different
// 32-vector column groups sharing each D fragment, i.e. a block covers 32 kPl output columns.
// The grid is one-dimensional and XCD-aware: workgroup L runs on XCD L mod 8, and each XCD
// takes every column block and K range of one row block in turn (row blocks x, x+8, ...), so
// the D tile they share is read from HBM once and then served from that XCD's L2.
// Steps by which the X tile's global loads run ahead of its use (kNX = x_ahead - 1 register
// buffers): three with two or more D steps in flight, two with one.
constexpr int x_ahead(int waves, int depth, int mr, int kb, int pl) {
  (void)waves; (void)mr; (void)kb; (void)pl;
  return depth >= 2 ? 3 : 2;
}

// kTiled: D is the tiled copy (see tile_rows_kernel): 16-row x 64-byte pieces, each 16-row
// group's whole K range contiguous, so a wave's load of 16 rows x 64 bytes is one contiguous
// kilobyte and a block streams long contiguous runs instead of 256-byte pieces of many rows.
template <int kW, int kDepth, int kMR, int kKB, int kPl, bool kWide, bool kTiled>
__device__ __forceinline__ void gemm_planes_body(
    const uint8_t* __restrict__ D, int rows, int cols, int pitch, const int8_t* __restrict__ Xs,
    const int32_t* __restrict__ colsum, int ncol, const int32_t* __restrict__ rowsum,
    uint32_t* __restrict__ out, int out_rowmajor, long long out_ld, int ksteps_per_block,
    int nrb, int ncb, int nkz) {
  static_assert(kWide || kPl == 4, "byte-plane mode has four planes");
  constexpr int kSl = kKB / 64;            // MFMA K slices per step
  constexpr int kStride = kKB + 32;        // LDS row stride; a 32-byte skew makes the fragment reads conflict-free
  __shared__ __attribute__((aligned(16))) int8_t xs[2][kPl * kBC][kStride];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, r = lane & 15;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per_rb = ncb * nkz;
  const int rbi = (slot / per_rb) * 8 + xcd;
  if (rbi >= nrb) return;
  const int u = slot % per_rb;
  const int cbi = u % ncb, kz = u / ncb;
  const int rowblk = rbi * 16 * kMR * kW;
  const int cblk = cbi * (kWide ? kPl * kBC : kBC);
  const int kstep0 = kz * ksteps_per_block;
  const int nsteps = min(ksteps_per_block, pitch / kKB - kstep0);
  if (nsteps <= 0) return;

  const uint8_t* dp[kMR];
#pragma unroll
  for (int mr = 0; mr < kMR; ++mr) {
    const int row = min(rowblk + 16 * kMR * wave + 16 * mr + r, rows - 1);
    dp[mr] = kTiled ? D + (size_t)(row >> 4) * 16 * pitch + (size_t)kstep0 * (kKB / 64) * 1024 + (row & 15) * 64 + 16 * g
                    : D + (size_t)row * pitch + (size_t)kstep0 * kKB + 16 * g;
  }
  constexpr int kPieces = kPl * kBC * (kKB / 16) / (64 * kW);
  static_assert(kPieces >= 1 && kPieces * 64 * kW == kPl * kBC * (kKB / 16), "X tile split");
  // The X tile's offsets are kept relative to the block's first vector: at most 32 kPl vectors
  // (one plane each, kWide) or 32 vectors of kPl planes, so below 128 pitch, which fits 32 bits
  // for every pitch the library accepts (at most 2^24).  Only the block base is 64-bit.
  const int8_t* __restrict__ xbase = Xs + (size_t)cblk * (kWide ? 1 : kPl) * pitch + (size_t)kstep0 * kKB;
  int xoff[kPieces], lrow[kPieces], lcol[kPieces];
  bool xval[kPieces];
#pragma unroll
  for (int t = 0; t < kPieces; ++t) {
    const int piece = tid + t * 64 * kW;
    lrow[t] = piece / (kKB / 16);
    lcol[t] = (piece % (kKB / 16)) * 16;
    const int b = lrow[t] >> 5;
    const int c = kWide ? cblk + lrow[t] : cblk + (lrow[t] & 31);
    xval[t] = c < ncol;
    // vectors beyond ncol read vector ncol-1 (a valid address) and are zeroed in the stash
    const int cr = min(c, ncol - 1) - cblk;
    xoff[t] = (kWide ? cr : cr * kPl + b) * pitch + lcol[t];
  }

  v4i acc[kMR][2][kPl];
#pragma unroll
  for (int mr = 0; mr < kMR; ++mr)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int b = 0; b < kPl; ++b) acc[mr][qb][b] = v4i{0, 0, 0, 0};

  // X steps are loaded kXA steps ahead into kNX register buffers (step j in buffer j % kNX)
  // and stashed into LDS one step ahead.  With two or more D steps in flight, X runs three
  // steps ahead and each step issues its X load before its D load: the in-order load counter
  // then lets the wait for X(i+1) pass while the younger D loads are still in flight.
  constexpr int kXA = x_ahead(kW, kDepth, kMR, kKB, kPl);
  constexpr int kNX = kXA - 1;
  static_assert(kDepth == 1 || (kDepth % 2 == 0 ? kDepth : 2 * kDepth) % kNX == 0,
                "X buffers must be static in the unrolled trip");
  // unroll so that ring slots and X buffers are static register indices
  constexpr int kU = kDepth == 1 ? 1 : (kDepth % 2 == 0 ? kDepth : 2 * kDepth);
  u32x4 ring[kDepth][kMR][kSl];
  u32x4 xn[kNX][kPieces];
  auto load_d = [&](int slot_, int st) {
#pragma unroll
    for (int mr = 0; mr < kMR; ++mr)
#pragma unroll
      for (int s = 0; s < kSl; ++s)
        ring[slot_][mr][s] = __builtin_nontemporal_load(
            reinterpret_cast<const u32x4*>(kTiled ? dp[mr] + (size_t)st * kKB * 16 + 1024 * s
                                                  : dp[mr] + (size_t)st * kKB + 64 * s));
  };
  auto load_x = [&](int xb, int st) {
#pragma unroll
    for (int t = 0; t < kPieces; ++t)
      xn[xb][t] = *reinterpret_cast<const u32x4*>(xbase + (size_t)xoff[t] + (size_t)st * kKB);
  };
  // Vectors beyond ncol are zeroed here, when the data is consumed: a select right after the
  // load would make the wave wait for it (and, the load counter being in order, for every
  // older load) in the step that issued it.
  auto stash = [&](int xb, int buf) {
#pragma unroll
    for (int t = 0; t < kPieces; ++t)
      *reinterpret_cast<u32x4*>(&xs[buf][lrow[t]][lcol[t]]) = xval[t] ? xn[xb][t] : u32x4{0u, 0u, 0u, 0u};
  };

  // Every load is issued unconditionally, with its step clamped to the last one (the
  // surplus loads near the end re-read that step and are never consumed), and the main loop
  // runs whole unrolled trips only: with loads under branches, or loop back edges from
  // several points, the compiler cannot count how many loads are younger than the one it
  // needs and waits for all of them, which would expose the full load latency every step.
  // The prologue issues its loads in the steady state's order for the same reason.
  const int last = nsteps - 1;
  load_x(0, 0);
#pragma unroll
  for (int a = 1; a < kNX; ++a) load_x(a, min(a, last));
  load_d(0, 0);
  if constexpr (kDepth >= 2) load_d(1, min(1, last));
  stash(0, 0);
  load_x(0, min(kNX, last));  // X(kXA - 1) into the buffer just stashed
#pragma unroll
  for (int d = 2; d < kDepth; ++d) load_d(d, min(d, last));
  lds_barrier();

  auto step = [&](int cur, int d) {
    // Keep the scheduler from hoisting work on later ring slots (their sign flips) into this
    // step, which would wait for those slots' loads here.
    __builtin_amdgcn_sched_barrier(0);
    const int buf = cur & 1;
    const int rs = d % kDepth;
    // With one step in flight the next load is issued before this step's MFMAs (from a
    // copy of the ring slot); with two or more it is issued after them, which saves the
    // copy's registers while the other slots keep HBM busy.
    u32x4 dc[kDepth == 1 ? kMR : 1][kSl];
    if constexpr (kDepth == 1) {
#pragma unroll
      for (int mr = 0; mr < kMR; ++mr)
#pragma unroll
        for (int s = 0; s < kSl; ++s) dc[mr][s] = ring[0][mr][s];
      load_d(0, min(cur + 1, last));
    }
#pragma unroll
    for (int s = 0; s < kSl; ++s) {
      v4i xf[2][kPl];
#pragma unroll
      for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int b = 0; b < kPl; ++b)
          xf[qb][b] = *reinterpret_cast<const v4i*>(&xs[buf][b * 32 + 16 * qb + r][16 * g + 64 * s]);
#pragma unroll
      for (int mr = 0; mr < kMR; ++mr) {
        u32x4 v = kDepth == 1 ? dc[kDepth == 1 ? mr : 0][s] : ring[rs][mr][s];
        v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
        const v4i a = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
          for (int b = 0; b < kPl; ++b)
            acc[mr][qb][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, xf[qb][b], acc[mr][qb][b], 0, 0, 0);
      }
    }
    // the other LDS buffer was last read in the previous step, before its barrier; after the
    // final step this stash writes surplus data that nothing reads
    stash((d + 1) % kNX, buf ^ 1);
    load_x((d + kXA) % kNX, min(cur + kXA, last));
    if constexpr (kDepth > 1) load_d(rs, min(cur + kDepth, last));
    lds_barrier();
  };
  int st = 0;
  for (; st + kU <= nsteps; st += kU) {
#pragma unroll
    for (int d = 0; d < kU; ++d) step(st + d, d);
  }
#pragma unroll
  for (int d = 0; d < kU - 1; ++d) {
    if (st + d >= nsteps) break;
    step(st + d, d);
  }

  const bool first = kz == 0;
  if constexpr (kWide) {
#pragma unroll
    for (int mr = 0; mr < kMR; ++mr)
#pragma unroll
      for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int b = 0; b < kPl; ++b) {
          const int c = cblk + 32 * b + 16 * qb + r;
          if (c >= ncol) continue;
          const uint32_t cs = first ? 128u * (uint32_t)colsum[c] : 0u;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int orow = rowblk + 16 * kMR * wave + 16 * mr + 4 * g + i;
            if (orow >= rows) continue;
            const uint32_t rterm = first ? 128u * (uint32_t)rowsum[orow] + 16384u * (uint32_t)cols : 0u;
            const uint32_t v = (uint32_t)acc[mr][qb][b][i] + cs + rterm;
            uint32_t* o = out_rowmajor ? out + (size_t)orow * ncol + c : out + (size_t)c * out_ld + orow;
            if (nkz == 1) *o = v; else atomicAdd(o, v);
          }
        }
    return;
  }
#pragma unroll
  for (int mr = 0; mr < kMR; ++mr)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const int c = cblk + 16 * qb + r;
      if (c >= ncol) continue;
      uint32_t cs[kPl];
#pragma unroll
      for (int b = 0; b < kPl; ++b) cs[b] = first ? 128u * (uint32_t)colsum[c * kPl + b] : 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int orow = rowblk + 16 * kMR * wave + 16 * mr + 4 * g + i;
        if (orow >= rows) continue;
        const uint32_t rterm = first ? 128u * (uint32_t)rowsum[orow] + 16384u * (uint32_t)cols : 0u;
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < kPl; ++b) v += ((uint32_t)acc[mr][qb][b][i] + cs[b] + rterm) << (8 * b);
        uint32_t* o = out_rowmajor ? out + (size_t)orow * ncol + c : out + (size_t)c * out_ld + orow;
        if (nkz == 1) *o = v; else atomicAdd(o, v);
      }
    }
}

#define ZP_GEMM_ARGS                                                                              \
  const uint8_t* __restrict__ D, int rows, int cols, int pitch, const int8_t* __restrict__ Xs,     \
      const int32_t* __restrict__ colsum, int ncol, const int32_t* __restrict__ rowsum,            \
      uint32_t* __restrict__ out, int out_rowmajor, long long out_ld, int ksteps_per_block,        \
      int nrb, int ncb, int nkz
#define ZP_GEMM_PASS D, rows, cols, pitch, Xs, colsum, ncol, rowsum, out, out_rowmajor, out_ld, \
                     ksteps_per_block, nrb, ncb, nkz

template <int kW, int kDepth, int kMR, int kKB, int kPl, bool kWide, bool kTiled = false>
__global__ __launch_bounds__(64 * kW) void gemm_planes_kernel(ZP_GEMM_ARGS) {
  gemm_planes_body<kW, kDepth, kMR, kKB, kPl, kWide, kTiled>(ZP_GEMM_PASS);
}

// Four row tiles per wave need more than half the register file: at most two waves per SIMD.
template <int kW, int kDepth, int kMR, int kKB, int kPl, bool kWide, bool kTiled = false>
__global__ __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(1, 2)))
void gemm_planes_kernel_wide_regs(ZP_GEMM_ARGS) {
  gemm_planes_body<kW, kDepth, kMR, kKB, kPl, kWide, kTiled>(ZP_GEMM_PASS);
}

// Dt[(j / 16) 16 pitch + (i / 64) 1024 + (j mod 16) 64 + i mod 64] = D[j pitch + i] for the listed
// rows j (rowlist == nullptr: rows 0 .. nrows-1); pitch is a multiple of 64.  One thread per
// 16 bytes.
__global__ void tile_rows_kernel(const uint8_t* __restrict__ D, int pitch, const uint32_t* __restrict__ rowlist,
                                 int nrows, uint8_t* __restrict__ Dt) {
  const long long per_row = pitch / 16;
  const long long n = (long long)nrows * per_row;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long li = i / per_row;
    const long long j = rowlist ? (long long)rowlist[li] : li;
    const int k = (int)(i - li * per_row) * 16;
    const u32x4 v = *reinterpret_cast<const u32x4*>(D + j * pitch + k);
    *reinterpret_cast<u32x4*>(Dt + (j >> 4) * 16LL * pitch + (long long)(k >> 6) * 1024 + (j & 15) * 64 + (k & 63)) = v;
  }
}

void launch_tile_rows(const uint8_t* D, int pitch, const uint32_t* rowlist, int nrows, uint8_t* Dt,
                      hipStream_t s) {
  if (nrows <= 0) return;
  const long long n = (long long)nrows * (pitch / 16);
  const int blocks = (int)std::min<long long>(8192, (n + 255) / 256);
  tile_rows_kernel<<<blocks, 256, 0, s>>>(D, pitch, rowlist, nrows, Dt);
}

// Clears the rows x ncol output block: out[j*ncol + c] (row-major) or out[c*ld + j].
__global__ void zero_out_kernel(uint32_t* __restrict__ p, int rows, int ncol, int rowmajor,
                                long long ld) {
  const long long n = (long long)rows * ncol;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (rowmajor) {
      p[i] = 0u;
    } else {
      const long long c = i / rows, j = i - c * rows;
      p[c * ld + j] = 0u;
    }
  }
}

// compare == 0: ref[c*rows + j] = element (j, c) of the output block (a snapshot);
// compare == 1: adds the number of elements that differ from the snapshot to *mism.
__global__ void gemm_snapshot_kernel(const uint32_t* __restrict__ out, int rows, int ncol,
                                     int rowmajor, long long ld, uint32_t* __restrict__ ref,
                                     int compare, unsigned* __restrict__ mism) {
  const long long n = (long long)rows * ncol;
  unsigned bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long c = i / rows, j = i - c * rows;
    const uint32_t v = rowmajor ? out[j * ncol + c] : out[c * ld + j];
    if (compare) bad += v != ref[i] ? 1u : 0u;
    else ref[i] = v;
  }
  if (compare && bad) atomicAdd(mism, bad);
}

void launch_gemm_snapshot(const uint32_t* out, int rows, int ncol, bool out_rowmajor,
                          long long out_ld, uint32_t* ref, bool compare, unsigned* mism,
                          hipStream_t s) {
  if ((long long)rows * ncol == 0) return;
  gemm_snapshot_kernel<<<1024, 256, 0, s>>>(out, rows, ncol, out_rowmajor ? 1 : 0, out_ld, ref,
                                            compare ? 1 : 0, mism);
}

bool gemm_shape_valid(const GemmShape& sh, int pitch, int planes) {
  const bool base = (sh.waves == 8 && sh.depth == 1 && sh.mr == 2 && sh.kb == 256) ||
                    (sh.waves == 8 && sh.depth == 2 && sh.mr == 2 && sh.kb == 256) ||
                    (sh.waves == 8 && sh.depth == 3 && sh.mr == 2 && sh.kb == 256) ||
                    (sh.waves == 8 && sh.depth == 1 && sh.mr == 1 && sh.kb == 256) ||
                    (sh.waves == 4 && sh.depth == 1 && sh.mr == 2 && sh.kb == 256) ||
                    (sh.waves == 4 && sh.depth == 4 && sh.mr == 2 && sh.kb == 256) ||
                    (sh.waves == 4 && sh.depth == 1 && sh.mr == 2 && sh.kb == 512);
  const bool mr4 = (sh.waves == 8 || sh.waves == 4) && sh.mr == 4 && sh.kb == 256 &&
                   (sh.depth == 2 || (planes == 1 && sh.depth == 1));
  // one plane, all nine 32-vector groups of a 260-column offset operand in one block
  const bool wide9 = planes == 1 && sh.cg == 9 && sh.mr == 2 && sh.depth >= 2 && sh.depth <= 4 &&
                     ((sh.waves == 4 && sh.kb == 128) || (sh.waves == 2 && sh.kb == 64));
  if (wide9) return sh.ksplit >= 1 && pitch % sh.kb == 0;
  const bool known = base || (planes == 4 && sh.waves == 2 && sh.depth == 2 && sh.mr == 2 && sh.kb == 256) || mr4;
  if (!known || sh.ksplit < 1) return false;
  if (planes == 1 && (sh.cg < 2 || sh.cg > 4)) return false;
  if (planes != 1 && planes != 4) return false;
  return pitch % sh.kb == 0;
}

void launch_gemm_planes(const uint8_t* D, int rows, int cols, int pitch, int planes,
                        const int8_t* Xs, const int32_t* colsum, int ncol, const int32_t* rowsum,
                        uint32_t* out, bool out_rowmajor, long long out_ld, const GemmShape& sh_in,
                        hipStream_t s, bool tiled) {
  if (tiled && planes != 4) return;  // the tiled copy serves the four-plane contraction only
  GemmShape sh = sh_in;
  if (!gemm_shape_valid(sh, pitch, planes))
    sh = planes == 4 ? GemmShape{8, 1, 2, 256, 2, 4} : GemmShape{8, 1, 2, 256, 1, 3};
  const int nsteps = pitch / sh.kb;
  const int per = std::min(kMaxBlockK / sh.kb, (nsteps + sh.ksplit - 1) / sh.ksplit);
  const int nkz = (nsteps + per - 1) / per;
  if (nkz > 1) zero_out_kernel<<<1024, 256, 0, s>>>(out, rows, ncol, out_rowmajor ? 1 : 0, out_ld);
  const int rows_per_block = 16 * sh.mr * sh.waves;
  const int nrb = (rows + rows_per_block - 1) / rows_per_block;
  const int cols_per_block = planes == 4 ? kBC : kBC * sh.cg;
  const int ncb = (ncol + cols_per_block - 1) / cols_per_block;
  const long long nblocks = (long long)((nrb + 7) / 8 * 8) * ncb * nkz;
  const dim3 grid((unsigned)nblocks);
#define ZP_LAUNCHT(W, DP, MR, KB, PL, WIDE, TL)                                                     \
  if constexpr (MR >= 4)                                                                            \
    gemm_planes_kernel_wide_regs<W, DP, MR, KB, PL, WIDE, TL><<<grid, 64 * W, 0, s>>>(               \
        D, rows, cols, pitch, Xs, colsum, ncol, rowsum, out, out_rowmajor, out_ld, per, nrb, ncb, nkz); \
  else                                                                                              \
    gemm_planes_kernel<W, DP, MR, KB, PL, WIDE, TL><<<grid, 64 * W, 0, s>>>(                         \
        D, rows, cols, pitch, Xs, colsum, ncol, rowsum, out, out_rowmajor, out_ld, per, nrb, ncb, nkz)
#define ZP_LAUNCH(W, DP, MR, KB, PL, WIDE) ZP_LAUNCHT(W, DP, MR, KB, PL, WIDE, false)
#define ZP_LAUNCH4(W, DP, MR, KB)                                                                   \
  do {                                                                                              \
    if (tiled) ZP_LAUNCHT(W, DP, MR, KB, 4, false, true);                                           \
    else ZP_LAUNCHT(W, DP, MR, KB, 4, false, false);                                                \
  } while (0)
#define ZP_G(W, DP, MR, KB)                                                                         \
  if (sh.waves == W && sh.depth == DP && sh.mr == MR && sh.kb == KB) {                              \
    if (planes == 4) ZP_LAUNCH4(W, DP, MR, KB);                                                     \
    else if (sh.cg == 2) ZP_LAUNCH(W, DP, MR, KB, 2, true);                                         \
    else if (sh.cg == 3) ZP_LAUNCH(W, DP, MR, KB, 3, true);                                         \
    else ZP_LAUNCH(W, DP, MR, KB, 4, true);                                                         \
    return;                                                                                         \
  }
  ZP_G(8, 1, 2, 256) ZP_G(8, 2, 2, 256) ZP_G(8, 3, 2, 256) ZP_G(8, 1, 1, 256) ZP_G(4, 1, 2, 256)
  ZP_G(4, 4, 2, 256) ZP_G(4, 1, 2, 512)
  if (planes == 1 && sh.cg == 9 && sh.waves == 4) {
    if (sh.depth == 2) ZP_LAUNCH(4, 2, 2, 128, 9, true);
    else if (sh.depth == 3) ZP_LAUNCH(4, 3, 2, 128, 9, true);
    else ZP_LAUNCH(4, 4, 2, 128, 9, true);
    return;
  }
  if (planes == 1 && sh.cg == 9 && sh.waves == 2) {
    if (sh.depth == 2) ZP_LAUNCH(2, 2, 2, 64, 9, true);
    else if (sh.depth == 3) ZP_LAUNCH(2, 3, 2, 64, 9, true);
    else ZP_LAUNCH(2, 4, 2, 64, 9, true);
    return;
  }
#define ZP_W(W, DP, MR, KB)                                                                         \
  if (planes == 1 && sh.waves == W && sh.depth == DP && sh.mr == MR && sh.kb == KB) {               \
    if (sh.cg == 2) ZP_LAUNCH(W, DP, MR, KB, 2, true);                                              \
    else if (sh.cg == 3) ZP_LAUNCH(W, DP, MR, KB, 3, true);                                         \
    else ZP_LAUNCH(W, DP, MR, KB, 4, true);                                                         \
    return;                                                                                         \
  }
  ZP_W(8, 1, 4, 256) ZP_W(4, 1, 4, 256)
#undef ZP_W
  ZP_G(8, 2, 4, 256) ZP_G(4, 2, 4, 256)
#undef ZP_G
  if (sh.waves == 2 && sh.depth == 2 && sh.mr == 2 && sh.kb == 256 && planes == 4) {
    ZP_LAUNCH4(2, 2, 2, 256);
    return;
  }
#undef ZP_LAUNCH4
#undef ZP_LAUNCH
#undef ZP_LAUNCHT
}

}  // namespace zp
