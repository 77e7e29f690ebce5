// Batched online answer B = D.Q mod 2^32 for many clients' queries at once (Alg. 5, Response,
// first line, over a batch; D is shared by every client, Sec. 4.3 "Reusability of the offline
// phase"), as one fused, persistent launch on int8 MFMA.
//
// Byte planes: with Q_b = byte b of Q,  D.Q = sum_b 2^(8b) (D . Q_b) mod 2^32, and with the
// shift to signed bytes D' = D - 128, Q_b' = Q_b - 128 (XOR 0x80),
//   D.Q_b = D'.Q_b' + 128 sum_i Q_b'[i] + 128 sum_i D'[i] + 16384 cols      (exact).
// Everything else of the batched path happens inside the one launch: each workgroup reads the
// raw uint32 queries of its K step, splits them into the four signed planes in registers (a
// 4 x 4 byte transpose by v_perm), stages them in LDS in MFMA fragment order, and keeps the
// column sums of the planes (v_dot4) for its epilogue; there is no packing launch, no plane
// buffer in HBM and no clearing of the output.  The grid is persistent: a workgroup takes work
// items (row block, 32-query column group, K range) in turn.
//
// D is read from the tiled copy (16-row x 64-byte pieces, each 16-row group contiguous over its
// K range), so a wavefront's load of one A fragment (16 rows x 64 bytes) is one contiguous
// kilobyte and each wavefront streams MR contiguous runs.
#include <algorithm>

#include "internal.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ void lds_fence_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Four words w0..w3 to the four byte planes: out[b] holds byte b of w0, w1, w2, w3 (in that
// order, from the low byte), by a 4 x 4 byte transpose in eight byte permutes.
__device__ __forceinline__ void planes4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t (&out)[4]) {
  const uint32_t t0 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);  // w0.0 w1.0 w0.1 w1.1
  const uint32_t t1 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);  // w0.2 w1.2 w0.3 w1.3
  const uint32_t t2 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);  // w2.0 w3.0 w2.1 w3.1
  const uint32_t t3 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);  // w2.2 w3.2 w2.3 w3.3
  out[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
  out[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
  out[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
  out[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

}  // namespace

constexpr int kBatchQG = 32;     // queries per column group: two 16-query tiles x four planes
constexpr int kBatchKStep = 128; // K bytes per step: two 64-byte MFMA slices

// Work item geometry shared by the kernel and its launcher.
struct BatchGrid {
  int nrb, ncg, nkz, steps_per_range, nitems;
};

// kVec: every query row starts 16-byte aligned and cols is a multiple of 16, so a thread's 16
// query entries are four aligned 16-byte loads (otherwise entries are loaded one by one and
// those at or beyond cols read as zero).
template <int MR, int kDE, bool kVec>
__global__ __launch_bounds__(256) void batch_answer_kernel(const uint8_t* __restrict__ Dt, int rows, int cols,
                                                           int pitch, const uint32_t* __restrict__ Q, int batch,
                                                           const int32_t* __restrict__ rowsum,
                                                           uint32_t* __restrict__ B, long long ldb, BatchGrid gd) {
  constexpr int kTiles = 8;                       // (query tile qb, plane b) = 2 x 4
  constexpr int kStepBytes = 2 * kTiles * 1024;   // one K step of X in LDS
  constexpr int kOutWords = kBatchQG * 16 * MR;   // one wavefront's output tile
  static_assert(4 * kOutWords * 4 <= 2 * kStepBytes, "the epilogue reuses the X buffers");
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kStepBytes];
  __shared__ int32_t csl[kBatchQG][4];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, r = lane & 15;
  // the X producer role of this thread: query xc of the group, 16 K entries from 16 xs
  const int xc = tid >> 3, xs = tid & 7;
  const int xsl = xs >> 2, xg = xs & 3;
  const int ngroups = (rows + 15) / 16;

  for (int item = blockIdx.x; item < gd.nitems; item += gridDim.x) {
    const int cg = item % gd.ncg;
    const int kz = (item / gd.ncg) % gd.nkz;
    const int rb = item / (gd.ncg * gd.nkz);
    const int step0 = kz * gd.steps_per_range;
    const int nsteps = min(gd.steps_per_range, pitch / kBatchKStep - step0);
    const int q = cg * kBatchQG + xc;  // this thread's query as X producer
    const bool qlive = q < batch;
    const uint32_t* qrow = Q + (size_t)min(q, batch - 1) * cols;

    // A streams: tile i of this wavefront is the 16-row group T; lane (g, r) reads row r,
    // bytes 16 g .. 16 g + 15 of each 64-byte piece
    const uint8_t* ap[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const int T = min((rb * 4 + wave) * MR + i, ngroups - 1);
      ap[i] = Dt + (size_t)T * 16 * pitch + (size_t)step0 * 2 * 1024 + r * 64 + 16 * g;
    }

    v4i acc[MR][kTiles];
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int t = 0; t < kTiles; ++t) acc[i][t] = v4i{0, 0, 0, 0};
    int32_t csum[4] = {0, 0, 0, 0};

    u32x4 ra[kDE][MR][2];
    uint32_t xr[16];
    const int last = nsteps - 1;
    auto load_a = [&](int slot_, int st) {
#pragma unroll
      for (int i = 0; i < MR; ++i)
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
          ra[slot_][i][sl] =
              __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(ap[i] + (size_t)st * 2048 + sl * 1024));
    };
    auto load_x = [&](int st) {
      const int k0 = (step0 + st) * kBatchKStep + 16 * xs;
      if constexpr (kVec) {
        const u32x4* p = reinterpret_cast<const u32x4*>(qrow + min(k0, cols - 16));
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const u32x4 v = p[m];
          xr[4 * m] = v.x; xr[4 * m + 1] = v.y; xr[4 * m + 2] = v.z; xr[4 * m + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) xr[u] = k0 + u < cols ? qrow[k0 + u] : 0u;
      }
    };
    // the planes of the loaded entries into LDS buffer buf (zero for a query beyond the batch or
    // entries at or beyond cols, which count for nothing in the column sums either)
    auto stash = [&](int buf, int st) {
      const int k0 = (step0 + st) * kBatchKStep + 16 * xs;
      const bool live = qlive && st <= last && k0 < cols;
      uint32_t pl[4][4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        uint32_t o[4];
        planes4(xr[4 * m], xr[4 * m + 1], xr[4 * m + 2], xr[4 * m + 3], o);
#pragma unroll
        for (int b = 0; b < 4; ++b) pl[b][m] = o[b];
      }
      // entries at or beyond cols must contribute the shifted zero (0 before XOR)
      const int nval = cols - k0;  // entries of this thread's 16 that lie below cols
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        uint32_t keep = 0xFFFFFFFFu;
        if (!kVec) {
          const int v = nval - 4 * m;
          keep = v >= 4 ? 0xFFFFFFFFu : v <= 0 ? 0u : (0xFFFFFFFFu >> (8 * (4 - v)));
        }
        if (!live) keep = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t sv = (pl[b][m] ^ 0x80808080u) & keep;
          pl[b][m] = sv;
          csum[b] = __builtin_amdgcn_sdot4((int)sv, 0x01010101, csum[b], false);
        }
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int tile = (xc >> 4) * 4 + b;
        *reinterpret_cast<u32x4*>(lds + buf * kStepBytes + ((xsl * kTiles + tile) * 64 + xg * 16 + (xc & 15)) * 16) =
            u32x4{pl[b][0], pl[b][1], pl[b][2], pl[b][3]};
      }
    };

    // prologue: X(0) into buffer 0, X(1) in registers, A(0 .. kDE - 1) in flight
    load_x(0);
#pragma unroll
    for (int d = 0; d < kDE; ++d) load_a(d, min(d, last));
    stash(0, 0);
    load_x(min(1, last));
    lds_fence_barrier();

    auto step = [&](int cur, int d) {
      __builtin_amdgcn_sched_barrier(0);
      const uint8_t* xb = lds + (cur & 1) * kStepBytes + lane * 16;
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        v4i bf[kTiles];
#pragma unroll
        for (int t = 0; t < kTiles; ++t) bf[t] = *reinterpret_cast<const v4i*>(xb + (sl * kTiles + t) * 1024);
#pragma unroll
        for (int i = 0; i < MR; ++i) {
          u32x4 v = ra[d][i][sl];
          v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
          const v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
          for (int t = 0; t < kTiles; ++t)
            acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[t], acc[i][t], 0, 0, 0);
        }
      }
      // the other buffer was last read in the previous step, before its barrier; past the last
      // step the stash writes zeros that nothing reads
      stash((cur + 1) & 1, cur + 1);
      load_x(min(cur + 2, last));
      load_a(d, min(cur + kDE, last));
      lds_fence_barrier();
    };
    // whole trips only: a step past the last multiplies a zero X tile (its stash wrote zeros)
    // and adds nothing, while its loads re-read the last step
    for (int st = 0; st < nsteps; st += kDE) {
#pragma unroll
      for (int d = 0; d < kDE; ++d) step(st + d, d);
    }

    // column sums of this item's K range: the eight producers of a query are adjacent lanes
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int32_t v = csum[b];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      if (xs == 0) csl[xc][b] = v;
    }
    lds_fence_barrier();

    // epilogue: combine the planes in registers, transpose through LDS so that each query's rows
    // are stored contiguously (atomic adds when the K range is split)
    uint32_t* ol = reinterpret_cast<uint32_t*>(lds) + wave * kOutWords;
    const bool first = kz == 0;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int lr = 16 * i + 4 * g + e;  // row within the wavefront's tile
        const int row = min(((rb * 4 + wave) * MR) * 16 + lr, rows - 1);
        const uint32_t rterm = first ? 128u * (uint32_t)rowsum[row] + 16384u * (uint32_t)cols : 0u;
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
          const int c = 16 * qb + r;
          uint32_t v = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b)
            v += ((uint32_t)acc[i][qb * 4 + b][e] + 128u * (uint32_t)csl[c][b] + rterm) << (8 * b);
          ol[c * (16 * MR) + lr] = v;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const int rowbase = ((rb * 4 + wave) * MR) * 16;
#pragma unroll
    for (int it = 0; it < kOutWords / 64; ++it) {
      const int idx = it * 64 + lane;
      const int c = idx / (16 * MR), lr = idx % (16 * MR);
      const int qq = cg * kBatchQG + c;
      const int row = rowbase + lr;
      if (qq < batch && row < rows) {
        uint32_t* o = B + (size_t)qq * ldb + row;
        if (gd.nkz == 1) *o = ol[idx];
        else atomicAdd(o, ol[idx]);
      }
    }
    lds_fence_barrier();  // before the next item's prologue overwrites LDS
  }
}

bool batch_answer_supported(int rows, int pitch) {
  (void)rows;
  return pitch % kBatchKStep == 0;
}

__global__ void batch_zero_kernel(uint32_t* __restrict__ B, long long ldb, int rows, int batch) {
  const long long n = (long long)rows * batch;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long c = i / rows, j = i - c * rows;
    B[c * ldb + j] = 0u;
  }
}

void launch_batch_answer(const uint8_t* Dt, int rows, int cols, int pitch, const uint32_t* Q, int batch,
                         const int32_t* rowsum, uint32_t* B, long long ldb, const BatchShape& sh,
                         int num_cus, hipStream_t s) {
  if (rows <= 0 || batch <= 0) return;
  const int MR = sh.mr;
  const int rows_per_block = 64 * MR;
  BatchGrid gd;
  gd.nrb = (rows + rows_per_block - 1) / rows_per_block;
  gd.ncg = (batch + kBatchQG - 1) / kBatchQG;
  const int steps = pitch / kBatchKStep;
  // split K only when row blocks and column groups leave CUs idle
  const int base = gd.nrb * gd.ncg;
  gd.nkz = std::max(1, std::min(sh.ksplit, steps));
  if (sh.ksplit == 0) gd.nkz = std::max(1, std::min(steps, (num_cus + base - 1) / base));
  gd.steps_per_range = (steps + gd.nkz - 1) / gd.nkz;
  gd.nkz = (steps + gd.steps_per_range - 1) / gd.steps_per_range;
  gd.nitems = base * gd.nkz;
  if (gd.nkz > 1) batch_zero_kernel<<<1024, 256, 0, s>>>(B, ldb, rows, batch);
  const int grid = std::max(1, std::min(gd.nitems, num_cus * sh.blocks_per_cu));
  const bool vec = cols % 16 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
#define ZP_BATCH(M, DE)                                                                                        \
  if (vec) batch_answer_kernel<M, DE, true><<<grid, 256, 0, s>>>(Dt, rows, cols, pitch, Q, batch, rowsum, B, ldb, gd); \
  else batch_answer_kernel<M, DE, false><<<grid, 256, 0, s>>>(Dt, rows, cols, pitch, Q, batch, rowsum, B, ldb, gd)
  if (MR == 1) {
    if (sh.depth <= 2) { ZP_BATCH(1, 2); } else if (sh.depth == 3) { ZP_BATCH(1, 3); } else { ZP_BATCH(1, 4); }
  } else {
    if (sh.depth <= 2) { ZP_BATCH(2, 2); } else if (sh.depth == 3) { ZP_BATCH(2, 3); } else { ZP_BATCH(2, 4); }
  }
#undef ZP_BATCH
}

}  // namespace zp
