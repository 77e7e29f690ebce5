// Online offset answer of the full protocol (Alg. 5, Response, second line):
//   t_j = (b_j + sum_k E_jk ck_o,k) mod N,   E = (-H) mod 2^32,  ck_o,k < 2^(32 h),
// the product of the shared hint matrix with one client's vector of big integers.
//
// The paper evaluates it in an RNS basis of small primes so that a CPU can use machine
// words (Sec. 4.3, "Faster matrix multiplication using RNS").  Here it is one exact integer
// contraction on int8 MFMA instead: write E_jk = sum_a 2^(8a) e_jk[a] and
// ck_o,k = sum_c 2^(8c) y_k[c] by bytes; then
//   sum_k E_jk ck_o,k = sum_pos 2^(8 pos) W[j][pos],
//   W[j][pos] = sum_{k, a} e_jk[a] y_k[pos - a]          (0 <= pos - a < 4h),
// i.e. four uint8 products, one per byte plane a of E, each with the n x 4h matrix of the
// offsets' bytes, added with shifts of a byte position.  Every W entry is below 4n 255^2 < 2^32,
// so the contraction is exact in 32-bit accumulators.  The offsets are first replaced by
// y_k = ck_o,k 2^96 mod N, so that a reduction kernel can fold the byte positions into limbs,
// add b_j 2^96 and finish modulo N with three Montgomery reduction steps (see below).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "rownum.h"
#include "stage.h"
#include "wavenum.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- operands of the offset contraction
//
// The contraction runs on v_mfma_i32_16x16x64_i8 over K' = 4 kpad entries, E's four byte planes
// laid end to end along K (plane a, entries k).  With the offsets' bytes shifted by one position
// per plane,
//   Y4[pos][(a, k)] = byte pos - a of y_k   (0 where pos - a is outside [0, 4h)),
// the four shifted plane products become one:
//   W[j][pos] = sum_{(a, k)} e_jk[a] Y4[pos][(a, k)],   pos < 4h + 3,
// so the accumulators hold W itself and nothing is added across planes afterwards.  The shifted
// copies are never stored: the B fragment of plane a is the unshifted one read a columns to the
// left, so each 64-entry slice of K stages Y once and serves all four planes.
// Both operands are int8 (XOR 0x80; padding 0) in MFMA fragment order:
//   Ep (E planes): piece (T, a, s) is 1 KiB, lane l's 16 bytes at 16 l hold
//     E'_a[16 T + l mod 16][64 s + 16 (l / 16) + u], u < 16; the pieces of eight consecutive
//     row tiles (one row block of the contraction) are ordered by slice, then plane, then tile:
//     piece (T, a, s) is number ((T / 8) S + s) 32 + 8 a + T mod 8, so a row block streams one
//     contiguous 32 KiB run per slice;
//   Yc (one client's offset bytes): per slice s, NTq + 1 pieces of 16 columns, piece u holding
//     columns c = 16 u - 16 ... 16 u - 1 (piece 0 is the zero padding left of column 0).  In a
//     piece, column c's 64 bytes Y'[c][64 s ...] sit at 64 (c mod 16), as four 16-byte runs
//     whose order is swizzled by bits 2-3 of the column: run g at 16 (g ^ ((c / 4) mod 4)).
//     Reading the 16 columns of a fragment then touches 16 distinct 16-byte bank groups.
// Entries beyond rows, n or 4h are 0 (the value 128 before the shift), which adds nothing to the
// signed product; the shift terms below count only the real entries.

// One thread per (tile, slice, lane): reads 16 entries of H once and writes the four planes.
__global__ __launch_bounds__(256) void e_planes_kernel(const uint32_t* __restrict__ H, int rows, int n,
                                                       int S, long long pieces, u32x4* __restrict__ Ep) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= pieces) return;  // pieces = tiles * S * 64
  const int l = (int)(p & 63);
  const long long q = p >> 6;
  const int s = (int)(q % S);
  const long long T = q / S;
  const long long row = 16 * T + (l & 15);
  const int k0 = 64 * s + 16 * (l >> 4);
  uint32_t w[4][4] = {};
  if (row < rows) {
    const uint32_t* hr = H + row * n;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + u;
      const uint32_t e = k < n ? 0u - hr[k] : 0u;
      // byte a of e, shifted (0 for padding, which the XOR below turns back into 0)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const uint32_t sb = k < n ? (((e >> (8 * a)) & 0xFFu) ^ 0x80u) : 0u;
        w[a][u >> 2] |= sb << (8 * (u & 3));
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
    Ep[(((T >> 3) * S + s) * 32 + 8 * a + (T & 7)) * 64 + l] = u32x4{w[a][0], w[a][1], w[a][2], w[a][3]};
}

// Ers[a * rows_pad + j] = sum_{k<n} (byte a of E_jk) - 128: one wavefront per row.
__global__ __launch_bounds__(256) void e_plane_sums_kernel(const uint32_t* __restrict__ H, int rows, int n,
                                                           int rows_pad, int32_t* __restrict__ Ers) {
  const int j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (j >= rows) return;
  const int lane = threadIdx.x & 63;
  int32_t sum[4] = {0, 0, 0, 0};
  for (int k = lane; k < n; k += 64) {
    const uint32_t e = 0u - H[(size_t)j * n + k];
#pragma unroll
    for (int a = 0; a < 4; ++a) sum[a] += (int32_t)((e >> (8 * a)) & 0xFFu) - 128;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int32_t v = sum[a];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) Ers[(size_t)a * rows_pad + j] = v;
  }
}

void launch_e_planes(const uint32_t* H, int rows, int n, int rows_pad, uint8_t* Ep, int32_t* Ers,
                     hipStream_t s) {
  const int S = offset_slices(n);
  const long long pieces = (long long)(rows_pad / 16) * S * 64;
  e_planes_kernel<<<(unsigned)((pieces + 255) / 256), 256, 0, s>>>(H, rows, n, S, pieces,
                                                                   reinterpret_cast<u32x4*>(Ep));
  e_plane_sums_kernel<<<(rows + 3) / 4, 256, 0, s>>>(H, rows, n, rows_pad, Ers);
}

// K slices of 64 entries, padded to a multiple of 4 (the contraction's loop runs whole trips of
// its slices in flight; the padding slices are zero and add nothing)
int offset_slices(int n) { return ((n + 63) / 64 + 3) / 4 * 4; }

// Column tiles of the contraction: the 4h + 3 output positions in tiles of 16, in column groups
// of offset_group(h) tiles (a multiple of 4, at most 20: the width that pads least, the wider
// on a tie), padded to whole groups.
int offset_group(int h) {
  const int nt = (4 * h + 3 + 15) / 16;
  int best = 4, pad = 1 << 30;
  for (int bc = 4; bc <= 20; bc += 4) {
    const int tiles = (nt + bc - 1) / bc * bc;
    if (tiles <= pad) {
      pad = tiles;
      best = bc;
    }
  }
  return best;
}

int offset_tiles(int h) {
  const int nt = (4 * h + 3 + 15) / 16, bc = offset_group(h);
  return (nt + bc - 1) / bc * bc;
}

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// One thread per 16-byte run (s, u, l) of client blockIdx.y: lane l of piece u holds column
// c = 16 u + l / 4 - 16, run g = (l mod 4) ^ ((l / 16) mod 4).  colsum[i 16 NTq + c] (zeroed
// first) = sum_{k<n} (byte c of y_k) - 128 for c < 4h: the four lanes of a column hold the
// slice's 64 entries, one atomic per column and slice.
__global__ __launch_bounds__(256) void pack_y_kernel(const uint32_t* __restrict__ ys, int n, int h, int S,
                                                     int NTq, u32x4* __restrict__ Yc,
                                                     int32_t* __restrict__ colsum) {
  const int i = blockIdx.y;
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long per = (long long)S * (NTq + 1) * 64;
  const bool live = p < per;
  const int l = (int)(p & 63);
  const long long q = p >> 6;
  const int u = (int)(q % (NTq + 1));
  const int s = (int)(q / (NTq + 1));
  const int c = 16 * u + (l >> 2) - 16;
  const int g = (l & 3) ^ ((l >> 4) & 3);
  const int k0 = 64 * s + 16 * g;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  int32_t part = 0;
  if (live && c >= 0 && c < 4 * h) {
    const uint32_t* y = ys + (size_t)i * n * h + (c >> 2);
    const int sh = 8 * (c & 3);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int k = k0 + v;
      if (k < n) {
        const uint32_t sb = ((y[(size_t)k * h] >> sh) & 0xFFu) ^ 0x80u;
        w[v >> 2] |= sb << (8 * (v & 3));
        part += (int32_t)(int8_t)sb;
      }
    }
  }
  if (live) Yc[(size_t)i * per + p] = u32x4{w[0], w[1], w[2], w[3]};
  part += __shfl_xor(part, 1, 64);
  part += __shfl_xor(part, 2, 64);
  if (live && (l & 3) == 0 && c >= 0 && c < 4 * h && part != 0) atomicAdd(colsum + (size_t)i * 16 * NTq + c, part);
}

void launch_pack_y(const uint32_t* ys, int batch, int n, int h, uint8_t* Yc, int32_t* colsum,
                   hipStream_t s) {
  const int S = offset_slices(n), NTq = offset_tiles(h);
  const int ncs = batch * 16 * NTq;
  zero_i32_kernel<<<(ncs + 255) / 256, 256, 0, s>>>(colsum, ncs);
  const long long per = (long long)S * (NTq + 1) * 64;
  dim3 grid((unsigned)((per + 255) / 256), batch);
  pack_y_kernel<<<grid, 256, 0, s>>>(ys, n, h, S, NTq, reinterpret_cast<u32x4*>(Yc), colsum);
}

long long offset_y_bytes(int n, int h) { return (long long)offset_slices(n) * (offset_tiles(h) + 1) * 1024; }

// A 64-bit value from another lane of the quad (DPP quad_perm C: kDppQuadXor1 takes lane i ^ 1,
// kDppQuadXor2 lane i ^ 2).
template <int C>
__device__ __forceinline__ uint64_t quad_from(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, C, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), C, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// ---- the contraction
//
// A workgroup of 2 WC wavefronts takes 128 rows (eight 16-row tiles), one column group of
// BC = WC CWV tiles and one client; wavefront (wr, wc) computes 4 x CWV accumulator tiles: row
// tiles of half wr, column tiles wc CWV ... of the group.  With WC = 2 each SIMD runs one
// wavefront with a wide tile; with WC = 4 two narrower ones, which hide each other's waits at
// the price of more LDS reads per MFMA.  Per 64-entry slice s of K, the operands pass through LDS
// in NS stages by direct global-to-LDS loads (stage.h): a stage holds the block's 32 E fragments
// (eight row tiles x four planes, each a kilobyte of Ep) and the BC + 1 pieces of Yc its columns
// need (one contiguous run); wavefront w issues the pieces w, w + 2 WC, ...  One barrier per
// slice; the four planes then run back to back on the staged slice (4 x 4 x CWV MFMAs per
// wavefront), plane a reading its B fragments a columns to the left.
// Then each accumulator becomes a W entry:
//   W = acc + 128 sum_{a in A(pos)} (colsum[pos - a] + Ers_a[j]) + 16384 n |A(pos)|,
//   A(pos) = {a < 4 : 0 <= pos - a < 4h}
// (exact modulo 2^32, and the true value is below 4 n 255^2 < 2^32 for n <= 16384), and the
// four positions of a 32-bit limb, which sit in four neighbouring lanes, are folded into one
// 64-bit word X_l = sum_u W[4l + u] 2^(8u) (below 2^57) by two DPP exchanges within the quad:
// the output holds limbs 0 .. h of each row (cpc words per client), half the bytes of W.
// The grid is XCD-aware: workgroup L runs on XCD L mod 8, and each XCD takes the (client, column
// group) items of its row blocks (x, x + 8, ...) one after the other, so a block's E stream comes
// from HBM once and from that XCD's L2 for the other items.
template <int CWV, int WC, int NS>
__global__ __launch_bounds__(128 * WC) __attribute__((amdgpu_waves_per_eu(WC / 2, WC / 2)))
void offset_gemm_kernel(const uint8_t* __restrict__ Ep, const int32_t* __restrict__ Ers, int rows_pad, int rows,
                        int n, int S, const uint8_t* __restrict__ Yc, const int32_t* __restrict__ colsum,
                        int batch, int nrb, int ncg, int NTq, int h, uint64_t* __restrict__ W, long long ldw,
                        int cpc) {
  constexpr int RW = 4, BR = 8, CW = CWV, BC = WC * CWV, NW = 2 * WC;
  constexpr int EA = 4 * BR;      // E pieces per stage: piece a BR + i is plane a of row tile i
  constexpr int YP = BC + 1;      // Yc pieces per stage
  constexpr int CH = EA + YP, PW = (CH + NW - 1) / NW, STAGE = CH * 1024;
  static_assert((NS - 2) * PW < 64 && PW >= 2, "loads per slice");
  __shared__ __attribute__((aligned(1024))) uint8_t lds[NS * STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w / WC, wc = w % WC;
  const int g = lane >> 4, r = lane & 15;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int items = batch * ncg;
  const int rb = (slot / items) * 8 + xcd;
  const int item = slot % items;
  const int ci = item / ncg, cg = item % ncg;
  if (rb >= nrb) return;
  const int T0 = rb * BR, t0 = cg * BC;

  // this wavefront's pieces of each slice: w, w + NW, ...; where that passes CH the wavefront
  // loads its previous piece once more (same bytes, same place), so that every wavefront issues
  // PW loads per slice.
  const uint8_t* src[PW];
  long long sstride[PW];
  int dst[PW];
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    const int c = w + NW * j < CH ? w + NW * j : w + NW * j - NW;
    dst[j] = c * 1024;
    if (c < EA) {  // piece c = 8 a + i of the row block's run for the slice
      src[j] = Ep + ((size_t)rb * S * 32 + c) * 1024 + lane * 16;
      sstride[j] = 32 * 1024;
    } else {
      src[j] = Yc + ((size_t)ci * S * (NTq + 1) + t0 + (c - EA)) * 1024 + lane * 16;
      sstride[j] = (long long)(NTq + 1) * 1024;
    }
  }
  auto issue = [&](int sl) {  // slice sl (clamped to the last) into its stage buffer
    const int sc = min(sl, S - 1);
    uint8_t* base = lds + (sl % NS) * STAGE;
#pragma unroll
    for (int j = 0; j < PW; ++j) g2l16(src[j] + (size_t)sc * sstride[j], base + dst[j]);
  };

  // where lane (g, r) finds its B bytes for plane a: column 16 t + r - a of the block's window
  // (window column 16 + the block's first output column), run g swizzled by that column's bits
  // 2-3 (independent of t, so tile t adds 1024 t)
  int boff[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int cw = 16 * (wc * CW) + r - a + 16;
    boff[a] = EA * 1024 + cw * 64 + ((g ^ ((cw >> 2) & 3)) << 4);
  }

  v4i acc[RW][CW];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int t = 0; t < CW; ++t) acc[i][t] = v4i{0, 0, 0, 0};

#pragma unroll
  for (int st = 0; st < NS - 1; ++st) issue(st);
  for (int s = 0; s < S; ++s) {
    wait_vmcnt<(NS - 2) * PW>();  // slice s has landed (later slices stay in flight)
    __builtin_amdgcn_s_barrier();  // ... for every wavefront; slice s - 1 is consumed
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    issue(s + NS - 1);
    const uint8_t* base = lds + (s % NS) * STAGE;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      v4i bf[CW];
#pragma unroll
      for (int t = 0; t < CW; ++t) bf[t] = *reinterpret_cast<const v4i*>(base + boff[a] + 1024 * t);
#pragma unroll
      for (int i = 0; i < RW; ++i) {
        const v4i af = *reinterpret_cast<const v4i*>(base + (a * BR + wr * RW + i) * 1024 + lane * 16);
#pragma unroll
        for (int t = 0; t < CW; ++t) acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[t], acc[i][t], 0, 0, 0);
      }
    }
  }
  wait_vmcnt<0>();  // the surplus loads past the last slice

  // epilogue: shift terms, then W entries straight from the accumulators
  const uint32_t nterm = 16384u * (uint32_t)n;
  const int npos = 4 * h + 3, nreal = 4 * h;
  const int32_t* cs = colsum + (size_t)ci * 16 * NTq;
  uint32_t cterm[CW];
  uint32_t amask[CW];  // bit a: pos - a is a real byte position
#pragma unroll
  for (int t = 0; t < CW; ++t) {
    const int pos = (t0 + wc * CW + t) * 16 + r;
    uint32_t c = 0, m = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (pos - a >= 0 && pos - a < nreal) {
        c += 128u * (uint32_t)cs[pos - a];
        m |= 1u << a;
      }
    cterm[t] = c;
    amask[t] = m;
  }
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int rowbase = (T0 + wr * RW + i) * 16 + 4 * g;
    uint32_t R[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int a = 0; a < 4; ++a)
        R[e][a] = rowbase + e < rows ? 128u * (uint32_t)Ers[(size_t)a * rows_pad + rowbase + e] + nterm : 0u;
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int pos = (t0 + wc * CW + t) * 16 + r;
      const int limb = pos >> 2;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = rowbase + e;
        uint32_t v = (uint32_t)acc[i][t][e] + cterm[t];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          if (amask[t] & (1u << a)) v += R[e][a];
        if (pos >= npos) v = 0u;
        // every lane takes part in the exchanges; only the quad's first lane stores
        uint64_t x = (uint64_t)v << (8 * (r & 3));
        x += quad_from<kDppQuadXor1>(x);
        x += quad_from<kDppQuadXor2>(x);
        if ((r & 3) == 0 && row < rows && limb <= h) W[(size_t)row * ldw + (size_t)ci * cpc + limb] = x;
      }
    }
  }
}

template <int CWV, int WC, int NS>
static void launch_offset_gemm_t(const uint8_t* Ep, const int32_t* Ers, int rows_pad, int rows, int n,
                                 const uint8_t* Yc, const int32_t* colsum, int batch, int h, uint64_t* W,
                                 long long ldw, int cpc, hipStream_t s) {
  const int S = offset_slices(n), NTq = offset_tiles(h);
  const int ncg = NTq / (WC * CWV);
  const int nrb = rows_pad / 128;  // rows_pad is a multiple of 128
  const long long nblocks = (long long)((nrb + 7) / 8 * 8) * batch * ncg;
  offset_gemm_kernel<CWV, WC, NS><<<(unsigned)nblocks, 128 * WC, 0, s>>>(Ep, Ers, rows_pad, rows, n, S, Yc, colsum,
                                                                          batch, nrb, ncg, NTq, h, W, ldw, cpc);
}

// Launch variants per column group width BC: four wavefronts of BC / 2 columns tiles or eight of
// BC / 4, each with three stages in flight, and four stages where LDS holds them (every variant
// gives identical bits; the runtime times them once per problem shape).
static bool offset_four_stages(int bc) { return 4 * (32 + bc + 1) * 1024 <= 163840; }

int offset_gemm_variants(int h) { return offset_four_stages(offset_group(h)) ? 4 : 2; }

void launch_offset_gemm(const uint8_t* Ep, const int32_t* Ers, int rows_pad, int rows, int n,
                        const uint8_t* Yc, const int32_t* colsum, int batch, int h, uint64_t* W,
                        long long ldw, int cpc, int variant, hipStream_t s) {
  const int BC = offset_group(h);
  const int v = (variant >= 0 && variant < offset_gemm_variants(h)) ? variant : 0;
  const int WC = (v & 1) ? 4 : 2, NS = v >= 2 ? 4 : 3;
#define ZP_OFF(B, C, N)                                                                                     \
  if (BC == B && WC == C && NS == N) {                                                                      \
    launch_offset_gemm_t<B / C, C, N>(Ep, Ers, rows_pad, rows, n, Yc, colsum, batch, h, W, ldw, cpc, s);     \
    return;                                                                                                 \
  }
#define ZP_OFF_B(B) ZP_OFF(B, 2, 3) ZP_OFF(B, 4, 3)
  ZP_OFF_B(4) ZP_OFF_B(8) ZP_OFF_B(12) ZP_OFF_B(16) ZP_OFF_B(20)
  ZP_OFF(4, 2, 4) ZP_OFF(4, 4, 4)
#undef ZP_OFF_B
#undef ZP_OFF
}

// The offsets enter the contraction scaled by 2^96 (mod N, which also makes them canonical):
//   y_k = ck_o,k 2^96 mod N,   v_j = b_j 2^96 + sum_k E_jk y_k  = 2^96 (b_j + sum_k E_jk ck_o,k)  (mod N).
// Three Montgomery reduction steps then give v_j 2^-96 mod N, which is t_j, and they shrink
// v_j < 2^128 + n 2^32 N to below v_j / 2^96 + N < 2N: one conditional subtraction finishes.
template <int PN>
__global__ __launch_bounds__(256) void scale_offsets_kernel(ClientDev cd, const uint32_t* __restrict__ cko,
                                                            int n, uint32_t* __restrict__ out) {
  const int k = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (k >= n) return;
  WNum<PN> Nn, c, x;
  wn_load(Nn, cd.Nn);
  wn_load(c, cd.C96);
  wn_load_n(x, cko + (size_t)k * cd.h, cd.h);
  mont_mul(x, x, c, Nn, cd.nprime);
  wn_store_n(out + (size_t)k * cd.h, x, cd.h);
}

void launch_scale_offsets(const ClientDev& cd, const uint32_t* cko, int n, uint32_t* out,
                          hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (n + 3) / 4;
  if (cd.PN == 1)
    scale_offsets_kernel<1><<<blocks, 256, 0, s>>>(cd, cko, n, out);
  else
    scale_offsets_kernel<2><<<blocks, 256, 0, s>>>(cd, cko, n, out);
}

// t_j from the folded limbs X[j][0 .. h] (X_l = sum_u W[4l + u] 2^(8u), below 2^57), four rows
// per wavefront (one per 16-lane row): numbers of 16 Q limbs, Q = 4 PN + 1, so that
// 16 Q >= h + 2 limbs hold the sum; modulus N zero above its h limbs.  Lane l of a row adds the
// words of its limbs [Q l, Q l + Q) with carries along its chunk and keeps the carry out of the
// chunk pending until the end, as the Montgomery steps expect.  The result goes out through the
// wavefront's own LDS slice, so that each lane stores four consecutive limbs of a row at once.
// With part non-null, b_j is not read from b but summed from the one-query matvec's nseg
// per-segment partials part[j nseg + s] (mod 2^32), and written to bout[j].
template <int Q>
__global__ __launch_bounds__(256) void offset_reduce_quad_kernel(ClientDev cd, const uint64_t* __restrict__ W,
                                                                 long long ldw, const uint32_t* __restrict__ b,
                                                                 const uint32_t* __restrict__ part, int nseg,
                                                                 uint32_t* __restrict__ bout, int rows,
                                                                 uint32_t* __restrict__ T) {
  __shared__ uint32_t out[4][4][16 * Q];  // [wavefront][row][limb]
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int widx = blockIdx.x * (blockDim.x >> 6) + wv;
  if (4 * widx >= rows) return;
  const int mine = 4 * widx + row_index();
  const int j = min(rows - 1, mine);  // rows past the end repeat the last one and store nothing
  const uint64_t* w = W + (size_t)j * ldw;
  uint32_t bj;
  if (part) {
    uint32_t sum = 0;
    for (int q = row_lane(); q < nseg; q += 16) sum += part[(size_t)j * nseg + q];
    bj = row_sum16(sum);
    if (row_lane() == 0 && mine < rows) bout[j] = bj;
  } else {
    bj = b[j];
  }
  RNum<Q> v, m;
  uint64_t carry = 0;
#pragma unroll
  for (int jj = 0; jj < Q; ++jj) {
    const int limb = Q * row_lane() + jj;
    uint64_t x = carry;
    if (limb <= cd.h) x += w[limb];
    if (limb == 3) x += bj;  // b_j 2^96
    v.v[jj] = (uint32_t)x;
    carry = x >> 32;
  }
  rn_load_n(m, cd.NP, cd.h);
#pragma unroll
  for (int i = 0; i < 3; ++i) rn_redc_step(v, carry, m, cd.nprime);
  const uint64_t ovf = rn_resolve(v, carry);
  rn_cond_sub(v, ovf, m);
  uint32_t* o = out[wv][row_index()];
#pragma unroll
  for (int jj = 0; jj < Q; ++jj) o[Q * row_lane() + jj] = v.v[jj];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  if (mine < rows) {
    uint32_t* t = T + (size_t)j * cd.h;
    for (int c = 4 * row_lane(); c < cd.h; c += 64) {
      if (c + 4 <= cd.h && (reinterpret_cast<uintptr_t>(t + c) & 15) == 0) {
        *reinterpret_cast<u32x4*>(t + c) = u32x4{o[c], o[c + 1], o[c + 2], o[c + 3]};
      } else {
        for (int i = c; i < min(c + 4, cd.h); ++i) t[i] = o[i];
      }
    }
  }
}

void launch_offset_reduce(const ClientDev& cd, const uint64_t* W, long long ldw, const uint32_t* b,
                          int rows, uint32_t* T, hipStream_t s, const uint32_t* part, int nseg, uint32_t* bout) {
  if (rows <= 0) return;
  const int blocks = (rows + 15) / 16;
  switch (cd.PN) {
    case 1: offset_reduce_quad_kernel<5><<<blocks, 256, 0, s>>>(cd, W, ldw, b, part, nseg, bout, rows, T); break;
    case 2: offset_reduce_quad_kernel<9><<<blocks, 256, 0, s>>>(cd, W, ldw, b, part, nseg, bout, rows, T); break;
  }
}

// Packed offset answer (batched compression, Sec. 4.3): for the group of rows
// g ell .. g ell + ell - 1, Tg = sum_j 2^(t j) t_{g ell + j} mod N.  The terms are independent:
// one wavefront per (group, j) forms 2^(t j) t mod N as one Montgomery product by
// PJ[j] = 2^(t j) R_N mod N, and a second kernel adds each group's terms modulo N.
template <int PN>
__global__ __launch_bounds__(256) void offset_terms_kernel(ClientDev cd, const uint32_t* __restrict__ T,
                                                           int rows, int ell,
                                                           const uint32_t* __restrict__ PJ,
                                                           uint32_t* __restrict__ Tmp) {
  const int w = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= rows) return;
  const int j = w % ell;
  WNum<PN> Nn, c, x;
  wn_load(Nn, cd.Nn);
  wn_load(c, PJ + (size_t)j * 64 * PN);
  wn_load_n(x, T + (size_t)w * cd.h, cd.h);
  mont_mul(x, x, c, Nn, cd.nprime);
  wn_store_n(Tmp + (size_t)w * cd.h, x, cd.h);
}

// offset_terms_kernel with four rows per wavefront, one per 16-lane row (rownum.h; QN = 4 PN
// limbs per lane, the same R_N).  Spare rows of the last wavefront repeat its last row and
// store nothing.
template <int PN>
__global__ __launch_bounds__(256) void offset_terms_quad_kernel(ClientDev cd, const uint32_t* __restrict__ T,
                                                                int rows, int ell,
                                                                const uint32_t* __restrict__ PJ,
                                                                uint32_t* __restrict__ Tmp) {
  constexpr int QN = 4 * PN;
  const int widx = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (4 * widx >= rows) return;
  const int mine = 4 * widx + row_index();
  const int w = min(rows - 1, mine);
  const int j = w % ell;
  RNum<QN> Nn, c, x;
  rn_load(Nn, cd.Nn);
  rn_load(c, PJ + (size_t)j * 64 * PN);
  rn_load_n(x, T + (size_t)w * cd.h, cd.h);
  rn_mont_mul(x, x, c, Nn, cd.nprime);
  if (mine < rows) rn_store_n(Tmp + (size_t)w * cd.h, x, cd.h);
}

template <int PN>
__global__ __launch_bounds__(256) void offset_sum_kernel(ClientDev cd, const uint32_t* __restrict__ Tmp,
                                                         int rows, int ell, uint32_t* __restrict__ Tg) {
  const int g = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = g * ell;
  if (r0 >= rows) return;
  const int r1 = min(rows, r0 + ell);
  WNum<PN> Nn, acc, x;
  wn_load(Nn, cd.Nn);
  wn_load_n(acc, Tmp + (size_t)r0 * cd.h, cd.h);
  for (int r = r0 + 1; r < r1; ++r) {
    wn_load_n(x, Tmp + (size_t)r * cd.h, cd.h);
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < PN; ++k) {
      const uint64_t s = (uint64_t)acc.v[k] + x.v[k] + c;
      acc.v[k] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    const uint64_t ovf = wn_resolve(acc, (uint64_t)c);
    wn_cond_sub(acc, ovf, Nn);
  }
  wn_store_n(Tg + (size_t)g * cd.h, acc, cd.h);
}

void launch_offset_pack(const ClientDev& cd, const uint32_t* T, int rows, int ell,
                        const uint32_t* PJ, uint32_t* Tmp, uint32_t* Tg, hipStream_t s) {
  if (rows <= 0) return;
  const int groups = (rows + ell - 1) / ell;
  // four rows per wavefront while that still leaves several wavefronts per SIMD
  const bool quad = rows >= 16384;
  const int tblocks = quad ? ((rows + 3) / 4 + 3) / 4 : (rows + 3) / 4;
  if (cd.PN == 1) {
    if (quad) offset_terms_quad_kernel<1><<<tblocks, 256, 0, s>>>(cd, T, rows, ell, PJ, Tmp);
    else offset_terms_kernel<1><<<tblocks, 256, 0, s>>>(cd, T, rows, ell, PJ, Tmp);
    offset_sum_kernel<1><<<(groups + 3) / 4, 256, 0, s>>>(cd, Tmp, rows, ell, Tg);
  } else {
    if (quad) offset_terms_quad_kernel<2><<<tblocks, 256, 0, s>>>(cd, T, rows, ell, PJ, Tmp);
    else offset_terms_kernel<2><<<tblocks, 256, 0, s>>>(cd, T, rows, ell, PJ, Tmp);
    offset_sum_kernel<2><<<(groups + 3) / 4, 256, 0, s>>>(cd, Tmp, rows, ell, Tg);
  }
}

}  // namespace zp
