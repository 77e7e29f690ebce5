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
#include "internal.h"
#include "rownum.h"
#include "stage.h"
#include "wavenum.h"

namespace zp {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- operands of the offset contraction
//
// The contraction runs on v_mfma_i32_16x16x64_i8 with E split into its four byte planes:
//   W_a[j][c] = sum_k e_jk[a] y_k[c]   (a < 4, c < 4h),    W[j][pos] = sum_a W_a[j][pos - a].
// Both operands are stored already in MFMA fragment order, shifted to int8 by XOR 0x80:
//   Ep (E planes): piece (T, a, s) is 1 KiB, lane l's 16 bytes at 16 l hold
//     E'_a[16 T + l mod 16][64 s + 16 (l / 16) + u], u < 16,
//   so the stream of one 16-row tile and one plane is contiguous over its S = kpad / 64 slices;
//   Yf (offset bytes of one client): piece (s, t) is 1 KiB, lane l's bytes
//     Y'[16 t + l mod 16][64 s + 16 (l / 16) + u] with Y'[c][k] = byte c of y_k,
//   so one K slice of every column tile is one contiguous NT KiB run.
// Entries beyond rows, n or 4h are 0 (the value 128 before the shift), which adds nothing to
// the signed product; the shift terms below count only the real entries.

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
    Ep[((T * 4 + a) * S + s) * 64 + l] = u32x4{w[a][0], w[a][1], w[a][2], w[a][3]};
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

int offset_tiles(int h) {
  const int c = 4 * h;
  return c <= 64 ? 4 : c <= 128 ? 8 : c <= 256 ? 16 : c <= 384 ? 24 : 32;
}

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// One thread per 16-byte piece of client blockIdx.y; colsum[i 16 NT + c] = sum_{k<n} Y'[c][k]
// (zeroed first) by one atomic per column and piece row.
__global__ __launch_bounds__(256) void pack_y_kernel(const uint32_t* __restrict__ ys, int n, int h, int S,
                                                     int NT, u32x4* __restrict__ Yf,
                                                     int32_t* __restrict__ colsum) {
  const int i = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;  // piece within the client: (s, t, l)
  const int per = S * NT * 64;
  const bool live = p < per;
  const int l = p & 63;
  const int q = p >> 6;
  const int t = q % NT, s = q / NT;
  const int c = 16 * t + (l & 15);
  const int k0 = 64 * s + 16 * (l >> 4);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  int32_t part = 0;
  if (live && c < 4 * h) {
    const uint32_t* y = ys + (size_t)i * n * h + (c >> 2);
    const int sh = 8 * (c & 3);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + u;
      if (k < n) {
        const uint32_t sb = ((y[(size_t)k * h] >> sh) & 0xFFu) ^ 0x80u;
        w[u >> 2] |= sb << (8 * (u & 3));
        part += (int32_t)(int8_t)sb;
      }
    }
  }
  if (live) Yf[(size_t)i * per + p] = u32x4{w[0], w[1], w[2], w[3]};
  // the four lanes l, l^16, l^32, l^48 hold the same column
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  if (live && l < 16 && c < 4 * h && part != 0) atomicAdd(colsum + (size_t)i * 16 * NT + c, part);
}

void launch_pack_y(const uint32_t* ys, int batch, int n, int h, uint8_t* Yf, int32_t* colsum,
                   hipStream_t s) {
  const int S = offset_slices(n), NT = offset_tiles(h);
  const int ncs = batch * 16 * NT;
  zero_i32_kernel<<<(ncs + 255) / 256, 256, 0, s>>>(colsum, ncs);
  const int per = S * NT * 64;
  dim3 grid((per + 255) / 256, batch);
  pack_y_kernel<<<grid, 256, 0, s>>>(ys, n, h, S, NT, reinterpret_cast<u32x4*>(Yf), colsum);
}

// ---- the contraction
//
// A workgroup of four wavefronts takes 16 MR rows and one client; wavefront a computes W_a for
// all 16 NT columns: MR x NT accumulator tiles.  Both operands pass through LDS in NS stages
// of one 64-byte K slice each, by direct global-to-LDS loads (stage.h): a stage holds the four
// planes' MR fragments of the block's rows (4 MR KiB, each one contiguous kilobyte of Ep) and
// the client's NT fragments of the offset bytes (NT KiB, contiguous in Yf).  No operand passes
// through VGPRs on its way in, so the only wait per slice is for that slice's own loads, and
// the NS - 2 later slices stay in flight; one barrier per slice.  Each B fragment read from
// LDS feeds MR MFMAs, each A fragment NT.  Then the four planes are added with their shifts
// through LDS, one 16-row tile at a time:
//   W_a = acc + 128 colsum_c + 128 Ers_a[j] + 16384 n (exact modulo 2^32, and the true value
//   is below 2^32), and W[j][pos] = sum_a W_a[j][pos - a] for pos < 4h + 3.
// The grid is XCD-aware: workgroup L runs on XCD L mod 8, and each XCD takes the clients of its
// row blocks (x, x + 8, ...) one after the other, so a block's E stream comes from HBM once and
// from that XCD's L2 for the other clients.
template <int MR, int NT, int NS>
struct OffsetGeom {
  static constexpr int kAChunks = 4 * MR;                 // (plane, row tile) fragments per slice
  static constexpr int kChunks = kAChunks + NT;           // plus the offset-byte fragments
  static constexpr int kPerWave = kChunks / 4;            // loads per lane per slice
  static constexpr int kStage = kChunks * 1024;
  static constexpr int kCW = 16 * NT + 4;                 // words per row of a plane in the epilogue
  static constexpr int kEpi = 4 * 16 * kCW * 4;
  static constexpr int kLds = NS * kStage > kEpi ? NS * kStage : kEpi;
  static_assert(kChunks % 4 == 0, "chunks are dealt to four wavefronts");
};

template <int MR, int NT, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, MR * NT <= 32 ? 2 : 1)))
void offset_gemm_kernel(const uint8_t* __restrict__ Ep, const int32_t* __restrict__ Ers, int rows_pad, int rows,
                        int n, int S, const uint8_t* __restrict__ Yf, const int32_t* __restrict__ colsum,
                        int batch, int nrb, int h, uint32_t* __restrict__ W, long long ldw, int cpc) {
  using Geo = OffsetGeom<MR, NT, NS>;
  __shared__ __attribute__((aligned(1024))) uint8_t lds[Geo::kLds];
  const int tid = threadIdx.x, lane = tid & 63;
  const int a = __builtin_amdgcn_readfirstlane(tid >> 6);  // the plane of this wavefront
  const int g = lane >> 4, r = lane & 15;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int rb = (slot / batch) * 8 + xcd;
  const int ci = slot % batch;
  if (rb >= nrb) return;
  const int T0 = rb * MR;

  // this wavefront's share of each slice's loads: chunks a, a + 4, ...
  const uint8_t* src[Geo::kPerWave];
  long long sstride[Geo::kPerWave];
#pragma unroll
  for (int j = 0; j < Geo::kPerWave; ++j) {
    const int c = a + 4 * j;
    if (c < Geo::kAChunks) {
      const int pa = c / MR, i = c % MR;
      src[j] = Ep + ((size_t)((T0 + i) * 4 + pa) * S) * 1024 + lane * 16;
      sstride[j] = 1024;
    } else {
      src[j] = Yf + ((size_t)ci * S * NT + (c - Geo::kAChunks)) * 1024 + lane * 16;
      sstride[j] = (long long)NT * 1024;
    }
  }
  auto issue = [&](int sl) {  // slice sl (clamped to the last) into its stage buffer
    const int sc = min(sl, S - 1);
    uint8_t* base = lds + (sl % NS) * Geo::kStage;
#pragma unroll
    for (int j = 0; j < Geo::kPerWave; ++j) g2l16(src[j] + (size_t)sc * sstride[j], base + (a + 4 * j) * 1024);
  };

  v4i acc[MR][NT];
#pragma unroll
  for (int i = 0; i < MR; ++i)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[i][t] = v4i{0, 0, 0, 0};

#pragma unroll
  for (int st = 0; st < NS - 1; ++st) issue(st);
  for (int s = 0; s < S; ++s) {
    wait_vmcnt<(NS - 2) * Geo::kPerWave>();  // slice s has landed (later slices stay in flight)
    __builtin_amdgcn_s_barrier();            // ... for every wavefront; slice s - 1 is consumed
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    issue(s + NS - 1);
    const uint8_t* base = lds + (s % NS) * Geo::kStage + lane * 16;
    v4i bf[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bf[t] = *reinterpret_cast<const v4i*>(base + (Geo::kAChunks + t) * 1024);
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const v4i af = *reinterpret_cast<const v4i*>(base + (a * MR + i) * 1024);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[t], acc[i][t], 0, 0, 0);
    }
  }
  wait_vmcnt<0>();  // the surplus loads past the last slice write LDS the epilogue reuses
  lds_barrier_sync();

  // epilogue: planes through LDS, one 16-row tile at a time
  uint32_t* wl = reinterpret_cast<uint32_t*>(lds);
  constexpr int CW = Geo::kCW;
  const uint32_t nterm = 16384u * (uint32_t)n;
  const int npos = 4 * h + 3;
  const int32_t* cs = colsum + (size_t)ci * 16 * NT;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int rowbase = (T0 + i) * 16;
    uint32_t rterm[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) rterm[e] = 128u * (uint32_t)Ers[(size_t)a * rows_pad + rowbase + 4 * g + e] + nterm;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = 16 * t + r;
      const uint32_t ct = 128u * (uint32_t)cs[c];
#pragma unroll
      for (int e = 0; e < 4; ++e) wl[(a * 16 + 4 * g + e) * CW + c] = (uint32_t)acc[i][t][e] + ct + rterm[e];
    }
    lds_barrier_sync();
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int rho = 4 * a + rr;
      const int row = rowbase + rho;
      if (row < rows) {
        uint32_t* wrow = W + (size_t)row * ldw + (size_t)ci * cpc;
        for (int pos = lane; pos < npos; pos += 64) {
          uint32_t v = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int p = pos - b;
            if (p >= 0 && p < 4 * h) v += wl[(b * 16 + rho) * CW + p];
          }
          wrow[pos] = v;
        }
      }
    }
    lds_barrier_sync();
  }
}

template <int MR, int NT, int NS>
static void launch_offset_gemm_t(const uint8_t* Ep, const int32_t* Ers, int rows_pad, int rows, int n,
                                 const uint8_t* Yf, const int32_t* colsum, int batch, int h, uint32_t* W,
                                 long long ldw, int cpc, hipStream_t s) {
  const int S = offset_slices(n);
  const int nrb = rows_pad / (16 * MR);
  const long long nblocks = (long long)((nrb + 7) / 8 * 8) * batch;
  offset_gemm_kernel<MR, NT, NS><<<(unsigned)nblocks, 256, 0, s>>>(Ep, Ers, rows_pad, rows, n, S, Yf, colsum,
                                                                    batch, nrb, h, W, ldw, cpc);
}

// Launch variants (row tiles per wavefront MR, stages in flight NS) per column-tile count; the
// runtime times them once per problem shape (every variant gives identical bits).
struct OffsetVariant {
  int mr, ns;
};
static const OffsetVariant* offset_variant_list(int NT, int* count) {
  static const OffsetVariant v4[] = {{4, 4}, {4, 3}, {2, 4}};
  static const OffsetVariant v8[] = {{4, 4}, {4, 3}, {2, 4}};
  static const OffsetVariant v16[] = {{4, 4}, {4, 3}, {2, 4}, {2, 3}, {1, 4}};
  static const OffsetVariant v24[] = {{2, 4}, {2, 3}, {1, 4}};
  static const OffsetVariant v32[] = {{2, 3}, {1, 4}, {1, 3}};
  switch (NT) {
    case 4: *count = 3; return v4;
    case 8: *count = 3; return v8;
    case 16: *count = 5; return v16;
    case 24: *count = 3; return v24;
    default: *count = 3; return v32;
  }
}

int offset_gemm_variants(int h) {
  int count = 0;
  (void)offset_variant_list(offset_tiles(h), &count);
  return count;
}

void launch_offset_gemm(const uint8_t* Ep, const int32_t* Ers, int rows_pad, int rows, int n,
                        const uint8_t* Yf, const int32_t* colsum, int batch, int h, uint32_t* W,
                        long long ldw, int cpc, int variant, hipStream_t s) {
  const int NT = offset_tiles(h);
  int count = 0;
  const OffsetVariant* vl = offset_variant_list(NT, &count);
  const OffsetVariant v = vl[(variant >= 0 && variant < count) ? variant : 0];
#define ZP_OFF(M, T, N)                                                                                       \
  if (NT == T && v.mr == M && v.ns == N) {                                                                    \
    launch_offset_gemm_t<M, T, N>(Ep, Ers, rows_pad, rows, n, Yf, colsum, batch, h, W, ldw, cpc, s);          \
    return;                                                                                                   \
  }
  ZP_OFF(4, 4, 4) ZP_OFF(4, 4, 3) ZP_OFF(2, 4, 4)
  ZP_OFF(4, 8, 4) ZP_OFF(4, 8, 3) ZP_OFF(2, 8, 4)
  ZP_OFF(4, 16, 4) ZP_OFF(4, 16, 3) ZP_OFF(2, 16, 4) ZP_OFF(2, 16, 3) ZP_OFF(1, 16, 4)
  ZP_OFF(2, 24, 4) ZP_OFF(2, 24, 3) ZP_OFF(1, 24, 4)
  ZP_OFF(2, 32, 3) ZP_OFF(1, 32, 4) ZP_OFF(1, 32, 3)
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

// t_j from W[j][0 .. 4h+3): one wavefront per row, numbers of S = 64 P limbs (S >= h + 2
// holds the sum), modulus N zero-padded to S limbs.
template <int P>
__global__ __launch_bounds__(256) void offset_reduce_kernel(ClientDev cd, const uint32_t* __restrict__ W,
                                                            long long ldw,
                                                            const uint32_t* __restrict__ b, int rows,
                                                            uint32_t* __restrict__ T) {
  const int j = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (j >= rows) return;
  const uint32_t* w = W + (size_t)j * ldw;
  const int npos = 4 * cd.h + 3;
  WNum<P> v, m;
  uint64_t carry = 0;
#pragma unroll
  for (int jj = 0; jj < P; ++jj) {
    const int limb = P * lane_id() + jj;
    uint64_t x = carry;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int pos = 4 * limb + u;
      if (pos < npos) x += (uint64_t)w[pos] << (8 * u);
    }
    if (limb == 3) x += b[j];  // b_j 2^96
    v.v[jj] = (uint32_t)x;
    carry = x >> 32;
  }
  wn_load(m, cd.NP);
#pragma unroll
  for (int i = 0; i < 3; ++i) redc_step(v, carry, m, cd.nprime);
  const uint64_t ovf = wn_resolve(v, carry);
  wn_cond_sub(v, ovf, m);
  wn_store_n(T + (size_t)j * cd.h, v, cd.h);
}

void launch_offset_reduce(const ClientDev& cd, const uint32_t* W, long long ldw, const uint32_t* b,
                          int rows, uint32_t* T, hipStream_t s) {
  if (rows <= 0) return;
  const int blocks = (rows + 3) / 4;
  switch (cd.P) {
    case 1: offset_reduce_kernel<1><<<blocks, 256, 0, s>>>(cd, W, ldw, b, rows, T); break;
    case 2: offset_reduce_kernel<2><<<blocks, 256, 0, s>>>(cd, W, ldw, b, rows, T); break;
    case 3: offset_reduce_kernel<3><<<blocks, 256, 0, s>>>(cd, W, ldw, b, rows, T); break;
    case 4: offset_reduce_kernel<4><<<blocks, 256, 0, s>>>(cd, W, ldw, b, rows, T); break;
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
