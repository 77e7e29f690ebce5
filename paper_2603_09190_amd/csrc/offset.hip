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
// which is the uint8 product of E's rows read as 4n bytes (little-endian, so the byte of
// E_jk with weight 2^(8a) sits at K index 4k + a) with a 4n x (4h + 3) byte matrix whose
// column pos holds the bytes y_k[pos - a].  Every W entry is below 4n 255^2 < 2^32, so the
// contraction is exact in 32-bit accumulators.  The offsets are first replaced by
// y_k = ck_o,k 2^96 mod N, so that a reduction kernel can fold the byte positions into limbs,
// add b_j 2^96 and finish modulo N with three Montgomery reduction steps (see below).
#include "internal.h"
#include "rownum.h"
#include "wavenum.h"

namespace zp {

// Eb row j = the 4n bytes of E row j (E_jk = -H_jk mod 2^32), zero up to the pitch.
__global__ __launch_bounds__(256) void e_bytes_kernel(const uint32_t* __restrict__ H, int rows,
                                                      int n, int epitch_words,
                                                      uint32_t* __restrict__ Eb) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)rows * epitch_words) return;
  const long long j = i / epitch_words;
  const int k = (int)(i - j * epitch_words);
  Eb[i] = k < n ? 0u - H[j * n + k] : 0u;
}

void launch_e_bytes(const uint32_t* H, int rows, int n, int epitch, uint8_t* Eb, hipStream_t s) {
  const long long words = (long long)rows * (epitch / 4);
  const int blocks = (int)((words + 255) / 256);
  e_bytes_kernel<<<blocks, 256, 0, s>>>(H, rows, n, epitch / 4, reinterpret_cast<uint32_t*>(Eb));
}

// Column col = i*cpc + pos of the shifted-byte operand for client i: X[col][4k + a] is byte
// (pos - a) of y_k (0 outside [0, 4h)), stored as X ^ 0x80 for K indices below 4n and 0
// beyond (the one-plane layout of launch_gemm_planes); colsum[col] sums the stored int8s.
__global__ __launch_bounds__(256) void pack_offset_kernel(const uint32_t* __restrict__ cko, int n,
                                                          int h, int cpc, int epitch,
                                                          int8_t* __restrict__ X,
                                                          int32_t* __restrict__ colsum) {
  const int col = blockIdx.x;
  const int client = col / cpc, pos = col - client * cpc;
  const int k = blockIdx.y * blockDim.x + threadIdx.x;  // one K quadruple (4k .. 4k+3)
  int32_t part = 0;
  if (4 * k < epitch) {
    uint32_t w = 0;
    if (k < n) {
      const uint32_t* y = cko + ((size_t)client * n + k) * h;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int idx = pos - a;
        uint32_t v = 0;
        if (idx >= 0 && idx < 4 * h) v = (y[idx >> 2] >> (8 * (idx & 3))) & 0xFFu;
        const uint32_t sb = v ^ 0x80u;
        w |= sb << (8 * a);
        part += (int32_t)(int8_t)sb;
      }
    }
    reinterpret_cast<uint32_t*>(X + (size_t)col * epitch)[k] = w;
  }
  __shared__ int32_t red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if (lane == 0) red[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(colsum + col, red[0] + red[1] + red[2] + red[3]);
}

void launch_pack_offset(const uint32_t* cko, int batch, int n, int h, int cpc, int epitch,
                        int8_t* X, int32_t* colsum, hipStream_t s) {
  (void)hipMemsetAsync(colsum, 0, sizeof(int32_t) * (size_t)batch * cpc, s);
  // columns on x (batch cpc reaches 66048 at batch 128 and 4096-bit N), K on y (at most 64)
  dim3 grid(batch * cpc, (epitch / 4 + 255) / 256);
  pack_offset_kernel<<<grid, 256, 0, s>>>(cko, n, h, cpc, epitch, X, colsum);
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
