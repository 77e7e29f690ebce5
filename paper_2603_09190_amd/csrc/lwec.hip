// Standalone compression of LWE ciphertexts and RLWE coefficients into Paillier ciphertexts.
//
// Alg. 2 (LWECompress): x = Enc(b; 1) (+) sum_i ((q - a_i) mod q) (x) ck_i
//                         = (1 + b N) prod_i ck_i^((q - a_i) mod q)   mod N^2.
// Alg. 8 (RLWECompressCoefficient, appendix B): the same product for coefficient k of an RLWE
// ciphertext (A, B) over Z_q[X]/(X^n + 1), with exponents (q - A[k-i]) mod q for i <= k and
// A[n+k-i] mod q for i > k, and b = B[k].
//
// The bases are fixed (the compression key), so the 8-bit fixed-base table of the client-hint
// kernel applies with as many windows as q has bytes: an exponent below 2^64 costs at most 8
// Montgomery products.  One ciphertext is spread over `parts` wavefronts (each multiplies the
// table entries of a contiguous range of bases), and the partial products are multiplied
// together in a tree of fan-in `fan`; with many ciphertexts one wavefront per ciphertext is
// enough to fill the GPU.

#include "internal.h"
#include "rownum.h"
#include "wavenum.h"

namespace zp {

__device__ __forceinline__ uint64_t lw_load(const uint32_t* p, size_t idx, int qw) {
  return qw == 2 ? ((uint64_t)p[2 * idx + 1] << 32) | p[2 * idx] : (uint64_t)p[idx];
}

__device__ __forceinline__ uint64_t lw_mod(uint64_t a, uint64_t q) { return q ? a % q : a; }

// (q - (a mod q)) mod q, q = 0 standing for 2^64
__device__ __forceinline__ uint64_t lw_neg(uint64_t a, uint64_t q) {
  const uint64_t r = lw_mod(a, q);
  return r == 0 ? 0 : (q ? q - r : 0 - r);
}

// exponent of base k for ciphertext `row`
__device__ __forceinline__ uint64_t lw_exponent(const LweBatch& lb, int row, int k) {
  if (!lb.ks) return lw_neg(lw_load(lb.A, (size_t)row * lb.n + k, lb.qw), lb.q);
  const int kk = (int)lb.ks[row];
  return k <= kk ? lw_neg(lw_load(lb.A, kk - k, lb.qw), lb.q)
                 : lw_mod(lw_load(lb.A, lb.n + kk - k, lb.qw), lb.q);
}

// x <- x (1 + b N) mod N^2 for x in Montgomery form (x = X R): the result is X (1 + b N),
// canonical.  1 + b N < N^2 because b < q <= 2^64 < N.
template <int P>
__device__ __forceinline__ void times_enc_b(const ClientDev& cd, WNum<P>& x, uint64_t b,
                                            const WNum<P>& M) {
  WNum<P> f, Nsh;
  wn_zero(f);
  if (lane_id() == 0) f.v[0] = 1;
  wn_load(Nsh, cd.NP);
  uint64_t pend = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // f += b_i N 2^(32 i)
    const uint32_t bi = (uint32_t)(b >> (32 * i));
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint64_t t = (uint64_t)bi * Nsh.v[j] + f.v[j] + c;
      f.v[j] = (uint32_t)t;
      c = (uint32_t)(t >> 32);
    }
    pend += c;
    const uint32_t in = from_prev_lane(Nsh.v[P - 1]);
#pragma unroll
    for (int j = P - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
    Nsh.v[0] = in;
  }
  (void)wn_resolve(f, pend);  // 1 + b N < N^2
  mont_mul(x, x, f, M, cd.m2prime);
}

__device__ __forceinline__ uint64_t lw_b(const LweBatch& lb, int row) {
  return lb.ks ? lw_mod(lw_load(lb.B, lb.ks[row], lb.qw), lb.q)
               : lw_mod(lw_load(lb.B, row, lb.qw), lb.q);
}

template <int P>
__global__ __launch_bounds__(256) void compress_lwe_kernel(ClientDev cd, LweBatch lb,
                                                           const uint32_t* __restrict__ table,
                                                           int parts, uint32_t* __restrict__ Part,
                                                           uint32_t* __restrict__ X) {
  constexpr int S = 64 * P;
  const int widx = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (widx >= lb.rows * parts) return;
  const int row = widx / parts, part = widx - row * parts;
  const int k0 = (int)((long long)lb.n * part / parts);
  const int k1 = (int)((long long)lb.n * (part + 1) / parts);
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  wn_load(acc, cd.R1);  // Montgomery form of 1
  for (int k = k0; k < k1; ++k) {
    const uint64_t e = lw_exponent(lb, row, k);
    const uint32_t* tk = table + (size_t)k * lb.windows * kDigits * S;
    for (int w = 0; w < lb.windows; ++w) {
      const uint32_t d = (uint32_t)(e >> (kWindowBits * w)) & kDigits;
      if (d != 0) {
        wn_load(b, tk + ((size_t)w * kDigits + (d - 1)) * S);
        mont_mul(acc, acc, b, M, cd.m2prime);
      }
    }
  }
  if (parts == 1) {
    times_enc_b<P>(cd, acc, lw_b(lb, row), M);
    wn_store_n(X + (size_t)row * cd.L, acc, cd.L);
  } else {
    wn_store(Part + (size_t)widx * S, acc);
  }
}

// x <- x (1 + b N) mod N^2 per row, x in Montgomery form (the row layout of times_enc_b).
template <int Q>
__device__ __forceinline__ void rn_times_enc_b(const ClientDev& cd, RNum<Q>& x, uint64_t b,
                                               const RNum<Q>& M) {
  RNum<Q> f, Nsh;
  rn_zero(f);
  if (row_lane() == 0) f.v[0] = 1;
  rn_load(Nsh, cd.NP);
  uint64_t pend = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // f += b_i N 2^(32 i)
    const uint32_t bi = (uint32_t)(b >> (32 * i));
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const uint64_t t = (uint64_t)bi * Nsh.v[j] + f.v[j] + c;
      f.v[j] = (uint32_t)t;
      c = (uint32_t)(t >> 32);
    }
    pend += c;
    const uint32_t in = row_from_prev(Nsh.v[Q - 1]);
#pragma unroll
    for (int j = Q - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
    Nsh.v[0] = in;
  }
  (void)rn_resolve(f, pend);  // 1 + b N < N^2
  rn_mont_mul(x, x, f, M, cd.m2prime);
}

// compress_lwe_kernel with four work items (ciphertext, part) per wavefront, one per 16-lane
// row (rownum.h).  Every row runs the longest part's base count; a row past its own range
// multiplies by R mod N^2 (the Montgomery form of 1).  Spare rows of the last wavefront repeat
// its last item and store nothing.
template <int P>
__global__ __launch_bounds__(256) void compress_lwe_quad_kernel(ClientDev cd, LweBatch lb,
                                                                const uint32_t* __restrict__ table,
                                                                int parts, uint32_t* __restrict__ Part,
                                                                uint32_t* __restrict__ X) {
  constexpr int S = 64 * P;
  constexpr int Q = 4 * P;
  const int items = lb.rows * parts;
  const int widx = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (4 * widx >= items) return;
  const int mine = 4 * widx + row_index();
  const int item = min(items - 1, mine);
  const int row = item / parts, part = item - row * parts;
  const int k0 = (int)((long long)lb.n * part / parts);
  const int k1 = (int)((long long)lb.n * (part + 1) / parts);
  const int span = (lb.n + parts - 1) / parts;  // the longest part, the same for every row
  RNum<Q> M, one, acc, b;
  rn_load(M, cd.N2);
  rn_load(one, cd.R1);
  acc = one;
  for (int i = 0; i < span; ++i) {
    const int k = k0 + i;
    const bool live = k < k1;
    const uint64_t e = live ? lw_exponent(lb, row, k) : 0;
    const uint32_t* tk = table + (size_t)(live ? k : 0) * lb.windows * kDigits * S;
    for (int w = 0; w < lb.windows; ++w) {
      const uint32_t d = (uint32_t)(e >> (kWindowBits * w)) & kDigits;
      if (d != 0) rn_load(b, tk + ((size_t)w * kDigits + (d - 1)) * S);
      else b = one;
      rn_mont_mul(acc, acc, b, M, cd.m2prime);
    }
  }
  if (parts == 1) {
    rn_times_enc_b<Q>(cd, acc, lw_b(lb, row), M);
    if (mine < items) rn_store_n(X + (size_t)row * cd.L, acc, cd.L);
  } else if (mine < items) {
    rn_store_n(Part + (size_t)item * S, acc, S);
  }
}

template <int P>
__global__ __launch_bounds__(256) void reduce_parts_kernel(ClientDev cd, LweBatch lb,
                                                           const uint32_t* __restrict__ Part,
                                                           int parts, int fan,
                                                           uint32_t* __restrict__ Out,
                                                           uint32_t* __restrict__ X) {
  constexpr int S = 64 * P;
  const int outs = (parts + fan - 1) / fan;
  const int widx = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (widx >= lb.rows * outs) return;
  const int row = widx / outs, o = widx - row * outs;
  const int p0 = o * fan, p1 = min(parts, p0 + fan);
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  wn_load(acc, Part + ((size_t)row * parts + p0) * S);
  for (int p = p0 + 1; p < p1; ++p) {
    wn_load(b, Part + ((size_t)row * parts + p) * S);
    mont_mul(acc, acc, b, M, cd.m2prime);
  }
  if (outs == 1) {
    times_enc_b<P>(cd, acc, lw_b(lb, row), M);
    wn_store_n(X + (size_t)row * cd.L, acc, cd.L);
  } else {
    wn_store(Out + (size_t)widx * S, acc);
  }
}

#define ZP_BY_P(KERNEL, GRID, ...)                                                   \
  switch (cd.P) {                                                                    \
    case 1: KERNEL<1><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 2: KERNEL<2><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 3: KERNEL<3><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;                      \
    case 4: KERNEL<4><<<GRID, 256, 0, s>>>(__VA_ARGS__); break;                      \
  }

void launch_compress_lwe(const ClientDev& cd, const LweBatch& lb, const uint32_t* table, int parts,
                         uint32_t* Part, uint32_t* X, hipStream_t s) {
  const long long items = (long long)lb.rows * parts;
  if (items <= 0) return;
  // four items per wavefront once that still leaves about four wavefronts per SIMD
  if (items >= kQuadItems) {
    const int blocks = (int)(((items + 3) / 4 + 3) / 4);
    ZP_BY_P(compress_lwe_quad_kernel, blocks, cd, lb, table, parts, Part, X)
    return;
  }
  const int blocks = (int)((items + 3) / 4);
  ZP_BY_P(compress_lwe_kernel, blocks, cd, lb, table, parts, Part, X)
}

void launch_reduce_parts(const ClientDev& cd, const LweBatch& lb, const uint32_t* Part, int parts,
                         int fan, uint32_t* Out, uint32_t* X, hipStream_t s) {
  const long long waves = (long long)lb.rows * ((parts + fan - 1) / fan);
  if (waves <= 0) return;
  const int blocks = (int)((waves + 3) / 4);
  ZP_BY_P(reduce_parts_kernel, blocks, cd, lb, Part, parts, fan, Out, X)
}

#undef ZP_BY_P

}  // namespace zp
