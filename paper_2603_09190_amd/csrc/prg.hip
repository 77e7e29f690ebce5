// Random hint keys of the silent offline phase (Sec. 4.3, "Lowering offline communication
// costs" and "Supporting multiple queries"): the client sends its Paillier modulus N and a
// seed; client and server expand the seed into the random ciphertexts ck_r of Alg. 5's Setup,
// one n-vector per query, uniform over Z_{N^2}.
//
// The PRG is the ChaCha20 keystream of RFC 8439 with the 32-byte seed as key.  Entry k of
// query q takes the keystream under nonce (q, k, r) -- three little-endian words, r the
// attempt -- from block 0 on as little-endian 32-bit words w_0 w_1 ...; the candidate
// sum_i w_i 2^(32 i) over W = ceil(bits(N^2) / 32) words, cut to its low bits(N^2) bits, is
// accepted when it is below N^2 (probability above 1/2 per attempt), else r increases.
#include "internal.h"

namespace zp {

__host__ __device__ __forceinline__ uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

__host__ __device__ __forceinline__ void qround(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
  a += b; d = rotl32(d ^ a, 16);
  c += d; b = rotl32(b ^ c, 12);
  a += b; d = rotl32(d ^ a, 8);
  c += d; b = rotl32(b ^ c, 7);
}

// One ChaCha20 block (RFC 8439, Sec. 2.3): constants, key, counter, nonce; twenty rounds;
// the input added back.
__host__ __device__ __forceinline__ void chacha20_block(const SeedKey& key, uint32_t counter, uint32_t n0,
                                               uint32_t n1, uint32_t n2, uint32_t (&out)[16]) {
  uint32_t x[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                    key.w[0], key.w[1], key.w[2], key.w[3], key.w[4], key.w[5], key.w[6], key.w[7],
                    counter, n0, n1, n2};
  uint32_t in[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) in[i] = x[i];
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    qround(x[0], x[4], x[8], x[12]);
    qround(x[1], x[5], x[9], x[13]);
    qround(x[2], x[6], x[10], x[14]);
    qround(x[3], x[7], x[11], x[15]);
    qround(x[0], x[5], x[10], x[15]);
    qround(x[1], x[6], x[11], x[12]);
    qround(x[2], x[7], x[8], x[13]);
    qround(x[3], x[4], x[9], x[14]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = x[i] + in[i];
}

// One thread per entry (query q = first_query + e / n, coordinate k = e % n).  The candidate
// is written straight into the entry's L limbs and compared with N^2 from the top word down.
// An entry still rejected after kMaxAttempts attempts (probability below 2^-64) counts in
// *failures and the host reports an error.
constexpr int kMaxAttempts = 64;

__global__ __launch_bounds__(256) void expand_key_kernel(SeedKey key, uint32_t first_query, int n,
                                                         long long entries, const uint32_t* __restrict__ N2,
                                                         int W, uint32_t top_mask, int L,
                                                         uint32_t* __restrict__ out,
                                                         unsigned* __restrict__ failures) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= entries) return;
  const uint32_t q = first_query + (uint32_t)(e / n);
  const uint32_t k = (uint32_t)(e % n);
  uint32_t* x = out + e * L;
  bool ok = false;
  for (int r = 0; r < kMaxAttempts && !ok; ++r) {
    for (int blk = 0; 16 * blk < W; ++blk) {
      uint32_t w[16];
      chacha20_block(key, (uint32_t)blk, q, k, (uint32_t)r, w);
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (16 * blk + i < W) x[16 * blk + i] = w[i];
    }
    x[W - 1] &= top_mask;
    int i = W - 1;
    while (i > 0 && x[i] == N2[i]) --i;
    ok = x[i] < N2[i];
  }
  for (int i = W; i < L; ++i) x[i] = 0u;
  if (!ok) atomicAdd(failures, 1u);
}

void launch_expand_key(const SeedKey& key, uint32_t first_query, int n, int count, const uint32_t* N2, int W,
                       uint32_t top_mask, int L, uint32_t* out, unsigned* failures, hipStream_t s) {
  const long long entries = (long long)count * n;
  if (entries <= 0) return;
  const int blocks = (int)((entries + 255) / 256);
  expand_key_kernel<<<blocks, 256, 0, s>>>(key, first_query, n, entries, N2, W, top_mask, L, out, failures);
}

}  // namespace zp
