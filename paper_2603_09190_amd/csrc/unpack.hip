// Unpacking a packed compression key (Alg. 6, UnpackCompressionKey): key entry i t + j is
// pck_i^(delta^(t-1-j)) mod N^2, and with delta = 2^dbits that is pck_i raised to 2^(dbits (t-1-j)):
// one chain of squarings per packed ciphertext, each key entry a stop along the chain.
//
// A chain cannot be split: squaring is the whole work and step k needs step k-1.  So each step
// (one Montgomery product modulo M = N^2, S = 64 P words, R = 2^(32 S)) is spread over a workgroup
// of 256 threads, and a chain runs on one workgroup:
//   1. column sums of a b: thread (bi, bj) of a 16 x 16 grid multiplies the K x K block
//      a[bi K ...] x b[bj K ...] (K = S / 16) into 2K - 1 column accumulators in registers and adds
//      them into LDS columns (two 64-bit LDS atomics per column: bits 0-31 and 32-); the columns
//      become words in two local passes and one carry-lookahead pass;
//   2. m = (a b mod R) n' mod R with n' = -M^-1 mod R, the same block product restricted to the
//      low S columns;
//   3. U = (a b + m M) / R: the block product m M added to a b's words, carried, the high half
//      taken, and M subtracted once if U >= M (U < 2M).
// Carry-lookahead: for a chunk of 64 words x_l < 2^33 - 1 (one per lane), G = ballot(x_l > 2^32 - 1)
// and P = ballot(x_l == 2^32 - 1); the carries into the lanes are the internal carries of the
// 64-bit addition G + (G | P) + c_in, i.e. (G + (G | P) + c_in) ^ G ^ (G | P), and the addition's
// own carry-out goes into the next chunk.  Borrows of a subtraction work the same way with
// "u < m" and "u == m".
#include "internal.h"

namespace zp {

namespace {

constexpr int kThreads = 256;

// Products have 2S - 1 columns; one more word (index 2S) takes the top bit of T + m M.
template <int S>
struct UnpackLds {
  static constexpr int kW = 2 * S + 64;
  uint32_t M[S], Ni[S], X[S], Y[S], m[S];
  uint32_t T[kW];                              // a b, then a b + m M, as words
  unsigned long long c0[kW], c1[kW];           // column sums: bits 0-31, bits 32- (as added)
  unsigned long long x[kW];                    // words before the carry-lookahead
};

// Carry-lookahead over `words` entries of v (each < 2^33 - 1), written as 32-bit words to out;
// returns the carry out of the top word.  Wave 0 only.
__device__ uint32_t carry_chain(const unsigned long long* v, int words, uint32_t* out) {
  const int lane = threadIdx.x & 63;
  unsigned long long cin = 0;
  for (int base = 0; base < words; base += 64) {
    const unsigned long long xv = base + lane < words ? v[base + lane] : 0ull;
    const unsigned long long G = __ballot(xv > 0xFFFFFFFFull);
    const unsigned long long P = __ballot(xv == 0xFFFFFFFFull);
    const unsigned long long B = G | P;
    const unsigned long long s1 = G + B;
    const unsigned long long s2 = s1 + cin;
    const unsigned long long C = s2 ^ G ^ B;
    const unsigned long long cout = (s1 < G) | (s2 < s1);
    if (base + lane < words) out[base + lane] = (uint32_t)(xv + ((C >> lane) & 1ull));
    cin = cout;
  }
  return (uint32_t)cin;
}

// Column sums of a x b into L.c0 / L.c1 (cleared by the caller): all columns, or only those
// below S (low = true).
template <int S, bool kLow>
__device__ void block_product(UnpackLds<S>& L, const uint32_t* a, const uint32_t* b) {
  constexpr int K = S / 16;
  const int bi = threadIdx.x >> 4, bj = threadIdx.x & 15;
  const int cb = (bi + bj) * K;
  if (kLow && cb >= S) return;
  uint32_t ar[K], br[K];
#pragma unroll
  for (int d = 0; d < K; ++d) {
    ar[d] = a[bi * K + d];
    br[d] = b[bj * K + d];
  }
  unsigned long long acc[2 * K - 1];
  uint32_t hi[2 * K - 1];
#pragma unroll
  for (int c = 0; c < 2 * K - 1; ++c) {
    acc[c] = 0ull;
    hi[c] = 0u;
  }
#pragma unroll
  for (int di = 0; di < K; ++di)
#pragma unroll
    for (int dj = 0; dj < K; ++dj) {
      if (kLow && cb + di + dj >= S) continue;
      const unsigned long long p = (unsigned long long)ar[di] * br[dj];
      const unsigned long long s = acc[di + dj] + p;
      hi[di + dj] += s < p ? 1u : 0u;
      acc[di + dj] = s;
    }
#pragma unroll
  for (int c = 0; c < 2 * K - 1; ++c) {
    if (kLow && cb + c >= S) continue;
    atomicAdd(&L.c0[cb + c], acc[c] & 0xFFFFFFFFull);
    atomicAdd(&L.c1[cb + c], (acc[c] >> 32) + ((unsigned long long)hi[c] << 32));
  }
}

// Column sums (c0, c1) over `cols` columns, plus `add` (cols words or nullptr), to words in x
// (each at most 2^32 + 6): two local passes.  Every thread; barriers inside.
template <int S>
__device__ void columns_to_x(UnpackLds<S>& L, int cols, const uint32_t* add) {
  // value of column c: c0[c] + c1[c] 2^32 with c0 < 2^37 and c1 < 2^42 (at most 32 blocks add
  // into a column); word c receives lo(c0[c]) + hi(c0[c-1]) + lo(c1[c-1]) + hi(c1[c-2])
  for (int c = threadIdx.x; c < cols; c += kThreads) {
    unsigned long long w = L.c0[c] & 0xFFFFFFFFull;
    if (c >= 1) w += (L.c0[c - 1] >> 32) + (L.c1[c - 1] & 0xFFFFFFFFull);
    if (c >= 2) w += L.c1[c - 2] >> 32;
    if (add) w += add[c];
    L.x[c] = w;  // < 2^35
  }
  __syncthreads();
  unsigned long long v[(2 * S + 1 + kThreads - 1) / kThreads];
  int k = 0;
  for (int c = threadIdx.x; c < cols; c += kThreads, ++k)
    v[k] = (L.x[c] & 0xFFFFFFFFull) + (c >= 1 ? L.x[c - 1] >> 32 : 0ull);
  __syncthreads();
  k = 0;
  for (int c = threadIdx.x; c < cols; c += kThreads, ++k) L.x[c] = v[k];  // <= 2^32 + 6
  __syncthreads();
}

template <int S>
__device__ void clear_columns(UnpackLds<S>& L, int cols) {
  for (int c = threadIdx.x; c < cols; c += kThreads) {
    L.c0[c] = 0ull;
    L.c1[c] = 0ull;
  }
}

// out = a b R^-1 mod M (a, b, out in LDS, S words; out may alias a or b).
template <int S>
__device__ void mont_mul_wg(UnpackLds<S>& L, const uint32_t* a, const uint32_t* b, uint32_t* out) {
  const int wave = threadIdx.x >> 6;
  // 1. T = a b (2S + 1 words, the top one 0)
  clear_columns(L, 2 * S + 1);
  __syncthreads();
  block_product<S, false>(L, a, b);
  __syncthreads();
  columns_to_x(L, 2 * S + 1, nullptr);
  if (wave == 0) (void)carry_chain(L.x, 2 * S + 1, L.T);
  __syncthreads();
  // 2. m = T_low n' mod R
  clear_columns(L, S);
  __syncthreads();
  block_product<S, true>(L, L.T, L.Ni);
  __syncthreads();
  columns_to_x(L, S, nullptr);
  if (wave == 0) (void)carry_chain(L.x, S, L.m);
  __syncthreads();
  // 3. U = (T + m M) / R, then U mod M
  clear_columns(L, 2 * S + 1);
  __syncthreads();
  block_product<S, false>(L, L.m, L.M);
  __syncthreads();
  columns_to_x(L, 2 * S + 1, L.T);
  if (wave == 0) {
    const int lane = threadIdx.x & 63;
    // T + m M < 2 R M: words 0 .. S-1 are zero by construction (their carry reaches word S
    // through the chain), U is words S .. 2S-1, and word 2S its top bit
    (void)carry_chain(L.x, 2 * S + 1, L.T);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    const uint32_t top = L.T[2 * S];
    const uint32_t* U = L.T + S;
    // U >= M ?  (U < 2M): compare from the top
    bool ge = top != 0;
    if (!ge) {
      int decided = 0;
      for (int base = S - 64; base >= 0 && !decided; base -= 64) {
        const uint32_t u = U[base + lane], mm = L.M[base + lane];
        const unsigned long long gt = __ballot(u > mm), lt = __ballot(u < mm);
        if (gt | lt) {
          const int hg = gt ? 63 - __builtin_clzll(gt) : -1, hl = lt ? 63 - __builtin_clzll(lt) : -1;
          ge = hg > hl;
          decided = 1;
        }
      }
      if (!decided) ge = true;  // U == M
    }
    // out = U - M (if ge) with borrow lookahead, else U
    unsigned long long bin = 0;
    for (int base = 0; base < S; base += 64) {
      const uint32_t u = U[base + lane], mm = ge ? L.M[base + lane] : 0u;
      const unsigned long long G = __ballot(u < mm), P = __ballot(u == mm);
      const unsigned long long B = G | P;
      const unsigned long long s1 = G + B, s2 = s1 + bin;
      const unsigned long long C = s2 ^ G ^ B;
      bin = (s1 < G) | (s2 < s1);
      out[base + lane] = u - mm - (uint32_t)((C >> lane) & 1ull);
    }
  }
  __syncthreads();
}

// One workgroup per packed ciphertext i: keys i t + t - 1, i t + t - 2, ..., i t (those below n),
// stopping to write each after dbits further squarings.
template <int S>
__global__ __launch_bounds__(kThreads) void unpack_chain_kernel(const uint32_t* __restrict__ M,
                                                                const uint32_t* __restrict__ RR,
                                                                const uint32_t* __restrict__ Ni,
                                                                const uint32_t* __restrict__ pck, int n, int t,
                                                                int dbits, int L, uint32_t* __restrict__ ck) {
  __shared__ UnpackLds<S> lds;
  const int i = blockIdx.x;
  for (int w = threadIdx.x; w < S; w += kThreads) {
    lds.M[w] = M[w];
    lds.Ni[w] = Ni[w];
    lds.Y[w] = RR[w];
    lds.X[w] = w < L ? pck[(size_t)i * L + w] : 0u;
  }
  __syncthreads();
  mont_mul_wg(lds, lds.X, lds.Y, lds.X);  // Montgomery form
  for (int j = t - 1; j >= 0; --j) {
    const int k = i * t + j;
    if (k < n) {
      // key k = X R^-1 (out of Montgomery form) via a product with 1
      for (int w = threadIdx.x; w < S; w += kThreads) lds.Y[w] = w == 0 ? 1u : 0u;
      __syncthreads();
      mont_mul_wg(lds, lds.X, lds.Y, lds.Y);
      for (int w = threadIdx.x; w < L; w += kThreads) ck[(size_t)k * L + w] = lds.Y[w];
      __syncthreads();
    }
    if (j > 0)
      for (int sq = 0; sq < dbits; ++sq) mont_mul_wg(lds, lds.X, lds.X, lds.X);
  }
}

}  // namespace

void launch_unpack_chains(const ClientDev& cd, const uint32_t* Ni, const uint32_t* pck, int n, int t, int dbits,
                          uint32_t* ck, hipStream_t s) {
  if (n <= 0) return;
  const int groups = (n + t - 1) / t;
  switch (cd.P) {
    case 1: unpack_chain_kernel<64><<<groups, kThreads, 0, s>>>(cd.N2, cd.RR, Ni, pck, n, t, dbits, cd.L, ck); break;
    case 2: unpack_chain_kernel<128><<<groups, kThreads, 0, s>>>(cd.N2, cd.RR, Ni, pck, n, t, dbits, cd.L, ck); break;
    case 3: unpack_chain_kernel<192><<<groups, kThreads, 0, s>>>(cd.N2, cd.RR, Ni, pck, n, t, dbits, cd.L, ck); break;
    case 4: unpack_chain_kernel<256><<<groups, kThreads, 0, s>>>(cd.N2, cd.RR, Ni, pck, n, t, dbits, cd.L, ck); break;
  }
}

}  // namespace zp
