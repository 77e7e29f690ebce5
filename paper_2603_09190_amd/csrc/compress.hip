// Combined response c_j = K_j * (1 + b_j N) mod N^2 (Sec. 4.3, "Smaller responses w/
// Paillier addition": the online answer b_j is folded into the offline hint K_j with one
// Paillier addition of Enc(b_j; 1) = (N+1)^b_j = 1 + b_j N mod N^2).
//
// Since K (1 + b N) = K + N (K b mod N)  (mod N^2), the combine needs only
//   r = K_j b_j mod N      -- one Montgomery step on kappa_j = K_j 2^32 mod N (precomputed
//                             with the hint), as (kappa_j b_j + q N) / 2^32 < 2N,
//   c = K_j + N r          -- an h x h limb product and an add, then one conditional
//                             subtraction of N^2 (the sum is below 2 N^2).
// One wavefront handles one row.
#include "internal.h"
#include "wavenum.h"

namespace zp {

template <int P, int PN>
__global__ __launch_bounds__(256) void compress_kernel(ClientDev cd, const uint32_t* __restrict__ K,
                                                       const uint32_t* __restrict__ kappa,
                                                       const uint32_t* __restrict__ b, int rows,
                                                       uint32_t* __restrict__ C) {
  const int row = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= rows) return;
  const uint32_t bj = b[row];

  WNum<PN> Nn, kap, r;
  wn_load(Nn, cd.Nn);
  wn_load_n(kap, kappa + (size_t)row * cd.h, cd.h);
  wn_zero(r);
  uint64_t c = 0;
  mont_step(r, c, bj, kap, Nn, cd.nprime);  // kappa * b / 2^32 = K b (mod N), below 2N
  uint64_t ovf = wn_resolve(r, c);
  wn_cond_sub(r, ovf, Nn);

  WNum<P> acc, Nsh;
  wn_load_n(acc, K + (size_t)row * cd.L, cd.L);
  wn_load(Nsh, cd.NP);
  uint64_t pend = 0;
  for (int i = 0; i < cd.h; ++i) {
    const uint32_t ri = wn_limb(r, i);
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint64_t x = (uint64_t)ri * Nsh.v[j] + acc.v[j] + carry;
      acc.v[j] = (uint32_t)x;
      carry = (uint32_t)(x >> 32);
    }
    pend += carry;
    // Nsh <- Nsh * 2^32 (N shifted up one limb for the next r limb)
    const uint32_t in = from_prev_lane(Nsh.v[P - 1]);
#pragma unroll
    for (int j = P - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
    Nsh.v[0] = in;
  }
  ovf = wn_resolve(acc, pend);
  WNum<P> M2;
  wn_load(M2, cd.N2);
  wn_cond_sub(acc, ovf, M2);
  wn_store_n(C + (size_t)row * cd.L, acc, cd.L);
}

void launch_compress(const ClientDev& cd, const uint32_t* K, const uint32_t* kappa,
                     const uint32_t* b, int rows, uint32_t* C, hipStream_t s) {
  if (rows <= 0) return;
  const int blocks = (rows + 3) / 4;
  switch (cd.P) {
    case 1: compress_kernel<1, 1><<<blocks, 256, 0, s>>>(cd, K, kappa, b, rows, C); break;
    case 2: compress_kernel<2, 1><<<blocks, 256, 0, s>>>(cd, K, kappa, b, rows, C); break;
    case 3: compress_kernel<3, 2><<<blocks, 256, 0, s>>>(cd, K, kappa, b, rows, C); break;
    case 4: compress_kernel<4, 2><<<blocks, 256, 0, s>>>(cd, K, kappa, b, rows, C); break;
  }
}

}  // namespace zp
