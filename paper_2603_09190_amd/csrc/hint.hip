// Client hint K_j = prod_k ck_k^{E_jk} mod N^2 with E = (-H) mod 2^32
// (Alg. 5 Hint = PaillierMatMul(H, ck); Alg. 2 multiplies ck[i] by (q - a[i]), Alg. 4 by
// (q - a[i]) mod q).
//
// Alg. 4 precomputes ck^(2^j) so that each plaintext multiplication becomes at most 32
// ciphertext multiplications selected by the exponent's bits.  Here the same fixed-base
// idea is taken to 8-bit windows: for every base k and window w the table holds
// ck_k^(v * 2^(8w)) for v = 1..255, so one 32-bit exponent costs at most 4 Montgomery
// multiplications, all bases being shared by every row of the database.  Any order of
// the multiplications gives the same residue.
//
// One wavefront computes one row; every value stays in Montgomery form (x R mod N^2) until
// the final conversion.
#include "internal.h"
#include "wavenum.h"

namespace zp {

__device__ __forceinline__ int wave_index() {
  return blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

template <int P>
__global__ __launch_bounds__(256) void build_table_kernel(ClientDev cd,
                                                          const uint32_t* __restrict__ ck, int n,
                                                          uint32_t* __restrict__ table) {
  constexpr int S = 64 * P;
  const int widx = wave_index();
  if (widx >= n * kWindows) return;
  const int k = widx / kWindows, w = widx % kWindows;
  WNum<P> M, RR, x, cur;
  wn_load(M, cd.N2);
  wn_load(RR, cd.RR);
  wn_load_n(x, ck + (size_t)k * cd.L, cd.L);
  mont_mul(x, x, RR, M, cd.m2prime);  // ck * R mod N^2
  for (int t = 0; t < kWindowBits * w; ++t) mont_mul(x, x, x, M, cd.m2prime);
  uint32_t* T = table + (size_t)widx * kDigits * S;
  wn_store(T, x);
  cur = x;
  for (int v = 2; v <= kDigits; ++v) {
    mont_mul(cur, cur, x, M, cd.m2prime);
    wn_store(T + (size_t)(v - 1) * S, cur);
  }
}

template <int P>
__global__ __launch_bounds__(256) void hint_rows_kernel(ClientDev cd, const uint32_t* __restrict__ H,
                                                        int n, const uint32_t* __restrict__ rowlist,
                                                        int nrows, const uint32_t* __restrict__ table,
                                                        uint32_t* __restrict__ K) {
  constexpr int S = 64 * P;
  const int widx = wave_index();
  if (widx >= nrows) return;
  const int row = rowlist ? (int)rowlist[widx] : widx;
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  wn_load(acc, cd.R1);  // Montgomery form of 1
  const uint32_t* hrow = H + (size_t)row * n;
  for (int k = 0; k < n; ++k) {
    const uint32_t e = 0u - hrow[k];  // (-H_jk) mod 2^32
    const uint32_t* tk = table + (size_t)k * kWindows * kDigits * S;
#pragma unroll
    for (int w = 0; w < kWindows; ++w) {
      const uint32_t d = (e >> (kWindowBits * w)) & kDigits;
      if (d != 0) {
        wn_load(b, tk + ((size_t)w * kDigits + (d - 1)) * S);
        mont_mul(acc, acc, b, M, cd.m2prime);
      }
    }
  }
  WNum<P> one;
  wn_zero(one);
  if (lane_id() == 0) one.v[0] = 1;
  mont_mul(acc, acc, one, M, cd.m2prime);  // leave Montgomery form
  wn_store_n(K + (size_t)row * cd.L, acc, cd.L);
}

// kappa_j = K_j * 2^32 mod N, the per-row constant the online combine needs
// (K_j mod N, pre-scaled so that a single Montgomery step yields K_j * b mod N).
template <int PN>
__global__ __launch_bounds__(256) void kappa_kernel(ClientDev cd, const uint32_t* __restrict__ K,
                                                    const uint32_t* __restrict__ rowlist,
                                                    int nrows, uint32_t* __restrict__ kappa) {
  constexpr int SN = 64 * PN;
  const int widx = wave_index();
  if (widx >= nrows) return;
  const int row = rowlist ? (int)rowlist[widx] : widx;
  WNum<PN> Nn, C1, C2, lo, hi, x, y;
  wn_load(Nn, cd.Nn);
  wn_load(C1, cd.C1);
  wn_load(C2, cd.C2);
  const uint32_t* kr = K + (size_t)row * cd.L;
  // K = lo + hi * R_N with lo < R_N and hi < N (since K < N^2 and N < R_N)
  wn_load_n(lo, kr, cd.L < SN ? cd.L : SN);
  if (cd.L > SN) wn_load_n(hi, kr + SN, cd.L - SN); else wn_zero(hi);
  mont_mul(x, lo, C1, Nn, cd.nprime);  // lo * 2^32 mod N
  mont_mul(y, hi, C2, Nn, cd.nprime);  // hi * R_N * 2^32 mod N
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < PN; ++j) {
    const uint64_t s = (uint64_t)x.v[j] + y.v[j] + carry;
    x.v[j] = (uint32_t)s;
    carry = (uint32_t)(s >> 32);
  }
  const uint64_t ovf = wn_resolve(x, (uint64_t)carry);
  wn_cond_sub(x, ovf, Nn);
  wn_store_n(kappa + (size_t)row * cd.h, x, cd.h);
}

void launch_build_table(const ClientDev& cd, const uint32_t* ck, int n, uint32_t* table,
                        hipStream_t s) {
  const int waves = n * kWindows;
  const int blocks = (waves + 3) / 4;
  switch (cd.P) {
    case 1: build_table_kernel<1><<<blocks, 256, 0, s>>>(cd, ck, n, table); break;
    case 2: build_table_kernel<2><<<blocks, 256, 0, s>>>(cd, ck, n, table); break;
    case 3: build_table_kernel<3><<<blocks, 256, 0, s>>>(cd, ck, n, table); break;
    case 4: build_table_kernel<4><<<blocks, 256, 0, s>>>(cd, ck, n, table); break;
  }
}

void launch_hint_rows(const ClientDev& cd, const uint32_t* H, int n, const uint32_t* rowlist,
                      int nrows, const uint32_t* table, uint32_t* K, hipStream_t s) {
  if (nrows <= 0) return;
  const int blocks = (nrows + 3) / 4;
  switch (cd.P) {
    case 1: hint_rows_kernel<1><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, K); break;
    case 2: hint_rows_kernel<2><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, K); break;
    case 3: hint_rows_kernel<3><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, K); break;
    case 4: hint_rows_kernel<4><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, K); break;
  }
}

void launch_kappa(const ClientDev& cd, const uint32_t* K, const uint32_t* rowlist, int nrows,
                  uint32_t* kappa, hipStream_t s) {
  if (nrows <= 0) return;
  const int blocks = (nrows + 3) / 4;
  switch (cd.PN) {
    case 1: kappa_kernel<1><<<blocks, 256, 0, s>>>(cd, K, rowlist, nrows, kappa); break;
    case 2: kappa_kernel<2><<<blocks, 256, 0, s>>>(cd, K, rowlist, nrows, kappa); break;
  }
}

}  // namespace zp
