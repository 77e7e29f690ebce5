// Client hint K_j = prod_k ck_k^{E_jk} mod N^2 with E = (-H) mod 2^32
// (Alg. 5 Hint = PaillierMatMul(H, ck); Alg. 2 multiplies ck[i] by (q - a[i]), Alg. 4 by
// (q - a[i]) mod q).
//
// Alg. 4 precomputes ck^(2^j) so that each plaintext multiplication becomes at most 32
// ciphertext multiplications selected by the exponent's bits.  Here the same fixed-base
// idea is taken to windows of wb bits: for every base k and window w the table holds
// ck_k^(v * 2^(wb w)) for v = 1..2^wb - 1, so one 32-bit exponent costs at most
// ceil(32 / wb) Montgomery multiplications, all bases being shared by every row of the
// database.  wb = 8 (4 windows, 255 entries each) suits a few rows; wb = 11 (3 windows, 2047
// entries each) costs a larger table and saves a quarter of the row products.  Any order of
// the multiplications gives the same residue.
//
// One wavefront computes one row (four rows, one per 16-lane row, when there are many rows);
// every value stays in Montgomery form (x R mod N^2) until the final conversion, which stores
// K'_j = K_j 2^32 mod N^2 (the form the online combine consumes; pir_get_client_hint converts
// back to K_j).
#include <algorithm>

#include "internal.h"
#include "rownum.h"
#include "wavenum.h"

namespace zp {

__device__ __forceinline__ int wave_index() {
  return blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// One wavefront per (base k, window w, segment): with digits = 2^wbits - 1 entries per window
// cut into `segs` runs, segment s computes x^v for v in its run, x = ck_k^(2^(wbits w)),
// starting from x^v0 by square-and-multiply and continuing by multiplications by x.
template <int P>
__global__ __launch_bounds__(256) void build_table_kernel(ClientDev cd,
                                                          const uint32_t* __restrict__ ck, int n,
                                                          int windows, int wbits, int segs,
                                                          uint32_t* __restrict__ table) {
  constexpr int S = 64 * P;
  const int widx = wave_index();
  if (widx >= n * windows * segs) return;
  const int seg = widx % segs, kw = widx / segs;
  const int k = kw / windows, w = kw % windows;
  const int digits = (1 << wbits) - 1;
  const int v0 = 1 + (int)((long long)digits * seg / segs);
  const int v1 = (int)((long long)digits * (seg + 1) / segs);  // inclusive
  WNum<P> M, RR, x, cur;
  wn_load(M, cd.N2);
  wn_load(RR, cd.RR);
  wn_load_n(x, ck + (size_t)k * cd.L, cd.L);
  mont_mul(x, x, RR, M, cd.m2prime);  // ck * R mod N^2
  for (int t = 0; t < wbits * w; ++t) mont_mul(x, x, x, M, cd.m2prime);
  // cur = x^v0: left-to-right binary exponentiation
  cur = x;
  for (int bit = 30 - __builtin_clz((unsigned)v0); bit >= 0; --bit) {
    mont_mul(cur, cur, cur, M, cd.m2prime);
    if ((v0 >> bit) & 1) mont_mul(cur, cur, x, M, cd.m2prime);
  }
  uint32_t* T = table + (size_t)kw * digits * S;
  wn_store(T + (size_t)(v0 - 1) * S, cur);
  for (int v = v0 + 1; v <= v1; ++v) {
    mont_mul(cur, cur, x, M, cd.m2prime);
    wn_store(T + (size_t)(v - 1) * S, cur);
  }
}

// build_table_kernel with four bases per wavefront (k = 4 kq .. 4 kq + 3, one per 16-lane
// row, rownum.h) sharing the window w and the segment, so every loop is uniform across the
// wavefront.  Spare rows past the last base repeat it and store nothing.
template <int P>
__global__ __launch_bounds__(256) void build_table_quad_kernel(ClientDev cd,
                                                               const uint32_t* __restrict__ ck, int n,
                                                               int windows, int wbits, int segs,
                                                               uint32_t* __restrict__ table) {
  constexpr int S = 64 * P;
  constexpr int Q = 4 * P;
  const int widx = wave_index();
  const int nq = (n + 3) / 4;
  if (widx >= nq * windows * segs) return;
  const int seg = widx % segs, rest = widx / segs;
  const int w = rest % windows, kq = rest / windows;
  const int kmine = 4 * kq + row_index();
  const int k = min(n - 1, kmine);
  const int digits = (1 << wbits) - 1;
  const int v0 = 1 + (int)((long long)digits * seg / segs);
  const int v1 = (int)((long long)digits * (seg + 1) / segs);  // inclusive
  RNum<Q> M, RR, x, cur;
  rn_load(M, cd.N2);
  rn_load(RR, cd.RR);
  rn_load_n(x, ck + (size_t)k * cd.L, cd.L);
  rn_mont_mul(x, x, RR, M, cd.m2prime);  // ck * R mod N^2
  for (int t = 0; t < wbits * w; ++t) rn_mont_mul(x, x, x, M, cd.m2prime);
  cur = x;
  for (int bit = 30 - __builtin_clz((unsigned)v0); bit >= 0; --bit) {
    rn_mont_mul(cur, cur, cur, M, cd.m2prime);
    if ((v0 >> bit) & 1) rn_mont_mul(cur, cur, x, M, cd.m2prime);
  }
  const bool live = kmine < n;
  uint32_t* T = table + ((size_t)k * windows + w) * digits * S;
  if (live) rn_store_n(T + (size_t)(v0 - 1) * S, cur, S);
  for (int v = v0 + 1; v <= v1; ++v) {
    rn_mont_mul(cur, cur, x, M, cd.m2prime);
    if (live) rn_store_n(T + (size_t)(v - 1) * S, cur, S);
  }
}

template <int P>
__global__ __launch_bounds__(256) void hint_rows_kernel(ClientDev cd, const uint32_t* __restrict__ H,
                                                        int n, const uint32_t* __restrict__ rowlist,
                                                        int nrows, const uint32_t* __restrict__ table,
                                                        int wbits, uint32_t* __restrict__ K) {
  constexpr int S = 64 * P;
  const int widx = wave_index();
  if (widx >= nrows) return;
  const int windows = (32 + wbits - 1) / wbits;
  const uint32_t digits = (1u << wbits) - 1;
  const int row = rowlist ? (int)rowlist[widx] : widx;
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  wn_load(acc, cd.R1);  // Montgomery form of 1
  const uint32_t* hrow = H + (size_t)row * n;
  for (int k = 0; k < n; ++k) {
    const uint32_t e = 0u - hrow[k];  // (-H_jk) mod 2^32
    const uint32_t* tk = table + (size_t)k * windows * digits * S;
    for (int w = 0; w < windows; ++w) {
      const uint32_t d = (e >> (wbits * w)) & digits;
      if (d != 0) {
        wn_load(b, tk + ((size_t)w * digits + (d - 1)) * S);
        mont_mul(acc, acc, b, M, cd.m2prime);
      }
    }
  }
  // leave Montgomery form scaled by 2^32: acc * 2^32 * R^{-1} = K_j * 2^32 mod N^2
  WNum<P> two32;
  wn_zero(two32);
  if (lane_id() == 1 / P) two32.v[1 % P] = 1;
  mont_mul(acc, acc, two32, M, cd.m2prime);
  wn_store_n(K + (size_t)row * cd.L, acc, cd.L);
}

// Few rows: each row's product over its n bases is split into `parts` chains of `span` bases,
// one wavefront per (row, part), and the parts are multiplied together afterwards.  A wave
// otherwise has to run all n W products of its row in sequence, each waiting for its table
// entry, and a few hundred rows cannot fill the chip.  Partial products stay in Montgomery
// form: partial[(i parts + part) S ..] for row index i < nrows.
template <int P>
__global__ __launch_bounds__(256) void hint_parts_kernel(ClientDev cd, const uint32_t* __restrict__ H,
                                                         int n, const uint32_t* __restrict__ rowlist,
                                                         int nrows, const uint32_t* __restrict__ table,
                                                         int wbits, int parts, int span,
                                                         uint32_t* __restrict__ partial) {
  constexpr int S = 64 * P;
  const int item = wave_index();
  if (item >= nrows * parts) return;
  const int i = item / parts, part = item - i * parts;
  const int row = rowlist ? (int)rowlist[i] : i;
  const int windows = (32 + wbits - 1) / wbits;
  const uint32_t digits = (1u << wbits) - 1;
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  wn_load(acc, cd.R1);  // Montgomery form of 1
  const uint32_t* hrow = H + (size_t)row * n;
  const int k1 = min(n, (part + 1) * span);
  for (int k = part * span; k < k1; ++k) {
    const uint32_t e = 0u - hrow[k];  // (-H_jk) mod 2^32
    const uint32_t* tk = table + (size_t)k * windows * digits * S;
    for (int w = 0; w < windows; ++w) {
      const uint32_t d = (e >> (wbits * w)) & digits;
      if (d != 0) {
        wn_load(b, tk + ((size_t)w * digits + (d - 1)) * S);
        mont_mul(acc, acc, b, M, cd.m2prime);
      }
    }
  }
  wn_store(partial + (size_t)item * S, acc);
}

// K'_j from row i's parts: their Montgomery product, left scaled by 2^32 as in hint_rows_kernel.
template <int P>
__global__ __launch_bounds__(256) void hint_join_kernel(ClientDev cd, const uint32_t* __restrict__ partial,
                                                        int parts, const uint32_t* __restrict__ rowlist,
                                                        int nrows, uint32_t* __restrict__ K) {
  constexpr int S = 64 * P;
  const int i = wave_index();
  if (i >= nrows) return;
  const int row = rowlist ? (int)rowlist[i] : i;
  WNum<P> M, acc, b;
  wn_load(M, cd.N2);
  const uint32_t* pr = partial + (size_t)i * parts * S;
  wn_load(acc, pr);
  for (int p = 1; p < parts; ++p) {
    wn_load(b, pr + (size_t)p * S);
    mont_mul(acc, acc, b, M, cd.m2prime);
  }
  WNum<P> two32;
  wn_zero(two32);
  if (lane_id() == 1 / P) two32.v[1 % P] = 1;
  mont_mul(acc, acc, two32, M, cd.m2prime);
  wn_store_n(K + (size_t)row * cd.L, acc, cd.L);
}

// Four rows per wavefront, one per 16-lane row (rownum.h): the same products as
// hint_rows_kernel, each row with its own table entries.  A zero digit multiplies by R mod N^2,
// the Montgomery form of 1, so the four rows stay in step.  When nrows is not a multiple of
// four, the last wavefront's spare rows repeat its last row and store nothing.
template <int P>
__global__ __launch_bounds__(256) void hint_rows_quad_kernel(ClientDev cd, const uint32_t* __restrict__ H,
                                                             int n, const uint32_t* __restrict__ rowlist,
                                                             int nrows, const uint32_t* __restrict__ table,
                                                             int wbits, uint32_t* __restrict__ K) {
  constexpr int S = 64 * P;
  constexpr int Q = 4 * P;  // limbs per lane, S = 16 Q
  const int widx = wave_index();
  if (4 * widx >= nrows) return;
  const int mine = 4 * widx + row_index();
  const int i = min(nrows - 1, mine);
  const int row = rowlist ? (int)rowlist[i] : i;
  const int windows = (32 + wbits - 1) / wbits;
  const uint32_t digits = (1u << wbits) - 1;
  RNum<Q> M, one, acc, b;
  rn_load(M, cd.N2);
  rn_load(one, cd.R1);  // Montgomery form of 1
  acc = one;
  const uint32_t* hrow = H + (size_t)row * n;
  for (int k = 0; k < n; ++k) {
    const uint32_t e = 0u - hrow[k];  // (-H_jk) mod 2^32
    const uint32_t* tk = table + (size_t)k * windows * digits * S;
    for (int w = 0; w < windows; ++w) {
      const uint32_t d = (e >> (wbits * w)) & digits;
      if (d != 0) rn_load(b, tk + ((size_t)w * digits + (d - 1)) * S);
      else b = one;
      rn_mont_mul(acc, acc, b, M, cd.m2prime);
    }
  }
  // leave Montgomery form scaled by 2^32: acc * 2^32 * R^{-1} = K_j * 2^32 mod N^2
  RNum<Q> two32;
  rn_zero(two32);
  if (row_lane() == 0) two32.v[1] = 1;
  rn_mont_mul(acc, acc, two32, M, cd.m2prime);
  if (mine < nrows) rn_store_n(K + (size_t)row * cd.L, acc, cd.L);
}

// The per-row key of the online combine: M'_j = N * (K'_j mod N), with K'_j = K_j 2^32 mod N^2.
// It is a plain product below N^2 and satisfies M'_j = N K_j 2^32 (mod N^2), so that
// K_j (1 + b N) 2^32 = K'_j + b M'_j (mod N^2).
template <int P, int PN>
__global__ __launch_bounds__(256) void combine_key_kernel(ClientDev cd,
                                                          const uint32_t* __restrict__ Kp,
                                                          const uint32_t* __restrict__ rowlist,
                                                          int nrows, uint32_t* __restrict__ Mp,
                                                          uint32_t* __restrict__ Y, int scaled) {
  constexpr int SN = 64 * PN;
  const int widx = wave_index();
  if (widx >= nrows) return;
  const int row = rowlist ? (int)rowlist[widx] : widx;
  WNum<PN> Nn, C1, C2, lo, hi, x, y;
  wn_load(Nn, cd.Nn);
  wn_load(C1, cd.C1);
  wn_load(C2, cd.C2);
  const uint32_t* kr = Kp + (size_t)row * cd.L;
  // K' = lo + hi R_N with lo < R_N and hi < N (K' < N^2 and N < R_N)
  wn_load_n(lo, kr, cd.L < SN ? cd.L : SN);
  if (cd.L > SN) wn_load_n(hi, kr + SN, cd.L - SN); else wn_zero(hi);
  mont_mul(x, lo, C1, Nn, cd.nprime);  // lo mod N          (C1 = R_N mod N)
  mont_mul(y, hi, C2, Nn, cd.nprime);  // hi R_N mod N      (C2 = R_N^2 mod N)
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < PN; ++j) {
    const uint64_t s = (uint64_t)x.v[j] + y.v[j] + carry;
    x.v[j] = (uint32_t)s;
    carry = (uint32_t)(s >> 32);
  }
  const uint64_t ovf = wn_resolve(x, (uint64_t)carry);
  wn_cond_sub(x, ovf, Nn);  // x = K' mod N
  if (Y) {
    // scaled: (K mod N) R_N = x 2^-32 R_N mod N = x D1 R_N^-1 (D1 = R_N^2 2^-32 mod N);
    // otherwise x R_N = x C2 R_N^-1 (C2 = R_N^2 mod N)
    WNum<PN> d, yv;
    wn_load(d, scaled ? cd.D1 : cd.C2);
    mont_mul(yv, x, d, Nn, cd.nprime);
    wn_store_n(Y + (size_t)row * cd.h, yv, cd.h);
  }
  // M' = N * x: h broadcast limbs of x times N shifted up one limb per step
  WNum<P> acc, Nsh;
  wn_zero(acc);
  wn_load(Nsh, cd.NP);
  uint64_t pend = 0;
  for (int i = 0; i < cd.h; ++i) {
    const uint32_t xi = wn_limb(x, i);
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint64_t t = (uint64_t)xi * Nsh.v[j] + acc.v[j] + c;
      acc.v[j] = (uint32_t)t;
      c = (uint32_t)(t >> 32);
    }
    pend += c;
    const uint32_t in = from_prev_lane(Nsh.v[P - 1]);
#pragma unroll
    for (int j = P - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
    Nsh.v[0] = in;
  }
  (void)wn_resolve(acc, pend);  // N x < N^2 fits in L limbs
  wn_store_n(Mp + (size_t)row * cd.L, acc, cd.L);
}

// K_j = K'_j 2^{-32} mod N^2 (one Montgomery reduction step), for hint export.
template <int P>
__global__ __launch_bounds__(256) void unscale_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                      int row0, int nrows, uint32_t* __restrict__ K) {
  const int widx = wave_index();
  if (widx >= nrows) return;
  WNum<P> M, t;
  wn_load(M, cd.N2);
  wn_load_n(t, Kp + (size_t)(row0 + widx) * cd.L, cd.L);
  uint64_t c = 0;
  redc_step(t, c, M, cd.m2prime);
  const uint64_t ovf = wn_resolve(t, c);
  wn_cond_sub(t, ovf, M);
  wn_store_n(K + (size_t)widx * cd.L, t, cd.L);
}

// Group key of the packed response (Alg. 3 with gamma = 2^t, offline part):
//   K_g = prod_{j < ell} K_{g ell + j}^{2^(t j)} mod N^2,
// by Horner from the last row of the group: acc <- acc^(2^t) * K_row (t squarings per row).
template <int P>
__global__ __launch_bounds__(256) void group_keys_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                         int rows, int ell, int t,
                                                         const uint32_t* __restrict__ glist,
                                                         int ngroups, uint32_t* __restrict__ Kg) {
  const int widx = wave_index();
  if (widx >= ngroups) return;
  const int g = glist ? (int)glist[widx] : widx;
  const int r0 = g * ell;
  const int r1 = min(rows, r0 + ell);
  WNum<P> M, CP, acc, x;
  wn_load(M, cd.N2);
  wn_load(CP, cd.CP);
  wn_load_n(acc, Kp + (size_t)(r1 - 1) * cd.L, cd.L);
  mont_mul(acc, acc, CP, M, cd.m2prime);  // K' 2^(64S-32) R^{-1} = K R
  for (int r = r1 - 2; r >= r0; --r) {
    for (int i = 0; i < t; ++i) mont_mul(acc, acc, acc, M, cd.m2prime);
    wn_load_n(x, Kp + (size_t)r * cd.L, cd.L);
    mont_mul(x, x, CP, M, cd.m2prime);
    mont_mul(acc, acc, x, M, cd.m2prime);
  }
  WNum<P> one;
  wn_zero(one);
  if (lane_id() == 0) one.v[0] = 1;
  mont_mul(acc, acc, one, M, cd.m2prime);
  wn_store_n(Kg + (size_t)g * cd.L, acc, cd.L);
}

// x <- x 2^(32 limbs) mod N^2: one Montgomery product by R^2 mod N^2 (x R), then one by the
// plain number 2^(32 limbs) (< N^2), which divides the R out again.
template <int P>
__global__ __launch_bounds__(256) void mul_pow2_limbs_kernel(ClientDev cd, uint32_t* __restrict__ x,
                                                             const uint32_t* __restrict__ rowlist, int nrows,
                                                             int limbs) {
  const int widx = wave_index();
  if (widx >= nrows) return;
  const int row = rowlist ? (int)rowlist[widx] : widx;
  WNum<P> M, RR, v;
  wn_load(M, cd.N2);
  wn_load(RR, cd.RR);
  wn_load_n(v, x + (size_t)row * cd.L, cd.L);
  mont_mul(v, v, RR, M, cd.m2prime);
  WNum<P> e;
#pragma unroll
  for (int j = 0; j < P; ++j) e.v[j] = P * lane_id() + j == limbs ? 1u : 0u;
  mont_mul(v, v, e, M, cd.m2prime);
  wn_store_n(x + (size_t)row * cd.L, v, cd.L);
}

void launch_group_keys(const ClientDev& cd, const uint32_t* Kp, int rows, int ell, int t,
                       const uint32_t* glist, int ngroups, uint32_t* Kg, hipStream_t s) {
  if (ngroups <= 0) return;
  const int blocks = (ngroups + 3) / 4;
  switch (cd.P) {
    case 1: group_keys_kernel<1><<<blocks, 256, 0, s>>>(cd, Kp, rows, ell, t, glist, ngroups, Kg); break;
    case 2: group_keys_kernel<2><<<blocks, 256, 0, s>>>(cd, Kp, rows, ell, t, glist, ngroups, Kg); break;
    case 3: group_keys_kernel<3><<<blocks, 256, 0, s>>>(cd, Kp, rows, ell, t, glist, ngroups, Kg); break;
    case 4: group_keys_kernel<4><<<blocks, 256, 0, s>>>(cd, Kp, rows, ell, t, glist, ngroups, Kg); break;
  }
}

void launch_mul_pow2_limbs(const ClientDev& cd, uint32_t* x, const uint32_t* rowlist, int nrows,
                           int limbs, hipStream_t s) {
  if (nrows <= 0) return;
  const int blocks = (nrows + 3) / 4;
  switch (cd.P) {
    case 1: mul_pow2_limbs_kernel<1><<<blocks, 256, 0, s>>>(cd, x, rowlist, nrows, limbs); break;
    case 2: mul_pow2_limbs_kernel<2><<<blocks, 256, 0, s>>>(cd, x, rowlist, nrows, limbs); break;
    case 3: mul_pow2_limbs_kernel<3><<<blocks, 256, 0, s>>>(cd, x, rowlist, nrows, limbs); break;
    case 4: mul_pow2_limbs_kernel<4><<<blocks, 256, 0, s>>>(cd, x, rowlist, nrows, limbs); break;
  }
}

void launch_build_table(const ClientDev& cd, const uint32_t* ck, int n, int windows,
                        uint32_t* table, hipStream_t s, int wbits) {
  // four segments per (base, window): four times the wavefronts, each with a quarter of the
  // chain of products
  const int segs = 4;
  if (n <= 0 || windows <= 0) return;
  // four bases per wavefront while that still leaves several wavefronts per SIMD
  const long long quad_waves = (long long)((n + 3) / 4) * windows * segs;
  if (quad_waves >= 3072) {
    const int blocks = (int)((quad_waves + 3) / 4);
    switch (cd.P) {
      case 1: build_table_quad_kernel<1><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
      case 2: build_table_quad_kernel<2><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
      case 3: build_table_quad_kernel<3><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
      case 4: build_table_quad_kernel<4><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
    }
    return;
  }
  const int waves = n * windows * segs;
  const int blocks = (waves + 3) / 4;
  switch (cd.P) {
    case 1: build_table_kernel<1><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
    case 2: build_table_kernel<2><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
    case 3: build_table_kernel<3><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
    case 4: build_table_kernel<4><<<blocks, 256, 0, s>>>(cd, ck, n, windows, wbits, segs, table); break;
  }
}

int hint_parts(int nrows, int n) {
  if (nrows >= kSplitRowsBelow || n < 2) return 1;
  // enough (row, part) items to fill the chip, but at most 64 parts: the join multiplies a
  // row's parts in sequence, so its chain grows with their number
  const int want = std::min({n, 64, (int)((kQuadItems + nrows - 1) / nrows)});
  const int span = (n + want - 1) / want;
  return (n + span - 1) / span;  // no empty part
}

void launch_hint_rows_split(const ClientDev& cd, const uint32_t* H, int n, const uint32_t* rowlist,
                            int nrows, const uint32_t* table, int wbits, int parts, uint32_t* partial,
                            uint32_t* K, hipStream_t s) {
  if (nrows <= 0) return;
  const int span = (n + parts - 1) / parts;
  const long long items = (long long)nrows * parts;
  const int blocks = (int)((items + 3) / 4), jblocks = (nrows + 3) / 4;
#define ZP_SPLIT(PP)                                                                                \
  hint_parts_kernel<PP><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, parts, span, partial); \
  hint_join_kernel<PP><<<jblocks, 256, 0, s>>>(cd, partial, parts, rowlist, nrows, K)
  switch (cd.P) {
    case 1: ZP_SPLIT(1); break;
    case 2: ZP_SPLIT(2); break;
    case 3: ZP_SPLIT(3); break;
    case 4: ZP_SPLIT(4); break;
  }
#undef ZP_SPLIT
}

void launch_hint_rows(const ClientDev& cd, const uint32_t* H, int n, const uint32_t* rowlist,
                      int nrows, const uint32_t* table, int wbits, uint32_t* K, hipStream_t s) {
  if (nrows <= 0) return;
  // four rows per wavefront while that still leaves several wavefronts per SIMD
  if (nrows >= 16384) {
    const int blocks = ((nrows + 3) / 4 + 3) / 4;
    switch (cd.P) {
      case 1: hint_rows_quad_kernel<1><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
      case 2: hint_rows_quad_kernel<2><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
      case 3: hint_rows_quad_kernel<3><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
      case 4: hint_rows_quad_kernel<4><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
    }
    return;
  }
  const int blocks = (nrows + 3) / 4;
  switch (cd.P) {
    case 1: hint_rows_kernel<1><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
    case 2: hint_rows_kernel<2><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
    case 3: hint_rows_kernel<3><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
    case 4: hint_rows_kernel<4><<<blocks, 256, 0, s>>>(cd, H, n, rowlist, nrows, table, wbits, K); break;
  }
}

void launch_combine_key(const ClientDev& cd, const uint32_t* Kp, const uint32_t* rowlist,
                        int nrows, uint32_t* Mp, uint32_t* Y, hipStream_t s, bool scaled) {
  if (nrows <= 0) return;
  const int blocks = (nrows + 3) / 4;
  switch (cd.P) {
    case 1: combine_key_kernel<1, 1><<<blocks, 256, 0, s>>>(cd, Kp, rowlist, nrows, Mp, Y, scaled ? 1 : 0); break;
    case 2: combine_key_kernel<2, 1><<<blocks, 256, 0, s>>>(cd, Kp, rowlist, nrows, Mp, Y, scaled ? 1 : 0); break;
    case 3: combine_key_kernel<3, 2><<<blocks, 256, 0, s>>>(cd, Kp, rowlist, nrows, Mp, Y, scaled ? 1 : 0); break;
    case 4: combine_key_kernel<4, 2><<<blocks, 256, 0, s>>>(cd, Kp, rowlist, nrows, Mp, Y, scaled ? 1 : 0); break;
  }
}

void launch_unscale(const ClientDev& cd, const uint32_t* Kp, int row0, int nrows, uint32_t* K,
                    hipStream_t s) {
  if (nrows <= 0) return;
  const int blocks = (nrows + 3) / 4;
  switch (cd.P) {
    case 1: unscale_kernel<1><<<blocks, 256, 0, s>>>(cd, Kp, row0, nrows, K); break;
    case 2: unscale_kernel<2><<<blocks, 256, 0, s>>>(cd, Kp, row0, nrows, K); break;
    case 3: unscale_kernel<3><<<blocks, 256, 0, s>>>(cd, Kp, row0, nrows, K); break;
    case 4: unscale_kernel<4><<<blocks, 256, 0, s>>>(cd, Kp, row0, nrows, K); break;
  }
}

}  // namespace zp
