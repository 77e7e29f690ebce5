// Combined response c_j = K_j (1 + b_j N) mod N^2 (Sec. 4.3, "Smaller responses w/ Paillier
// addition": the online answer b_j is folded into the offline hint K_j with one Paillier
// addition of Enc(b_j; 1) = (N+1)^b_j = 1 + b_j N mod N^2).
//
// K (1 + bN) = K + b N (K mod N)  (mod N^2), because N r = N K b (mod N^2) for r = K b mod N.
// The hint step stores, per row, K' = K 2^32 mod N^2 and M' = N (K' mod N) (a plain product
// below N^2, congruent to N K 2^32), so the combine is a single Montgomery step:
//   t = K' + b M'            (< N^2 2^32)
//   c = (t + q N^2) / 2^32   with q = -t N^{-2} mod 2^32, so c = K (1 + bN) mod N^2, c < 2 N^2,
// followed by one conditional subtraction of N^2.  About 2 L word products per row; the
// kernel is bound by reading K' and M' and writing c.
#include "internal.h"
#include "rownum.h"
#include "wavenum.h"

namespace zp {

// Each wave combines kRowsPerWave consecutive rows, loading the modulus once and the next
// row's K', M' and b while it reduces the current one.
constexpr int kRowsPerWave = 8;

template <int P>
__global__ __launch_bounds__(256) void compress_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                       const uint32_t* __restrict__ Mp,
                                                       const uint32_t* __restrict__ b, int rows,
                                                       uint32_t* __restrict__ C) {
  const int wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = wave * kRowsPerWave;
  if (row0 >= rows) return;
  const int row1 = min(rows, row0 + kRowsPerWave);
  WNum<P> M2, t, m, tn, mn;
  wn_load(M2, cd.N2);
  wn_load_n(t, Kp + (size_t)row0 * cd.L, cd.L);
  wn_load_n(m, Mp + (size_t)row0 * cd.L, cd.L);
  uint32_t bj = b[row0], bn = 0;
  for (int row = row0; row < row1; ++row) {
    if (row + 1 < row1) {
      wn_load_n(tn, Kp + (size_t)(row + 1) * cd.L, cd.L);
      wn_load_n(mn, Mp + (size_t)(row + 1) * cd.L, cd.L);
      bn = b[row + 1];
    }
    uint64_t c = 0;
    mont_step(t, c, bj, m, M2, cd.m2prime);
    const uint64_t ovf = wn_resolve(t, c);
    wn_cond_sub(t, ovf, M2);
    wn_store_n(C + (size_t)row * cd.L, t, cd.L);
    t = tn;
    m = mn;
    bj = bn;
  }
}

// compress_kernel with four rows per wavefront, one per 16-lane row (rownum.h): Q = 4P limbs
// per lane, 16-byte row pieces when the rows fill the lanes (kFull), and every row's K', M'
// and b requested before the first row is reduced.
template <int P, bool kFull>
__global__ __launch_bounds__(256) void compress_quad_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                            const uint32_t* __restrict__ Mp,
                                                            const uint32_t* __restrict__ b, int rows,
                                                            uint32_t* __restrict__ C) {
  constexpr int Q = 4 * P;
  constexpr int kPasses = kRowsPerWave / 4;
  const int wave = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = wave * kRowsPerWave;
  if (row0 >= rows) return;
  RNum<Q> t[kPasses], m[kPasses];
  uint32_t bj[kPasses];
#pragma unroll
  for (int i = 0; i < kPasses; ++i) {
    const int row = min(rows - 1, row0 + 4 * i + row_index());
    rn_load_row<P, kFull>(t[i], Kp + (size_t)row * cd.L, cd.L);
    rn_load_row<P, kFull>(m[i], Mp + (size_t)row * cd.L, cd.L);
    bj[i] = b[row];
  }
  RNum<Q> M2;
  rn_load(M2, cd.N2);
#pragma unroll
  for (int i = 0; i < kPasses; ++i) {
    if (row0 + 4 * i >= rows) break;
    const int mine = row0 + 4 * i + row_index();
    rn_zero_above<P, kFull>(t[i], cd.L);
    rn_zero_above<P, kFull>(m[i], cd.L);
    uint64_t c = 0;
    rn_mont_step(t[i], c, bj[i], m[i], M2, cd.m2prime);
    const uint64_t ovf = rn_resolve(t[i], c);
    rn_cond_sub(t[i], ovf, M2);
    if (mine < rows) rn_store_row<P, kFull>(C + (size_t)mine * cd.L, t[i], cd.L);
  }
}

void launch_compress(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Mp,
                     const uint32_t* b, int rows, uint32_t* C, hipStream_t s) {
  if (rows <= 0) return;
  const int waves = (rows + kRowsPerWave - 1) / kRowsPerWave;
  const int blocks = (waves + 3) / 4;
  if (rows >= kQuadItems) {  // four rows per wavefront once that still leaves several per SIMD
    // 16-byte pieces need rows that fill the lanes and 16-byte aligned arrays
    const bool full = cd.L == 64 * cd.P && ((reinterpret_cast<uintptr_t>(Kp) | reinterpret_cast<uintptr_t>(Mp) |
                                              reinterpret_cast<uintptr_t>(C)) & 15) == 0;
#define ZP_COMPRESS_QUAD(PP)                                                                        \
  (full ? compress_quad_kernel<PP, true><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C)               \
        : compress_quad_kernel<PP, false><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C))
    switch (cd.P) {
      case 1: ZP_COMPRESS_QUAD(1); break;
      case 2: ZP_COMPRESS_QUAD(2); break;
      case 3: ZP_COMPRESS_QUAD(3); break;
      case 4: ZP_COMPRESS_QUAD(4); break;
    }
#undef ZP_COMPRESS_QUAD
    return;
  }
  switch (cd.P) {
    case 1: compress_kernel<1><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C); break;
    case 2: compress_kernel<2><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C); break;
    case 3: compress_kernel<3><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C); break;
    case 4: compress_kernel<4><<<blocks, 256, 0, s>>>(cd, Kp, Mp, b, rows, C); break;
  }
}

// Packed response (Alg. 3, online part, gamma = 2^t): for group g of ell rows,
//   c_g = K_g (1 + beta_g N) mod N^2 = K_g + beta_g M_g mod N^2,  beta_g = sum_j b_{g ell + j} 2^(t j),
// with M_g = N (K_g mod N) < N^2 kept as Mr = M_g 2^(32h) mod N^2.  beta_g < gamma^ell < N has
// at most h limbs, so a Montgomery product truncated after those h steps (each dividing by
// 2^32) gives beta_g M_g mod N^2: half the serial steps of a full product with R = 2^(32 S).
// Since t >= 32 the answers occupy disjoint bit ranges of beta_g: each limb takes at most two
// of them.  One wavefront per group.
template <int P>
__global__ __launch_bounds__(256) void compress_packed_kernel(
    ClientDev cd, const uint32_t* __restrict__ Kg, const uint32_t* __restrict__ Mr,
    const uint32_t* __restrict__ b, int rows, int ell, int t, uint32_t* __restrict__ C) {
  const int g = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = g * ell;
  if (r0 >= rows) return;
  const int nj = min(ell, rows - r0);
  WNum<P> beta, mr, M2, acc;
#pragma unroll
  for (int jj = 0; jj < P; ++jj) {
    const int w = P * lane_id() + jj;  // limb index: bits [32w, 32w + 32)
    uint32_t v = 0;
    const int jlo = max(0, (32 * w - 31 + t - 1) / t);
    const int jhi = min(nj - 1, (32 * w + 31) / t);
    for (int j = jlo; j <= jhi; ++j) {
      const int sh = t * j - 32 * w;
      const uint32_t bj = b[r0 + j];
      v |= sh >= 0 ? (bj << sh) : (bj >> (-sh));
    }
    beta.v[jj] = v;
  }
  wn_load_n(mr, Mr + (size_t)g * cd.L, cd.L);
  wn_load(M2, cd.N2);
  mont_mul_trunc(acc, beta, cd.h, mr, M2, cd.m2prime);  // beta_g M_g mod N^2
  WNum<P> k;
  wn_load_n(k, Kg + (size_t)g * cd.L, cd.L);
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t s = (uint64_t)acc.v[j] + k.v[j] + carry;
    acc.v[j] = (uint32_t)s;
    carry = (uint32_t)(s >> 32);
  }
  const uint64_t ovf = wn_resolve(acc, (uint64_t)carry);
  wn_cond_sub(acc, ovf, M2);
  wn_store_n(C + (size_t)g * cd.L, acc, cd.L);
}

void launch_compress_packed(const ClientDev& cd, const uint32_t* Kg, const uint32_t* Mr,
                            const uint32_t* b, int rows, int ell, int t, uint32_t* C, hipStream_t s) {
  if (rows <= 0) return;
  const int groups = (rows + ell - 1) / ell;
  const int blocks = (groups + 3) / 4;
  switch (cd.P) {
    case 1: compress_packed_kernel<1><<<blocks, 256, 0, s>>>(cd, Kg, Mr, b, rows, ell, t, C); break;
    case 2: compress_packed_kernel<2><<<blocks, 256, 0, s>>>(cd, Kg, Mr, b, rows, ell, t, C); break;
    case 3: compress_packed_kernel<3><<<blocks, 256, 0, s>>>(cd, Kg, Mr, b, rows, ell, t, C); break;
    case 4: compress_packed_kernel<4><<<blocks, 256, 0, s>>>(cd, Kg, Mr, b, rows, ell, t, C); break;
  }
}

// Combined response of the full protocol (Alg. 5 Response with the Sec. 4.3 Paillier
// addition): c_j = K_j (+) Enc(t_j; 1) = K_j (1 + t_j N) mod N^2 for an h-limb offset answer t_j.
//   K (1 + tN) = K + N (t (K mod N) mod N)   (mod N^2).
// With y = (K mod N) R_N mod N stored by the hint step:
//   z = t (K mod N) mod N    = t y R_N^{-1}   (one Montgomery product mod N, h multiplier limbs),
//   K = K' 2^{-32} mod N^2                   (one Montgomery reduction step; packed group
//                                             keys are stored as K itself),
//   c = K + N z mod N^2.
// One wavefront per row.
template <int P, int PN>
__global__ __launch_bounds__(256) void compress_offset_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                              const uint32_t* __restrict__ Y,
                                                              const uint32_t* __restrict__ T, int rows,
                                                              uint32_t* __restrict__ C, int scaled) {
  const int row = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= rows) return;
  const uint32_t* kr = Kp + (size_t)row * cd.L;
  WNum<PN> Nn, y, tv, z;
  wn_load(Nn, cd.Nn);
  wn_load_n(y, Y + (size_t)row * cd.h, cd.h);
  wn_load_n(tv, T + (size_t)row * cd.h, cd.h);
  mont_mul_short(z, tv, cd.h, y, Nn, cd.nprime);
  // N z: the h limbs of z times N, N shifted up one limb per step
  WNum<P> acc, Nsh, k, M2;
  wn_zero(acc);
  wn_load(Nsh, cd.NP);
  uint64_t pend = 0;
  for (int i = 0; i < cd.h; ++i) {
    const uint32_t zi = wn_limb(z, i);
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint64_t t = (uint64_t)zi * Nsh.v[j] + acc.v[j] + c;
      acc.v[j] = (uint32_t)t;
      c = (uint32_t)(t >> 32);
    }
    pend += c;
    const uint32_t in = from_prev_lane(Nsh.v[P - 1]);
#pragma unroll
    for (int j = P - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
    Nsh.v[0] = in;
  }
  (void)wn_resolve(acc, pend);  // N z < N^2
  // K = K' 2^{-32} mod N^2
  wn_load(M2, cd.N2);
  wn_load_n(k, kr, cd.L);
  uint64_t ovf;
  if (scaled) {
    uint64_t kc = 0;
    redc_step(k, kc, M2, cd.m2prime);
    ovf = wn_resolve(k, kc);
    wn_cond_sub(k, ovf, M2);
  }
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t s = (uint64_t)acc.v[j] + k.v[j] + carry;
    acc.v[j] = (uint32_t)s;
    carry = (uint32_t)(s >> 32);
  }
  ovf = wn_resolve(acc, (uint64_t)carry);
  wn_cond_sub(acc, ovf, M2);
  wn_store_n(C + (size_t)row * cd.L, acc, cd.L);
}

// The same combine with four rows per wavefront, one per 16-lane row (rownum.h): Q = 4 P limbs
// per lane for numbers mod N^2 and QN = 4 PN for numbers mod N, so R and R_N are those of the
// one-row layout.  Spare rows of the last wavefront repeat its last row and store nothing.
template <int P, int PN>
__global__ __launch_bounds__(256) void compress_offset_quad_kernel(ClientDev cd, const uint32_t* __restrict__ Kp,
                                                                   const uint32_t* __restrict__ Y,
                                                                   const uint32_t* __restrict__ T, int rows,
                                                                   uint32_t* __restrict__ C, int scaled) {
  constexpr int Q = 4 * P, QN = 4 * PN;
  const int widx = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (4 * widx >= rows) return;
  const int mine = 4 * widx + row_index();
  const int row = min(rows - 1, mine);
  RNum<QN> Nn, y, tv, z;
  rn_load(Nn, cd.Nn);
  rn_load_n(y, Y + (size_t)row * cd.h, cd.h);
  rn_load_n(tv, T + (size_t)row * cd.h, cd.h);
  rn_mont_mul(z, tv, y, Nn, cd.nprime);  // z = t (K mod N) mod N
  // N z: the limbs of z (broadcast from their lane) times N, N shifted up one limb per step
  RNum<Q> acc, Nsh, k, M2;
  rn_zero(acc);
  rn_load(Nsh, cd.NP);
  uint64_t pend = 0;
  for (int src = 0; src < 16; ++src) {
    const int addr = row_src_addr(src);
    uint32_t zl[QN];
#pragma unroll
    for (int jj = 0; jj < QN; ++jj) zl[jj] = row_pick(addr, z.v[jj]);
#pragma unroll
    for (int jj = 0; jj < QN; ++jj) {
      uint32_t c = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const uint64_t t = (uint64_t)zl[jj] * Nsh.v[j] + acc.v[j] + c;
        acc.v[j] = (uint32_t)t;
        c = (uint32_t)(t >> 32);
      }
      pend += c;
      const uint32_t in = row_from_prev(Nsh.v[Q - 1]);
#pragma unroll
      for (int j = Q - 1; j > 0; --j) Nsh.v[j] = Nsh.v[j - 1];
      Nsh.v[0] = in;
    }
  }
  (void)rn_resolve(acc, pend);  // N z < N^2
  rn_load(M2, cd.N2);
  rn_load_n(k, Kp + (size_t)row * cd.L, cd.L);
  uint64_t ovf;
  if (scaled) {  // K = K' 2^{-32} mod N^2
    uint64_t kc = 0;
    rn_redc_step(k, kc, M2, cd.m2prime);
    ovf = rn_resolve(k, kc);
    rn_cond_sub(k, ovf, M2);
  }
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const uint64_t sum = (uint64_t)acc.v[j] + k.v[j] + carry;
    acc.v[j] = (uint32_t)sum;
    carry = (uint32_t)(sum >> 32);
  }
  ovf = rn_resolve(acc, (uint64_t)carry);
  rn_cond_sub(acc, ovf, M2);
  if (mine < rows) rn_store_n(C + (size_t)row * cd.L, acc, cd.L);
}

void launch_compress_offset(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Y,
                            const uint32_t* T, int rows, uint32_t* C, hipStream_t s, bool scaled) {
  if (rows <= 0) return;
  const int sc = scaled ? 1 : 0;
  // four rows per wavefront while that still leaves several wavefronts per SIMD
  if (rows >= 16384) {
    const int blocks = ((rows + 3) / 4 + 3) / 4;
    switch (cd.P) {
      case 1: compress_offset_quad_kernel<1, 1><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
      case 2: compress_offset_quad_kernel<2, 1><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
      case 3: compress_offset_quad_kernel<3, 2><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
      case 4: compress_offset_quad_kernel<4, 2><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
    }
    return;
  }
  const int blocks = (rows + 3) / 4;
  switch (cd.P) {
    case 1: compress_offset_kernel<1, 1><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
    case 2: compress_offset_kernel<2, 1><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
    case 3: compress_offset_kernel<3, 2><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
    case 4: compress_offset_kernel<4, 2><<<blocks, 256, 0, s>>>(cd, Kp, Y, T, rows, C, sc); break;
  }
}

}  // namespace zp
