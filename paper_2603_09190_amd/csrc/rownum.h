// Row-distributed multiprecision arithmetic for gfx950: four big integers per wavefront, one
// per 16-lane row.
//
// Lane l of row r (lanes 16r .. 16r + 15) owns limbs [P (l mod 16), P (l mod 16) + P) of row
// r's number, S = 16 P little-endian 32-bit limbs in all, zero padded above the modulus, so
// Montgomery arithmetic uses R = 2^(32 S).  The algorithms are those of wavenum.h (CIOS with
// a pending carry word per lane, resolved at the end), with moves inside a row done by DPP row
// operations and broadcasts of a row's lane by ds_bpermute.  Compared with one number per
// wavefront, a CIOS step amortises its fixed work (the broadcast of a_i, the quotient, the
// one-limb shift) over four times as many limbs per lane.
//
// The four rows are independent: each routine works on every row at once, with per-row
// operands, and must be called by all 64 lanes of a wave with wave-uniform modulus arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wavenum.h"

namespace zp {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // as in internal.h

// DPP row controls: row_shl:1 gives lane i of a row the value of lane i+1, row_shr:1 that of
// lane i-1 (a lane without a source in its row keeps `old`, here 0); row_newbcast:k gives
// every lane of a row the value of that row's lane k.
constexpr int kDppRowShl1 = 0x101;
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowBcast = 0x150;

__device__ __forceinline__ int row_lane() { return lane_id() & 15; }
__device__ __forceinline__ int row_index() { return lane_id() >> 4; }

__device__ __forceinline__ uint32_t row_from_next(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShl1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t row_from_prev(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowShr1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t row_from_prev64(uint64_t x) {
  return ((uint64_t)row_from_prev((uint32_t)(x >> 32)) << 32) | row_from_prev((uint32_t)x);
}
template <int K>
__device__ __forceinline__ uint32_t row_bcast(uint32_t x) {
  static_assert(K >= 0 && K < 16, "row lane");
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppRowBcast + K, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t row_bcast_top64(uint64_t x) {
  return ((uint64_t)row_bcast<15>((uint32_t)(x >> 32)) << 32) | row_bcast<15>((uint32_t)x);
}
// value of lane `src` of this lane's row (src may vary between iterations); `addr` is the
// byte address ds_bpermute takes, row_src_addr(src)
__device__ __forceinline__ int row_src_addr(int src) { return ((lane_id() & ~15) | src) << 2; }
__device__ __forceinline__ uint32_t row_pick(int addr, uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)x);
}

template <int P>
struct RNum {
  uint32_t v[P];
};

template <int P>
__device__ __forceinline__ void rn_zero(RNum<P>& x) {
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = 0;
}

// `src` points at this row's number (each row passes its own); the first nl limbs are read
// and the rest are zero.
template <int P>
__device__ __forceinline__ void rn_load_n(RNum<P>& x, const uint32_t* __restrict__ src, int nl) {
  const int base = P * row_lane();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = (base + j < nl) ? src[base + j] : 0u;
}

template <int P>
__device__ __forceinline__ void rn_load(RNum<P>& x, const uint32_t* __restrict__ src) {
  const uint32_t* p = src + P * row_lane();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = p[j];
}

template <int P>
__device__ __forceinline__ void rn_store_n(uint32_t* __restrict__ dst, const RNum<P>& x, int nl) {
  const int base = P * row_lane();
#pragma unroll
  for (int j = 0; j < P; ++j)
    if (base + j < nl) dst[base + j] = x.v[j];
}

// A row of 4P limbs per lane (Q = 4P) from a row array of nl limbs, for kernels that request
// several rows' operands before using the first: with kFull (nl == 16 Q, 16-byte aligned
// rows) each lane reads its limbs as 16-byte pieces; otherwise every lane loads at indices
// clamped to the row, with no branch between the loads, and rn_zero_above clears the limbs at
// or beyond nl before use.
template <int P, bool kFull>
__device__ __forceinline__ void rn_load_row(RNum<4 * P>& x, const uint32_t* __restrict__ src, int nl) {
  constexpr int Q = 4 * P;
  if (kFull) {
    const u32x4* p = reinterpret_cast<const u32x4*>(src + Q * row_lane());
#pragma unroll
    for (int v = 0; v < Q / 4; ++v) {
      const u32x4 w = p[v];
      x.v[4 * v] = w.x; x.v[4 * v + 1] = w.y; x.v[4 * v + 2] = w.z; x.v[4 * v + 3] = w.w;
    }
  } else {
    const int base = Q * row_lane();
#pragma unroll
    for (int j = 0; j < Q; ++j) x.v[j] = src[min(base + j, nl - 1)];
  }
}

template <int P, bool kFull>
__device__ __forceinline__ void rn_zero_above(RNum<4 * P>& x, int nl) {
  if (kFull) return;
  const int base = 4 * P * row_lane();
#pragma unroll
  for (int j = 0; j < 4 * P; ++j) x.v[j] = base + j < nl ? x.v[j] : 0u;
}

// The counterpart of rn_load_row for stores (kFull: 16-byte pieces).
template <int P, bool kFull>
__device__ __forceinline__ void rn_store_row(uint32_t* __restrict__ dst, const RNum<4 * P>& x, int nl) {
  constexpr int Q = 4 * P;
  if (kFull) {
    u32x4* p = reinterpret_cast<u32x4*>(dst + Q * row_lane());
#pragma unroll
    for (int v = 0; v < Q / 4; ++v) p[v] = u32x4{x.v[4 * v], x.v[4 * v + 1], x.v[4 * v + 2], x.v[4 * v + 3]};
  } else {
    rn_store_n(dst, x, nl);
  }
}

// Resolve pending per-lane carries; returns each row's carry out of its top limb.
template <int P>
__device__ __forceinline__ uint64_t rn_resolve(RNum<P>& t, uint64_t c) {
  uint64_t ovf = 0;
  while (true) {
    ovf += row_bcast_top64(c);
    uint64_t acc = row_from_prev64(c);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      acc += t.v[j];
      t.v[j] = (uint32_t)acc;
      acc >>= 32;
    }
    c = acc;
    if (!wave_any(c != 0)) break;
  }
  return ovf;
}

// Per row: if (x + ovf 2^(32S)) >= m then x -= m.  Requires the value to be < 2m.
template <int P>
__device__ __forceinline__ void rn_cond_sub(RNum<P>& x, uint64_t ovf, const RNum<P>& m) {
  RNum<P> d;
  uint32_t br = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t s = (uint64_t)x.v[j] - m.v[j] - br;
    d.v[j] = (uint32_t)s;
    br = (uint32_t)(s >> 63);
  }
  uint32_t final_borrow = 0;
  while (true) {
    final_borrow += row_bcast<15>(br);
    uint32_t b = row_from_prev(br);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const uint64_t u = (uint64_t)d.v[j] - b;
      d.v[j] = (uint32_t)u;
      b = (uint32_t)(u >> 63);
    }
    br = b;
    if (!wave_any(br != 0)) break;
  }
  if (ovf != 0 || final_borrow == 0) {
#pragma unroll
    for (int j = 0; j < P; ++j) x.v[j] = d.v[j];
  }
}

// t = (t + q m) / 2^32 with q = t_0 mprime mod 2^32 (per row).
template <int P>
__device__ __forceinline__ void rn_redc_step(RNum<P>& t, uint64_t& c, const RNum<P>& m,
                                             uint32_t mprime) {
  const uint32_t q = row_bcast<0>(t.v[0]) * mprime;
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t x = (uint64_t)q * m.v[j] + t.v[j];
    unsigned int c1;
    t.v[j] = __builtin_addc((uint32_t)x, carry, 0u, &c1);
    carry = (uint32_t)(x >> 32) + c1;
  }
  c += carry;
  const uint32_t up = row_from_next(t.v[0]);
#pragma unroll
  for (int j = 0; j < P - 1; ++j) t.v[j] = t.v[j + 1];
  const uint64_t top = (uint64_t)up + c;
  t.v[P - 1] = (uint32_t)top;
  c = top >> 32;
}

template <int P>
__device__ __forceinline__ void rn_mont_step(RNum<P>& t, uint64_t& c, uint32_t ai,
                                             const RNum<P>& b, const RNum<P>& m, uint32_t mprime) {
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t x = (uint64_t)ai * b.v[j] + t.v[j];
    unsigned int c1;
    t.v[j] = __builtin_addc((uint32_t)x, carry, 0u, &c1);
    carry = (uint32_t)(x >> 32) + c1;
  }
  c += carry;
  rn_redc_step(t, c, m, mprime);
}

// out = a b R^{-1} mod m per row, canonical, for a < R and b < m (m odd, m < R).  The limbs of
// a are broadcast one source lane ahead of their use.
template <int P>
__device__ __forceinline__ void rn_mont_mul(RNum<P>& out, const RNum<P>& a, const RNum<P>& b,
                                            const RNum<P>& m, uint32_t mprime) {
  RNum<P> t;
  rn_zero(t);
  uint64_t c = 0;
  uint32_t cur[P], nxt[P];
#pragma unroll
  for (int jj = 0; jj < P; ++jj) cur[jj] = row_pick(row_src_addr(0), a.v[jj]);
  for (int src = 0; src < 16; ++src) {
    const int addr = row_src_addr((src + 1) & 15);
#pragma unroll
    for (int jj = 0; jj < P; ++jj) nxt[jj] = row_pick(addr, a.v[jj]);
#pragma unroll
    for (int jj = 0; jj < P; ++jj) rn_mont_step(t, c, cur[jj], b, m, mprime);
#pragma unroll
    for (int jj = 0; jj < P; ++jj) cur[jj] = nxt[jj];
  }
  const uint64_t ovf = rn_resolve(t, c);
  rn_cond_sub(t, ovf, m);
  out = t;
}

}  // namespace zp
