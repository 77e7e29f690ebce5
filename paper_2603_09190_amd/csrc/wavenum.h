// Wave-distributed multiprecision arithmetic for gfx950 (wave64).
//
// One wavefront holds one big integer of S = 64*P little-endian 32-bit limbs: lane l owns
// limbs [P*l, P*l + P) in registers ("P-layout").  Moduli shorter than S limbs are zero
// padded, so Montgomery arithmetic uses R = 2^(32*S).
//
// Montgomery multiplication is the coarsely integrated operand scanning (CIOS) method of
// Koc, Acar and Kaliski (1996): for each limb a_i of the first operand, t += a_i*b, then
// t += q*M with q = t_0 * (-M^{-1}) mod 2^32, then t /= 2^32.  Here the division by 2^32 is
// a one-limb shift across lanes, and each lane keeps the carry out of its own P-limb chain
// as a pending 64-bit word (positioned just above its top limb) instead of propagating it
// through the whole wave every step; pending carries are resolved once at the end.
//
// Every routine must be called by all 64 lanes of a wave with wave-uniform arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zp {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// One-lane moves use DPP wavefront shifts, a VALU operand modifier (no LDS round trip):
// wave_shl:1 gives lane l the value of lane l+1, wave_shr:1 the value of lane l-1; a lane
// without a source keeps the `old` operand, here 0.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

// Lane l receives lane l+1's value; lane 63 receives 0.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppWaveShl1, 0xF, 0xF, false);
}

// Lane l receives lane l-1's value; lane 0 receives 0.
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppWaveShr1, 0xF, 0xF, false);
}

__device__ __forceinline__ uint64_t from_prev_lane64(uint64_t x) {
  uint32_t lo = from_prev_lane((uint32_t)x);
  uint32_t hi = from_prev_lane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Sums by DPP quad permutes and row mirrors, VALU operand modifiers with no LDS round trip:
// quad_perm [1,0,3,2] and [2,3,0,1] give every lane its quad's sum; row_half_mirror (lane i of
// an 8-lane half takes lane 7-i) and row_mirror (lane i of a 16-lane row takes lane 15-i) then
// pair each lane with the other quad and the other half.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

// Wrapping sum over the 16 lanes of each row, in every lane of that row.
__device__ __forceinline__ uint32_t row_sum16(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppQuadXor1, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppQuadXor2, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowHalfMirror, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowMirror, 0xF, 0xF, false);
  return v;
}

// Wrapping sum over all 64 lanes, wave-uniform: the four row sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ uint32_t wave_sum64(uint32_t v) {
  v = row_sum16(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

__device__ __forceinline__ uint32_t bcast(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

template <int P>
struct WNum {
  uint32_t v[P];
};

template <int P>
__device__ __forceinline__ void wn_zero(WNum<P>& x) {
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = 0;
}

// Load/store S = 64*P limbs from a contiguous little-endian array (fully coalesced).
template <int P>
__device__ __forceinline__ void wn_load(WNum<P>& x, const uint32_t* __restrict__ src) {
  const uint32_t* p = src + P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = p[j];
}

// Load the first `nl` limbs and zero the rest (nl <= S).
template <int P>
__device__ __forceinline__ void wn_load_n(WNum<P>& x, const uint32_t* __restrict__ src, int nl) {
  const int base = P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j) x.v[j] = (base + j < nl) ? src[base + j] : 0u;
}

template <int P>
__device__ __forceinline__ void wn_store(uint32_t* __restrict__ dst, const WNum<P>& x) {
  uint32_t* p = dst + P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j) p[j] = x.v[j];
}

template <int P>
__device__ __forceinline__ void wn_store_n(uint32_t* __restrict__ dst, const WNum<P>& x, int nl) {
  const int base = P * lane_id();
#pragma unroll
  for (int j = 0; j < P; ++j)
    if (base + j < nl) dst[base + j] = x.v[j];
}

// Limb i of a distributed number, as a wave-uniform value.
template <int P>
__device__ __forceinline__ uint32_t wn_limb(const WNum<P>& x, int i) {
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < P; ++j)
    if (i % P == j) r = bcast(x.v[j], i / P);
  return r;
}

// Resolve pending per-lane carries: value = sum_l (chunk_l + c_l * 2^(32P)) * 2^(32Pl).
// Returns the carry out of the top limb (the part at and above 2^(32S)), wave-uniform.
template <int P>
__device__ __forceinline__ uint64_t wn_resolve(WNum<P>& t, uint64_t c) {
  uint64_t ovf = 0;
  while (true) {
    ovf += bcast((uint32_t)c, 63) | ((uint64_t)bcast((uint32_t)(c >> 32), 63) << 32);
    uint64_t cin = from_prev_lane64(c);
    uint64_t acc = cin;
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

// If (x + ovf*2^(32S)) >= m then x -= m.  Requires the value to be < 2m.
template <int P>
__device__ __forceinline__ void wn_cond_sub(WNum<P>& x, uint64_t ovf, const WNum<P>& m) {
  WNum<P> d;
  uint32_t br = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint64_t s = (uint64_t)x.v[j] - m.v[j] - br;
    d.v[j] = (uint32_t)s;
    br = (uint32_t)(s >> 63);
  }
  // ripple borrows across lanes; borrows leaving lane 63 are counted in final_borrow
  uint32_t final_borrow = 0;
  while (true) {
    final_borrow += bcast(br, 63);
    uint32_t b = from_prev_lane(br);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      uint64_t u = (uint64_t)d.v[j] - b;
      d.v[j] = (uint32_t)u;
      b = (uint32_t)(u >> 63);
    }
    br = b;
    if (!wave_any(br != 0)) break;
  }
  // value >= m  <=>  ovf*2^(32S) + x - m >= 0  <=>  not (ovf == 0 and a borrow left the top)
  const bool ge = (ovf != 0) || (final_borrow == 0);
  if (ge) {
#pragma unroll
    for (int j = 0; j < P; ++j) x.v[j] = d.v[j];
  }
}

// The reduction half of a CIOS step: t = (t + q*m) / 2^32 with q = t_0 * mprime mod 2^32, so
// the division is exact.  c is the lane's pending carry word (see file comment).
template <int P>
__device__ __forceinline__ void redc_step(WNum<P>& t, uint64_t& c, const WNum<P>& m,
                                          uint32_t mprime) {
  const uint32_t q = bcast(t.v[0], 0) * mprime;
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t x = (uint64_t)q * m.v[j] + t.v[j];
    unsigned int c1;
    t.v[j] = __builtin_addc((uint32_t)x, carry, 0u, &c1);
    carry = (uint32_t)(x >> 32) + c1;
  }
  c += carry;
  // lane 0's limb 0 is now zero: shift the whole number down one limb
  const uint32_t up = from_next_lane(t.v[0]);
#pragma unroll
  for (int j = 0; j < P - 1; ++j) t.v[j] = t.v[j + 1];
  const uint64_t top = (uint64_t)up + c;
  t.v[P - 1] = (uint32_t)top;
  c = top >> 32;
}

// One CIOS step: t = (t + a_i*b + q*m) / 2^32 with q chosen so the division is exact.
// c is the lane's pending carry word (see file comment).
template <int P>
__device__ __forceinline__ void mont_step(WNum<P>& t, uint64_t& c, uint32_t ai, const WNum<P>& b,
                                          const WNum<P>& m, uint32_t mprime) {
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const uint64_t x = (uint64_t)ai * b.v[j] + t.v[j];
    unsigned int c1;
    t.v[j] = __builtin_addc((uint32_t)x, carry, 0u, &c1);
    carry = (uint32_t)(x >> 32) + c1;
  }
  c += carry;
  redc_step(t, c, m, mprime);
}

// out = a * b * R^{-1} mod m, canonical, for a < R and b < m (m odd, m < R).
template <int P>
__device__ __forceinline__ void mont_mul(WNum<P>& out, const WNum<P>& a, const WNum<P>& b,
                                         const WNum<P>& m, uint32_t mprime) {
  WNum<P> t;
  wn_zero(t);
  uint64_t c = 0;
  for (int src = 0; src < 64; ++src) {
#pragma unroll
    for (int jj = 0; jj < P; ++jj) {
      const uint32_t ai = bcast(a.v[jj], src);
      mont_step(t, c, ai, b, m, mprime);
    }
  }
  const uint64_t ovf = wn_resolve(t, c);
  wn_cond_sub(t, ovf, m);
  out = t;
}

// a b 2^(-32 na) mod m, canonical, for a < 2^(32 na) given by its first na limbs and b < m:
// the first na CIOS steps only (each divides by 2^32).  The CIOS bound keeps every partial
// value below 2m, so one conditional subtraction finishes.
template <int P>
__device__ __forceinline__ void mont_mul_trunc(WNum<P>& out, const WNum<P>& a, int na,
                                               const WNum<P>& b, const WNum<P>& m, uint32_t mprime) {
  WNum<P> t;
  wn_zero(t);
  uint64_t c = 0;
  for (int i = 0; i < na; ++i) mont_step(t, c, wn_limb(a, i), b, m, mprime);
  const uint64_t ovf = wn_resolve(t, c);
  wn_cond_sub(t, ovf, m);
  out = t;
}

// Montgomery multiplication by a number given only through its first `na` limbs
// (the remaining limbs are zero): skips the zero limbs of a.
template <int P>
__device__ __forceinline__ void mont_mul_short(WNum<P>& out, const WNum<P>& a, int na,
                                               const WNum<P>& b, const WNum<P>& m,
                                               uint32_t mprime) {
  WNum<P> t;
  wn_zero(t);
  uint64_t c = 0;
  for (int i = 0; i < na; ++i) mont_step(t, c, wn_limb(a, i), b, m, mprime);
  // the remaining S - na steps have a_i = 0: only the reduction part remains
  for (int i = na; i < 64 * P; ++i) redc_step(t, c, m, mprime);
  const uint64_t ovf = wn_resolve(t, c);
  wn_cond_sub(t, ovf, m);
  out = t;
}

}  // namespace zp
