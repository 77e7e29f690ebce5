// Host-side multiprecision helpers for per-modulus constants (little-endian uint32 limbs), and
// the constant block every wave-distributed Montgomery kernel reads (zp::ClientDev).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace zp {

using Big = std::vector<uint32_t>;

inline Big big_resize(Big a, size_t n) {
  a.resize(n, 0u);
  return a;
}

inline int big_cmp(const Big& a, const Big& b) {
  const size_t n = std::max(a.size(), b.size());
  for (size_t i = n; i-- > 0;) {
    const uint32_t x = i < a.size() ? a[i] : 0u, y = i < b.size() ? b[i] : 0u;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

inline void big_sub_inplace(Big& a, const Big& b) {  // a -= b, requires a >= b
  uint64_t br = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    const uint64_t y = (i < b.size() ? b[i] : 0u) + br;
    const uint64_t x = a[i];
    a[i] = (uint32_t)(x - y);
    br = x < y ? 1 : 0;
  }
}

inline Big big_mul(const Big& a, const Big& b) {
  Big r(a.size() + b.size(), 0u);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      const uint64_t t = (uint64_t)a[i] * b[j] + r[i + j] + carry;
      r[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    size_t k = i + b.size();
    while (carry) {
      const uint64_t t = (uint64_t)r[k] + carry;
      r[k] = (uint32_t)t;
      carry = t >> 32;
      ++k;
    }
  }
  return r;
}

// 2^k mod m by repeated doubling (m odd, m > 1).
inline Big big_pow2_mod(uint64_t k, const Big& m) {
  Big x(m.size() + 1, 0u);
  x[0] = 1;
  if (big_cmp(x, m) >= 0) big_sub_inplace(x, m);
  for (uint64_t t = 0; t < k; ++t) {
    uint32_t carry = 0;
    for (size_t i = 0; i < x.size(); ++i) {
      const uint32_t nc = x[i] >> 31;
      x[i] = (x[i] << 1) | carry;
      carry = nc;
    }
    if (big_cmp(x, m) >= 0) big_sub_inplace(x, m);
  }
  x.resize(m.size());
  return x;
}

inline uint32_t neg_inv32(uint32_t m0) {  // -m0^{-1} mod 2^32 for odd m0 (Newton iteration)
  uint32_t inv = m0;                      // correct to 3 bits
  for (int i = 0; i < 5; ++i) inv *= 2u - m0 * inv;
  return 0u - inv;
}

// -m^{-1} mod 2^(32 words) for odd m, by Newton's iteration x <- x (2 - m x), which doubles the
// number of correct low bits each step, from the 32-bit inverse; checked by m n' + 1 = 0.
inline Big big_neg_inv_pow2(const Big& m, size_t words) {
  const Big mw = big_resize(m, words);
  Big x(words, 0u);
  x[0] = 0u - neg_inv32(mw[0]);
  auto negate = [](Big& v) {  // v <- -v mod 2^(32 |v|)
    uint64_t carry = 1;
    for (auto& w : v) {
      const uint64_t t = (uint64_t)(uint32_t)~w + carry;
      w = (uint32_t)t;
      carry = t >> 32;
    }
  };
  for (size_t bits = 32; bits < 32 * words; bits *= 2) {
    Big e = big_resize(big_mul(mw, x), words);  // m x
    negate(e);                                  // -m x
    uint64_t carry = 2;                         // 2 - m x
    for (size_t i = 0; i < words && carry; ++i) {
      const uint64_t t = (uint64_t)e[i] + carry;
      e[i] = (uint32_t)t;
      carry = t >> 32;
    }
    x = big_resize(big_mul(x, e), words);
  }
  negate(x);
  Big chk = big_resize(big_mul(mw, x), words);
  uint64_t carry = 1;
  bool zero = true;
  for (auto& w : chk) {
    const uint64_t t = (uint64_t)w + carry;
    zero = zero && (uint32_t)t == 0u;
    carry = t >> 32;
  }
  if (!zero) x.clear();
  return x;
}

// Bits 7k .. 7k + 6 of a (the k-th base-128 digit).
inline uint8_t big_digit7(const Big& a, size_t k) {
  const size_t bit = 7 * k, wi = bit / 32, sh = bit % 32;
  uint64_t v = wi < a.size() ? a[wi] : 0u;
  if (wi + 1 < a.size()) v |= (uint64_t)a[wi + 1] << 32;
  return (uint8_t)((v >> sh) & 0x7Fu);
}

inline size_t bit_length(const Big& a) {
  for (size_t i = a.size(); i-- > 0;)
    if (a[i]) return 32 * i + (32 - __builtin_clz(a[i]));
  return 0;
}

// Sizes and constants of one Paillier modulus N (h limbs): L = 2h limbs modulo N^2, numbers
// of S = 64 P limbs modulo N^2 and SN = 64 PN limbs modulo N.  `host` is the device block
//   N2 | R1 | RR | NP (S each) | Nn | C1 | C2 (SN each) | CP (S) | D1 | D2 | C96 | CT (SN each)
// (the meaning of each is listed at zp::ClientDev).
struct ModConsts {
  uint32_t n_bits = 0, h = 0, L = 0, P = 0, PN = 0, S = 0, SN = 0;
  uint32_t m2prime = 0, nprime = 0;
  Big N;
  std::vector<uint32_t> host;
};

// t_bits: the packing shift t of packed offset answers (CT = 2^t R_N mod N); 0 if unused.
inline ModConsts mod_constants(const Big& N_in, uint32_t n_bits, uint32_t t_bits = 0) {
  ModConsts c;
  c.n_bits = n_bits;
  c.h = (n_bits + 31) / 32;
  c.L = 2 * c.h;
  c.P = (c.L + 63) / 64;
  c.PN = (c.h + 63) / 64;
  c.S = 64 * c.P;
  c.SN = 64 * c.PN;
  c.N = big_resize(N_in, c.h);
  const Big N2 = big_resize(big_mul(c.N, c.N), c.S);
  const Big N2L = big_resize(N2, c.L);
  const Big Nn = big_resize(c.N, c.SN);
  const Big R1 = big_pow2_mod(32ull * c.S, N2L);
  const Big RR = big_pow2_mod(64ull * c.S, N2L);
  const Big C1 = big_pow2_mod(32ull * c.SN, c.N);
  const Big C2 = big_pow2_mod(64ull * c.SN, c.N);
  const Big CP = big_pow2_mod(64ull * c.S - 32, N2L);
  const Big D1 = big_pow2_mod(64ull * c.SN - 32, c.N);
  const Big D2 = big_pow2_mod(96ull * c.SN - 32, c.N);
  const Big C96 = big_pow2_mod(32ull * c.SN + 96, c.N);
  const Big CT = big_pow2_mod(32ull * c.SN + t_bits, c.N);
  c.m2prime = neg_inv32(N2[0]);
  c.nprime = neg_inv32(c.N[0]);
  c.host.assign(5 * (size_t)c.S + 7 * (size_t)c.SN, 0u);
  auto put = [&](size_t off, const Big& v, size_t width) {
    for (size_t i = 0; i < std::min(width, v.size()); ++i) c.host[off + i] = v[i];
  };
  put(0, N2, c.S);
  put(c.S, R1, c.S);
  put(2 * (size_t)c.S, RR, c.S);
  put(3 * (size_t)c.S, c.N, c.S);
  put(4 * (size_t)c.S, Nn, c.SN);
  put(4 * (size_t)c.S + c.SN, C1, c.SN);
  put(4 * (size_t)c.S + 2 * c.SN, C2, c.SN);
  put(4 * (size_t)c.S + 3 * c.SN, CP, c.S);
  put(5 * (size_t)c.S + 3 * c.SN, D1, c.SN);
  put(5 * (size_t)c.S + 4 * c.SN, D2, c.SN);
  put(5 * (size_t)c.S + 5 * c.SN, C96, c.SN);
  put(5 * (size_t)c.S + 6 * c.SN, CT, c.SN);
  return c;
}

// The kernels' view of a constant block `consts` (device copy of ModConsts::host).
inline ClientDev dev_view(const ModConsts& c, const uint32_t* consts) {
  ClientDev d;
  const size_t S = c.S, SN = c.SN;
  d.N2 = consts;
  d.R1 = consts + S;
  d.RR = consts + 2 * S;
  d.NP = consts + 3 * S;
  d.Nn = consts + 4 * S;
  d.C1 = consts + 4 * S + SN;
  d.C2 = consts + 4 * S + 2 * SN;
  d.CP = consts + 4 * S + 3 * SN;
  d.D1 = consts + 5 * S + 3 * SN;
  d.D2 = consts + 5 * S + 4 * SN;
  d.C96 = consts + 5 * S + 5 * SN;
  d.CT = consts + 5 * S + 6 * SN;
  d.m2prime = c.m2prime;
  d.nprime = c.nprime;
  d.L = (int)c.L;
  d.h = (int)c.h;
  d.P = (int)c.P;
  d.PN = (int)c.PN;
  return d;
}

}  // namespace zp
