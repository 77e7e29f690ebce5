// Unpacking a packed compression key (Alg. 6, UnpackCompressionKey): key entry i t + j is
// pck_i^(delta^(t-1-j)) mod N^2, and with delta = 2^dbits that is pck_i raised to 2^(dbits (t-1-j)):
// one chain of squarings per packed ciphertext, each key entry a stop along the chain.
//
// A chain cannot be split: squaring is the whole work and step k needs step k-1.  So each step,
// one Montgomery product modulo M = N^2, is spread over a workgroup of 256 threads, and a chain
// runs on one workgroup.  Its latency is what counts, so the chain stays in one representation:
//   - a residue is DP = unpack_digits(S) balanced 7-bit digits d_k in [-64, 64] (int8), value
//     sum d_k 128^k, possibly negative, and the Montgomery radix is R = 128^DP > 4M.  With
//     |a|, |b| < M, T = a b, m = (T mod R) n' taken as the balanced low DP digits of T n'
//     (|m| < 0.51 R, m = -T M^-1 mod R) and n' = -M^-1 mod R, the value T + m M is a multiple of R
//     whose low DP balanced digits have a value below R / 2 in magnitude, so they sum to exactly
//     zero and U = (T + m M) / R is the high DP digits, with |U| < M^2 / R + 0.51 M < M.  The chain
//     needs no carry propagation and no subtraction; only a key written out is made canonical
//     (its words, plus M when negative);
//   - the three multiprecision products (a b; T n'; m M) run on the int8 matrix cores.  The
//     digit coefficients c_k = sum_i x_i y_(k-i) are a matrix product: with k = 16 u + r and
//     i = 16 v + s, c_(16u+r) = sum_w sum_s Y_w[r][s] X[s][u-w], Y_w[r][s] = y_(16w+r-s) a 16 x 16
//     Toeplitz block of y and X[s][v] = x_(16v+s) x's v-th 16-digit block.  One
//     v_mfma_i32_16x16x64_i8 covers 16 coefficient rows r, 16 blocks u and four w's along K: its
//     A operand (lane: row r, one w) is 16 consecutive bytes of y's digits stored in reverse,
//     read at a byte offset and aligned with v_alignbyte; its B operand (lane: column u, one w)
//     is one aligned 16-digit block of x.  Each of the eight wavefronts computes whole column
//     tiles over all K steps (pairs with zero operands read zero padding, which costs less than
//     branching around them) and writes its coefficients to LDS;
//   - coefficients (magnitude below 2^25) become balanced digits locally: each digit depends on
//     the coefficients at most five places below it, so each thread turns its own run of
//     digits around with no exchange (see normalize).
#include "internal.h"

namespace zp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

template <int S>
struct Dig {
  static constexpr int DP = unpack_digits(S);            // digits of a residue; R = 128^DP
  static constexpr int NB = DP / 16;                     // 16-digit blocks
  static constexpr int NT = (2 * NB + 15) / 16;          // 16-block column tiles of a product
  static constexpr int CF = 256 * NT;                    // coefficient slots (>= 2 DP)
  // Operand buffers carry zeros around the digits, so that every block an MFMA step can touch
  // is a valid address and the out-of-range ones read as zero: forward digits start at PX
  // (blocks v in [-(NB + 3), 16 NT) are readable), reversed digits at PY (64 zero bytes below,
  // 32 above).
  static constexpr int PX = 16 * (NB + 4);
  static constexpr int XB = PX + 256 * NT;
  static constexpr int PY = 64;
  static constexpr int RB = PY + DP + 32;
  static constexpr int RUN = 4 * ((2 * DP + 4 * kThreads - 1) / (4 * kThreads));  // digits per thread
};

// Where a normalised product goes.
enum NormMode { kModeT, kModeM, kModeU, kModeOut };

template <int S>
struct UnpackLds {
  using D = Dig<S>;
  int cf[D::CF];                       // digit coefficients of a product
  alignas(16) uint8_t xa[D::XB];       // digits of the chain value (B operand of a b), from PX
  alignas(16) uint8_t xb[D::XB];       // digits of T mod R, then of m (B operands), from PX
  alignas(16) uint8_t td[2 * D::DP];   // digits of T = a b
  alignas(16) uint8_t yr[D::RB];       // reversed digits of the chain value (byte PY + DP - 1 - k: digit k)
  alignas(16) uint8_t nr[D::RB];       // reversed digits of n'
  alignas(16) uint8_t mr[D::RB];       // reversed digits of M
  alignas(16) uint8_t rr[D::RB];       // reversed digits of R^2 mod M
  alignas(16) uint8_t one[D::RB];      // reversed digits of 1
  uint32_t X[S];                       // packed ciphertext words
  uint32_t Mw[S];                      // M's words
  uint32_t ow[S + 2];                  // a key entry's words
};

// Digit coefficients of x y for the 16-digit blocks u < ulim (NTL = ceil(ulim / 16) column
// tiles): x's digits in xd (blocks), y's reversed in yr.  Wavefront w takes column tiles
// w kT .. w kT + kT - 1 (kT = 1 up to 6144-bit moduli, 2 at 8192; wavefronts past the last
// tile idle, tiles in [NTL, NT) get zeros) over all K steps ks = 0 .. (min(NB, ulim - 1)) / 4,
// so every coefficient is computed whole by one wavefront and written once.  The next K step's
// operand reads are in flight during each step's products, and pairs whose operands are zero
// read the zero padding (for the low product, the extra terms only reach blocks u >= ulim).
// Every thread; no barrier inside.
template <int S, int NTL>
__device__ void mfma_product(const uint8_t* xd, const uint8_t* yr, int ulim, int* cf) {
  using D = Dig<S>;
  constexpr int kT = (D::NT + kWaves - 1) / kWaves;  // column tiles per wavefront
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int kn = (min(D::NB, ulim - 1) >> 2) + 1;
  const int nt0 = wave * kT;
  // Lane (g, c) in K step ks: A = y_(16w + c - s), s = 0..15, w = 4 ks + g, i.e. the reversed
  // bytes from PY + DP - 1 - 16 w - c on; B = x's block v = 16 nt + c - w.  Both move down by
  // 64 bytes per K step; the A window's misalignment (o & 3) is the lane's for every step.
  const int oA = D::PY + D::DP - 1 - 16 * g - c;
  const int aA = oA & ~3, sh = oA & 3;
  const uint8_t* pb = xd + D::PX + 16 * (c - g) + 256 * nt0;
  v4i acc[kT];
#pragma unroll
  for (int j = 0; j < kT; ++j) acc[j] = v4i{0, 0, 0, 0};
  if (nt0 < NTL) {
    auto load = [&](int ks, uint32_t (&y)[5], v4i (&bf)[kT]) {
      const uint32_t* pa = reinterpret_cast<const uint32_t*>(yr + aA - 64 * ks);
#pragma unroll
      for (int i = 0; i < 5; ++i) y[i] = pa[i];
#pragma unroll
      for (int j = 0; j < kT; ++j)
        if (nt0 + j < NTL) bf[j] = *reinterpret_cast<const v4i*>(pb + 256 * j - 64 * ks);
    };
    uint32_t y[5], yn[5];
    v4i bf[kT], bn[kT];
    load(0, y, bf);
    for (int ks = 0; ks < kn; ++ks) {
      if (ks + 1 < kn) load(ks + 1, yn, bn);
      const v4i af = v4i{(int)__builtin_amdgcn_alignbyte(y[1], y[0], sh), (int)__builtin_amdgcn_alignbyte(y[2], y[1], sh),
                         (int)__builtin_amdgcn_alignbyte(y[3], y[2], sh), (int)__builtin_amdgcn_alignbyte(y[4], y[3], sh)};
#pragma unroll
      for (int j = 0; j < kT; ++j)
        if (nt0 + j < NTL) acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[j], acc[j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 5; ++i) y[i] = yn[i];
#pragma unroll
      for (int j = 0; j < kT; ++j) bf[j] = bn[j];
    }
  }
  // acc[j][e]: coefficient row 4 g + e of block 16 (nt0 + j) + c (zero past the NTL tiles)
  int* dst = cf + 16 * c + 4 * g;
#pragma unroll
  for (int j = 0; j < kT; ++j)
    if (nt0 + j < D::NT) *reinterpret_cast<v4i*>(dst + 256 * (nt0 + j)) = acc[j];
}

// Balanced digits of sum_k c_k 128^k (c_k in L.cf, plus the digits
// td for kModeU and kModeOut) for k < K (K = DP for kModeM, else 2 DP; what lies above is
// dropped), written where MODE says:
//   kModeT: T's digits to td, and T mod R's to xb;   kModeM: m's digits to xb;
//   kModeU: digits DP .. 2DP - 1 (U = (T + m M) / R) to xa and, reversed, to yr;
//   kModeOut: the same U to xb.
// Each digit is found from the coefficients at most five places below it, so every thread
// works alone on its run: e_k takes the 7-bit pieces of c_k, c_(k-1), c_(k-2) and c_(k-3) that
// land on digit k (with c_k below 2^25 in magnitude, e_k is in [-73, 454]); f_k = (e_k mod 128)
// + floor(e_(k-1) / 128) is in [-1, 130] and sum f_k 128^k equals the value; and
// d_k = f_k - 128 g_k + g_(k-1) with g_k = [f_k >= 64] is in [-64, 64].  Every thread; no barrier
// inside.
template <int S, int MODE>
__device__ void normalize(UnpackLds<S>& L) {
  using D = Dig<S>;
  constexpr int K = MODE == kModeM ? D::DP : 2 * D::DP;
  constexpr int RUN = D::RUN;
  const int k0 = RUN * threadIdx.x;
  if (k0 >= K) return;
  // c_(k0-8) .. c_(k0+RUN-1); below 0 there is nothing
  int cv[RUN + 8];
#pragma unroll
  for (int i = 0; i < RUN + 8; i += 4) {
    const int k = k0 - 8 + i;
    v4i v = v4i{0, 0, 0, 0};
    if (k >= 0) v = *reinterpret_cast<const v4i*>(&L.cf[k]);
#pragma unroll
    for (int j = 0; j < 4; ++j) cv[i + j] = v[j];
  }
  // e_k for k = k0 - 2 .. k0 + RUN - 1 (index k - k0 + 2); c_k is cv[k - k0 + 8]
  int e[RUN + 2];
#pragma unroll
  for (int i = 0; i < RUN + 2; ++i) {
    const int b = i + 6;  // c_(k0 - 2 + i)
    e[i] = (cv[b] & 127) + ((cv[b - 1] >> 7) & 127) + ((cv[b - 2] >> 14) & 127) + (cv[b - 3] >> 21);
  }
  if (MODE == kModeU || MODE == kModeOut) {
    // T's digits k0 - 4 .. k0 + RUN - 1 (signed bytes), added to e for k >= k0 - 2
#pragma unroll
    for (int i = 0; i < RUN + 4; i += 4) {
      const int k = k0 - 4 + i;
      if (k >= 0 && k < 2 * D::DP) {
        const uint32_t dw = *reinterpret_cast<const uint32_t*>(L.td + k);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (i + j >= 2) e[i + j - 2] += (int)(int8_t)(uint8_t)(dw >> (8 * j));
      }
    }
  }
  // f_k for k = k0 - 1 .. k0 + RUN - 1 (index k - k0 + 1), then the balanced digits
  int f[RUN + 1];
#pragma unroll
  for (int i = 0; i < RUN + 1; ++i) f[i] = (e[i + 1] & 127) + (e[i] >> 7);
  if (k0 == 0) f[0] = 0;  // no digit below 0
#pragma unroll
  for (int i = 0; i < RUN; i += 4) {
    uint32_t dw = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int fk = f[i + j + 1], fp = f[i + j];
      const int d = fk - (fk >= 64 ? 128 : 0) + (fp >= 64 ? 1 : 0);
      dw |= (uint32_t)(uint8_t)(int8_t)d << (8 * j);
    }
    const int k = k0 + i;
    if (k >= K) continue;
    if (MODE == kModeT) {
      *reinterpret_cast<uint32_t*>(L.td + k) = dw;
      if (k < D::DP) *reinterpret_cast<uint32_t*>(L.xb + D::PX + k) = dw;
    } else if (MODE == kModeM) {
      *reinterpret_cast<uint32_t*>(L.xb + D::PX + k) = dw;
    } else if (k >= D::DP) {
      const int j = k - D::DP;
      if (MODE == kModeU) {
        *reinterpret_cast<uint32_t*>(L.xa + D::PX + j) = dw;
        *reinterpret_cast<uint32_t*>(L.yr + D::PY + D::DP - 4 - j) = __builtin_bswap32(dw);
      } else {
        *reinterpret_cast<uint32_t*>(L.xb + D::PX + j) = dw;
      }
    }
  }
}

// U = a b R^-1 (mod M) for a = the chain value (digits in xa) and b given by its reversed digits
// br, with |U| < M when |a|, |b| < M; U goes to xa / yr (kModeU) or xb (kModeOut).
template <int S, int OUT>
__device__ void mont_mul_wg(UnpackLds<S>& L, const uint8_t* br) {
  using D = Dig<S>;
  constexpr int kLowTiles = (D::NB + 15) / 16;
  // 1. T = a b
  mfma_product<S, D::NT>(L.xa, br, 2 * D::NB, L.cf);
  __syncthreads();
  normalize<S, kModeT>(L);
  __syncthreads();
  // 2. m = (T mod R) n' mod R, up to a multiple of R (|m| < 0.51 R)
  mfma_product<S, kLowTiles>(L.xb, L.nr, D::NB, L.cf);
  __syncthreads();
  normalize<S, kModeM>(L);
  __syncthreads();
  // 3. U = (T + m M) / R: in balanced digits the low DP digits of T + m M sum to exactly zero
  //    (their value is a multiple of R below R / 2 in magnitude), so U is the high half
  mfma_product<S, D::NT>(L.xb, L.mr, 2 * D::NB, L.cf);
  __syncthreads();
  normalize<S, OUT>(L);
  __syncthreads();
}

// Reversed digits (byte PY + DP - 1 - k holds digit k) from DP forward digits in global memory.
template <int S>
__device__ void load_reversed(const uint8_t* dig, uint8_t* rev) {
  using D = Dig<S>;
  for (int q = threadIdx.x; q < D::DP / 4; q += kThreads)
    reinterpret_cast<uint32_t*>(rev + D::PY)[(D::DP - 4 - 4 * q) >> 2] =
        __builtin_bswap32(reinterpret_cast<const uint32_t*>(dig)[q]);
}

// One workgroup per packed ciphertext i: keys i t + t - 1, i t + t - 2, ..., i t (those below n),
// stopping to write each after dbits further squarings.
template <int S>
__global__ __launch_bounds__(kThreads) void unpack_chain_kernel(const uint32_t* __restrict__ M,
                                                                const uint8_t* __restrict__ cdig,
                                                                const uint32_t* __restrict__ pck, int n, int t,
                                                                int dbits, int L, uint32_t* __restrict__ ck) {
  __shared__ UnpackLds<S> lds;
  using D = Dig<S>;
  const int i = blockIdx.x;
  for (int w = threadIdx.x; w < S; w += kThreads) {
    lds.X[w] = w < L ? pck[(size_t)i * L + w] : 0u;
    lds.Mw[w] = M[w];
  }
  for (int w = threadIdx.x; w < D::RB / 4; w += kThreads) {
    reinterpret_cast<uint32_t*>(lds.yr)[w] = 0u;
    reinterpret_cast<uint32_t*>(lds.nr)[w] = 0u;
    reinterpret_cast<uint32_t*>(lds.mr)[w] = 0u;
    reinterpret_cast<uint32_t*>(lds.rr)[w] = 0u;
    reinterpret_cast<uint32_t*>(lds.one)[w] = 0u;
  }
  for (int w = threadIdx.x; w < D::XB / 16; w += kThreads) {
    reinterpret_cast<v4i*>(lds.xa)[w] = v4i{0, 0, 0, 0};
    reinterpret_cast<v4i*>(lds.xb)[w] = v4i{0, 0, 0, 0};
  }
  __syncthreads();
  // the packed ciphertext's digits, and the constants reversed
  for (int q = threadIdx.x; q < D::DP / 4; q += kThreads) {
    uint32_t dw = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int bit = 7 * (4 * q + j), wi = bit >> 5, sh = bit & 31;
      uint32_t d = 0;
      if (wi < S) {
        d = lds.X[wi] >> sh;
        if (sh > 25 && wi + 1 < S) d |= lds.X[wi + 1] << (32 - sh);
      }
      dw |= (d & 0x7Fu) << (8 * j);
    }
    reinterpret_cast<uint32_t*>(lds.xa + D::PX)[q] = dw;
  }
  load_reversed<S>(cdig, lds.mr);
  load_reversed<S>(cdig + D::DP, lds.nr);
  load_reversed<S>(cdig + 2 * D::DP, lds.rr);
  if (threadIdx.x == 0) lds.one[D::PY + D::DP - 1] = 1;
  __syncthreads();
  mont_mul_wg<S, kModeU>(lds, lds.rr);  // Montgomery form: pck R mod M (magnitude below M)
  for (int j = t - 1; j >= 0; --j) {
    const int k = i * t + j;
    if (k < n) {
      // key k: X R^-1 (magnitude below 0.51 M) via a product with 1, its balanced digits in xb;
      // as words: partial sums per word (digits starting in it, 64-bit, in the coefficient
      // buffer, free until the next product), then one thread propagates the carries over
      // S + 2 two's-complement words and adds M when the value is negative
      mont_mul_wg<S, kModeOut>(lds, lds.one);
      long long* pw = reinterpret_cast<long long*>(lds.cf);
      for (int w = threadIdx.x; w < S + 2; w += kThreads) {
        const int kb = (32 * w + 6) / 7, ke = min((32 * w + 31) / 7, D::DP - 1);
        long long acc = 0;
        for (int kk = kb; kk <= ke; ++kk)
          acc += (long long)(int8_t)lds.xb[D::PX + kk] * (1LL << (7 * kk - 32 * w));
        pw[w] = acc;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        long long c = 0;
        for (int w = 0; w < S + 2; ++w) {
          const long long v = pw[w] + c;
          lds.ow[w] = (uint32_t)v;
          c = v >> 32;
        }
        if ((int32_t)lds.ow[S + 1] < 0) {
          unsigned long long cy = 0;
          for (int w = 0; w < S; ++w) {
            const unsigned long long v = (unsigned long long)lds.ow[w] + lds.Mw[w] + cy;
            lds.ow[w] = (uint32_t)v;
            cy = v >> 32;
          }
        }
      }
      __syncthreads();
      for (int w = threadIdx.x; w < L; w += kThreads) ck[(size_t)k * L + w] = lds.ow[w];
      __syncthreads();
    }
    if (j > 0)
      for (int sq = 0; sq < dbits; ++sq) mont_mul_wg<S, kModeU>(lds, lds.yr);
  }
}

}  // namespace

void launch_unpack_chains(const ClientDev& cd, const uint8_t* cdig, const uint32_t* pck, int n, int t, int dbits,
                          uint32_t* ck, hipStream_t s) {
  if (n <= 0) return;
  const int groups = (n + t - 1) / t;
  switch (cd.P) {
    case 1: unpack_chain_kernel<64><<<groups, kThreads, 0, s>>>(cd.N2, cdig, pck, n, t, dbits, cd.L, ck); break;
    case 2: unpack_chain_kernel<128><<<groups, kThreads, 0, s>>>(cd.N2, cdig, pck, n, t, dbits, cd.L, ck); break;
    case 3: unpack_chain_kernel<192><<<groups, kThreads, 0, s>>>(cd.N2, cdig, pck, n, t, dbits, cd.L, ck); break;
    case 4: unpack_chain_kernel<256><<<groups, kThreads, 0, s>>>(cd.N2, cdig, pck, n, t, dbits, cd.L, ck); break;
  }
}

}  // namespace zp
