// Host side of the standalone compressor (pir_compressor_* and pir_compress_lwe/rlwe in
// zippir.h): the compression key and its fixed-base table stay resident; each call compresses
// a batch of LWE ciphertexts or RLWE coefficients (Alg. 2, Alg. 8; packed keys of Alg. 6).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hostbig.h"
#include "internal.h"
#include "zippir.h"

struct pir_compressor {
  int device = 0;
  hipStream_t stream = nullptr;
  uint32_t n = 0;
  uint64_t q = 0;  // 0 stands for 2^64
  int qw = 1, windows = 4;
  zp::ModConsts mc;
  uint32_t* consts = nullptr;
  uint32_t* ck = nullptr;     // n x L
  uint32_t* table = nullptr;  // n x windows x 255 x S
  std::map<void*, size_t> allocs;
  uint64_t bytes = 0;
  // device time of the setup steps, from events on the compressor's stream
  float unpack_ms = 0.0f, table_ms = 0.0f;
  // growable scratch
  void* s_in = nullptr;
  size_t s_in_bytes = 0;
  void* s_out = nullptr;
  size_t s_out_bytes = 0;
  void* s_part[2] = {nullptr, nullptr};
  size_t s_part_bytes[2] = {0, 0};

  zp::ClientDev dev() const { return zp::dev_view(mc, consts); }

  pir_status alloc(void** p, size_t b) {
    *p = nullptr;
    if (b == 0) b = 256;
    if (hipMalloc(p, b) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      zp::set_error("hipMalloc failed in the compressor");
      return PIR_ENOMEM;
    }
    allocs[*p] = b;
    bytes += b;
    return PIR_OK;
  }
  void release(void* p) {
    if (!p) return;
    auto it = allocs.find(p);
    if (it != allocs.end()) {
      bytes -= it->second;
      allocs.erase(it);
    }
    (void)hipFree(p);
  }
  pir_status grow(void*& p, size_t& have, size_t need) {
    if (have >= need) return PIR_OK;
    if (p) {
      (void)hipStreamSynchronize(stream);
      release(p);
      p = nullptr;
      have = 0;
    }
    pir_status st = alloc(&p, need);
    if (st == PIR_OK) have = need;
    return st;
  }
};

namespace {

pir_status cfail(pir_status st, const std::string& m) {
  zp::set_error(m.c_str());
  return st;
}

#define ZC_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return cfail(e_ == hipErrorOutOfMemory ? PIR_ENOMEM : PIR_EDEVICE,                   \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                     \
  } while (0)

#define ZC_TRY(expr)                 \
  do {                               \
    pir_status st_ = (expr);         \
    if (st_ != PIR_OK) return st_;   \
  } while (0)

// Largest exponent (q - 1) in bits; 8-bit windows cover it.
int exponent_windows(uint64_t q) {
  const uint64_t qm1 = q ? q - 1 : ~0ull;
  int bits = 0;
  for (uint64_t v = qm1; v; v >>= 1) ++bits;
  return std::max(1, (bits + zp::kWindowBits - 1) / zp::kWindowBits);
}

// Common part of both constructors: checks, constants, resident key (device copy in c->ck
// must be filled by the caller), table.
pir_status setup_common(pir_compressor* c, int device, void* stream, uint32_t n, uint64_t q,
                        const uint32_t* N, uint32_t N_bits, uint32_t ptr_flags) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return cfail(PIR_EINVAL, "no such device");
  if (n < 1) return cfail(PIR_EINVAL, "n must be positive");
  if (q == 1) return cfail(PIR_EINVAL, "q must be at least 2");
  if (N_bits < 64 || N_bits > 4096) return cfail(PIR_EINVAL, "N_bits must be in [64, 4096]");
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->n = n;
  c->q = q;
  c->qw = (q == 0 || q > (1ull << 32)) ? 2 : 1;
  c->windows = exponent_windows(q);
  ZC_HIP(hipSetDevice(device));
  const uint32_t h = (N_bits + 31) / 32;
  zp::Big Nb(h, 0u);
  if (ptr_flags == PIR_PTR_DEVICE)
    ZC_HIP(hipMemcpy(Nb.data(), N, h * sizeof(uint32_t), hipMemcpyDeviceToHost));
  else
    std::memcpy(Nb.data(), N, h * sizeof(uint32_t));
  if (zp::bit_length(Nb) != N_bits) return cfail(PIR_EINVAL, "N does not have exactly N_bits bits");
  if ((Nb[0] & 1u) == 0) return cfail(PIR_EINVAL, "N must be odd");
  // Theorem 1: N > q + n (q-1)^2 >= the largest plaintext b + sum (q - a_i) s_i with s_i < q
  {
    zp::Big qb = {(uint32_t)(q ? q : 0), (uint32_t)(q ? q >> 32 : 0), q ? 0u : 1u};
    zp::Big qm1 = {(uint32_t)((q ? q : 0) - 1), (uint32_t)((q ? q - 1 : ~0ull) >> 32), 0u};
    zp::Big bound = zp::big_mul(zp::big_mul(qm1, qm1), zp::Big{n});
    // bound += q
    uint64_t carry = 0;
    bound.resize(std::max(bound.size(), qb.size()) + 1, 0u);
    for (size_t i = 0; i < bound.size(); ++i) {
      const uint64_t t = (uint64_t)bound[i] + (i < qb.size() ? qb[i] : 0u) + carry;
      bound[i] = (uint32_t)t;
      carry = t >> 32;
    }
    if (zp::big_cmp(Nb, bound) <= 0)
      return cfail(PIR_EINVAL, "N too small: compression needs N > q + n (q-1)^2 (Theorem 1)");
  }
  c->mc = zp::mod_constants(Nb, N_bits);
  ZC_TRY(c->alloc((void**)&c->consts, c->mc.host.size() * sizeof(uint32_t)));
  ZC_HIP(hipMemcpyAsync(c->consts, c->mc.host.data(), c->mc.host.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice, c->stream));
  ZC_TRY(c->alloc((void**)&c->ck, (size_t)n * c->mc.L * sizeof(uint32_t)));
  return PIR_OK;
}

// Device milliseconds of the work `fn` enqueues on the compressor's stream (0 if events fail).
template <typename F>
float time_on_stream(pir_compressor* c, F fn) {
  hipEvent_t a = nullptr, b = nullptr;
  const bool ev = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  if (ev) (void)hipEventRecord(a, c->stream);
  fn();
  float ms = 0.0f;
  if (ev) {
    (void)hipEventRecord(b, c->stream);
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.0f;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return ms;
}

pir_status build_table(pir_compressor* c) {
  const size_t tb = (size_t)c->n * c->windows * zp::kDigits * c->mc.S * sizeof(uint32_t);
  ZC_TRY(c->alloc((void**)&c->table, tb));
  c->table_ms = time_on_stream(c, [&] { zp::launch_build_table(c->dev(), c->ck, (int)c->n, c->windows, c->table, c->stream); });
  ZC_HIP(hipGetLastError());
  ZC_HIP(hipStreamSynchronize(c->stream));
  return PIR_OK;
}

pir_status check_key(pir_compressor* c) {
  // every key entry must be a residue mod N^2
  std::vector<uint32_t> h((size_t)c->n * c->mc.L);
  ZC_HIP(hipMemcpyAsync(h.data(), c->ck, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  ZC_HIP(hipStreamSynchronize(c->stream));
  const zp::Big N2 = zp::big_resize(zp::big_mul(c->mc.N, c->mc.N), c->mc.L);
  for (uint32_t k = 0; k < c->n; ++k) {
    zp::Big v(h.begin() + (size_t)k * c->mc.L, h.begin() + (size_t)(k + 1) * c->mc.L);
    if (zp::big_cmp(v, N2) >= 0) return cfail(PIR_EINVAL, "key entry " + std::to_string(k) + " is not below N^2");
  }
  return PIR_OK;
}

// Parts per ciphertext: enough work items to fill the GPU when few ciphertexts are
// compressed, down to one base per part (a lone ciphertext's latency is then the window
// products of one base plus a tree of fan-in kFan).
int choose_parts(uint32_t rows, uint32_t n) {
  const long long target = zp::kQuadItems;
  long long p = (target + rows - 1) / rows;
  p = std::min<long long>(p, std::max<uint32_t>(1, n));
  return (int)std::max<long long>(1, p);
}

pir_status run(pir_compressor* c, zp::LweBatch lb, uint32_t* X, uint32_t ptr_flags, size_t in_words_A,
               size_t in_words_B, const uint32_t* ks_host) {
  hipStream_t st = c->stream;
  const size_t L = c->mc.L, S = c->mc.S;
  const size_t xbytes = (size_t)lb.rows * L * sizeof(uint32_t);
  // inputs
  size_t ks_words = lb.ks ? (size_t)lb.rows : 0;
  if (ptr_flags == PIR_PTR_HOST || ks_host) {
    const size_t in_bytes = (in_words_A + in_words_B + ks_words) * sizeof(uint32_t);
    ZC_TRY(c->grow(c->s_in, c->s_in_bytes, in_bytes));
    auto* base = (uint32_t*)c->s_in;
    const hipMemcpyKind kind = ptr_flags == PIR_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    ZC_HIP(hipMemcpyAsync(base, lb.A, in_words_A * sizeof(uint32_t), kind, st));
    ZC_HIP(hipMemcpyAsync(base + in_words_A, lb.B, in_words_B * sizeof(uint32_t), kind, st));
    lb.A = base;
    lb.B = base + in_words_A;
    if (ks_host) {
      ZC_HIP(hipMemcpyAsync(base + in_words_A + in_words_B, ks_host, ks_words * sizeof(uint32_t),
                            hipMemcpyHostToDevice, st));
      lb.ks = base + in_words_A + in_words_B;
    }
  }
  uint32_t* dX = X;
  if (ptr_flags == PIR_PTR_HOST) {
    ZC_TRY(c->grow(c->s_out, c->s_out_bytes, xbytes));
    dX = (uint32_t*)c->s_out;
  }
  const zp::ClientDev cd = c->dev();
  const int parts = choose_parts((uint32_t)lb.rows, c->n);
  if (parts == 1) {
    zp::launch_compress_lwe(cd, lb, c->table, 1, nullptr, dX, st);
  } else {
    const size_t pbytes = (size_t)lb.rows * parts * S * sizeof(uint32_t);
    ZC_TRY(c->grow(c->s_part[0], c->s_part_bytes[0], pbytes));
    ZC_TRY(c->grow(c->s_part[1], c->s_part_bytes[1], pbytes));
    zp::launch_compress_lwe(cd, lb, c->table, parts, (uint32_t*)c->s_part[0], dX, st);
    int cur = 0, p = parts;
    constexpr int kFan = 4;
    while (true) {
      const int outs = (p + kFan - 1) / kFan;
      zp::launch_reduce_parts(cd, lb, (const uint32_t*)c->s_part[cur], p, kFan,
                              (uint32_t*)c->s_part[cur ^ 1], dX, st);
      if (outs == 1) break;
      cur ^= 1;
      p = outs;
    }
  }
  ZC_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) ZC_HIP(hipMemcpyAsync(X, dX, xbytes, hipMemcpyDeviceToHost, st));
  ZC_HIP(hipStreamSynchronize(st));
  return PIR_OK;
}

}  // namespace

extern "C" {

pir_status pir_compressor_create(pir_compressor** out, int device, void* stream, uint32_t n, uint64_t q,
                                 const uint32_t* N, uint32_t N_bits, const uint32_t* ck,
                                 uint32_t ptr_flags) {
  if (!out || !N || !ck) return cfail(PIR_EINVAL, "NULL argument");
  *out = nullptr;
  if (ptr_flags != PIR_PTR_HOST && ptr_flags != PIR_PTR_DEVICE) return cfail(PIR_EINVAL, "bad ptr_flags");
  auto* c = new pir_compressor();
  pir_status st = setup_common(c, device, stream, n, q, N, N_bits, ptr_flags);
  if (st == PIR_OK) {
    const hipMemcpyKind kind = ptr_flags == PIR_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(c->ck, ck, (size_t)n * c->mc.L * sizeof(uint32_t), kind, c->stream) != hipSuccess)
      st = cfail(PIR_EDEVICE, "copying the compression key");
  }
  if (st == PIR_OK) st = check_key(c);
  if (st == PIR_OK) st = build_table(c);
  if (st != PIR_OK) {
    pir_compressor_destroy(c);
    return st;
  }
  *out = c;
  return PIR_OK;
}

pir_status pir_compressor_create_packed(pir_compressor** out, int device, void* stream, uint32_t n,
                                        uint64_t q, const uint32_t* N, uint32_t N_bits,
                                        const uint32_t* pck, uint32_t t, uint32_t delta_log2,
                                        uint32_t ptr_flags) {
  if (!out || !N || !pck) return cfail(PIR_EINVAL, "NULL argument");
  *out = nullptr;
  if (ptr_flags != PIR_PTR_HOST && ptr_flags != PIR_PTR_DEVICE) return cfail(PIR_EINVAL, "bad ptr_flags");
  if (t < 1 || delta_log2 < 1 || (uint64_t)delta_log2 * (t - 1) > 1u << 20)
    return cfail(PIR_EINVAL, "bad packing parameters");
  auto* c = new pir_compressor();
  pir_status st = setup_common(c, device, stream, n, q, N, N_bits, ptr_flags);
  uint32_t* dp = nullptr;
  const uint32_t npck = (n + t - 1) / t;
  if (st == PIR_OK) st = c->alloc((void**)&dp, (size_t)npck * c->mc.L * sizeof(uint32_t));
  if (st == PIR_OK) {
    const hipMemcpyKind kind = ptr_flags == PIR_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(dp, pck, (size_t)npck * c->mc.L * sizeof(uint32_t), kind, c->stream) != hipSuccess)
      st = cfail(PIR_EDEVICE, "copying the packed key");
  }
  // the unpacking's constants as 7-bit digits: N^2, -(N^2)^{-1} mod R and R^2 mod N^2 for
  // R = 2^(7 DP)
  uint8_t* cdig = nullptr;
  if (st == PIR_OK) {
    const int DP = zp::unpack_digits((int)c->mc.S);
    const zp::Big N2 = zp::big_resize(zp::big_mul(c->mc.N, c->mc.N), c->mc.L);
    const zp::Big Ni = zp::big_neg_inv_pow2(N2, (7 * (size_t)DP + 31) / 32);
    const zp::Big RR = zp::big_pow2_mod(14ull * DP, N2);
    if (Ni.empty()) st = cfail(PIR_EINVAL, "no inverse of N^2 modulo the Montgomery radix");
    std::vector<uint8_t> host(3 * (size_t)DP, 0);
    if (st == PIR_OK) {
      const zp::Big* parts[3] = {&N2, &Ni, &RR};
      for (int p = 0; p < 3; ++p)
        for (int k = 0; k < DP; ++k) host[(size_t)p * DP + k] = zp::big_digit7(*parts[p], k);
      st = c->alloc((void**)&cdig, host.size());
    }
    if (st == PIR_OK && (hipMemcpyAsync(cdig, host.data(), host.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
                         hipStreamSynchronize(c->stream) != hipSuccess))
      st = cfail(PIR_EDEVICE, "copying the packed key constants");
  }
  if (st == PIR_OK) {
    c->unpack_ms = time_on_stream(
        c, [&] { zp::launch_unpack_chains(c->dev(), cdig, dp, (int)n, (int)t, (int)delta_log2, c->ck, c->stream); });
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      st = cfail(PIR_EDEVICE, "unpacking the compression key");
  }
  if (dp) c->release(dp);
  if (cdig) c->release(cdig);
  if (st == PIR_OK) st = check_key(c);
  if (st == PIR_OK) st = build_table(c);
  if (st != PIR_OK) {
    pir_compressor_destroy(c);
    return st;
  }
  *out = c;
  return PIR_OK;
}

pir_status pir_compressor_setup_ms(const pir_compressor* c, float* unpack_ms, float* table_ms) {
  if (!c) return cfail(PIR_EINVAL, "NULL compressor");
  if (unpack_ms) *unpack_ms = c->unpack_ms;
  if (table_ms) *table_ms = c->table_ms;
  return PIR_OK;
}

void pir_compressor_destroy(pir_compressor* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->allocs) (void)hipFree(kv.first);
  delete c;
}

pir_status pir_compressor_key(pir_compressor* c, uint32_t k0, uint32_t nk, uint32_t* ck,
                              uint32_t ptr_flags) {
  if (!c || !ck) return cfail(PIR_EINVAL, "NULL argument");
  if ((uint64_t)k0 + nk > c->n) return cfail(PIR_EINVAL, "key range out of bounds");
  ZC_HIP(hipSetDevice(c->device));
  const hipMemcpyKind kind = ptr_flags == PIR_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  ZC_HIP(hipMemcpyAsync(ck, c->ck + (size_t)k0 * c->mc.L, (size_t)nk * c->mc.L * sizeof(uint32_t), kind,
                        c->stream));
  ZC_HIP(hipStreamSynchronize(c->stream));
  return PIR_OK;
}

pir_status pir_compressor_info(pir_compressor* c, uint32_t* L, uint32_t* windows, uint64_t* device_bytes) {
  if (!c) return cfail(PIR_EINVAL, "NULL compressor");
  if (L) *L = c->mc.L;
  if (windows) *windows = (uint32_t)c->windows;
  if (device_bytes) *device_bytes = c->bytes;
  return PIR_OK;
}

pir_status pir_compress_lwe(pir_compressor* c, const uint32_t* A, const uint32_t* B, uint32_t rows,
                            uint32_t* X, uint32_t ptr_flags) {
  if (!c || !A || !B || !X) return cfail(PIR_EINVAL, "NULL argument");
  if (ptr_flags != PIR_PTR_HOST && ptr_flags != PIR_PTR_DEVICE) return cfail(PIR_EINVAL, "bad ptr_flags");
  if (rows == 0) return PIR_OK;
  ZC_HIP(hipSetDevice(c->device));
  zp::LweBatch lb{A, B, nullptr, (int)rows, (int)c->n, c->qw, c->windows, c->q};
  return run(c, lb, X, ptr_flags, (size_t)rows * c->n * c->qw, (size_t)rows * c->qw, nullptr);
}

pir_status pir_compress_rlwe(pir_compressor* c, const uint32_t* A, const uint32_t* B, const uint32_t* ks,
                             uint32_t nk, uint32_t* X, uint32_t ptr_flags) {
  if (!c || !A || !B || !ks || !X) return cfail(PIR_EINVAL, "NULL argument");
  if (ptr_flags != PIR_PTR_HOST && ptr_flags != PIR_PTR_DEVICE) return cfail(PIR_EINVAL, "bad ptr_flags");
  for (uint32_t i = 0; i < nk; ++i)
    if (ks[i] >= c->n) return cfail(PIR_EINVAL, "coefficient index out of range");
  if (nk == 0) return PIR_OK;
  ZC_HIP(hipSetDevice(c->device));
  zp::LweBatch lb{A, B, ks, (int)nk, (int)c->n, c->qw, c->windows, c->q};
  return run(c, lb, X, ptr_flags, (size_t)c->n * c->qw, (size_t)c->n * c->qw, ks);
}

}  // extern "C"
