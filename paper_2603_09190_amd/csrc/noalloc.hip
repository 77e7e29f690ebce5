// pir_answer_compress_noalloc: the one-call online step (pir_answer_compress: the matvec
// b = D . qu mod 2^32, then c_j = K_j (1 + b_j N) mod N^2) for callers that cannot allocate
// device memory at call time.  The step's only scratch, the per-(row, column segment) partial
// sums of the matvec, lives in a static device array instead of the server's growable buffer.
//
// The array is one per GPU, held from the library's load until the process ends.  Host code
// never passes the array's name to a kernel (on the host that name is only a stand-in): the
// device address comes from hipGetSymbolAddress, once per device with that device current
// (pir_setup does it for its device), and is kept per device.
#include <mutex>
#include <string>

#include "internal.h"

namespace {

// 4 Mi words (16 MiB): nseg x rows partials, i.e. 131072 rows at up to 131072 columns
// (32 segments of 4096), or any database whose rows x segments stays within it.
constexpr size_t kScratchWords = size_t(4) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint32_t scratch[kScratchWords];

std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace zp {

// With `device` current: look up (once) and return that device's address of the scratch array.
pir_status scratch_init(int device, uint32_t** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("no-alloc scratch: device index beyond 63");
    return PIR_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error((std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
      return PIR_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<uint32_t*>(p);
  }
  if (out) *out = g_scratch_ptr[device];
  return PIR_OK;
}

size_t scratch_words() { return kScratchWords; }

}  // namespace zp

extern "C" pir_status pir_answer_compress_noalloc(pir_server* s, const uint32_t* Q, uint32_t client_id,
                                                  uint32_t* B, uint32_t* C) {
  zp::set_error("");
  if (!s || !Q || !B || !C) {
    zp::set_error("NULL argument");
    return PIR_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(Q) % 16 != 0) {
    zp::set_error("Q must be 16-byte aligned (the matvec reads the query 16 bytes at a time)");
    return PIR_EINVAL;
  }
  uint32_t rows = 0, cols = 0;
  zp::server_shape(s, &rows, &cols);
  const size_t need = (size_t)zp::answer_segments((int)((cols + 255u) & ~255u)) * rows;
  if (need > kScratchWords) {
    zp::set_error(("the no-alloc step needs " + std::to_string(need) + " scratch words (rows x column segments), above its " +
                   std::to_string(kScratchWords) + "-word limit: use pir_answer_compress")
                      .c_str());
    return PIR_EINVAL;
  }
  int nseg = 0;
  pir_status st = zp::answer_compress_check(s, client_id, &nseg);  // makes the server's device current
  if (st != PIR_OK) return st;
  uint32_t* part = nullptr;
  st = zp::scratch_init(zp::server_device(s), &part);
  if (st != PIR_OK) return st;
  return zp::answer_compress_launch(s, client_id, Q, B, C, part, false);
}
