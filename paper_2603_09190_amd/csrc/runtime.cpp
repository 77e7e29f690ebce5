// Host runtime behind zippir.h: server state, device residency, per-client constants and
// the C entry points.  All device work is enqueued on the server's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "hostbig.h"
#include "internal.h"
#include "zippir.h"

namespace {

using zp::Big;
using zp::big_cmp;
using zp::big_mul;
using zp::big_pow2_mod;
using zp::big_resize;
using zp::bit_length;

thread_local std::string g_last_error;

pir_status fail(pir_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define ZP_HIP(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(e_ == hipErrorOutOfMemory ? PIR_ENOMEM : PIR_EDEVICE,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

#define ZP_TRY(expr)                 \
  do {                               \
    pir_status st_ = (expr);         \
    if (st_ != PIR_OK) return st_;   \
  } while (0)

// ----------------------------------------------------------------------------- state

struct DevAlloc {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct ClientState {
  uint32_t id = 0;
  uint32_t n_bits = 0, h = 0, L = 0, P = 0, PN = 0, S = 0, SN = 0;
  Big N;
  uint32_t* ck = nullptr;      // n x L
  uint32_t* consts = nullptr;  // the device copy of mc.host (layout at zp::mod_constants)
  uint32_t* Kp = nullptr;      // rows x L: K_j 2^32 mod N^2
  uint32_t* Mp = nullptr;      // rows x L: N (K'_j mod N), the combine key
  uint32_t* Y = nullptr;       // rows x h: (K_j mod N) R_N mod N, the offset-combine key
  uint32_t m2prime = 0, nprime = 0;
  uint32_t hint_wbits = 0;     // window width of the last pir_hint's table (0: none yet)
  std::vector<uint8_t> valid;  // per row: K' and M' up to date
  int64_t stale = 0;
  // packed responses (batched compression): ell rows per ciphertext, gamma = 2^t
  uint32_t ell = 1, t = 0, ell_max = 1;
  uint32_t* Kg = nullptr;      // groups x L: group keys K_g
  uint32_t* Mr = nullptr;      // groups x L: N (K_g mod N) 2^(32h) mod N^2
  uint32_t* Yg = nullptr;      // groups x h: (K_g mod N) R_N mod N, the packed offset-combine key
  uint32_t* PJ = nullptr;      // ell_max x SN: 2^(t j) R_N mod N, the packed offset-answer weights
  std::vector<uint8_t> gvalid; // per group
  int64_t gstale = 0;

  zp::ModConsts mc;            // sizes and constants of N (mc.host is the device block `consts`)

  zp::ClientDev dev() const { return zp::dev_view(mc, consts); }
};

struct pir_server {
  int device = 0;
  int num_cus = 256;            // compute units of the device (sizes persistent grids)
  // a second stream (default priority) and two events for pir_answer_offset, which runs the
  // offset contraction beside the answer
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t stream = nullptr;
  uint32_t rows = 0, cols = 0, n = 0, pitch = 0;
  uint8_t* D = nullptr;         // rows x pitch, zero beyond cols
  // D again in 16-row x 64-byte tiles (launch_tile_rows), read by the four-plane contraction;
  // nullptr when switched off or when HBM had no room for it (the contraction then reads D)
  uint8_t* Dt = nullptr;
  uint32_t* A = nullptr;        // cols x n
  uint8_t* Apt = nullptr;       // A's signed byte planes in fragment order (launch_a_planes)
  int32_t* Acolsum = nullptr;   // n x 4
  int32_t* rowsum = nullptr;    // rows: sum_i (D[j][i] - 128)
  uint32_t* H = nullptr;        // rows x n
  std::vector<uint8_t> H_valid;
  int64_t H_stale = 0;
  // E = -H mod 2^32 as four signed byte planes in MFMA fragment order (launch_e_planes) for the
  // offset answer, built on first use after H changes
  uint8_t* Ep = nullptr;        // rows_pad x 4 x 64 S bytes
  int32_t* Ers = nullptr;       // 4 x rows_pad: per plane and row, sum_{k<n} (byte - 128)
  uint32_t rows_pad = 0;        // rows rounded up to 128 (the contraction's row blocks)
  bool E_ready = false;
  std::map<uint32_t, std::unique_ptr<ClientState>> clients;
  uint32_t next_id = 1;
  std::map<void*, size_t> allocs;
  uint64_t bytes = 0;
  // attached to a serving engine: shapes not yet tuned run with the default launch shape
  // instead of being tuned in place (the engine tunes its shapes when the database is added)
  bool serving = false;
  // per-kernel event timing (pir_profile)
  bool prof = false;
  struct ProfRecord {
    hipEvent_t begin, end;
    int launches;
  };
  std::vector<ProfRecord> prof_ev[PIR_KERNEL_COUNT];
  // growable scratch
  DevAlloc s_planes, s_colsum, s_q, s_b, s_rows, s_gath, s_gsum, s_h, s_c, s_x, s_xcs, s_w, s_t, s_ys, s_tmp,
      s_part, s_aq, s_ak, s_ab;

  pir_status alloc(void** p, size_t bytes_) {
    *p = nullptr;
    if (bytes_ == 0) bytes_ = 256;
    hipError_t e = hipMalloc(p, bytes_);
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return fail(PIR_ENOMEM, std::string("hipMalloc(") + std::to_string(bytes_) +
                                  " bytes): " + hipGetErrorString(e));
    }
    allocs[*p] = bytes_;
    bytes += bytes_;
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
  pir_status scratch(DevAlloc& a, size_t need) {
    if (a.bytes >= need) return PIR_OK;
    if (a.p) {
      (void)hipStreamSynchronize(stream);
      release(a.p);
      a.p = nullptr;
      a.bytes = 0;
    }
    ZP_TRY(alloc(&a.p, need));
    a.bytes = need;
    return PIR_OK;
  }
};

namespace {

hipMemcpyKind kind_to_dev(uint32_t flags) {
  return flags == PIR_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_from_dev(uint32_t flags) {
  return flags == PIR_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

pir_status check_flags(uint32_t flags) {
  if (flags != PIR_PTR_HOST && flags != PIR_PTR_DEVICE)
    return fail(PIR_EINVAL, "ptr_flags must be PIR_PTR_HOST or PIR_PTR_DEVICE");
  return PIR_OK;
}

// Records an event pair around one launch when profiling is on.
struct ProfScope {
  pir_server* s;
  int k;
  int launches;
  hipEvent_t b = nullptr, e = nullptr;
  hipStream_t on;
  ProfScope(pir_server* s_, int k_, int launches_ = 1, hipStream_t on_ = nullptr)
      : s(s_), k(k_), launches(launches_), on(on_ ? on_ : s_->stream) {
    if (!s->prof) return;
    if (hipEventCreate(&b) != hipSuccess || hipEventCreate(&e) != hipSuccess) {
      b = e = nullptr;
      return;
    }
    (void)hipEventRecord(b, on);
  }
  ~ProfScope() {
    if (!b) return;
    (void)hipEventRecord(e, on);
    s->prof_ev[k].push_back(pir_server::ProfRecord{b, e, launches});
  }
};

void prof_clear(pir_server* s) {
  for (auto& v : s->prof_ev) {
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.begin);
      (void)hipEventDestroy(pr.end);
    }
    v.clear();
  }
}

// ----------------------------------------------------------------------------- autotuner
// Launch shape of the byte-plane contraction per problem shape.  The first contraction of a
// shape runs every candidate once as a warm-up, checks that its output equals the first
// candidate's element for element (every shape must compute identical bits; a difference is
// reported as PIR_EDEVICE), times three more launches with events on the server's stream and
// keeps the fastest.  ZIPPIR_AUTOTUNE=0 disables tuning (default shape);
// ZIPPIR_TUNE_CACHE=<file> persists choices as lines
// "rows pitch ncol rowmajor planes tiled waves depth mr kb ksplit cg".
using TuneKey = std::tuple<int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, zp::GemmShape> g_tune;
bool g_tune_loaded = false;

constexpr zp::GemmShape kDefaultShape4{8, 2, 2, 256, 2, 4};
constexpr zp::GemmShape kDefaultShape1{4, 2, 2, 128, 1, 9};
// byte-plane problems (batched answers, H)
const std::vector<zp::GemmShape> kCandidates4 = {{8, 2, 2, 256, 2, 4}, {8, 1, 2, 256, 2, 4}, {8, 1, 2, 256, 4, 4},
                                                 {8, 2, 2, 256, 4, 4}, {8, 1, 1, 256, 2, 4}, {4, 1, 2, 512, 1, 4},
                                                 {4, 4, 2, 256, 1, 4}, {4, 1, 2, 256, 1, 4}, {2, 2, 2, 256, 1, 4},
                                                 {4, 2, 4, 256, 1, 4}};
// one-plane problems (the offset answer): column groups per block as well
const std::vector<zp::GemmShape> kCandidates1 = {{4, 2, 2, 128, 1, 9}, {4, 3, 2, 128, 1, 9}, {4, 4, 2, 128, 1, 9},
                                                 {2, 4, 2, 64, 1, 9},  {8, 1, 2, 256, 1, 3}, {8, 1, 1, 256, 1, 4},
                                                 {8, 2, 2, 256, 1, 3}, {4, 1, 2, 256, 1, 3}, {4, 4, 2, 256, 1, 3},
                                                 {8, 1, 2, 256, 1, 2}, {4, 1, 4, 256, 1, 3}, {4, 2, 4, 256, 1, 4}};

const char* tune_cache_path() {
  const char* p = std::getenv("ZIPPIR_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

using BatchKey = std::tuple<int, int, int>;
bool batch_shape_valid(const zp::BatchShape& b) {
  if (b.mr == 0) return (b.depth == 1 || b.depth == 2) && (b.ksplit == 2 || b.ksplit == 4);
  return (b.mr == 1 || b.mr == 2) && b.depth >= 2 && b.depth <= 4 && b.ksplit >= 0 && b.ksplit <= 64 &&
         b.blocks_per_cu >= 1 && b.blocks_per_cu <= 4;
}
std::map<BatchKey, zp::BatchShape> g_btune;

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {  // lines of any other layout (an older cache) are skipped
    std::istringstream in(line);
    if (line.compare(0, 6, "batch ") == 0) {
      std::string tag;
      int br, bp, ncg, mr, d, k, bpc, bextra;
      in >> tag;
      if (!(in >> br >> bp >> ncg >> mr >> d >> k >> bpc) || (in >> bextra)) continue;
      const zp::BatchShape bs{mr, d, k, bpc};
      if (batch_shape_valid(bs)) g_btune[BatchKey(br, bp, ncg)] = bs;
      continue;
    }
    int r, p, n, m, pl, tl, w, d, mr, kb, k, cg, extra;
    if (!(in >> r >> p >> n >> m >> pl >> tl >> w >> d >> mr >> kb >> k >> cg) || (in >> extra)) continue;
    if ((tl != 0 && tl != 1) || (tl == 1 && pl != 4)) continue;
    const zp::GemmShape sh{w, d, mr, kb, k, cg};
    if (zp::gemm_shape_valid(sh, p, pl)) g_tune[TuneKey(r, p, n, m, pl, tl)] = sh;
  }
}

// Rewrites the cache file with both tables: the contraction's lines, then the fused batched
// answer's ("batch ..." lines).
void tune_store_locked() {
  const char* path = tune_cache_path();
  if (!path) return;
  std::ofstream f(path, std::ios::trunc);
  for (auto& kv : g_tune)
    f << std::get<0>(kv.first) << " " << std::get<1>(kv.first) << " " << std::get<2>(kv.first) << " "
      << std::get<3>(kv.first) << " " << std::get<4>(kv.first) << " " << std::get<5>(kv.first) << " "
      << kv.second.waves << " "
      << kv.second.depth << " "
      << kv.second.mr << " " << kv.second.kb << " " << kv.second.ksplit << " " << kv.second.cg << "\n";
  for (auto& kv : g_btune)
    f << "batch " << std::get<0>(kv.first) << " " << std::get<1>(kv.first) << " " << std::get<2>(kv.first) << " "
      << kv.second.mr << " " << kv.second.depth << " " << kv.second.ksplit << " " << kv.second.blocks_per_cu << "\n";
}

bool autotune_enabled(const pir_server* s) {
  if (s->serving) return false;
  const char* e = std::getenv("ZIPPIR_AUTOTUNE");
  return !(e && std::strcmp(e, "0") == 0);
}

// out = D . X (mod 2^32 for four planes) with the tuned launch shape; tiled: D is the tiled
// copy (four planes, rows from a multiple of 16).
pir_status run_gemm_x(pir_server* s, const uint8_t* D, int rows, int cols, int pitch, int planes,
                      const int8_t* Xs, const int32_t* colsum, int ncol, const int32_t* rowsum,
                      uint32_t* out, bool rowmajor, long long ld, bool tiled = false) {
  hipStream_t st = s->stream;
  if (tiled && planes != 4) return fail(PIR_EINVAL, "the tiled copy serves the four-plane contraction only");
  const TuneKey key((int)rows, pitch, ncol, rowmajor ? 1 : 0, planes, tiled ? 1 : 0);
  zp::GemmShape shape = planes == 4 ? kDefaultShape4 : kDefaultShape1;
  bool need_tune = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) shape = it->second;
    else need_tune = autotune_enabled(s);
  }
  if (need_tune) {
    const size_t nout = (size_t)rows * (size_t)ncol;
    const size_t refbytes = (nout * sizeof(uint32_t) + 255) / 256 * 256;
    void* tmp = nullptr;
    ZP_TRY(s->alloc(&tmp, refbytes + 256));
    auto* ref = static_cast<uint32_t*>(tmp);
    auto* mism = reinterpret_cast<unsigned*>(static_cast<char*>(tmp) + refbytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pir_status rc = PIR_OK;
    auto check = [&](hipError_t e) {
      if (e != hipSuccess && rc == PIR_OK) rc = fail(PIR_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    };
    check(hipEventCreate(&e0));
    check(hipEventCreate(&e1));
    check(hipMemsetAsync(mism, 0, sizeof(unsigned), st));
    float best = 1e30f;
    bool have_ref = false;
    for (const zp::GemmShape& c : planes == 4 ? kCandidates4 : kCandidates1) {
      if (rc != PIR_OK) break;
      if (!zp::gemm_shape_valid(c, pitch, planes)) continue;
      zp::launch_gemm_planes(D, rows, cols, pitch, planes, Xs, colsum, ncol, rowsum, out, rowmajor,
                             ld, c, st, tiled);
      zp::launch_gemm_snapshot(out, rows, ncol, rowmajor, ld, ref, have_ref, mism, st);
      have_ref = true;
      float ms = 1e30f;
      for (int rep = 0; rep < 3 && rc == PIR_OK; ++rep) {
        check(hipEventRecord(e0, st));
        zp::launch_gemm_planes(D, rows, cols, pitch, planes, Xs, colsum, ncol, rowsum, out, rowmajor,
                               ld, c, st, tiled);
        check(hipEventRecord(e1, st));
        check(hipEventSynchronize(e1));
        float t = 0;
        check(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, t);
      }
      if (ms < best) {
        best = ms;
        shape = c;
      }
    }
    unsigned bad = 0;
    check(hipMemcpyAsync(&bad, mism, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    check(hipStreamSynchronize(st));
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->release(tmp);
    ZP_TRY(rc);
    if (bad != 0)
      return fail(PIR_EDEVICE, "autotune: launch shapes disagree on " + std::to_string(bad) +
                                   " output elements");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = shape;
    tune_store_locked();
  }
  ProfScope ps(s, planes == 4 ? PIR_KERNEL_GEMM : PIR_KERNEL_OFFSET_GEMM);
  zp::launch_gemm_planes(D, rows, cols, pitch, planes, Xs, colsum, ncol, rowsum, out, rowmajor, ld,
                         shape, st, tiled);
  return PIR_OK;
}

// The database contraction: out = D . X mod 2^32 over the rows of D starting at D (row-major,
// or the tiled copy from a multiple of 16 rows when tiled).
pir_status run_gemm(pir_server* s, const uint8_t* D, int rows, const int8_t* Xs,
                    const int32_t* colsum, int ncol, const int32_t* rowsum, uint32_t* out,
                    bool rowmajor, long long ld, bool tiled = false) {
  return run_gemm_x(s, D, rows, (int)s->cols, (int)s->pitch, 4, Xs, colsum, ncol, rowsum, out,
                    rowmajor, ld, tiled);
}

// ----------------------------------------------------------------------------- batch tuner
// Launch shape of the fused batched answer per (rows, pitch, column groups of 32 queries), chosen
// like the contraction's: every candidate runs once and must give the first one's bits
// (PIR_EDEVICE otherwise), then the fastest of three timed launches wins.  Batches of 2..32
// queries share one key, so a database is tuned once for them.  Persisted in the same cache
// file as lines "batch rows pitch ncg mr depth ksplit blocks_per_cu".
constexpr zp::BatchShape kDefaultBatch{0, 1, 2, 0};
// mr 0: the split form (pack launch + byte-plane contraction with depth and ksplit as given),
// the default: it measured faster than the fused form (186-194 us against 282-315 us for 32
// queries on the 1 GiB database)
const std::vector<zp::BatchShape> kBatchCandidates = {
    {2, 4, 0, 1}, {2, 2, 0, 1}, {2, 4, 2, 1}, {1, 4, 0, 2}, {1, 2, 2, 2},
    {0, 1, 2, 0}, {0, 2, 2, 0}, {0, 1, 4, 0}};


// Times `ncand` launch variants of one problem and returns the fastest in *best: every variant
// runs once and must leave the first one's bits in the rows x ncol output block (out with
// leading dimension ld, row-major or column-major; PIR_EDEVICE otherwise), then the fastest of
// three event-timed launches wins.
pir_status tune_variants(pir_server* s, const char* what, int ncand, const std::function<void(int)>& launch,
                         const uint32_t* out, int rows, int ncol, bool rowmajor, long long ld, int* best) {
  hipStream_t st = s->stream;
  const size_t nout = (size_t)rows * (size_t)ncol;
  const size_t refbytes = (nout * sizeof(uint32_t) + 255) / 256 * 256;
  void* tmp = nullptr;
  ZP_TRY(s->alloc(&tmp, refbytes + 256));
  auto* ref = static_cast<uint32_t*>(tmp);
  auto* mism = reinterpret_cast<unsigned*>(static_cast<char*>(tmp) + refbytes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  pir_status rc = PIR_OK;
  auto check = [&](hipError_t e) {
    if (e != hipSuccess && rc == PIR_OK) rc = fail(PIR_EDEVICE, std::string(what) + " autotune: " + hipGetErrorString(e));
  };
  check(hipEventCreate(&e0));
  check(hipEventCreate(&e1));
  check(hipMemsetAsync(mism, 0, sizeof(unsigned), st));
  float best_ms = 1e30f;
  *best = 0;
  for (int c = 0; c < ncand && rc == PIR_OK; ++c) {
    launch(c);
    zp::launch_gemm_snapshot(out, rows, ncol, rowmajor, ld, ref, c > 0, mism, st);
    float ms = 1e30f;
    for (int rep = 0; rep < 3 && rc == PIR_OK; ++rep) {
      check(hipEventRecord(e0, st));
      launch(c);
      check(hipEventRecord(e1, st));
      check(hipEventSynchronize(e1));
      float t = 0;
      check(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    if (ms < best_ms) {
      best_ms = ms;
      *best = c;
    }
  }
  unsigned bad = 0;
  check(hipMemcpyAsync(&bad, mism, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  check(hipStreamSynchronize(st));
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  s->release(tmp);
  ZP_TRY(rc);
  if (bad != 0)
    return fail(PIR_EDEVICE, std::string(what) + " autotune: launch shapes disagree on " + std::to_string(bad) +
                                 " output elements");
  return PIR_OK;
}

// Offset contraction variant per (rows, n, h, batch), tuned on first use (in memory only).
using OffsetKey = std::tuple<int, int, int, int>;
std::map<OffsetKey, int> g_otune;

// H = D.A for `rows` rows (tiled copy or row-major rows), the launch shape tuned once per
// (rows bucket, tiled, n): row counts are bucketed by powers of two so that updates of different
// sizes share a choice.
using HKey = std::tuple<int, int, int>;
std::map<HKey, int> g_htune;

pir_status run_hgemm(pir_server* s, const uint8_t* D, bool tiled, int rows, const int32_t* rowsum, uint32_t* H) {
  hipStream_t st = s->stream;
  auto launch = [&](int variant) {
    zp::launch_hgemm(D, tiled, rows, (int)s->cols, (int)s->pitch, s->Apt, (int)s->n, s->Acolsum, rowsum, H, variant, st);
  };
  int bucket = 1;
  while (bucket < rows) bucket <<= 1;
  const HKey key(bucket, tiled ? 1 : 0, (int)s->n);
  int variant = 0;
  bool need_tune = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_htune.find(key);
    if (it != g_htune.end()) variant = it->second;
    else need_tune = autotune_enabled(s);
  }
  if (need_tune) {
    ZP_TRY(tune_variants(s, "hint contraction", zp::hgemm_variants(), launch, H, rows, (int)s->n, true, s->n, &variant));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_htune[key] = variant;
  }
  ProfScope ps(s, PIR_KERNEL_GEMM);
  launch(variant);
  return PIR_OK;
}

// B = D.Q for `rows` rows of the tiled copy from a multiple of 256 rows (B column-major, ld).
pir_status run_batch(pir_server* s, const uint8_t* Dt, int rows, const uint32_t* Q, int batch,
                     const int32_t* rowsum, uint32_t* out, long long ld) {
  hipStream_t st = s->stream;
  const int ncg = (batch + 31) / 32;
  const BatchKey key(rows, (int)s->pitch, ncg);
  zp::BatchShape shape = kDefaultBatch;
  bool need_tune = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_btune.find(key);
    if (it != g_btune.end()) shape = it->second;
    else need_tune = autotune_enabled(s);
  }
  // The split form: planes packed by their own launch, then the byte-plane contraction with
  // split-K atomics (shape.mr == 0 marks it; depth and ksplit pick its launch shape).
  const size_t pbytes = (size_t)batch * 4 * s->pitch, cbytes = (size_t)batch * 4 * sizeof(int32_t);
  auto launch = [&](const zp::BatchShape& c) {
    if (c.mr != 0) {
      zp::launch_batch_answer(Dt, rows, (int)s->cols, (int)s->pitch, Q, batch, rowsum, out, ld, c, s->num_cus, st);
      return;
    }
    zp::launch_pack_planes_s8(Q, s->cols, 1, batch, (int)s->cols, (int)s->pitch, (int8_t*)s->s_planes.p,
                              (int32_t*)s->s_colsum.p, st);
    const zp::GemmShape gs{8, c.depth, 2, 256, c.ksplit, 4};
    zp::launch_gemm_planes(Dt, rows, (int)s->cols, (int)s->pitch, 4, (const int8_t*)s->s_planes.p,
                           (const int32_t*)s->s_colsum.p, batch, rowsum, out, false, ld, gs, st, true);
  };
  ZP_TRY(s->scratch(s->s_planes, pbytes));
  ZP_TRY(s->scratch(s->s_colsum, cbytes));
  if (need_tune) {
    int best = 0;
    ZP_TRY(tune_variants(s, "batch", (int)kBatchCandidates.size(), [&](int c) { launch(kBatchCandidates[c]); }, out,
                         rows, batch, false, ld, &best));
    shape = kBatchCandidates[best];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_btune[key] = shape;
    tune_store_locked();
  }
  ProfScope ps(s, PIR_KERNEL_GEMM);
  launch(shape);
  return PIR_OK;
}

pir_status use_device(pir_server* s) {
  ZP_HIP(hipSetDevice(s->device));
  return PIR_OK;
}

// Allocate and fill the contraction's tiled copy of D (rows rounded up to 16; the rows past
// the last are never read).  PIR_ENOMEM leaves the server without one.  With headroom, the
// copy is only made if at least an eighth of the device's memory (and 4 GiB) stays free for
// hints, tables and batches after it.
pir_status build_tiled(pir_server* s, bool headroom) {
  if (s->Dt) return PIR_OK;
  const size_t rows16 = ((size_t)s->rows + 15) / 16 * 16;
  const size_t need = rows16 * s->pitch;
  if (headroom) {
    size_t free_b = 0, total_b = 0;
    ZP_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t keep = std::max<size_t>(size_t(4) << 30, total_b / 8);
    if (free_b < need + keep) return fail(PIR_ENOMEM, "no room for the tiled copy of D");
  }
  ZP_TRY(s->alloc((void**)&s->Dt, need));
  zp::launch_tile_rows(s->D, (int)s->pitch, nullptr, (int)s->rows, s->Dt, s->stream);
  ZP_HIP(hipGetLastError());
  return PIR_OK;
}

// Recompute H for the given rows (all rows if the list covers most of them).
pir_status refresh_H(pir_server* s, const std::vector<uint32_t>& rows_in) {
  if (rows_in.empty()) return PIR_OK;
  hipStream_t st = s->stream;
  if (rows_in.size() * 4 >= s->rows) {
    ZP_TRY(run_hgemm(s, s->Dt ? s->Dt : s->D, s->Dt != nullptr, (int)s->rows, s->rowsum, s->H));
  } else {
    const size_t m = rows_in.size();
    ZP_TRY(s->scratch(s->s_rows, m * sizeof(uint32_t)));
    ZP_TRY(s->scratch(s->s_gath, m * (size_t)s->pitch));
    ZP_TRY(s->scratch(s->s_gsum, m * sizeof(int32_t)));
    ZP_TRY(s->scratch(s->s_h, m * (size_t)s->n * sizeof(uint32_t)));
    auto* drows = (uint32_t*)s->s_rows.p;
    ZP_HIP(hipMemcpyAsync(drows, rows_in.data(), m * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    zp::launch_gather_rows_u8(s->D, (int)s->pitch, drows, (int)m, (uint8_t*)s->s_gath.p, st);
    zp::launch_gather_rowsum(s->rowsum, drows, (int)m, (int32_t*)s->s_gsum.p, st);
    ZP_TRY(run_hgemm(s, (const uint8_t*)s->s_gath.p, false, (int)m, (const int32_t*)s->s_gsum.p,
                     (uint32_t*)s->s_h.p));
    zp::launch_scatter_rows_u32((const uint32_t*)s->s_h.p, (int)s->n, drows, (int)m, s->H, st);
    // the scratch is reused by later calls: finish before returning
    ZP_HIP(hipStreamSynchronize(st));
  }
  ZP_HIP(hipGetLastError());
  for (uint32_t r : rows_in)
    if (!s->H_valid[r]) {
      s->H_valid[r] = 1;
      --s->H_stale;
    }
  s->E_ready = false;
  return PIR_OK;
}

pir_status refresh_all_stale_H(pir_server* s) {
  if (s->H_stale == 0) return PIR_OK;
  std::vector<uint32_t> rows;
  rows.reserve((size_t)s->H_stale);
  for (uint32_t r = 0; r < s->rows; ++r)
    if (!s->H_valid[r]) rows.push_back(r);
  return refresh_H(s, rows);
}

ClientState* find_client(pir_server* s, uint32_t id) {
  auto it = s->clients.find(id);
  return it == s->clients.end() ? nullptr : it->second.get();
}

}  // namespace

hipStream_t zp::server_stream(pir_server* s) { return s->stream; }
int zp::server_device(pir_server* s) { return s->device; }
void zp::set_error(const char* msg) { g_last_error = msg; }

// E bytes and their row sums for the offset answer (H must be valid).
pir_status ensure_E(pir_server* s) {
  if (s->E_ready) return PIR_OK;
  hipStream_t st = s->stream;
  if (!s->Ep) {
    s->rows_pad = (s->rows + 127u) / 128u * 128u;
    const size_t bytes = (size_t)s->rows_pad * 4 * 64 * zp::offset_slices((int)s->n);
    ZP_TRY(s->alloc((void**)&s->Ep, bytes));
    ZP_TRY(s->alloc((void**)&s->Ers, (size_t)4 * s->rows_pad * sizeof(int32_t)));
    // rows past the last stay zero (every plane sum is read for whole 16-row tiles)
    ZP_HIP(hipMemsetAsync(s->Ers, 0, (size_t)4 * s->rows_pad * sizeof(int32_t), st));
  }
  zp::launch_e_planes(s->H, (int)s->rows, (int)s->n, (int)s->rows_pad, s->Ep, s->Ers, st);
  ZP_HIP(hipGetLastError());
  s->E_ready = true;
  return PIR_OK;
}

// Recompute the packed group keys of `groups` (all groups when empty) for a client whose rows
// in those groups are valid.  Synchronizes the stream.
pir_status refresh_groups(pir_server* s, ClientState* c, std::vector<uint32_t> groups) {
  if (c->ell <= 1) return PIR_OK;
  const uint32_t G = (s->rows + c->ell - 1) / c->ell;
  const bool all = groups.empty();
  hipStream_t st = s->stream;
  const zp::ClientDev cd = c->dev();
  uint32_t* dg = nullptr;
  const int ng = all ? (int)G : (int)groups.size();
  if (!all) {
    ZP_TRY(s->alloc((void**)&dg, groups.size() * sizeof(uint32_t)));
    (void)hipMemcpyAsync(dg, groups.data(), groups.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st);
  }
  zp::launch_group_keys(cd, c->Kp, (int)s->rows, (int)c->ell, (int)c->t, dg, ng, c->Kg, st);
  zp::launch_combine_key(cd, c->Kg, dg, ng, c->Mr, c->Yg, st, false);
  // M_g 2^(32h): the packed combine's Montgomery product then takes only beta_g's h limbs
  zp::launch_mul_pow2_limbs(cd, c->Mr, dg, ng, (int)cd.h, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (dg) s->release(dg);
  if (e != hipSuccess) return fail(PIR_EDEVICE, std::string("group keys: ") + hipGetErrorString(e));
  if (all) {
    std::fill(c->gvalid.begin(), c->gvalid.end(), 1);
    c->gstale = 0;
  } else {
    for (uint32_t g : groups)
      if (!c->gvalid[g]) {
        c->gvalid[g] = 1;
        --c->gstale;
      }
  }
  return PIR_OK;
}

// The one-call step's checks and launches, shared by pir_answer_compress and its no-alloc
// variant.  answer_compress_check: the client exists with a complete hint and the database
// has at most 64 column segments (nseg receives their number); makes the server's device
// current.  answer_compress_launch: the two launches on device arrays, the query 16-byte
// aligned, part holding nseg x rows words.
pir_status zp::answer_compress_check(pir_server* s, uint32_t id, int* nseg) {
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id " + std::to_string(id));
  if (c->stale != 0)
    return fail(PIR_ESTALE, "client " + std::to_string(id) + " has " + std::to_string(c->stale) +
                                " stale hint rows");
  *nseg = zp::answer_segments((int)s->pitch);
  if (*nseg > 64) return fail(PIR_EINVAL, "database wider than 262144 columns: use pir_answer and pir_compress");
  return use_device(s);
}

pir_status zp::answer_compress_launch(pir_server* s, uint32_t id, const uint32_t* dQ, uint32_t* dB, uint32_t* dC,
                                      uint32_t* part, bool events) {
  ClientState* c = find_client(s, id);
  hipStream_t st = s->stream;
  const int nseg = zp::answer_segments((int)s->pitch);
  // the profiling events (pir_profile) are created per launch, so the no-alloc caller skips them
  pir_server* ps_srv = events ? s : nullptr;
  {
    std::unique_ptr<ProfScope> ps(ps_srv ? new ProfScope(ps_srv, PIR_KERNEL_STEP_MATVEC) : nullptr);
    zp::launch_matvec_part(s->D, (int)s->rows, (int)s->pitch, dQ, (int)s->cols, part, st);
  }
  {
    std::unique_ptr<ProfScope> ps(ps_srv ? new ProfScope(ps_srv, PIR_KERNEL_STEP_COMBINE) : nullptr);
    zp::launch_combine_parts(c->dev(), c->Kp, c->Mp, part, nseg, (int)s->rows, dB, dC, st);
  }
  ZP_HIP(hipGetLastError());
  return PIR_OK;
}

void zp::server_shape(pir_server* s, uint32_t* rows, uint32_t* cols) {
  *rows = s->rows;
  *cols = s->cols;
}

// ============================================================================= C ABI

extern "C" {

const char* pir_strerror(pir_status st) {
  switch (st) {
    case PIR_OK: return "ok";
    case PIR_EINVAL: return "invalid argument";
    case PIR_ENOMEM: return "out of memory";
    case PIR_EDEVICE: return "device error";
    case PIR_ESTALE: return "hint missing or stale";
    case PIR_EBUSY: return "resource busy";
    default: return "unknown status";
  }
}

const char* pir_last_error(void) { return g_last_error.c_str(); }

pir_status pir_setup(pir_server** out, int device, void* hip_stream, const uint8_t* D,
                     uint32_t rows, uint32_t cols, const uint32_t* A, uint32_t n,
                     uint32_t ptr_flags) {
  g_last_error.clear();
  if (!out) return fail(PIR_EINVAL, "out is NULL");
  *out = nullptr;
  ZP_TRY(check_flags(ptr_flags));
  if (!D || !A || rows == 0 || cols == 0 || n == 0)
    return fail(PIR_EINVAL, "D and A must be non-NULL and rows, cols, n >= 1");
  // cols <= 2^24 keeps every in-kernel offset within a column block below 2^31 and every
  // grid dimension below its hardware limit
  if (cols > (1u << 24) || rows > (1u << 30) || n > (1u << 16))
    return fail(PIR_EINVAL, "shape too large (cols <= 2^24, rows <= 2^30, n <= 2^16)");
  int ndev = 0;
  ZP_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(PIR_EINVAL, "no such device");
  auto s = std::make_unique<pir_server>();
  s->device = device;
  s->stream = (hipStream_t)hip_stream;
  s->rows = rows;
  s->cols = cols;
  s->n = n;
  s->pitch = (cols + 255u) & ~255u;
  ZP_TRY(use_device(s.get()));
  // the device address of pir_answer_compress_noalloc's static scratch, looked up once per device
  ZP_TRY(zp::scratch_init(device, nullptr));
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
      s->num_cus = cus;
  }
  ZP_HIP(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
  ZP_HIP(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
  ZP_HIP(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
  hipStream_t st = s->stream;
  const size_t dbytes = (size_t)rows * s->pitch;
  ZP_TRY(s->alloc((void**)&s->D, dbytes));
  if (s->pitch != cols) ZP_HIP(hipMemsetAsync(s->D, 0, dbytes, st));
  ZP_HIP(hipMemcpy2DAsync(s->D, s->pitch, D, cols, cols, rows, kind_to_dev(ptr_flags), st));
  ZP_TRY(s->alloc((void**)&s->A, (size_t)cols * n * sizeof(uint32_t)));
  ZP_HIP(hipMemcpyAsync(s->A, A, (size_t)cols * n * sizeof(uint32_t), kind_to_dev(ptr_flags), st));
  ZP_TRY(s->alloc((void**)&s->rowsum, (size_t)rows * sizeof(int32_t)));
  zp::launch_rowsum(s->D, (int)rows, (int)cols, (int)s->pitch, s->rowsum, st);
  ZP_TRY(s->alloc((void**)&s->Apt, (size_t)4 * zp::hgemm_npad((int)n) * s->pitch));
  ZP_TRY(s->alloc((void**)&s->Acolsum, (size_t)n * 4 * sizeof(int32_t)));
  zp::launch_a_planes(s->A, (int)cols, (int)n, (int)s->pitch, s->Apt, st);
  zp::launch_a_colsum(s->A, (int)cols, (int)n, s->Acolsum, st);
  ZP_TRY(s->alloc((void**)&s->H, (size_t)rows * n * sizeof(uint32_t)));
  s->H_valid.assign(rows, 0);
  s->H_stale = rows;
  // the contraction's tiled copy, when HBM has room for it (otherwise it reads D)
  if (build_tiled(s.get(), true) != PIR_OK) g_last_error.clear();
  ZP_HIP(hipGetLastError());
  ZP_HIP(hipStreamSynchronize(st));
  *out = s.release();
  return PIR_OK;
}

void pir_destroy(pir_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  prof_clear(s);
  if (s->side) {
    (void)hipStreamSynchronize(s->side);
    (void)hipStreamDestroy(s->side);
  }
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  for (auto& kv : s->allocs) (void)hipFree(kv.first);
  s->allocs.clear();
  delete s;
}

pir_status pir_set_tiled_copy(pir_server* s, int32_t enable) {
  g_last_error.clear();
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ZP_TRY(use_device(s));
  if (enable) {
    ZP_TRY(build_tiled(s, false));
  } else if (s->Dt) {
    ZP_HIP(hipStreamSynchronize(s->stream));  // no launch may still read it
    s->release(s->Dt);
    s->Dt = nullptr;
  }
  ZP_HIP(hipStreamSynchronize(s->stream));
  return PIR_OK;
}

int32_t pir_tiled_copy(const pir_server* s) { return s && s->Dt ? 1 : 0; }

}  // extern "C"

// Frees every device buffer of a client (null pointers are skipped).
static void release_client(pir_server* s, ClientState* c) {
  for (void* p : {(void*)c->ck, (void*)c->consts, (void*)c->Kp, (void*)c->Mp, (void*)c->Y, (void*)c->PJ,
                  (void*)c->Kg, (void*)c->Mr, (void*)c->Yg})
    s->release(p);
}

// A new client of modulus N (h host limbs) without its key: checks N against Theorem 1,
// derives the Montgomery constants and packing weights, and allocates the key (n x L limbs,
// filled by the caller), K', M' and Y.  On failure nothing stays allocated.
static pir_status new_client(pir_server* s, const Big& Nin, uint32_t N_bits, std::unique_ptr<ClientState>& out) {
  auto c = std::make_unique<ClientState>();
  c->n_bits = N_bits;
  c->h = (N_bits + 31) / 32;
  c->L = 2 * c->h;
  c->P = (c->L + 63) / 64;
  c->PN = (c->h + 63) / 64;
  c->S = 64 * c->P;
  c->SN = 64 * c->PN;
  c->N = Nin;
  if (bit_length(c->N) != N_bits) return fail(PIR_EINVAL, "N does not have exactly N_bits bits");
  if ((c->N[0] & 1u) == 0) return fail(PIR_EINVAL, "N must be odd");
  // Theorem 1: N > q + n q^2 with q = 2^32, i.e. N > 2^32 + n * 2^64
  {
    Big bound(4, 0u);
    bound[1] = 1;
    bound[2] = s->n;
    if (big_cmp(c->N, bound) <= 0)
      return fail(PIR_EINVAL, "N too small: compression needs N > q + n q^2 (q = 2^32)");
  }
  // packing scale gamma = 2^t >= q + n q^2 (q = 2^32): t = 64 + bitlen(n); ell t <= N_bits - 1
  {
    uint32_t bl = 0;
    for (uint32_t v = s->n; v; v >>= 1) ++bl;
    c->t = 64 + bl;
    c->ell_max = std::max<uint32_t>(1, (N_bits - 1) / c->t);
  }
  c->mc = zp::mod_constants(c->N, N_bits, c->t);
  c->m2prime = c->mc.m2prime;
  c->nprime = c->mc.nprime;
  const std::vector<uint32_t>& host = c->mc.host;
  std::vector<uint32_t> pj((size_t)c->ell_max * c->SN, 0u);
  for (uint32_t j = 0; j < c->ell_max; ++j) {
    const Big v = big_pow2_mod((uint64_t)c->t * j + 32ull * c->SN, c->N);
    std::copy(v.begin(), v.begin() + std::min<size_t>(v.size(), c->SN), pj.begin() + (size_t)j * c->SN);
  }
  pir_status a = s->alloc((void**)&c->PJ, pj.size() * sizeof(uint32_t));
  if (a == PIR_OK) a = s->alloc((void**)&c->consts, host.size() * sizeof(uint32_t));
  if (a == PIR_OK) a = s->alloc((void**)&c->ck, (size_t)s->n * c->L * sizeof(uint32_t));
  if (a == PIR_OK) a = s->alloc((void**)&c->Kp, (size_t)s->rows * c->L * sizeof(uint32_t));
  if (a == PIR_OK) a = s->alloc((void**)&c->Mp, (size_t)s->rows * c->L * sizeof(uint32_t));
  if (a == PIR_OK) a = s->alloc((void**)&c->Y, (size_t)s->rows * c->h * sizeof(uint32_t));
  hipError_t e = hipSuccess;
  if (a == PIR_OK) e = hipMemcpy(c->PJ, pj.data(), pj.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (a == PIR_OK && e == hipSuccess)
    e = hipMemcpyAsync(c->consts, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream);
  if (a == PIR_OK && e != hipSuccess) a = fail(PIR_EDEVICE, std::string("client constants: ") + hipGetErrorString(e));
  if (a != PIR_OK) {
    release_client(s, c.get());
    return a;
  }
  c->valid.assign(s->rows, 0);
  c->stale = s->rows;
  out = std::move(c);
  return PIR_OK;
}

static pir_status read_modulus(const uint32_t* N, uint32_t N_bits, uint32_t ptr_flags, Big& out) {
  if (N_bits < 64 || N_bits > 4096) return fail(PIR_EINVAL, "N_bits must be in [64, 4096]");
  const uint32_t h = (N_bits + 31) / 32;
  out.assign(h, 0u);
  if (ptr_flags == PIR_PTR_DEVICE)
    ZP_HIP(hipMemcpy(out.data(), N, h * sizeof(uint32_t), hipMemcpyDeviceToHost));
  else
    std::memcpy(out.data(), N, h * sizeof(uint32_t));
  return PIR_OK;
}

extern "C" {

pir_status pir_add_client(pir_server* s, const uint32_t* N, uint32_t N_bits, const uint32_t* ck,
                          uint32_t ptr_flags, uint32_t* client_id) {
  g_last_error.clear();
  if (!s || !N || !ck || !client_id) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  ZP_TRY(use_device(s));
  Big Nh;
  ZP_TRY(read_modulus(N, N_bits, ptr_flags, Nh));
  std::unique_ptr<ClientState> c;
  ZP_TRY(new_client(s, Nh, N_bits, c));
  hipStream_t st = s->stream;
  const size_t ckbytes = (size_t)s->n * c->L * sizeof(uint32_t);
  // every ciphertext must be a residue mod N^2
  std::vector<uint32_t> hck((size_t)s->n * c->L);
  hipError_t e = hipMemcpyAsync(c->ck, ck, ckbytes, kind_to_dev(ptr_flags), st);
  if (e == hipSuccess) e = hipMemcpyAsync(hck.data(), c->ck, ckbytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    release_client(s, c.get());
    return fail(PIR_EDEVICE, std::string("copying ck: ") + hipGetErrorString(e));
  }
  const Big N2L = big_resize(big_mul(c->N, c->N), c->L);
  for (uint32_t k = 0; k < s->n; ++k) {
    Big v(hck.begin() + (size_t)k * c->L, hck.begin() + (size_t)(k + 1) * c->L);
    if (big_cmp(v, N2L) >= 0) {
      release_client(s, c.get());
      return fail(PIR_EINVAL, "ck[" + std::to_string(k) + "] is not below N^2");
    }
  }
  c->id = s->next_id++;
  *client_id = c->id;
  s->clients[c->id] = std::move(c);
  return PIR_OK;
}

pir_status pir_add_client_seeded(pir_server* s, const uint32_t* N, uint32_t N_bits, const uint8_t* seed,
                                 uint32_t first_query, uint32_t count, uint32_t ptr_flags,
                                 uint32_t* client_ids) {
  g_last_error.clear();
  if (!s || !N || !seed || !client_ids) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (count < 1 || count > 4096) return fail(PIR_EINVAL, "count must be in [1, 4096]");
  if ((uint64_t)first_query + count > (1ull << 32)) return fail(PIR_EINVAL, "query indices beyond 2^32");
  ZP_TRY(use_device(s));
  Big Nh;
  ZP_TRY(read_modulus(N, N_bits, ptr_flags, Nh));
  zp::SeedKey key;
  for (int i = 0; i < 8; ++i)
    key.w[i] = (uint32_t)seed[4 * i] | ((uint32_t)seed[4 * i + 1] << 8) | ((uint32_t)seed[4 * i + 2] << 16) |
               ((uint32_t)seed[4 * i + 3] << 24);
  const Big N2 = big_mul(Nh, Nh);
  const uint32_t nbits2 = bit_length(N2);
  const int W = (int)((nbits2 + 31) / 32);
  const uint32_t top_mask = (nbits2 % 32) ? ((1u << (nbits2 % 32)) - 1u) : 0xFFFFFFFFu;
  unsigned* fails = nullptr;
  ZP_TRY(s->alloc((void**)&fails, sizeof(unsigned)));
  hipStream_t st = s->stream;
  std::vector<std::unique_ptr<ClientState>> made;
  pir_status rc = PIR_OK;
  hipError_t e = hipMemsetAsync(fails, 0, sizeof(unsigned), st);
  if (e != hipSuccess) rc = fail(PIR_EDEVICE, std::string("seeded keys: ") + hipGetErrorString(e));
  for (uint32_t i = 0; i < count && rc == PIR_OK; ++i) {
    std::unique_ptr<ClientState> c;
    rc = new_client(s, Nh, N_bits, c);
    if (rc != PIR_OK) break;
    const zp::ClientDev cd = c->dev();
    zp::launch_expand_key(key, first_query + i, (int)s->n, 1, cd.N2, W, top_mask, (int)c->L, c->ck, fails, st);
    made.push_back(std::move(c));
  }
  unsigned bad = 0;
  if (rc == PIR_OK) {
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, fails, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(PIR_EDEVICE, std::string("seeded keys: ") + hipGetErrorString(e));
    else if (bad != 0) rc = fail(PIR_EDEVICE, "seeded keys: an entry was rejected 64 times in a row");
  }
  (void)hipStreamSynchronize(st);
  s->release(fails);
  if (rc != PIR_OK) {
    for (auto& c : made) release_client(s, c.get());
    return rc;
  }
  for (uint32_t i = 0; i < count; ++i) {
    made[i]->id = s->next_id++;
    client_ids[i] = made[i]->id;
    s->clients[made[i]->id] = std::move(made[i]);
  }
  return PIR_OK;
}

pir_status pir_get_client_key(pir_server* s, uint32_t id, uint32_t k0, uint32_t nk, uint32_t* ck,
                              uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ck) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  if ((uint64_t)k0 + nk > s->n) return fail(PIR_EINVAL, "key range out of bounds");
  ZP_TRY(use_device(s));
  ZP_HIP(hipMemcpyAsync(ck, c->ck + (size_t)k0 * c->L, (size_t)nk * c->L * sizeof(uint32_t),
                        kind_from_dev(ptr_flags), s->stream));
  if (ptr_flags == PIR_PTR_HOST) ZP_HIP(hipStreamSynchronize(s->stream));
  return PIR_OK;
}

pir_status pir_remove_client(pir_server* s, uint32_t id) {
  g_last_error.clear();
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  ZP_TRY(use_device(s));
  ZP_HIP(hipStreamSynchronize(s->stream));
  release_client(s, c);
  s->clients.erase(id);
  return PIR_OK;
}

pir_status pir_hint(pir_server* s, uint32_t id, const uint32_t* rows, uint32_t nrows) {
  g_last_error.clear();
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  ZP_TRY(use_device(s));
  std::vector<uint32_t> sel;
  const bool all = (rows == nullptr || nrows == 0);
  if (!all) {
    sel.assign(rows, rows + nrows);
    for (uint32_t r : sel)
      if (r >= s->rows) return fail(PIR_EINVAL, "row index out of range");
    std::sort(sel.begin(), sel.end());
    sel.erase(std::unique(sel.begin(), sel.end()), sel.end());
  }
  ZP_TRY(refresh_all_stale_H(s));
  hipStream_t st = s->stream;
  const zp::ClientDev cd = c->dev();
  const int m = all ? (int)s->rows : (int)sel.size();
  // Window width of the fixed-base table: building it costs n W (2^wb - 1) products (each
  // about 1.5 row products, one chain per wavefront), the rows m n W with W = ceil(32 / wb).
  // 11-bit windows (W = 3) win once there are a few thousand rows; if their table does not
  // fit, 8-bit windows (W = 4) are used.
  auto cost = [&](int wb) {
    const double W = (32 + wb - 1) / wb;
    return 1.5 * s->n * W * ((1 << wb) - 1) + (double)m * s->n * W;
  };
  int wbits = cost(11) < cost(zp::kWindowBits) ? 11 : zp::kWindowBits;
  uint32_t* table = nullptr;
  auto table_bytes = [&](int wb) {
    return (size_t)s->n * ((32 + wb - 1) / wb) * (((size_t)1 << wb) - 1) * c->S * sizeof(uint32_t);
  };
  if (wbits != zp::kWindowBits && s->alloc((void**)&table, table_bytes(wbits)) != PIR_OK) {
    g_last_error.clear();
    wbits = zp::kWindowBits;
  }
  if (!table) ZP_TRY(s->alloc((void**)&table, table_bytes(wbits)));
  {
    ProfScope ps(s, PIR_KERNEL_TABLE);
    zp::launch_build_table(cd, c->ck, (int)s->n, (32 + wbits - 1) / wbits, table, st, wbits);
  }
  c->hint_wbits = (uint32_t)wbits;
  uint32_t* drows = nullptr;
  if (!all) {
    pir_status a = s->alloc((void**)&drows, sel.size() * sizeof(uint32_t));
    if (a != PIR_OK) {
      s->release(table);
      return a;
    }
    (void)hipMemcpyAsync(drows, sel.data(), sel.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st);
  }
  const int parts = zp::hint_parts(m, (int)s->n);
  uint32_t* partial = nullptr;
  if (parts > 1 && s->alloc((void**)&partial, (size_t)m * parts * c->S * sizeof(uint32_t)) != PIR_OK) {
    g_last_error.clear();  // no room for the partial products: one wavefront per row
    partial = nullptr;
  }
  {
    ProfScope ps(s, PIR_KERNEL_HINT);
    if (partial)
      zp::launch_hint_rows_split(cd, s->H, (int)s->n, drows, m, table, wbits, parts, partial, c->Kp, st);
    else
      zp::launch_hint_rows(cd, s->H, (int)s->n, drows, m, table, wbits, c->Kp, st);
  }
  {
    ProfScope ps(s, PIR_KERNEL_KEY);
    zp::launch_combine_key(cd, c->Kp, drows, m, c->Mp, c->Y, st);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  s->release(table);
  if (partial) s->release(partial);
  if (drows) s->release(drows);
  if (e != hipSuccess) return fail(PIR_EDEVICE, std::string("hint kernels: ") + hipGetErrorString(e));
  if (all) {
    std::fill(c->valid.begin(), c->valid.end(), 1);
    c->stale = 0;
  } else {
    for (uint32_t r : sel)
      if (!c->valid[r]) {
        c->valid[r] = 1;
        --c->stale;
      }
  }
  if (c->ell > 1) {
    // refresh the groups whose rows are now all valid
    std::vector<uint32_t> groups;
    const uint32_t G = (s->rows + c->ell - 1) / c->ell;
    for (uint32_t g = 0; g < G; ++g) {
      if (c->gvalid[g]) continue;
      bool ok = true;
      for (uint32_t r = g * c->ell; r < std::min(s->rows, (g + 1) * c->ell) && ok; ++r) ok = c->valid[r] != 0;
      if (ok) groups.push_back(g);
    }
    if (!groups.empty()) {
      if (groups.size() == G) groups.clear();
      ZP_TRY(refresh_groups(s, c, groups));
    }
  }
  return PIR_OK;
}

pir_status pir_update_rows(pir_server* s, const uint32_t* rows, uint32_t nrows,
                           const uint8_t* new_rows, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ZP_TRY(check_flags(ptr_flags));
  if (nrows == 0) return PIR_OK;
  if (!rows || !new_rows) return fail(PIR_EINVAL, "NULL argument");
  std::vector<uint32_t> sel(rows, rows + nrows);
  {
    std::vector<uint32_t> sorted = sel;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(PIR_EINVAL, "row indices must be distinct");
    if (sorted.back() >= s->rows) return fail(PIR_EINVAL, "row index out of range");
  }
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  ZP_TRY(s->scratch(s->s_rows, sel.size() * sizeof(uint32_t)));
  ZP_TRY(s->scratch(s->s_gath, (size_t)nrows * s->cols));
  auto* drows = (uint32_t*)s->s_rows.p;
  ZP_HIP(hipMemcpyAsync(drows, sel.data(), sel.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  ZP_HIP(hipMemcpyAsync(s->s_gath.p, new_rows, (size_t)nrows * s->cols, kind_to_dev(ptr_flags), st));
  zp::launch_scatter_rows_u8((const uint8_t*)s->s_gath.p, (int)s->cols, (int)s->cols, drows,
                             (int)nrows, s->D, (int)s->pitch, st);
  if (s->Dt) zp::launch_tile_rows(s->D, (int)s->pitch, drows, (int)nrows, s->Dt, st);
  // row sums: recompute the changed rows through a gathered copy
  ZP_TRY(s->scratch(s->s_c, (size_t)nrows * s->pitch));
  ZP_TRY(s->scratch(s->s_gsum, (size_t)nrows * sizeof(int32_t)));
  zp::launch_gather_rows_u8(s->D, (int)s->pitch, drows, (int)nrows, (uint8_t*)s->s_c.p, st);
  zp::launch_rowsum((const uint8_t*)s->s_c.p, (int)nrows, (int)s->cols, (int)s->pitch,
                    (int32_t*)s->s_gsum.p, st);
  // scatter the new sums (int32 rows of width 1)
  zp::launch_scatter_rows_u32((const uint32_t*)s->s_gsum.p, 1, drows, (int)nrows,
                              (uint32_t*)s->rowsum, st);
  ZP_HIP(hipGetLastError());
  ZP_HIP(hipStreamSynchronize(st));
  for (uint32_t r : sel) {
    if (s->H_valid[r]) {
      s->H_valid[r] = 0;
      ++s->H_stale;
    }
    for (auto& kv : s->clients) {
      ClientState* c = kv.second.get();
      if (c->valid[r]) {
        c->valid[r] = 0;
        ++c->stale;
      }
      if (c->ell > 1 && c->gvalid[r / c->ell]) {
        c->gvalid[r / c->ell] = 0;
        ++c->gstale;
      }
    }
  }
  return PIR_OK;
}

// The answer's first step on device queries: picks the path (PIR_PATH_AUTO: the matvec for one
// query, the contraction otherwise) and sizes the scratch the row ranges use.  Nothing is
// enqueued: every row range packs what it reads itself, so the ranges of batches interleaved on
// one stream (the serving engine's two slots per database) never share packed operands.
static pir_status answer_begin_impl(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t* path) {
  (void)dQ;
  (void)dB;
  if (*path == PIR_PATH_AUTO) *path = batch == 1 ? PIR_PATH_MATVEC : PIR_PATH_MFMA;
  if (*path != PIR_PATH_MATVEC && *path != PIR_PATH_MFMA) return fail(PIR_EINVAL, "unknown answer path");
  ZP_TRY(s->scratch(s->s_planes, (size_t)batch * 4 * s->pitch));
  ZP_TRY(s->scratch(s->s_colsum, (size_t)batch * 4 * sizeof(int32_t)));
  return PIR_OK;
}

// Rows [r0, r0 + nr) of the answer (r0 a multiple of 256), after answer_begin_impl: the query
// planes packed (and, for the matvec, B's rows of the range cleared), then the range's launches.
static pir_status answer_rows_impl(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t path,
                                   uint32_t r0, uint32_t nr) {
  hipStream_t st = s->stream;
  if (r0 % 256 != 0 || r0 > s->rows || nr > s->rows - r0) return fail(PIR_EINVAL, "bad answer row range");
  if (nr == 0) return PIR_OK;
  uint8_t* planes = (uint8_t*)s->s_planes.p;
  if (path == PIR_PATH_MATVEC) {
    for (uint32_t c = 0; c < batch; ++c)
      zp::launch_pack_planes_u8(dQ + (size_t)c * s->cols, (int)s->cols, (int)s->pitch,
                                planes + (size_t)c * 4 * s->pitch, dB + (size_t)c * s->rows + r0, (int)nr, st);
    ProfScope ps(s, PIR_KERNEL_MATVEC, (int)batch);
    for (uint32_t c = 0; c < batch; ++c)
      zp::launch_matvec(s->D + (size_t)r0 * s->pitch, (int)nr, (int)s->pitch, planes + (size_t)c * 4 * s->pitch,
                        dB + (size_t)c * s->rows + r0, st);
  } else if (s->Dt && zp::batch_answer_supported((int)s->rows, (int)s->pitch)) {
    // the contraction on the tiled copy packs the planes itself (run_batch)
    ZP_TRY(run_batch(s, s->Dt + (size_t)r0 * s->pitch, (int)nr, dQ, (int)batch, s->rowsum + r0, dB + r0,
                     (long long)s->rows));
  } else {
    zp::launch_pack_planes_s8(dQ, s->cols, 1, (int)batch, (int)s->cols, (int)s->pitch, (int8_t*)planes,
                              (int32_t*)s->s_colsum.p, st);
    const uint8_t* base = s->Dt ? s->Dt : s->D;
    ZP_TRY(run_gemm(s, base + (size_t)r0 * s->pitch, (int)nr, (const int8_t*)planes, (const int32_t*)s->s_colsum.p,
                    (int)batch, s->rowsum + r0, dB + r0, false, (long long)s->rows, s->Dt != nullptr));
  }
  ZP_HIP(hipGetLastError());
  return PIR_OK;
}

// Rows of D per launch when a whole answer is enqueued at once: at most kLaunchBytes of D, a
// multiple of 256 rows.
static uint32_t rows_per_launch(const pir_server* s, long long bytes) {
  const long long per = std::max<long long>(256, bytes / s->pitch / 256 * 256);
  return (uint32_t)std::min<long long>(per, 1LL << 30);
}

static pir_status answer_impl(pir_server* s, const uint32_t* Q, uint32_t batch, uint32_t* B,
                              uint32_t ptr_flags, int32_t path) {
  hipStream_t st = s->stream;
  const uint32_t* dQ = Q;
  uint32_t* dB = B;
  const size_t qbytes = (size_t)batch * s->cols * sizeof(uint32_t);
  const size_t bbytes = (size_t)batch * s->rows * sizeof(uint32_t);
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_q, qbytes));
    ZP_TRY(s->scratch(s->s_b, bbytes));
    ZP_HIP(hipMemcpyAsync(s->s_q.p, Q, qbytes, hipMemcpyHostToDevice, st));
    dQ = (const uint32_t*)s->s_q.p;
    dB = (uint32_t*)s->s_b.p;
  }
  ZP_TRY(answer_begin_impl(s, dQ, batch, dB, &path));
  // D is streamed in row ranges of at most kLaunchBytes per launch, so that work queued on
  // other streams is dispatched between them
  const uint32_t per = rows_per_launch(s, zp::kLaunchBytes);
  for (uint32_t r0 = 0; r0 < s->rows; r0 += per)
    ZP_TRY(answer_rows_impl(s, dQ, batch, dB, path, r0, std::min(per, s->rows - r0)));
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(B, dB, bbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

}  // extern "C"

pir_status zp::answer_begin(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t* path) {
  return answer_begin_impl(s, dQ, batch, dB, path);
}

pir_status zp::answer_rows(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t path,
                           uint32_t r0, uint32_t nr) {
  return answer_rows_impl(s, dQ, batch, dB, path, r0, nr);
}

// Attach to (on) or detach from (off) a serving engine.  Attaching first runs the engine's
// batched answer shapes once on zero queries -- every batch size from 2 to max_batch falls in
// one of ceil(max_batch / 32) column-group shapes, answered in row ranges of `step_rows` rows
// as the engine does -- so that each contraction shape is tuned (and its scratch sized) before
// serving; afterwards shapes are no longer tuned in place.
pir_status zp::server_serving(pir_server* s, bool on, uint32_t max_batch, uint32_t step_rows) {
  ZP_TRY(use_device(s));
  if (!on) {
    s->serving = false;
    return PIR_OK;
  }
  if (max_batch >= 2) {
    if (step_rows == 0 || step_rows % 256 != 0) return fail(PIR_EINVAL, "step rows must be a multiple of 256");
    void* q = nullptr;
    void* b = nullptr;
    ZP_TRY(s->alloc(&q, (size_t)max_batch * s->cols * sizeof(uint32_t)));
    pir_status rc = s->alloc(&b, (size_t)max_batch * s->rows * sizeof(uint32_t));
    if (rc == PIR_OK && hipMemsetAsync(q, 0, (size_t)max_batch * s->cols * sizeof(uint32_t), s->stream) != hipSuccess)
      rc = fail(PIR_EDEVICE, "hipMemsetAsync failed");
    for (uint32_t g = 1; rc == PIR_OK && 32 * (g - 1) + 2 <= max_batch; ++g) {
      const uint32_t batch = std::min(max_batch, 32 * g);
      int32_t path = PIR_PATH_AUTO;
      rc = answer_begin_impl(s, (const uint32_t*)q, batch, (uint32_t*)b, &path);
      for (uint32_t r0 = 0; rc == PIR_OK && r0 < s->rows; r0 += step_rows)
        rc = answer_rows_impl(s, (const uint32_t*)q, batch, (uint32_t*)b, path, r0, std::min(step_rows, s->rows - r0));
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess && rc == PIR_OK) rc = fail(PIR_EDEVICE, "hipStreamSynchronize failed");
    s->release(q);
    s->release(b);
    ZP_TRY(rc);
  }
  s->serving = true;
  return PIR_OK;
}

extern "C" {

pir_status pir_answer_path(pir_server* s, const uint32_t* Q, uint32_t batch, uint32_t* B,
                           uint32_t ptr_flags, int32_t path) {
  g_last_error.clear();
  if (!s || !Q || !B) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (batch < 1 || batch > 1024) return fail(PIR_EINVAL, "batch must be in [1, 1024]");
  ZP_TRY(use_device(s));
  return answer_impl(s, Q, batch, B, ptr_flags, path);
}

pir_status pir_answer(pir_server* s, const uint32_t* Q, uint32_t batch, uint32_t* B,
                      uint32_t ptr_flags) {
  return pir_answer_path(s, Q, batch, B, ptr_flags, PIR_PATH_AUTO);
}

pir_status pir_compress(pir_server* s, const uint32_t* ids, uint32_t batch, const uint32_t* B,
                        uint32_t* C, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ids || !B || !C) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (batch < 1 || batch > 1024) return fail(PIR_EINVAL, "batch must be in [1, 1024]");
  std::vector<ClientState*> cs(batch);
  for (uint32_t i = 0; i < batch; ++i) {
    cs[i] = find_client(s, ids[i]);
    if (!cs[i]) return fail(PIR_EINVAL, "unknown client id " + std::to_string(ids[i]));
    if (cs[i]->L != cs[0]->L) return fail(PIR_EINVAL, "clients in one call must share L");
    if (cs[i]->stale != 0)
      return fail(PIR_ESTALE, "client " + std::to_string(ids[i]) + " has " +
                                  std::to_string(cs[i]->stale) + " stale hint rows");
  }
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t L = cs[0]->L;
  const uint32_t* dB = B;
  uint32_t* dC = C;
  const size_t bbytes = (size_t)batch * s->rows * sizeof(uint32_t);
  const size_t cbytes = (size_t)batch * s->rows * L * sizeof(uint32_t);
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_b, bbytes));
    ZP_TRY(s->scratch(s->s_c, cbytes));
    ZP_HIP(hipMemcpyAsync(s->s_b.p, B, bbytes, hipMemcpyHostToDevice, st));
    dB = (const uint32_t*)s->s_b.p;
    dC = (uint32_t*)s->s_c.p;
  }
  for (uint32_t i = 0; i < batch; ++i) {
    ProfScope ps(s, PIR_KERNEL_COMPRESS);
    zp::launch_compress(cs[i]->dev(), cs[i]->Kp, cs[i]->Mp, dB + (size_t)i * s->rows,
                        (int)s->rows, dC + (size_t)i * s->rows * L, st);
  }
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(C, dC, cbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_answer_compress(pir_server* s, const uint32_t* Q, uint32_t id, uint32_t* B,
                               uint32_t* C, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !Q || !B || !C) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  int nseg = 0;
  ZP_TRY(zp::answer_compress_check(s, id, &nseg));
  ClientState* c = find_client(s, id);
  hipStream_t st = s->stream;
  const uint32_t L = c->L;
  const uint32_t* dQ = Q;
  uint32_t* dB = B;
  uint32_t* dC = C;
  const size_t qbytes = (size_t)s->cols * sizeof(uint32_t);
  const size_t bbytes = (size_t)s->rows * sizeof(uint32_t);
  const size_t cbytes = (size_t)s->rows * L * sizeof(uint32_t);
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_q, qbytes));
    ZP_TRY(s->scratch(s->s_b, bbytes));
    ZP_TRY(s->scratch(s->s_c, cbytes));
    ZP_HIP(hipMemcpyAsync(s->s_q.p, Q, qbytes, hipMemcpyHostToDevice, st));
    dQ = (const uint32_t*)s->s_q.p;
    dB = (uint32_t*)s->s_b.p;
    dC = (uint32_t*)s->s_c.p;
  }
  if (reinterpret_cast<uintptr_t>(dQ) % 16 != 0) {  // the matvec reads the query 16 bytes at a time
    ZP_TRY(s->scratch(s->s_q, qbytes));
    ZP_HIP(hipMemcpyAsync(s->s_q.p, dQ, qbytes, hipMemcpyDeviceToDevice, st));
    dQ = (const uint32_t*)s->s_q.p;
  }
  ZP_TRY(s->scratch(s->s_part, (size_t)nseg * s->rows * sizeof(uint32_t)));
  ZP_TRY(zp::answer_compress_launch(s, id, dQ, dB, dC, (uint32_t*)s->s_part.p));
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(B, dB, bbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipMemcpyAsync(C, dC, cbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_set_packing(pir_server* s, uint32_t id, uint32_t ell) {
  g_last_error.clear();
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  if (ell < 1 || ell > c->ell_max)
    return fail(PIR_EINVAL, "ell must be in [1, " + std::to_string(c->ell_max) + "] (gamma^ell < N)");
  ZP_TRY(use_device(s));
  ZP_HIP(hipStreamSynchronize(s->stream));
  s->release(c->Kg);
  s->release(c->Mr);
  s->release(c->Yg);
  c->Kg = c->Mr = c->Yg = nullptr;
  c->ell = ell;
  c->gvalid.clear();
  c->gstale = 0;
  if (ell == 1) return PIR_OK;
  const uint32_t G = (s->rows + ell - 1) / ell;
  ZP_TRY(s->alloc((void**)&c->Kg, (size_t)G * c->L * sizeof(uint32_t)));
  ZP_TRY(s->alloc((void**)&c->Mr, (size_t)G * c->L * sizeof(uint32_t)));
  ZP_TRY(s->alloc((void**)&c->Yg, (size_t)G * c->h * sizeof(uint32_t)));
  c->gvalid.assign(G, 0);
  c->gstale = G;
  if (c->stale == 0) ZP_TRY(refresh_groups(s, c, {}));
  return PIR_OK;
}

pir_status pir_packing_info(pir_server* s, uint32_t id, uint32_t* ell, uint32_t* ell_max,
                            uint32_t* log2_gamma, uint32_t* groups) {
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  if (ell) *ell = c->ell;
  if (ell_max) *ell_max = c->ell_max;
  if (log2_gamma) *log2_gamma = c->t;
  if (groups) *groups = (s->rows + c->ell - 1) / c->ell;
  return PIR_OK;
}

pir_status pir_compress_packed(pir_server* s, const uint32_t* ids, uint32_t batch,
                               const uint32_t* B, uint32_t* C, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ids || !B || !C) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (batch < 1 || batch > 1024) return fail(PIR_EINVAL, "batch must be in [1, 1024]");
  std::vector<ClientState*> cs(batch);
  for (uint32_t i = 0; i < batch; ++i) {
    cs[i] = find_client(s, ids[i]);
    if (!cs[i]) return fail(PIR_EINVAL, "unknown client id " + std::to_string(ids[i]));
    if (cs[i]->ell <= 1) return fail(PIR_EINVAL, "client " + std::to_string(ids[i]) + " has no packing set");
    if (cs[i]->L != cs[0]->L || cs[i]->ell != cs[0]->ell)
      return fail(PIR_EINVAL, "clients in one call must share L and ell");
    if (cs[i]->stale != 0 || cs[i]->gstale != 0)
      return fail(PIR_ESTALE, "client " + std::to_string(ids[i]) + " has stale hint rows or groups");
  }
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t L = cs[0]->L, ell = cs[0]->ell;
  const uint32_t G = (s->rows + ell - 1) / ell;
  const uint32_t* dB = B;
  uint32_t* dC = C;
  const size_t bbytes = (size_t)batch * s->rows * sizeof(uint32_t);
  const size_t cbytes = (size_t)batch * G * L * sizeof(uint32_t);
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_b, bbytes));
    ZP_TRY(s->scratch(s->s_c, cbytes));
    ZP_HIP(hipMemcpyAsync(s->s_b.p, B, bbytes, hipMemcpyHostToDevice, st));
    dB = (const uint32_t*)s->s_b.p;
    dC = (uint32_t*)s->s_c.p;
  }
  for (uint32_t i = 0; i < batch; ++i) {
    ProfScope ps(s, PIR_KERNEL_COMPRESS);
    zp::launch_compress_packed(cs[i]->dev(), cs[i]->Kg, cs[i]->Mr, dB + (size_t)i * s->rows,
                               (int)s->rows, (int)ell, (int)cs[i]->t, dC + (size_t)i * G * L, st);
  }
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(C, dC, cbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

// Shared by the plain and the packed offset answer: checks, then T (batch x rows x h on the
// device) from device offsets and answers.  `packed`: every client must have the same ell > 1.
static pir_status offset_clients(pir_server* s, const uint32_t* ids, uint32_t batch, bool packed,
                                 std::vector<ClientState*>& cs) {
  if (batch < 1 || batch > 128) return fail(PIR_EINVAL, "batch must be in [1, 128]");
  if (s->n > 16384) return fail(PIR_EINVAL, "the offset answer needs n <= 16384");
  cs.assign(batch, nullptr);
  for (uint32_t i = 0; i < batch; ++i) {
    cs[i] = find_client(s, ids[i]);
    if (!cs[i]) return fail(PIR_EINVAL, "unknown client id " + std::to_string(ids[i]));
    if (cs[i]->h != cs[0]->h) return fail(PIR_EINVAL, "clients in one call must share the limb count");
    if (packed && (cs[i]->ell <= 1 || cs[i]->ell != cs[0]->ell))
      return fail(PIR_EINVAL, "clients in one packed call must share a packing factor ell > 1");
  }
  return PIR_OK;
}

// The offset contraction of the full protocol's online step: the folded limbs X (rows x batch
// (h + 1) 64-bit words in s_w) from the clients' offsets dK, launched on stream cst (the launch
// shape is tuned on the server's stream first, on the first call of a shape).
static pir_status offset_contract(pir_server* s, const std::vector<ClientState*>& cs, const uint32_t* dK,
                                  hipStream_t cst) {
  const uint32_t batch = (uint32_t)cs.size();
  ZP_TRY(refresh_all_stale_H(s));
  ZP_TRY(ensure_E(s));
  const uint32_t h = cs[0]->h;
  const int cpc = (int)(h + 1);
  const long long ncol = (long long)batch * cpc;
  const size_t kbytes = (size_t)batch * s->n * h * sizeof(uint32_t);
  const int NT = zp::offset_tiles((int)h);
  ZP_TRY(s->scratch(s->s_x, (size_t)batch * zp::offset_y_bytes((int)s->n, (int)h)));
  ZP_TRY(s->scratch(s->s_xcs, (size_t)batch * 16 * NT * sizeof(int32_t)));
  ZP_TRY(s->scratch(s->s_w, (size_t)s->rows * ncol * sizeof(uint64_t)));
  ZP_TRY(s->scratch(s->s_ys, kbytes));
  auto* X = (uint8_t*)s->s_x.p;
  auto* xcs = (int32_t*)s->s_xcs.p;
  auto* W = (uint64_t*)s->s_w.p;
  auto* ys = (uint32_t*)s->s_ys.p;
  auto prepare = [&](hipStream_t on) {
    ProfScope ps(s, PIR_KERNEL_OFFSET, (int)batch, on);
    for (uint32_t i = 0; i < batch; ++i)
      zp::launch_scale_offsets(cs[i]->dev(), dK + (size_t)i * s->n * h, (int)s->n, ys + (size_t)i * s->n * h, on);
    zp::launch_pack_y(ys, (int)batch, (int)s->n, (int)h, X, xcs, on);
  };
  auto launch = [&](int variant, hipStream_t on) {
    zp::launch_offset_gemm(s->Ep, s->Ers, (int)s->rows_pad, (int)s->rows, (int)s->n, X, xcs, (int)batch, (int)h,
                           W, ncol, cpc, variant, on);
  };
  const OffsetKey key((int)s->rows, (int)s->n, (int)h, (int)batch);
  int variant = 0;
  bool need_tune = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_otune.find(key);
    if (it != g_otune.end()) variant = it->second;
    else need_tune = autotune_enabled(s);
  }
  if (need_tune) {
    prepare(s->stream);
    // the snapshot compares the 64-bit words as pairs of 32-bit ones
    ZP_TRY(tune_variants(s, "offset", zp::offset_gemm_variants((int)h), [&](int v) { launch(v, s->stream); },
                         reinterpret_cast<const uint32_t*>(W), (int)s->rows, (int)(2 * ncol), true, 2 * ncol,
                         &variant));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_otune[key] = variant;
  }
  if (cst != s->stream) {  // everything above (H, E, tuning) is ordered before the other stream's work
    ZP_HIP(hipEventRecord(s->ev_fork, s->stream));
    ZP_HIP(hipStreamWaitEvent(cst, s->ev_fork, 0));
  }
  prepare(cst);
  {
    ProfScope ps(s, PIR_KERNEL_OFFSET_GEMM, 1, cst);
    launch(variant, cst);
  }
  ZP_HIP(hipGetLastError());
  return PIR_OK;
}

// T[i] = (B[i] + X_i) mod N_i for the contraction's folded limbs in s_w, on the server's stream.
static pir_status offset_reduce_all(pir_server* s, const std::vector<ClientState*>& cs, const uint32_t* dB,
                                    uint32_t* dT) {
  const uint32_t batch = (uint32_t)cs.size();
  const uint32_t h = cs[0]->h;
  const int cpc = (int)(h + 1);
  const long long ncol = (long long)batch * cpc;
  const auto* W = (const uint64_t*)s->s_w.p;
  {
    ProfScope ps(s, PIR_KERNEL_OFFSET, (int)batch);
    for (uint32_t i = 0; i < batch; ++i)
      zp::launch_offset_reduce(cs[i]->dev(), W + (size_t)i * cpc, ncol, dB + (size_t)i * s->rows, (int)s->rows,
                               dT + (size_t)i * s->rows * h, s->stream);
  }
  ZP_HIP(hipGetLastError());
  return PIR_OK;
}

static pir_status offset_answer_dev(pir_server* s, const std::vector<ClientState*>& cs,
                                    const uint32_t* dK, const uint32_t* dB, uint32_t* dT) {
  ZP_TRY(offset_contract(s, cs, dK, s->stream));
  return offset_reduce_all(s, cs, dB, dT);
}

static pir_status offset_answer_common(pir_server* s, const uint32_t* ids, uint32_t batch,
                                      const uint32_t* CKO, const uint32_t* B, uint32_t* T,
                                      uint32_t ptr_flags, bool packed) {
  g_last_error.clear();
  if (!s || !ids || !CKO || !B || !T) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  std::vector<ClientState*> cs;
  ZP_TRY(offset_clients(s, ids, batch, packed, cs));
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t h = cs[0]->h;
  const uint32_t ell = packed ? cs[0]->ell : 1;
  const uint32_t G = (s->rows + ell - 1) / ell;
  const size_t kbytes = (size_t)batch * s->n * h * sizeof(uint32_t);
  const size_t bbytes = (size_t)batch * s->rows * sizeof(uint32_t);
  const size_t tbytes = (size_t)batch * s->rows * h * sizeof(uint32_t);
  const size_t obytes = (size_t)batch * G * h * sizeof(uint32_t);
  const uint32_t* dK = CKO;
  const uint32_t* dB = B;
  uint32_t* dOut = T;
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_q, kbytes));
    ZP_TRY(s->scratch(s->s_b, bbytes));
    ZP_HIP(hipMemcpyAsync(s->s_q.p, CKO, kbytes, hipMemcpyHostToDevice, st));
    ZP_HIP(hipMemcpyAsync(s->s_b.p, B, bbytes, hipMemcpyHostToDevice, st));
    dK = (const uint32_t*)s->s_q.p;
    dB = (const uint32_t*)s->s_b.p;
  }
  uint32_t* dT = nullptr;
  if (packed || ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_t, tbytes));
    dT = (uint32_t*)s->s_t.p;
  } else {
    dT = T;
  }
  ZP_TRY(offset_answer_dev(s, cs, dK, dB, dT));
  if (packed) {
    if (ptr_flags == PIR_PTR_HOST) {
      ZP_TRY(s->scratch(s->s_c, obytes));
      dOut = (uint32_t*)s->s_c.p;
    }
    ZP_TRY(s->scratch(s->s_tmp, (size_t)s->rows * h * sizeof(uint32_t)));
    ProfScope ps(s, PIR_KERNEL_OFFSET, (int)batch);
    for (uint32_t i = 0; i < batch; ++i)
      zp::launch_offset_pack(cs[i]->dev(), dT + (size_t)i * s->rows * h, (int)s->rows, (int)ell, cs[i]->PJ,
                             (uint32_t*)s->s_tmp.p, dOut + (size_t)i * G * h, st);
  } else {
    dOut = dT;
  }
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(T, dOut, obytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_offset_answer(pir_server* s, const uint32_t* ids, uint32_t batch, const uint32_t* CKO,
                             const uint32_t* B, uint32_t* T, uint32_t ptr_flags) {
  return offset_answer_common(s, ids, batch, CKO, B, T, ptr_flags, false);
}

pir_status pir_answer_offset(pir_server* s, const uint32_t* ids, uint32_t batch, const uint32_t* Q,
                             const uint32_t* CKO, uint32_t* B, uint32_t* T, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ids || !Q || !CKO || !B || !T) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  std::vector<ClientState*> cs;
  ZP_TRY(offset_clients(s, ids, batch, false, cs));
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t h = cs[0]->h;
  const size_t qbytes = (size_t)batch * s->cols * sizeof(uint32_t);
  const size_t kbytes = (size_t)batch * s->n * h * sizeof(uint32_t);
  const size_t bbytes = (size_t)batch * s->rows * sizeof(uint32_t);
  const size_t tbytes = (size_t)batch * s->rows * h * sizeof(uint32_t);
  const uint32_t* dQ = Q;
  const uint32_t* dK = CKO;
  uint32_t* dB = B;
  uint32_t* dT = T;
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_aq, qbytes));
    ZP_TRY(s->scratch(s->s_ak, kbytes));
    ZP_TRY(s->scratch(s->s_ab, bbytes));
    ZP_TRY(s->scratch(s->s_t, tbytes));
    ZP_HIP(hipMemcpyAsync(s->s_aq.p, Q, qbytes, hipMemcpyHostToDevice, st));
    ZP_HIP(hipMemcpyAsync(s->s_ak.p, CKO, kbytes, hipMemcpyHostToDevice, st));
    dQ = (const uint32_t*)s->s_aq.p;
    dK = (const uint32_t*)s->s_ak.p;
    dB = (uint32_t*)s->s_ab.p;
    dT = (uint32_t*)s->s_t.p;
  }
  // One query with at most 64 column segments: the matvec writes per-segment partial sums (no
  // packing of the query), and the reduction sums them into B as it folds W.
  const int nseg = zp::answer_segments((int)s->pitch);
  const bool parts = batch == 1 && nseg <= 64;
  if (parts) {
    if (reinterpret_cast<uintptr_t>(dQ) % 16 != 0) {  // the matvec reads the query 16 bytes at a time
      ZP_TRY(s->scratch(s->s_q, qbytes));
      ZP_HIP(hipMemcpyAsync(s->s_q.p, dQ, qbytes, hipMemcpyDeviceToDevice, st));
      dQ = (const uint32_t*)s->s_q.p;
    }
    ZP_TRY(s->scratch(s->s_part, (size_t)nseg * s->rows * sizeof(uint32_t)));
  }
  // the offset contraction (independent of B) on the second stream, the answer meanwhile on the
  // server's stream; the reduction needs both
  ZP_TRY(offset_contract(s, cs, dK, s->side));
  ZP_HIP(hipEventRecord(s->ev_join, s->side));
  if (parts) {
    auto* part = (uint32_t*)s->s_part.p;
    {
      ProfScope ps(s, PIR_KERNEL_STEP_MATVEC);
      zp::launch_matvec_part(s->D, (int)s->rows, (int)s->pitch, dQ, (int)s->cols, part, st);
    }
    ZP_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
    {
      ProfScope ps(s, PIR_KERNEL_OFFSET);
      zp::launch_offset_reduce(cs[0]->dev(), (const uint64_t*)s->s_w.p, h + 1, nullptr, (int)s->rows, dT, st,
                               part, nseg, dB);
    }
    ZP_HIP(hipGetLastError());
  } else {
    ZP_TRY(answer_impl(s, dQ, batch, dB, PIR_PTR_DEVICE, PIR_PATH_AUTO));
    ZP_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
    ZP_TRY(offset_reduce_all(s, cs, dB, dT));
  }
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(B, dB, bbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipMemcpyAsync(T, dT, tbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_offset_answer_packed(pir_server* s, const uint32_t* ids, uint32_t batch,
                                    const uint32_t* CKO, const uint32_t* B, uint32_t* Tg,
                                    uint32_t ptr_flags) {
  return offset_answer_common(s, ids, batch, CKO, B, Tg, ptr_flags, true);
}

pir_status pir_compress_offset_packed(pir_server* s, const uint32_t* ids, uint32_t batch,
                                      const uint32_t* Tg, uint32_t* Cg, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ids || !Tg || !Cg) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (batch < 1 || batch > 1024) return fail(PIR_EINVAL, "batch must be in [1, 1024]");
  std::vector<ClientState*> cs(batch);
  for (uint32_t i = 0; i < batch; ++i) {
    cs[i] = find_client(s, ids[i]);
    if (!cs[i]) return fail(PIR_EINVAL, "unknown client id " + std::to_string(ids[i]));
    if (cs[i]->ell <= 1 || cs[i]->ell != cs[0]->ell || cs[i]->L != cs[0]->L)
      return fail(PIR_EINVAL, "clients in one packed call must share L and a packing factor ell > 1");
    if (cs[i]->stale != 0 || cs[i]->gstale != 0)
      return fail(PIR_ESTALE, "client " + std::to_string(ids[i]) + " has stale hint rows or groups");
  }
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t L = cs[0]->L, h = cs[0]->h, G = (s->rows + cs[0]->ell - 1) / cs[0]->ell;
  const size_t tbytes = (size_t)batch * G * h * sizeof(uint32_t);
  const size_t cbytes = (size_t)batch * G * L * sizeof(uint32_t);
  const uint32_t* dT = Tg;
  uint32_t* dC = Cg;
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_t, tbytes));
    ZP_TRY(s->scratch(s->s_c, cbytes));
    ZP_HIP(hipMemcpyAsync(s->s_t.p, Tg, tbytes, hipMemcpyHostToDevice, st));
    dT = (const uint32_t*)s->s_t.p;
    dC = (uint32_t*)s->s_c.p;
  }
  for (uint32_t i = 0; i < batch; ++i) {
    ProfScope ps(s, PIR_KERNEL_COMPRESS);
    zp::launch_compress_offset(cs[i]->dev(), cs[i]->Kg, cs[i]->Yg, dT + (size_t)i * G * h, (int)G,
                               dC + (size_t)i * G * L, st, false);
  }
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(Cg, dC, cbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_compress_offset(pir_server* s, const uint32_t* ids, uint32_t batch, const uint32_t* T,
                               uint32_t* C, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !ids || !T || !C) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if (batch < 1 || batch > 1024) return fail(PIR_EINVAL, "batch must be in [1, 1024]");
  std::vector<ClientState*> cs(batch);
  for (uint32_t i = 0; i < batch; ++i) {
    cs[i] = find_client(s, ids[i]);
    if (!cs[i]) return fail(PIR_EINVAL, "unknown client id " + std::to_string(ids[i]));
    if (cs[i]->L != cs[0]->L) return fail(PIR_EINVAL, "clients in one call must share L");
    if (cs[i]->stale != 0)
      return fail(PIR_ESTALE, "client " + std::to_string(ids[i]) + " has stale hint rows");
  }
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const uint32_t L = cs[0]->L, h = cs[0]->h;
  const size_t tbytes = (size_t)batch * s->rows * h * sizeof(uint32_t);
  const size_t cbytes = (size_t)batch * s->rows * L * sizeof(uint32_t);
  const uint32_t* dT = T;
  uint32_t* dC = C;
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_t, tbytes));
    ZP_TRY(s->scratch(s->s_c, cbytes));
    ZP_HIP(hipMemcpyAsync(s->s_t.p, T, tbytes, hipMemcpyHostToDevice, st));
    dT = (const uint32_t*)s->s_t.p;
    dC = (uint32_t*)s->s_c.p;
  }
  for (uint32_t i = 0; i < batch; ++i) {
    ProfScope ps(s, PIR_KERNEL_COMPRESS);
    zp::launch_compress_offset(cs[i]->dev(), cs[i]->Kp, cs[i]->Y, dT + (size_t)i * s->rows * h,
                               (int)s->rows, dC + (size_t)i * s->rows * L, st);
  }
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(C, dC, cbytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

pir_status pir_get_global_hint(pir_server* s, uint32_t row0, uint32_t nrows, uint32_t* H,
                               uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !H) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  if ((uint64_t)row0 + nrows > s->rows) return fail(PIR_EINVAL, "row range out of bounds");
  for (uint32_t r = row0; r < row0 + nrows; ++r)
    if (!s->H_valid[r]) return fail(PIR_ESTALE, "H row " + std::to_string(r) + " is stale");
  ZP_TRY(use_device(s));
  ZP_HIP(hipMemcpyAsync(H, s->H + (size_t)row0 * s->n, (size_t)nrows * s->n * sizeof(uint32_t),
                        kind_from_dev(ptr_flags), s->stream));
  if (ptr_flags == PIR_PTR_HOST) ZP_HIP(hipStreamSynchronize(s->stream));
  return PIR_OK;
}

pir_status pir_get_client_hint(pir_server* s, uint32_t id, uint32_t row0, uint32_t nrows,
                               uint32_t* K, uint32_t ptr_flags) {
  g_last_error.clear();
  if (!s || !K) return fail(PIR_EINVAL, "NULL argument");
  ZP_TRY(check_flags(ptr_flags));
  ClientState* c = find_client(s, id);
  if (!c) return fail(PIR_EINVAL, "unknown client id");
  if ((uint64_t)row0 + nrows > s->rows) return fail(PIR_EINVAL, "row range out of bounds");
  for (uint32_t r = row0; r < row0 + nrows; ++r)
    if (!c->valid[r]) return fail(PIR_ESTALE, "K row " + std::to_string(r) + " is stale");
  ZP_TRY(use_device(s));
  hipStream_t st = s->stream;
  const size_t bytes = (size_t)nrows * c->L * sizeof(uint32_t);
  uint32_t* dK = K;
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_TRY(s->scratch(s->s_c, bytes));
    dK = (uint32_t*)s->s_c.p;
  }
  zp::launch_unscale(c->dev(), c->Kp, (int)row0, (int)nrows, dK, st);
  ZP_HIP(hipGetLastError());
  if (ptr_flags == PIR_PTR_HOST) {
    ZP_HIP(hipMemcpyAsync(K, dK, bytes, hipMemcpyDeviceToHost, st));
    ZP_HIP(hipStreamSynchronize(st));
  }
  return PIR_OK;
}

uint32_t pir_client_limbs(pir_server* s, uint32_t id) {
  if (!s) return 0;
  ClientState* c = find_client(s, id);
  return c ? c->L : 0;
}

uint32_t pir_hint_window_bits(pir_server* s, uint32_t id) {
  if (!s) return 0;
  ClientState* c = find_client(s, id);
  return c ? c->hint_wbits : 0;
}

int64_t pir_stale_rows(pir_server* s, uint32_t id) {
  if (!s) return -1;
  if (id == UINT32_MAX) return s->H_stale;
  ClientState* c = find_client(s, id);
  return c ? c->stale : -1;
}

pir_status pir_shape(pir_server* s, uint32_t* rows, uint32_t* cols, uint32_t* n,
                     uint64_t* device_bytes) {
  if (!s) return fail(PIR_EINVAL, "NULL server");
  if (rows) *rows = s->rows;
  if (cols) *cols = s->cols;
  if (n) *n = s->n;
  if (device_bytes) *device_bytes = s->bytes;
  return PIR_OK;
}

pir_status pir_profile(pir_server* s, int32_t enable) {
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ZP_TRY(use_device(s));
  ZP_HIP(hipStreamSynchronize(s->stream));
  if (enable) prof_clear(s);
  s->prof = enable != 0;
  return PIR_OK;
}

pir_status pir_profile_read(pir_server* s, int32_t kernel, double* total_ms, uint64_t* launches) {
  if (!s) return fail(PIR_EINVAL, "NULL server");
  if (kernel < 0 || kernel >= PIR_KERNEL_COUNT) return fail(PIR_EINVAL, "unknown kernel id");
  ZP_TRY(use_device(s));
  ZP_HIP(hipStreamSynchronize(s->stream));
  double tot = 0;
  uint64_t cnt = 0;
  for (auto& pr : s->prof_ev[kernel]) {
    float ms = 0;
    ZP_HIP(hipEventElapsedTime(&ms, pr.begin, pr.end));
    tot += ms;
    cnt += (uint64_t)pr.launches;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return PIR_OK;
}

pir_status pir_sync(pir_server* s) {
  if (!s) return fail(PIR_EINVAL, "NULL server");
  ZP_TRY(use_device(s));
  ZP_HIP(hipStreamSynchronize(s->stream));
  return PIR_OK;
}

}  // extern "C"
