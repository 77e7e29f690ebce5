// Serving engine behind the pir_engine_* calls of zippir.h: continuous batching of PIR
// requests over several resident databases, admitted against a device-memory budget.
//
// A request is (database, client, query, result buffer, arrival time).  The scheduler thread
// keeps one FIFO queue per database.  Each database has two batch slots (device buffers for
// the queries, the answers and the compressed responses of one batch); whenever a slot is
// free and arrived requests are waiting, it takes up to max_batch of them whose clients
// share a limb count and a packing factor.  A batch is a list of steps enqueued on the
// database's stream: query uploads and packing, the answer in row ranges of at most
// step_bytes of D (matvec for one request, one int8-MFMA contraction otherwise),
// pir_compress (or pir_compress_packed for clients with packed responses), and the
// downloads in pieces of at most copy_bytes.  With more than one database registered, a
// batch keeps at most kDepth steps queued on its stream and the scheduler enqueues the next
// one as an earlier one completes, so a large database's answer never stands more than a
// couple of steps ahead of a small database's request on the device.  The scheduler polls
// the step events and hands completions to pir_engine_poll.  Databases use different
// streams, so their batches overlap on the device, and a database with a batch in flight
// forms its next one meanwhile.
//
// Device buffers of batches come from a pool: a slot that needs a larger buffer hands its
// old one back, and buffers are only freed (hipFree synchronises the device) when the budget
// cannot otherwise admit a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "zippir.h"

namespace {

using Clock = std::chrono::steady_clock;

// D bytes per answer step and response bytes per download step (defaults; pir_engine_set_steps).
constexpr uint64_t kStepBytes = 256ull << 20;
constexpr uint64_t kCopyBytes = 8ull << 20;
// Steps of one batch queued ahead on its stream when several databases share the device.
constexpr size_t kDepth = 2;

struct Request {
  uint64_t id = 0;
  uint32_t db = 0, client = 0, L = 0;
  uint32_t ell = 1;            // packing factor of the client's responses, read at submit
  double arrival_ms = 0;
  uint32_t* host_q = nullptr;  // pinned copy of the query
  uint32_t* result = nullptr;
};

enum StepKind : uint8_t { kBegin, kRows, kCompress, kCopy };

struct Step {
  StepKind kind;
  uint32_t a = 0, b = 0;  // kRows: first row, rows; kCopy: request, byte offset / kCopyBytes
};

struct Slot {
  uint32_t* dev = nullptr;  // queries | answers | responses of the batch
  uint64_t bytes = 0;
  bool busy = false;
  std::vector<Request> reqs;
  uint32_t L = 0, ell = 1;
  int32_t path = PIR_PATH_AUTO;
  std::vector<Step> steps;
  size_t next = 0;                  // first step not yet enqueued
  std::deque<hipEvent_t> pending;   // events after enqueued steps, oldest first
  std::vector<hipEvent_t> spare;    // recorded-and-passed events for reuse
  double start_ms = 0;
  int32_t status = PIR_OK;
};

struct PoolBuf {
  uint32_t* dev;
  uint64_t bytes;
  int device;
};

struct Db {
  pir_server* srv = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  uint32_t rows = 0, cols = 0;
  uint32_t step_rows = 0;        // rows of D per answer step (a multiple of 256)
  std::deque<Request> queue;
  Slot slots[2];
  std::vector<uint32_t*> qpool;  // free pinned query buffers (cols words each)
};

// Rows of one response: one ciphertext per database row, or per group of ell rows.
uint64_t response_rows(const Db& d, uint32_t ell) { return (d.rows + ell - 1) / ell; }

uint64_t bytes_per_request(const Db& d, uint32_t L, uint32_t ell) {
  return 4ull * d.cols + 4ull * d.rows + 4ull * response_rows(d, ell) * L;
}

// Requests can share a batch when their clients have the same limb count and packing.
uint32_t batch_key(const Request& r) { return r.L | (r.ell << 16); }

}  // namespace

struct pir_engine {
  Clock::time_point t0 = Clock::now();
  uint32_t max_batch = 32;
  uint64_t step_bytes = kStepBytes, copy_bytes = kCopyBytes;
  uint64_t budget = 0, in_use = 0, peak = 0;  // in_use counts slot and pool buffers
  std::vector<PoolBuf> pool;                   // idle device buffers
  uint64_t pooled = 0;
  std::vector<std::unique_ptr<Db>> dbs;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Request> incoming;
  std::deque<pir_completion> done;
  std::vector<double> lat;
  uint64_t next_id = 1, submitted = 0, completed = 0, failed = 0, batches = 0, waits = 0;
  uint64_t batched_reqs = 0;
  bool stop = false, started = false;
  std::thread th;

  double now() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  void run();
  bool launch(Db& d, Slot& slot, uint32_t n);
  bool advance(Db& d, Slot& slot);
  int32_t run_step(Db& d, Slot& slot, const Step& st);
  void complete(Db& d, Slot& slot);
  bool reserve(Db& d, Slot& slot, uint64_t need, uint64_t full);
  void free_pool(int device, uint64_t target);
};

namespace {
pir_status efail(pir_status st, const std::string& m) {
  zp::set_error(m.c_str());
  return st;
}
}  // namespace

extern "C" uint32_t pir_engine_capacity(uint64_t budget_free, uint64_t bytes_per_request,
                                        uint32_t max_batch) {
  if (bytes_per_request == 0) return max_batch;
  const uint64_t fit = budget_free / bytes_per_request;
  return (uint32_t)std::min<uint64_t>(fit, max_batch);
}

extern "C" uint32_t pir_engine_plan(const uint32_t* queued_limbs, uint32_t nqueued,
                                    uint32_t capacity) {
  if (nqueued == 0 || capacity == 0 || !queued_limbs) return 0;
  uint32_t n = 1;
  while (n < nqueued && n < capacity && queued_limbs[n] == queued_limbs[0]) ++n;
  return n;
}

// Free pooled buffers (largest first) until in_use + target fits the budget or the pool is
// empty.  Called with mu held, only when the budget is short.
void pir_engine::free_pool(int device, uint64_t target) {
  std::sort(pool.begin(), pool.end(), [](const PoolBuf& x, const PoolBuf& y) { return x.bytes < y.bytes; });
  while (in_use + target > budget && !pool.empty()) {
    PoolBuf pb = pool.back();
    pool.pop_back();
    (void)hipSetDevice(pb.device);
    (void)hipFree(pb.dev);
    in_use -= pb.bytes;
    pooled -= pb.bytes;
  }
  (void)hipSetDevice(device);
}

// Make sure `slot` holds at least `need` bytes of device memory within the budget: its own
// buffer, else the smallest pooled buffer that is large enough, else a new one of `full`
// bytes (a max_batch batch of the same kind) when the budget has room for that, else of
// `need` bytes.  Called with mu held.
bool pir_engine::reserve(Db& d, Slot& slot, uint64_t need, uint64_t full) {
  if (slot.bytes >= need) return true;
  if (slot.dev) {
    pool.push_back(PoolBuf{slot.dev, slot.bytes, d.device});
    pooled += slot.bytes;
    slot.dev = nullptr;
    slot.bytes = 0;
  }
  int best = -1;
  for (size_t i = 0; i < pool.size(); ++i)
    if (pool[i].device == d.device && pool[i].bytes >= need && (best < 0 || pool[i].bytes < pool[(size_t)best].bytes))
      best = (int)i;
  if (best >= 0) {
    slot.dev = pool[(size_t)best].dev;
    slot.bytes = pool[(size_t)best].bytes;
    pooled -= slot.bytes;
    pool.erase(pool.begin() + best);
    return true;
  }
  uint64_t want = std::max(need, full);
  if (in_use + want > budget) want = need;
  if (in_use + want > budget) free_pool(d.device, want);
  if (in_use + want > budget) {
    // idle slots elsewhere give their buffers up too
    for (auto& other : dbs)
      for (Slot& o : other->slots)
        if (!o.busy && &o != &slot && o.dev) {
          pool.push_back(PoolBuf{o.dev, o.bytes, other->device});
          pooled += o.bytes;
          o.dev = nullptr;
          o.bytes = 0;
        }
    free_pool(d.device, want);
  }
  if (in_use + want > budget) return false;
  (void)hipSetDevice(d.device);
  if (hipMalloc((void**)&slot.dev, want) != hipSuccess) {
    (void)hipGetLastError();
    slot.dev = nullptr;
    return false;
  }
  slot.bytes = want;
  in_use += want;
  peak = std::max(peak, in_use);
  return true;
}

// Form the batch of the first n queued requests in `slot` and enqueue its first steps.
bool pir_engine::launch(Db& d, Slot& slot, uint32_t n) {
  const uint32_t L = d.queue.front().L, ell = d.queue.front().ell;
  const uint64_t per = bytes_per_request(d, L, ell);
  if (!reserve(d, slot, per * n, per * max_batch)) return false;
  slot.reqs.assign(d.queue.begin(), d.queue.begin() + n);
  d.queue.erase(d.queue.begin(), d.queue.begin() + n);
  slot.L = L;
  slot.ell = ell;
  slot.path = PIR_PATH_AUTO;
  slot.steps.clear();
  slot.steps.push_back(Step{kBegin});
  for (uint32_t r0 = 0; r0 < d.rows; r0 += d.step_rows)
    slot.steps.push_back(Step{kRows, r0, std::min(d.step_rows, d.rows - r0)});
  slot.steps.push_back(Step{kCompress});
  const uint64_t rbytes = 4ull * response_rows(d, ell) * L;
  for (uint32_t i = 0; i < n; ++i)
    for (uint64_t off = 0; off < rbytes; off += copy_bytes) slot.steps.push_back(Step{kCopy, i, (uint32_t)(off / copy_bytes)});
  slot.next = 0;
  slot.status = PIR_OK;
  slot.start_ms = now();
  slot.busy = true;
  ++batches;
  batched_reqs += n;
  advance(d, slot);
  return true;
}

int32_t pir_engine::run_step(Db& d, Slot& slot, const Step& st) {
  const uint32_t n = (uint32_t)slot.reqs.size();
  uint32_t* dQ = slot.dev;
  uint32_t* dB = dQ + (size_t)n * d.cols;
  uint32_t* dC = dB + (size_t)n * d.rows;
  (void)hipSetDevice(d.device);
  switch (st.kind) {
    case kBegin:
      for (uint32_t i = 0; i < n; ++i)
        if (hipMemcpyAsync(dQ + (size_t)i * d.cols, slot.reqs[i].host_q, 4ull * d.cols, hipMemcpyHostToDevice,
                           d.stream) != hipSuccess)
          return PIR_EDEVICE;
      return zp::answer_begin(d.srv, dQ, n, dB, &slot.path);
    case kRows:
      return zp::answer_rows(d.srv, dQ, n, dB, slot.path, st.a, st.b);
    case kCompress: {
      std::vector<uint32_t> ids(n);
      for (uint32_t i = 0; i < n; ++i) ids[i] = slot.reqs[i].client;
      return slot.ell > 1 ? pir_compress_packed(d.srv, ids.data(), n, dB, dC, PIR_PTR_DEVICE)
                          : pir_compress(d.srv, ids.data(), n, dB, dC, PIR_PTR_DEVICE);
    }
    case kCopy: {
      const uint64_t rbytes = 4ull * response_rows(d, slot.ell) * slot.L;
      const uint64_t off = (uint64_t)st.b * copy_bytes;
      const uint64_t len = std::min(copy_bytes, rbytes - off);
      const char* src = reinterpret_cast<const char*>(dC) + (uint64_t)st.a * rbytes + off;
      char* dst = reinterpret_cast<char*>(slot.reqs[st.a].result) + off;
      return hipMemcpyAsync(dst, src, len, hipMemcpyDefault, d.stream) == hipSuccess ? PIR_OK : PIR_EDEVICE;
    }
  }
  return PIR_EINVAL;
}

// Retire the slot's passed step events and enqueue further steps while fewer than kDepth are
// outstanding (every step at once when only one database is registered).  A step that fails
// marks the batch failed and the rest are skipped.  Returns true if anything changed.
bool pir_engine::advance(Db& d, Slot& slot) {
  bool changed = false;
  while (!slot.pending.empty()) {
    const hipError_t q = hipEventQuery(slot.pending.front());
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      (void)hipGetLastError();
      slot.status = PIR_EDEVICE;
    }
    slot.spare.push_back(slot.pending.front());
    slot.pending.pop_front();
    changed = true;
  }
  const bool paced = dbs.size() > 1;
  while (slot.next < slot.steps.size() && (!paced || slot.pending.size() < kDepth)) {
    if (slot.status == PIR_OK) slot.status = run_step(d, slot, slot.steps[slot.next]);
    ++slot.next;
    changed = true;
    if (!paced && slot.next < slot.steps.size()) continue;
    hipEvent_t ev = nullptr;
    if (!slot.spare.empty()) {
      ev = slot.spare.back();
      slot.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ev = nullptr;
    }
    if (ev && hipEventRecord(ev, d.stream) == hipSuccess) {
      slot.pending.push_back(ev);
    } else {
      // no event to poll: wait for the stream here instead
      (void)hipGetLastError();
      if (ev) slot.spare.push_back(ev);
      if (hipStreamSynchronize(d.stream) != hipSuccess) {
        (void)hipGetLastError();
        slot.status = PIR_EDEVICE;
      }
    }
  }
  return changed;
}

void pir_engine::complete(Db& d, Slot& slot) {
  const double t = now();
  for (Request& r : slot.reqs) {
    pir_completion c;
    c.request_id = r.id;
    c.db = r.db;
    c.client_id = r.client;
    c.status = slot.status;
    c.batch = (uint32_t)slot.reqs.size();
    c.arrival_ms = r.arrival_ms;
    c.start_ms = slot.start_ms;
    c.done_ms = t;
    done.push_back(c);
    if (slot.status == PIR_OK) {
      ++completed;
      lat.push_back(t - r.arrival_ms);
    } else {
      ++failed;
    }
    d.qpool.push_back(r.host_q);
  }
  slot.reqs.clear();
  slot.busy = false;
}

void pir_engine::run() {
  std::unique_lock<std::mutex> lk(mu);
  std::vector<uint32_t> limbs;
  bool waited_for_budget = false;
  while (true) {
    while (!incoming.empty()) {
      Request r = incoming.front();
      incoming.pop_front();
      dbs[r.db]->queue.push_back(r);
    }
    bool progress = false, inflight = false, queued = false;
    double next_arrival = 1e300;
    const double t = now();
    for (auto& dp : dbs) {
      Db& d = *dp;
      for (Slot& s : d.slots)
        if (s.busy) {
          if (advance(d, s)) progress = true;
          if (s.next == s.steps.size() && s.pending.empty()) {
            complete(d, s);
            progress = true;
          } else {
            inflight = true;
          }
        }
      for (Slot& s : d.slots) {
        if (s.busy || d.queue.empty()) continue;
        // requests that have arrived, in FIFO order
        limbs.clear();
        for (const Request& r : d.queue) {
          if (r.arrival_ms > t) {
            next_arrival = std::min(next_arrival, r.arrival_ms);
            break;
          }
          limbs.push_back(batch_key(r));
        }
        if (limbs.empty()) continue;
        const uint64_t per = bytes_per_request(d, d.queue.front().L, d.queue.front().ell);
        uint64_t avail = budget - std::min(budget, in_use) + s.bytes + pooled;
        uint32_t cap = pir_engine_capacity(avail, per, max_batch);
        if (cap == 0) {
          // idle slots elsewhere can be released to make room
          uint64_t idle = 0;
          for (auto& other : dbs)
            for (Slot& o : other->slots)
              if (!o.busy && &o != &s) idle += o.bytes;
          cap = pir_engine_capacity(avail + idle, per, max_batch);
        }
        const uint32_t n = pir_engine_plan(limbs.data(), (uint32_t)limbs.size(), cap);
        if (n > 0 && launch(d, s, n)) {
          progress = true;
          inflight = true;
          waited_for_budget = false;
        } else {
          queued = true;
          if (!waited_for_budget) {
            ++waits;
            waited_for_budget = true;
          }
          if (!inflight) {
            // nothing in flight anywhere can free memory: this request can never run
            bool any_busy = false;
            for (auto& other : dbs)
              for (Slot& o : other->slots) any_busy |= o.busy;
            if (!any_busy) {
              Request r = d.queue.front();
              d.queue.pop_front();
              pir_completion c{r.id, r.db, r.client, PIR_ENOMEM, 0, r.arrival_ms, t, t};
              done.push_back(c);
              ++failed;
              d.qpool.push_back(r.host_q);
              progress = true;
            }
          }
        }
      }
      if (!d.queue.empty()) queued = true;
    }
    if (progress) cv_done.notify_all();
    if (stop && !inflight && !queued && incoming.empty()) break;
    if (!progress) {
      if (inflight) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else if (next_arrival < 1e299) {
        const double wait = std::max(0.0, next_arrival - now());
        cv_sched.wait_for(lk, std::chrono::duration<double, std::milli>(wait));
      } else {
        cv_sched.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
  }
}

extern "C" {

pir_status pir_engine_create(pir_engine** out, uint32_t max_batch, uint64_t hbm_budget_bytes) {
  if (!out) return efail(PIR_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 1024) return efail(PIR_EINVAL, "max_batch must be in [1, 1024]");
  auto e = std::make_unique<pir_engine>();
  e->max_batch = max_batch;
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return efail(PIR_EDEVICE, "hipMemGetInfo failed");
    hbm_budget_bytes = fr > (1ull << 30) ? fr - (1ull << 30) : fr / 2;
  }
  e->budget = hbm_budget_bytes;
  *out = e.release();
  return PIR_OK;
}

pir_status pir_engine_set_steps(pir_engine* e, uint64_t step_bytes, uint64_t copy_bytes) {
  if (!e) return efail(PIR_EINVAL, "NULL engine");
  if (step_bytes == 0 || copy_bytes == 0) return efail(PIR_EINVAL, "step sizes must be positive");
  std::lock_guard<std::mutex> lk(e->mu);
  if (!e->dbs.empty()) return efail(PIR_EINVAL, "step sizes must be set before the first database is added");
  e->step_bytes = step_bytes;
  e->copy_bytes = copy_bytes;
  return PIR_OK;
}

pir_status pir_engine_add_db(pir_engine* e, pir_server* srv, uint32_t* db_index) {
  if (!e || !srv || !db_index) return efail(PIR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->started) return efail(PIR_EINVAL, "databases must be added before the first request");
  auto d = std::make_unique<Db>();
  d->srv = srv;
  d->stream = zp::server_stream(srv);
  d->device = zp::server_device(srv);
  if (!d->stream) return efail(PIR_EINVAL, "the server needs its own (non-NULL) stream");
  uint32_t rows = 0, cols = 0, n = 0;
  uint64_t b = 0;
  if (pir_shape(srv, &rows, &cols, &n, &b) != PIR_OK) return efail(PIR_EINVAL, "bad server");
  d->rows = rows;
  d->cols = cols;
  const uint64_t pitch = ((uint64_t)cols + 255) / 256 * 256;
  d->step_rows = (uint32_t)std::min<uint64_t>(1u << 30, std::max<uint64_t>(256, e->step_bytes / pitch / 256 * 256));
  // tune and size the batched answer's shapes now, not while serving
  const pir_status st = zp::server_serving(srv, true, e->max_batch, d->step_rows);
  if (st != PIR_OK) return st;
  *db_index = (uint32_t)e->dbs.size();
  e->dbs.push_back(std::move(d));
  return PIR_OK;
}

pir_status pir_engine_submit(pir_engine* e, uint32_t db, uint32_t client, const uint32_t* query,
                             uint32_t* result, double arrival_ms, uint64_t* request_id) {
  if (!e || !query || !result) return efail(PIR_EINVAL, "NULL argument");
  uint32_t* qbuf = nullptr;
  Request r;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    if (db >= e->dbs.size()) return efail(PIR_EINVAL, "unknown database index");
    Db& d = *e->dbs[db];
    r.L = pir_client_limbs(d.srv, client);
    if (r.L == 0) return efail(PIR_EINVAL, "unknown client id");
    if (pir_packing_info(d.srv, client, &r.ell, nullptr, nullptr, nullptr) != PIR_OK)
      return efail(PIR_EINVAL, "unknown client id");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    const hipError_t pe = hipPointerGetAttributes(&attr, result);
    if (pe != hipSuccess || attr.type == hipMemoryTypeUnregistered) {
      (void)hipGetLastError();
      return efail(PIR_EINVAL, "result must be pinned host memory (pir_host_alloc) or device memory");
    }
    if (!d.qpool.empty()) {
      qbuf = d.qpool.back();
      d.qpool.pop_back();
    }
  }
  const uint32_t cols = e->dbs[db]->cols;
  if (!qbuf && hipHostMalloc((void**)&qbuf, 4ull * cols, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return efail(PIR_ENOMEM, "pinned query buffer");
  }
  std::memcpy(qbuf, query, 4ull * cols);
  std::lock_guard<std::mutex> lk(e->mu);
  r.id = e->next_id++;
  r.db = db;
  r.client = client;
  r.host_q = qbuf;
  r.result = result;
  const double t = e->now();
  r.arrival_ms = arrival_ms < 0 ? t : arrival_ms;
  e->incoming.push_back(r);
  ++e->submitted;
  if (request_id) *request_id = r.id;
  if (!e->started) {
    e->started = true;
    e->th = std::thread([e] { e->run(); });
  }
  e->cv_sched.notify_one();
  return PIR_OK;
}

pir_status pir_engine_poll(pir_engine* e, pir_completion* out, uint32_t max, uint32_t* count,
                           int32_t timeout_ms) {
  if (!e || !count || (max > 0 && !out)) return efail(PIR_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(e->mu);
  if (e->done.empty() && timeout_ms != 0) {
    if (timeout_ms < 0)
      e->cv_done.wait(lk, [&] { return !e->done.empty(); });
    else
      e->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !e->done.empty(); });
  }
  uint32_t n = 0;
  while (n < max && !e->done.empty()) {
    out[n++] = e->done.front();
    e->done.pop_front();
  }
  *count = n;
  return PIR_OK;
}

pir_status pir_engine_drain(pir_engine* e, int32_t timeout_ms) {
  if (!e) return efail(PIR_EINVAL, "NULL engine");
  std::unique_lock<std::mutex> lk(e->mu);
  auto finished = [&] { return e->completed + e->failed == e->submitted; };
  if (timeout_ms < 0) {
    e->cv_done.wait(lk, finished);
    return PIR_OK;
  }
  return e->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished)
             ? PIR_OK
             : efail(PIR_EBUSY, "requests still pending");
}

pir_status pir_engine_stats_get(pir_engine* e, pir_engine_stats* st) {
  if (!e || !st) return efail(PIR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(e->mu);
  st->submitted = e->submitted;
  st->completed = e->completed;
  st->failed = e->failed;
  st->batches = e->batches;
  st->admission_waits = e->waits;
  st->device_bytes_peak = e->peak;
  st->mean_batch = e->batches ? (double)e->batched_reqs / e->batches : 0.0;
  std::vector<double> v = e->lat;
  std::sort(v.begin(), v.end());
  auto rank = [&](double q) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::ceil(q * v.size());
    k = std::min(v.size(), std::max<size_t>(k, 1));
    return v[k - 1];
  };
  st->p50_ms = rank(0.50);
  st->p99_ms = rank(0.99);
  return PIR_OK;
}

double pir_engine_now_ms(pir_engine* e) { return e ? e->now() : 0.0; }

void pir_engine_destroy(pir_engine* e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
  }
  e->cv_sched.notify_all();
  if (e->th.joinable()) e->th.join();
  for (auto& d : e->dbs) {
    (void)hipSetDevice(d->device);
    (void)hipStreamSynchronize(d->stream);
    for (Slot& s : d->slots) {
      if (s.dev) (void)hipFree(s.dev);
      for (hipEvent_t ev : s.pending) (void)hipEventDestroy(ev);
      for (hipEvent_t ev : s.spare) (void)hipEventDestroy(ev);
    }
    (void)zp::server_serving(d->srv, false, 0, 0);
    for (uint32_t* q : d->qpool) (void)hipHostFree(q);
    for (Request& r : d->queue) (void)hipHostFree(r.host_q);
  }
  for (Request& r : e->incoming) (void)hipHostFree(r.host_q);
  for (const PoolBuf& pb : e->pool) {
    (void)hipSetDevice(pb.device);
    (void)hipFree(pb.dev);
  }
  delete e;
}

void* pir_host_alloc(uint64_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes ? bytes : 1, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pir_host_free(void* p) {
  if (p) (void)hipHostFree(p);
}

}  // extern "C"
