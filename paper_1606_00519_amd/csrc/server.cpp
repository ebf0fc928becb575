// Request loop of the C ABI (gmp_server_*): continuous batching of
// decompression requests on one GPU.
//
// Requests arrive at any time from any host thread.  A scheduler thread
// admits them first come first served while the bytes of everything in
// flight (compressed + decompressed + token workspace) stay within the
// budget, and whenever one of its launch slots is free it launches every
// admitted request not yet running as ONE kernel over all their blocks
// (largest blocks first), on that slot's stream.  Requests that arrive while
// others run join the next launch; launches of different slots overlap on
// the device.  (One launch per request would leave the device mostly idle:
// a request has only a handful of blocks, and the runtime runs few kernels
// at once.)  When a launch completes, its requests' budget and workspace are
// released and more are admitted.
//
// Token workspace comes from one device arena owned by the server, handed
// out first-fit in 256-byte units; everything else (compressed input,
// output, status words) is the caller's, already resident on the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/gompresso.h"
#include "inflate.h"

namespace {

constexpr uint32_t kMagicStream = 0x46504D47u;  // 'GMPF'
constexpr uint32_t kMagicBlock = 0x42504D47u;   // 'GMPB'
constexpr uint64_t kUnit = 256;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint32_t rd32(const uint8_t* p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
uint64_t rd64(const uint8_t* p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}

// First-fit allocator over [0, size) in kUnit units; free ranges are kept
// merged in an ordered map (offset -> length).
class Arena {
 public:
  explicit Arena(uint64_t size) { if (size) free_[0] = size; }
  bool alloc(uint64_t n, uint64_t* off) {
    n = (n + kUnit - 1) / kUnit * kUnit;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = (n + kUnit - 1) / kUnit * kUnit;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  std::map<uint64_t, uint64_t> free_;
};

struct Request {
  gmp_request r;
  std::vector<gmpk::DevJob> jobs;  // device pointers filled in at submission, except ws
  uint64_t ws_bytes = 0, bytes = 0, t_submit = 0, ws_off = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  gmpk::DevJob* d_jobs = nullptr;
  gmpk::DevJob* h_jobs = nullptr;  // pinned
  size_t cap = 0;
  bool busy = false;
  std::vector<Request> reqs;  // requests of the running launch
  uint64_t t_launch = 0;
};

}  // namespace

struct gmp_server {
  int device = 0;
  uint64_t budget = 0;
  gmp_tuning tuning{};
  uint8_t* d_arena = nullptr;
  Arena* arena = nullptr;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;  // submitted, not admitted (guarded by mu)
  std::vector<Request> ready;   // admitted, waiting for a launch slot
  std::vector<gmp_completion> completed;  // guarded by mu
  uint64_t in_flight_bytes = 0, peak_bytes = 0, submitted = 0, finished = 0, launches = 0;
  uint32_t peak_slots = 0;
  int32_t error = GMP_OK;  // first device error of the scheduler
  std::atomic<bool> stop{false};
  std::thread worker;
};

namespace {

void complete(gmp_server* s, const Request& rq, int32_t status, uint64_t t_launch) {
  gmp_completion c{};
  c.tag = rq.r.tag;
  c.status = status;
  c.t_submit_ns = rq.t_submit;
  c.t_admit_ns = t_launch;
  c.t_done_ns = now_ns();
  c.bytes = rq.r.out_len;
  s->completed.push_back(c);
  s->finished++;
}

// Launch every ready request as one kernel on slot `sl`.
gmp_status launch_ready(gmp_server* s, Slot& sl) {
  size_t n = 0;
  for (const Request& rq : s->ready) n += rq.jobs.size();
  if (n > sl.cap) {
    if (sl.d_jobs) (void)hipFree(sl.d_jobs);
    if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
    sl.d_jobs = nullptr;
    sl.h_jobs = nullptr;
    sl.cap = 0;
    const size_t cap = n + n / 2 + 16;
    if (hipMalloc(&sl.d_jobs, cap * sizeof(gmpk::DevJob)) != hipSuccess ||
        hipHostMalloc(&sl.h_jobs, cap * sizeof(gmpk::DevJob), hipHostMallocDefault) != hipSuccess)
      return GMP_ENOMEM;
    sl.cap = cap;
  }
  size_t k = 0;
  for (const Request& rq : s->ready) {
    uint64_t o = rq.ws_off;
    for (const gmpk::DevJob& j : rq.jobs) {
      sl.h_jobs[k] = j;
      sl.h_jobs[k].ws = s->d_arena + o;
      o += j.ws_len;
      k++;
    }
  }
  // largest blocks first, so the long ones start early
  std::stable_sort(sl.h_jobs, sl.h_jobs + n,
                   [](const gmpk::DevJob& x, const gmpk::DevJob& y) { return x.out_len > y.out_len; });
  if (n) {
    if (hipMemcpyAsync(sl.d_jobs, sl.h_jobs, n * sizeof(gmpk::DevJob), hipMemcpyHostToDevice, sl.stream) !=
            hipSuccess ||
        gmpk_launch(sl.d_jobs, (uint32_t)n, GMP_MODE_AUTO, s->tuning.waves_per_block, 0, 0, nullptr, sl.stream) != 0)
      return GMP_EDEVICE;
  }
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return GMP_EDEVICE;
  return GMP_OK;
}

// Scheduler thread body.
void serve(gmp_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool progress = false;
    // completed launches: their requests finish, budget and workspace return
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      for (const Request& rq : sl.reqs) {
        complete(s, rq, q == hipSuccess ? GMP_OK : GMP_EDEVICE, sl.t_launch);
        if (rq.ws_bytes) s->arena->release(rq.ws_off, rq.ws_bytes);
        s->in_flight_bytes -= rq.bytes;
      }
      if (q != hipSuccess && s->error == GMP_OK) s->error = GMP_EDEVICE;
      sl.reqs.clear();
      sl.busy = false;
      progress = true;
    }
    // admissions, first come first served, within the budget and the arena
    while (!s->pending.empty()) {
      Request& rq = s->pending.front();
      if (s->in_flight_bytes + rq.bytes > s->budget) break;
      if (rq.ws_bytes && !s->arena->alloc(rq.ws_bytes, &rq.ws_off)) break;
      s->in_flight_bytes += rq.bytes;
      if (s->in_flight_bytes > s->peak_bytes) s->peak_bytes = s->in_flight_bytes;
      s->ready.push_back(std::move(rq));
      s->pending.pop_front();
      progress = true;
    }
    // one launch for everything admitted, on a free slot
    if (!s->ready.empty()) {
      Slot* free_slot = nullptr;
      uint32_t busy = 0;
      for (Slot& sl : s->slots) {
        if (sl.busy) busy++;
        else if (!free_slot) free_slot = &sl;
      }
      if (free_slot) {
        Slot& sl = *free_slot;
        const gmp_status st = launch_ready(s, sl);
        sl.t_launch = now_ns();
        if (st != GMP_OK) {
          for (const Request& rq : s->ready) {
            complete(s, rq, st, sl.t_launch);
            if (rq.ws_bytes) s->arena->release(rq.ws_off, rq.ws_bytes);
            s->in_flight_bytes -= rq.bytes;
          }
          s->ready.clear();
          if (s->error == GMP_OK) s->error = st;
        } else {
          sl.reqs = std::move(s->ready);
          s->ready.clear();
          sl.busy = true;
          if (++busy > s->peak_slots) s->peak_slots = busy;
          s->launches++;
        }
        progress = true;
      }
    }
    if (progress) {
      s->cv.notify_all();
      continue;
    }
    // nothing to do right now: wait for a submission, or poll the device again shortly
    bool any_busy = false;
    for (Slot& sl : s->slots) any_busy |= sl.busy;
    if (any_busy)
      s->cv.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace

extern "C" gmp_status gmp_server_create(gmp_ctx* ctx, uint64_t budget_bytes, uint64_t workspace_bytes,
                                        uint32_t n_slots, const gmp_tuning* tuning, gmp_server** out) {
  (void)ctx;
  if (!ctx || !out || budget_bytes == 0 || n_slots == 0 || n_slots > 64) return GMP_EINVAL;
  *out = nullptr;
  gmp_tuning t{1u, 0u, 0u, 0u};
  if (tuning) t = *tuning;
  if (t.waves_per_block != 1 && t.waves_per_block != 2 && t.waves_per_block != 4 && t.waves_per_block != 7)
    return GMP_EINVAL;
  if (t.persistent) return GMP_EINVAL;  // requests launch one workgroup per block
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMP_EDEVICE;
  gmp_server* s = new (std::nothrow) gmp_server();
  if (!s) return GMP_ENOMEM;
  s->device = dev;
  s->budget = budget_bytes;
  s->tuning = t;
  if (workspace_bytes == 0) workspace_bytes = budget_bytes / 2;
  workspace_bytes = (workspace_bytes + kUnit - 1) / kUnit * kUnit;
  s->arena = new (std::nothrow) Arena(workspace_bytes);
  s->slots.resize(n_slots);
  bool ok = s->arena && hipMalloc(&s->d_arena, workspace_bytes) == hipSuccess;
  for (Slot& sl : s->slots) {
    ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    gmp_server_destroy(s);
    return GMP_ENOMEM;
  }
  s->worker = std::thread(serve, s);
  *out = s;
  return GMP_OK;
}

extern "C" gmp_status gmp_server_submit(gmp_server* s, const gmp_request* req) {
  if (!s || !req || !req->d_stream || !req->h_stream || !req->d_status) return GMP_EINVAL;
  const uint32_t mode = req->flags & GMP_MODE_MASK;
  if ((req->flags & ~GMP_MODE_MASK) != 0 || mode == 3u) return GMP_EINVAL;
  const uint8_t* hs = static_cast<const uint8_t*>(req->h_stream);
  if (req->len < 32 || rd32(hs) != kMagicStream) return GMP_EFORMAT;
  const uint32_t bs = rd32(hs + 8), nb = rd32(hs + 12);
  const uint64_t total = rd64(hs + 16);
  if (bs == 0 || nb != (total + bs - 1) / bs || 32 + 8 * ((uint64_t)nb + 1) > req->len) return GMP_EFORMAT;
  if (req->out_len != total) return GMP_ESIZE;
  if (nb && !req->d_out) return GMP_EINVAL;
  Request rq;
  rq.r = *req;
  rq.jobs.resize(nb);
  for (uint32_t b = 0; b < nb; b++) {
    const uint64_t o0 = rd64(hs + 32 + 8 * (size_t)b), o1 = rd64(hs + 32 + 8 * (size_t)b + 8);
    if (o0 > o1 || o1 > req->len || (o0 & 15) || o1 - o0 < 192) return GMP_EFORMAT;
    const uint8_t* blk = hs + o0;
    if (rd32(blk) != kMagicBlock) return GMP_EFORMAT;
    gmp_block_info info;
    gmp_status st = gmp_block_info_parse(blk, o1 - o0, &info);
    if (st != GMP_OK) return st;
    const uint64_t want = (b + 1 < nb) ? bs : total - (uint64_t)b * bs;
    if (info.raw_len != want) return GMP_ESIZE;
    if (mode == GMP_MODE_DE && !(info.mode == 1 && info.group % 64 == 0)) return GMP_EINVAL;
    gmpk::DevJob& j = rq.jobs[b];
    j.comp = req->d_stream + o0;
    j.comp_len = o1 - o0;
    j.out = req->d_out + (uint64_t)b * bs;
    j.out_len = info.raw_len;
    j.ws = nullptr;
    j.ws_len = gmpk::workspace_bytes(info.n_seq, info.n_lit, o1 - o0);
    j.rounds = nullptr;
    j.times = nullptr;
    j.status = req->d_status + b;
    j.n_seq = info.n_seq;
    j.n_lit = info.n_lit;
    rq.ws_bytes += j.ws_len;
  }
  rq.bytes = req->len + req->out_len + rq.ws_bytes;
  if (rq.bytes > s->budget) return GMP_EBUSY;  // could never be admitted
  rq.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error != GMP_OK) return s->error;
    s->pending.push_back(std::move(rq));
    s->submitted++;
  }
  s->cv.notify_all();
  return GMP_OK;
}

extern "C" uint32_t gmp_server_poll(gmp_server* s, gmp_completion* out, uint32_t max) {
  if (!s || !out || max == 0) return 0;
  std::lock_guard<std::mutex> g(s->mu);
  const uint32_t n = (uint32_t)std::min<size_t>(max, s->completed.size());
  std::memcpy(out, s->completed.data(), n * sizeof(gmp_completion));
  s->completed.erase(s->completed.begin(), s->completed.begin() + n);
  return n;
}

extern "C" gmp_status gmp_server_drain(gmp_server* s, uint32_t timeout_ms) {
  if (!s) return GMP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  while (s->finished < s->submitted) {
    if (s->cv.wait_until(lk, until) == std::cv_status::timeout && s->finished < s->submitted) return GMP_EBUSY;
  }
  return s->error;
}

extern "C" gmp_status gmp_server_stats(gmp_server* s, gmp_server_info* out) {
  if (!s || !out) return GMP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->finished = s->finished;
  out->pending = s->pending.size();
  out->in_flight_bytes = s->in_flight_bytes;
  out->peak_in_flight_bytes = s->peak_bytes;
  out->peak_slots = s->peak_slots;
  out->launches = s->launches;
  out->budget = s->budget;
  return GMP_OK;
}

extern "C" void gmp_server_destroy(gmp_server* s) {
  if (!s) return;
  if (s->worker.joinable()) {
    // let everything admitted finish, then stop the scheduler
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->pending.clear();
    }
    for (;;) {
      bool busy = false;
      {
        std::lock_guard<std::mutex> g(s->mu);
        for (Slot& sl : s->slots) busy |= sl.busy;
      }
      if (!busy) break;
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    s->stop.store(true);
    s->cv.notify_all();
    s->worker.join();
  }
  (void)hipSetDevice(s->device);
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.d_jobs) (void)hipFree(sl.d_jobs);
    if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->d_arena) (void)hipFree(s->d_arena);
  delete s->arena;
  delete s;
}
