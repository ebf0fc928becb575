// Request loop of the C ABI (gmp_server_*): continuous batching of
// decompression requests on one GPU.
//
// Requests arrive at any time from any host thread.  A scheduler thread
// admits them first come first served while the bytes of everything in
// flight (compressed + decompressed + token workspace) stay within the
// budget, and whenever one of its launch slots is free it launches every
// admitted request not yet running as ONE kernel over all their blocks
// (largest blocks first; one kernel per flag set), on that slot's stream.
// Requests that arrive while others run join the next launch; launches of
// different slots overlap on the device.  (One launch per request would
// leave the device mostly idle: a request has only a handful of blocks, and
// the runtime runs few kernels at once.)  Each block adds one to its
// request's completion counter in host-visible memory when it has finished,
// so a request completes, and its budget and workspace return, as soon as
// its own blocks are done, not when its launch ends.
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
#include "host_internal.h"
#include "inflate.h"

namespace {

constexpr uint32_t kMagicStream = 0x46504D47u;  // 'GMPF'
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
  std::vector<gmpk::DevJob> jobs;  // device pointers filled in at submission, except ws and done
  uint64_t ws_bytes = 0, bytes = 0, t_submit = 0, t_launch = 0, ws_off = 0;
  uint32_t ctr = 0;    // its completion counter (host-visible memory)
  bool finished = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  gmpk::DevJob* d_jobs = nullptr;
  gmpk::DevJob* h_jobs = nullptr;  // pinned
  size_t cap = 0;
  bool busy = false;
  std::vector<Request> reqs;  // requests of the running launch(es)
};

}  // namespace

struct gmp_server {
  int device = 0;
  uint64_t budget = 0, arena_bytes = 0;
  gmp_tuning tuning{};
  int32_t* d_first_err = nullptr;  // the context's first-error word
  uint8_t* d_arena = nullptr;
  Arena* arena = nullptr;
  // Completion counters, one per request in flight, in pinned host memory that
  // the kernels update: each block adds one when it has finished, so the
  // scheduler sees a request complete as soon as its last block is done,
  // while other requests of the same launch still run.
  uint32_t* h_done = nullptr;
  uint32_t* d_done = nullptr;  // the same memory, as the device sees it
  std::vector<uint32_t> free_ctr;
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

constexpr uint32_t kCounters = 4096;  // most requests admitted at once

// A request leaves the server: completion record, budget, workspace and counter back.
void retire(gmp_server* s, Request& rq, int32_t status) {
  gmp_completion c{};
  c.tag = rq.r.tag;
  c.status = status;
  c.t_submit_ns = rq.t_submit;
  c.t_admit_ns = rq.t_launch;
  c.t_done_ns = now_ns();
  c.bytes = rq.r.out_len;
  s->completed.push_back(c);
  s->finished++;
  if (rq.ws_bytes) s->arena->release(rq.ws_off, rq.ws_bytes);
  s->in_flight_bytes -= rq.bytes;
  s->free_ctr.push_back(rq.ctr);
  rq.finished = true;
}

// Launch every ready request on slot `sl`: one kernel per distinct flag set
// (resolution mode, DE check) over all the blocks of the requests that use it.
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
  std::vector<uint32_t> flag_sets;
  for (const Request& rq : s->ready)
    if (std::find(flag_sets.begin(), flag_sets.end(), rq.r.flags) == flag_sets.end()) flag_sets.push_back(rq.r.flags);
  size_t k = 0;
  for (uint32_t f : flag_sets) {
    const size_t k0 = k;
    for (const Request& rq : s->ready) {
      if (rq.r.flags != f) continue;
      uint64_t o = rq.ws_off;
      for (const gmpk::DevJob& j : rq.jobs) {
        sl.h_jobs[k] = j;
        sl.h_jobs[k].ws = s->d_arena + o;
        sl.h_jobs[k].done = s->d_done + rq.ctr;
        o += j.ws_len;
        k++;
      }
    }
    // largest blocks first, so the long ones start early
    std::stable_sort(sl.h_jobs + k0, sl.h_jobs + k,
                     [](const gmpk::DevJob& x, const gmpk::DevJob& y) { return x.out_len > y.out_len; });
    if (k > k0) {
      if (hipMemcpyAsync(sl.d_jobs + k0, sl.h_jobs + k0, (k - k0) * sizeof(gmpk::DevJob), hipMemcpyHostToDevice,
                         sl.stream) != hipSuccess ||
          gmpk_launch(sl.d_jobs + k0, (uint32_t)(k - k0), f, s->tuning.waves_per_block, 0, 0, nullptr,
                      s->d_first_err, sl.stream) != 0)
        return GMP_EDEVICE;
    }
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
    // requests whose blocks have all finished, and launches that completed
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      for (Request& rq : sl.reqs) {
        if (rq.finished) continue;
        const uint32_t d = __atomic_load_n(&s->h_done[rq.ctr], __ATOMIC_ACQUIRE);
        if (d >= rq.jobs.size()) {
          retire(s, rq, GMP_OK);
          progress = true;
        }
      }
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      // the launch is over: a request still unfinished here was ended by a HIP error
      for (Request& rq : sl.reqs) {
        if (rq.finished) continue;
        const uint32_t d = __atomic_load_n(&s->h_done[rq.ctr], __ATOMIC_ACQUIRE);
        retire(s, rq, (q == hipSuccess && d >= rq.jobs.size()) ? GMP_OK : GMP_EDEVICE);
        if (q != hipSuccess && s->error == GMP_OK) s->error = GMP_EDEVICE;
      }
      sl.reqs.clear();
      sl.busy = false;
      progress = true;
    }
    // admissions, first come first served, within the budget, the arena and the counters
    while (!s->pending.empty() && !s->free_ctr.empty()) {
      Request& rq = s->pending.front();
      if (s->in_flight_bytes + rq.bytes > s->budget) break;
      if (rq.ws_bytes && !s->arena->alloc(rq.ws_bytes, &rq.ws_off)) break;
      rq.ctr = s->free_ctr.back();
      s->free_ctr.pop_back();
      s->h_done[rq.ctr] = 0;
      s->in_flight_bytes += rq.bytes;
      if (s->in_flight_bytes > s->peak_bytes) s->peak_bytes = s->in_flight_bytes;
      s->ready.push_back(std::move(rq));
      s->pending.pop_front();
      progress = true;
    }
    // one launch (per flag set) for everything admitted, on a free slot
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
        const uint64_t t = now_ns();
        for (Request& rq : s->ready) rq.t_launch = t;
        if (st != GMP_OK) {
          // kernels of other flag sets may have started: let them end before
          // their requests' counters and workspace are handed out again
          (void)hipStreamSynchronize(sl.stream);
          for (Request& rq : s->ready) retire(s, rq, st);
          s->ready.clear();
          if (s->error == GMP_OK) s->error = st;
        } else {
          sl.reqs = std::move(s->ready);
          s->ready.clear();
          // requests without blocks are complete at once
          for (Request& rq : sl.reqs)
            if (rq.jobs.empty()) retire(s, rq, GMP_OK);
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
    // nothing to do right now: wait for a submission, or look at the device again shortly
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
  const int dev = gmp_ctx_device(ctx);
  if (hipSetDevice(dev) != hipSuccess) return GMP_EDEVICE;
  gmp_server* s = new (std::nothrow) gmp_server();
  if (!s) return GMP_ENOMEM;
  s->device = dev;
  s->budget = budget_bytes;
  s->tuning = t;
  s->d_first_err = gmp_ctx_first_err_word(ctx);
  if (workspace_bytes == 0) workspace_bytes = budget_bytes / 2;
  workspace_bytes = (workspace_bytes + kUnit - 1) / kUnit * kUnit;
  s->arena_bytes = workspace_bytes;
  s->arena = new (std::nothrow) Arena(workspace_bytes);
  s->slots.resize(n_slots);
  bool ok = s->arena && hipMalloc(&s->d_arena, workspace_bytes) == hipSuccess &&
            hipHostMalloc(&s->h_done, kCounters * sizeof(uint32_t), hipHostMallocDefault) == hipSuccess &&
            hipHostGetDevicePointer((void**)&s->d_done, s->h_done, 0) == hipSuccess;
  if (ok) {
    for (uint32_t i = 0; i < kCounters; i++) s->h_done[i] = 0;
    for (uint32_t i = kCounters; i-- > 0;) s->free_ctr.push_back(i);
  }
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
  if ((req->flags & ~(GMP_MODE_MASK | GMP_FLAG_VERIFY_DE | GMP_FLAG_PLAIN_MRR)) != 0) return GMP_EINVAL;
  if (reinterpret_cast<uintptr_t>(req->d_stream) & 15) return GMP_EINVAL;
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
    if (o0 > o1 || o1 > req->len || (o0 & 15) || o1 - o0 < 32) return GMP_EFORMAT;
    const uint8_t* blk = hs + o0;
    gmp_block_info info;
    gmp_status st = gmp_block_info_parse(blk, o1 - o0, &info);
    if (st != GMP_OK) return st;
    if (info.block_bytes > o1 - o0) return GMP_EFORMAT;
    const uint64_t want = (b + 1 < nb) ? bs : total - (uint64_t)b * bs;
    if (info.raw_len != want) return GMP_ESIZE;
    if (mode == GMP_MODE_DE && !(info.mode == 1 && info.group % 64 == 0)) return GMP_EINVAL;
    gmpk::DevJob& j = rq.jobs[b];
    j.comp = req->d_stream + o0;
    j.comp_len = o1 - o0;
    j.out = req->d_out + (uint64_t)b * bs;
    j.out_len = info.raw_len;
    j.ws = nullptr;
    j.ws_len = gmpk::block_workspace_bytes(info.format, info.n_seq, info.n_lit, o1 - o0);
    j.rounds = nullptr;
    j.times = nullptr;
    j.status = req->d_status + b;
    j.stats = nullptr;
    j.done = nullptr;
    j.n_seq = info.n_seq;
    j.n_lit = info.n_lit;
    rq.ws_bytes += j.ws_len;
  }
  rq.bytes = req->len + req->out_len + rq.ws_bytes;
  // could never be admitted: more bytes than the budget, or more workspace than the arena
  if (rq.bytes > s->budget || rq.ws_bytes > s->arena_bytes) return GMP_EBUSY;
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
  if (s->h_done) (void)hipHostFree(s->h_done);
  delete s->arena;
  delete s;
}
