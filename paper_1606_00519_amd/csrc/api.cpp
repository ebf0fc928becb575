// Host side of the C ABI declared in include/gompresso.h: header parsing,
// job tables, token workspace, launches.  Every decode step runs in the
// kernels of inflate.hip; this file only marshals arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/gompresso.h"
#include "compress.h"
#include "host_internal.h"
#include "inflate.h"

namespace {

constexpr uint32_t kMagicBlock = 0x42504D47u;   // 'GMPB'
constexpr uint32_t kMagicByte = 0x59504D47u;    // 'GMPY'
constexpr size_t kByteHdr = 32;
constexpr uint32_t kMagicStream = 0x46504D47u;  // 'GMPF'
constexpr size_t kHdrBytes = 192;
constexpr size_t kIdxBytes = 16;

uint32_t rd32(const uint8_t* p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
uint16_t rd16(const uint8_t* p) {
  uint16_t v;
  std::memcpy(&v, p, 2);
  return v;
}
uint64_t rd64(const uint8_t* p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}

#define HIP_OK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return GMP_EDEVICE;     \
  } while (0)

}  // namespace

struct gmp_ctx {
  int device = 0;
  int num_cu = 0;
  gmpk::DevJob* d_jobs = nullptr;  // job table of the single-call paths
  gmpk::DevJob* h_jobs = nullptr;  // pinned staging for it
  size_t jobs_cap = 0;
  uint8_t* d_ws = nullptr;  // token workspace of the single-call paths
  size_t ws_cap = 0;
  uint32_t* d_queue = nullptr;
  int32_t* d_first_err = nullptr;  // [0]: first device error since the last poll, [1]: poll staging
  int32_t* h_poll = nullptr;       // pinned
  hipEvent_t done = nullptr;       // recorded after the last single-call launch
  bool pending = false;
  gmpc::CompressJob* d_cjobs = nullptr;  // job table of the compressor
  gmpc::CompressJob* h_cjobs = nullptr;  // pinned staging for it
  size_t cjobs_cap = 0;
  uint8_t* d_cws = nullptr;              // the compressor's workspace
  size_t cws_cap = 0;
};

struct gmp_batch {
  int device = 0;
  uint32_t n = 0;
  gmpk::DevJob* d_jobs = nullptr;
  std::vector<gmpk::DevJob> h_jobs;  // host copy of the job table (spill areas are added to it on first use)
  uint8_t* d_spill = nullptr;        // spill lists of multi-launch resolution (allocated on first use)
  uint8_t* d_ws = nullptr;
  uint32_t* d_queue = nullptr;
  int32_t* d_first_err = nullptr;  // the context's first-error word
  int num_cu = 0;
  hipStream_t capture = nullptr;  // stream used for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" const char* gmp_strerror(gmp_status s) {
  switch (s) {
    case GMP_OK: return "ok";
    case GMP_EINVAL: return "invalid argument";
    case GMP_EFORMAT: return "malformed block or stream layout";
    case GMP_ECODE: return "invalid Huffman code or symbol";
    case GMP_EDIST: return "invalid back-reference distance";
    case GMP_ELEN: return "invalid match length";
    case GMP_ESIZE: return "output size differs from the decompressed size";
    case GMP_ESUB: return "sub-block bitstream does not match its index entry";
    case GMP_EDEVICE: return "HIP runtime error";
    case GMP_ENOMEM: return "out of memory";
    case GMP_EBUSY: return "no capacity";
    case GMP_ENOSYS: return "format feature not supported by this decoder";
    case GMP_ESTALL: return "device-side wait exceeded its bound (internal error)";
    case GMP_ERANGE: return "block too large for the fixed workspace of the allocation-free call";
    default: return "unknown status";
  }
}

extern "C" gmp_status gmp_block_info_parse(const void* h_block, size_t len, gmp_block_info* out) {
  if (!h_block || !out) return GMP_EINVAL;
  const uint8_t* b = static_cast<const uint8_t*>(h_block);
  if (len >= 4 && rd32(b) == kMagicByte) {
    // Gompresso/Byte: header, records, literals
    if (len < kByteHdr || b[4] != 1) return GMP_EFORMAT;
    gmp_block_info i{};
    i.format = 1;
    i.mode = b[5];
    i.group = b[6];
    i.raw_len = rd32(b + 8);
    i.window = rd32(b + 12);
    i.max_match = rd16(b + 16);
    i.n_seq = rd32(b + 20);
    i.n_lit = rd32(b + 24);
    if (i.mode > 1 || i.group < 1 || b[7] != 0 || i.window < 1 || i.window > 32768 || i.max_match < 3 ||
        i.max_match > 258 || rd16(b + 18) != 0 || rd32(b + 28) != 0 || i.n_seq > 0x3FFFFFFFu)
      return GMP_EFORMAT;
    const uint64_t payload = ((4ull * i.n_seq + 15) & ~15ull) + (((uint64_t)i.n_lit + 15) & ~15ull) + 16;
    if (payload > 0xFFFFFFFFull) return GMP_EFORMAT;
    i.payload_bytes = (uint32_t)payload;
    i.block_bytes = kByteHdr + payload;
    *out = i;
    return GMP_OK;
  }
  if (len < kHdrBytes) return GMP_EFORMAT;
  if (rd32(b) != kMagicBlock || b[4] != 1) return GMP_EFORMAT;
  gmp_block_info i{};
  i.mode = b[5];
  i.group = b[6];
  i.lmax = b[7];
  i.raw_len = rd32(b + 8);
  i.window = rd32(b + 12);
  i.max_match = rd16(b + 16);
  i.n_sub = rd32(b + 20);
  i.n_seq = rd32(b + 24);
  i.n_lit = rd32(b + 28);
  if (i.mode > 1 || i.group < 1 || i.lmax < 1 || i.lmax > 15 || i.window < 1 || i.window > 32768 ||
      i.max_match < 3 || i.max_match > 258 || rd16(b + 18) != 0)
    return GMP_EFORMAT;
  const uint64_t idx_end = kHdrBytes + kIdxBytes * (uint64_t)i.n_sub;
  if (idx_end + 4 > len) return GMP_EFORMAT;
  i.payload_bytes = rd32(b + idx_end);
  i.block_bytes = idx_end + 16 + i.payload_bytes;
  *out = i;
  return GMP_OK;
}

extern "C" uint64_t gmp_workspace_bytes(uint32_t n_seq, uint32_t n_lit, uint64_t comp_len) {
  return gmpk::workspace_bytes(n_seq, n_lit, comp_len);
}

extern "C" gmp_status gmp_stream_info(const void* h_stream, size_t len, uint32_t* n_blocks, uint32_t* block_size,
                                      uint64_t* raw_total) {
  if (!h_stream) return GMP_EINVAL;
  const uint8_t* s = static_cast<const uint8_t*>(h_stream);
  if (len < 32 || rd32(s) != kMagicStream || rd16(s + 4) != 1) return GMP_EFORMAT;
  const uint32_t bs = rd32(s + 8), nb = rd32(s + 12);
  const uint64_t total = rd64(s + 16);
  if (bs == 0 || nb != (total + bs - 1) / bs || 32 + 8 * ((uint64_t)nb + 1) > len) return GMP_EFORMAT;
  if (n_blocks) *n_blocks = nb;
  if (block_size) *block_size = bs;
  if (raw_total) *raw_total = total;
  return GMP_OK;
}

extern "C" gmp_status gmp_ctx_create(int device, gmp_ctx** out) {
  if (!out) return GMP_EINVAL;
  *out = nullptr;
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return GMP_EINVAL;
  HIP_OK(hipSetDevice(device));
  gmp_ctx* c = new (std::nothrow) gmp_ctx();
  if (!c) return GMP_ENOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess || hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->d_queue, 256) != hipSuccess || hipMalloc(&c->d_first_err, 256) != hipSuccess ||
      hipHostMalloc(&c->h_poll, 64, hipHostMallocDefault) != hipSuccess ||
      gmpk_clear_word(c->d_first_err, nullptr) != 0 || hipDeviceSynchronize() != hipSuccess) {
    gmp_ctx_destroy(c);
    return GMP_EDEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  // the allocation-free call's workspace address on this device, resolved now
  // (outside any graph capture the caller may start later)
  if (gmp_noalloc_init() != GMP_OK) {
    gmp_ctx_destroy(c);
    return GMP_EDEVICE;
  }
  *out = c;
  return GMP_OK;
}

extern "C" void gmp_ctx_destroy(gmp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->pending) (void)hipEventSynchronize(c->done);
  if (c->d_jobs) (void)hipFree(c->d_jobs);
  if (c->h_jobs) (void)hipHostFree(c->h_jobs);
  if (c->d_ws) (void)hipFree(c->d_ws);
  if (c->d_cjobs) (void)hipFree(c->d_cjobs);
  if (c->h_cjobs) (void)hipHostFree(c->h_cjobs);
  if (c->d_cws) (void)hipFree(c->d_cws);
  if (c->d_queue) (void)hipFree(c->d_queue);
  if (c->d_first_err) (void)hipFree(c->d_first_err);
  if (c->h_poll) (void)hipHostFree(c->h_poll);
  if (c->done) (void)hipEventDestroy(c->done);
  delete c;
}

int32_t* gmp_ctx_first_err_word(gmp_ctx* c) { return c ? c->d_first_err : nullptr; }
int gmp_ctx_device(gmp_ctx* c) { return c ? c->device : 0; }

extern "C" gmp_status gmp_poll(gmp_ctx* c, void* stream, int32_t* h_first_error) {
  if (!c || !h_first_error) return GMP_EINVAL;
  HIP_OK(hipSetDevice(c->device));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // the word is taken and cleared in one atomic exchange on the device, so an
  // error recorded by a launch still running on another stream is not lost
  if (gmpk_take_word(c->d_first_err, c->d_first_err + 1, s) != 0) return GMP_EDEVICE;
  HIP_OK(hipMemcpyAsync(c->h_poll, c->d_first_err + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *h_first_error = *c->h_poll;
  return GMP_OK;
}

namespace {

// Make the context's single-call buffers large enough; waits for the previous
// single call first, since it may still read them.
gmp_status ctx_reserve(gmp_ctx* c, size_t n_jobs, size_t ws_bytes) {
  if (c->pending) {
    HIP_OK(hipEventSynchronize(c->done));
    c->pending = false;
  }
  if (n_jobs > c->jobs_cap) {
    if (c->d_jobs) (void)hipFree(c->d_jobs);
    if (c->h_jobs) (void)hipHostFree(c->h_jobs);
    c->d_jobs = nullptr;
    c->h_jobs = nullptr;
    c->jobs_cap = 0;
    if (hipMalloc(&c->d_jobs, n_jobs * sizeof(gmpk::DevJob)) != hipSuccess) return GMP_ENOMEM;
    if (hipHostMalloc(&c->h_jobs, n_jobs * sizeof(gmpk::DevJob), hipHostMallocDefault) != hipSuccess) return GMP_ENOMEM;
    c->jobs_cap = n_jobs;
  }
  if (ws_bytes > c->ws_cap) {
    if (c->d_ws) (void)hipFree(c->d_ws);
    c->d_ws = nullptr;
    c->ws_cap = 0;
    if (hipMalloc(&c->d_ws, ws_bytes) != hipSuccess) return GMP_ENOMEM;
    c->ws_cap = ws_bytes;
  }
  return GMP_OK;
}

gmp_status ctx_launch(gmp_ctx* c, size_t n_jobs, uint32_t flags, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(c->d_jobs, c->h_jobs, n_jobs * sizeof(gmpk::DevJob), hipMemcpyHostToDevice, s));
  // the single-block and single-stream calls use the workgroup shape the
  // benchmark times: seven decoder wavefronts (two per SIMD)
  if (gmpk_launch(c->d_jobs, (uint32_t)n_jobs, flags, 7, 0, 0, c->d_queue, c->d_first_err, s) != 0)
    return GMP_EDEVICE;
  HIP_OK(hipEventRecord(c->done, s));
  c->pending = true;
  return GMP_OK;
}

static_assert(GMP_FLAG_STATS == GMPK_FLAG_STATS && GMP_FLAG_VERIFY_DE == GMPK_FLAG_VERIFY_DE &&
                  GMP_FLAG_PLAIN_MRR == GMPK_FLAG_PLAIN_MRR,
              "the kernels take the API's flags as they are");
bool valid_flags(uint32_t flags) {
  return (flags & ~(GMP_MODE_MASK | GMP_FLAG_STATS | GMP_FLAG_VERIFY_DE | GMP_FLAG_PLAIN_MRR)) == 0;
}

// Device blocks are read with 16-byte asynchronous copies into LDS.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" gmp_status gmp_decompress_block(gmp_ctx* c, const uint8_t* d_block, size_t block_len, const void* h_block,
                                           size_t h_len, uint8_t* d_out, size_t out_len, int32_t* d_status,
                                           uint32_t flags, void* stream) {
  if (!c || !d_block || !h_block || !d_status || !valid_flags(flags) || (flags & GMP_FLAG_STATS)) return GMP_EINVAL;
  if (!aligned16(d_block)) return GMP_EINVAL;
  gmp_block_info info;
  gmp_status st = gmp_block_info_parse(h_block, h_len, &info);
  if (st != GMP_OK) return st;
  if (info.block_bytes > block_len) return GMP_EFORMAT;
  if (out_len != info.raw_len) return GMP_ESIZE;
  if (!d_out && out_len) return GMP_EINVAL;
  HIP_OK(hipSetDevice(c->device));
  const size_t ws = gmpk::block_workspace_bytes(info.format, info.n_seq, info.n_lit, block_len);
  if ((st = ctx_reserve(c, 1, ws)) != GMP_OK) return st;
  gmpk::DevJob& j = c->h_jobs[0];
  j.comp = d_block;
  j.comp_len = block_len;
  j.out = d_out;
  j.out_len = out_len;
  j.ws = c->d_ws;
  j.ws_len = ws;
  j.rounds = nullptr;
  j.times = nullptr;
  j.status = d_status;
  j.stats = nullptr;
  j.done = nullptr;
  j.n_seq = info.n_seq;
  j.n_lit = info.n_lit;
  j.spill = nullptr;
  return ctx_launch(c, 1, flags, static_cast<hipStream_t>(stream));
}

extern "C" gmp_status gmp_decompress_stream(gmp_ctx* c, const uint8_t* d_stream, const void* h_stream, size_t len,
                                            uint8_t* d_out, size_t out_len, int32_t* d_status, uint32_t flags,
                                            void* stream) {
  if (!c || !d_stream || !h_stream || !d_status || !valid_flags(flags) || (flags & GMP_FLAG_STATS)) return GMP_EINVAL;
  if (!aligned16(d_stream)) return GMP_EINVAL;
  uint32_t nb = 0, bs = 0;
  uint64_t total = 0;
  gmp_status st = gmp_stream_info(h_stream, len, &nb, &bs, &total);
  if (st != GMP_OK) return st;
  if (out_len != total) return GMP_ESIZE;
  if (nb == 0) return GMP_OK;
  if (!d_out) return GMP_EINVAL;
  const uint8_t* hs = static_cast<const uint8_t*>(h_stream);
  std::vector<gmp_block_info> infos(nb);
  std::vector<uint64_t> offs(nb + 1);
  uint64_t ws_total = 0;
  for (uint32_t b = 0; b <= nb; b++) offs[b] = rd64(hs + 32 + 8 * (size_t)b);
  for (uint32_t b = 0; b < nb; b++) {
    if (offs[b] > offs[b + 1] || offs[b + 1] > len || (offs[b] & 15)) return GMP_EFORMAT;
    if ((st = gmp_block_info_parse(hs + offs[b], offs[b + 1] - offs[b], &infos[b])) != GMP_OK) return st;
    if (infos[b].block_bytes > offs[b + 1] - offs[b]) return GMP_EFORMAT;
    const uint64_t want = (b + 1 < nb) ? bs : total - (uint64_t)b * bs;
    if (infos[b].raw_len != want) return GMP_ESIZE;
    ws_total += gmpk::block_workspace_bytes(infos[b].format, infos[b].n_seq, infos[b].n_lit, offs[b + 1] - offs[b]);
  }
  HIP_OK(hipSetDevice(c->device));
  if ((st = ctx_reserve(c, nb, ws_total)) != GMP_OK) return st;
  uint64_t ws_off = 0;
  for (uint32_t b = 0; b < nb; b++) {
    gmpk::DevJob& j = c->h_jobs[b];
    j.comp = d_stream + offs[b];
    j.comp_len = offs[b + 1] - offs[b];
    j.out = d_out + (uint64_t)b * bs;
    j.out_len = infos[b].raw_len;
    j.ws = c->d_ws + ws_off;
    j.ws_len = gmpk::block_workspace_bytes(infos[b].format, infos[b].n_seq, infos[b].n_lit, j.comp_len);
    j.rounds = nullptr;
    j.times = nullptr;
    j.status = d_status + b;
    j.stats = nullptr;
    j.done = nullptr;
    j.n_seq = infos[b].n_seq;
    j.n_lit = infos[b].n_lit;
    j.spill = nullptr;
    ws_off += j.ws_len;
  }
  return ctx_launch(c, nb, flags, static_cast<hipStream_t>(stream));
}

extern "C" gmp_status gmp_batch_create(gmp_ctx* c, const gmp_job* h_jobs, uint32_t n_jobs, int32_t* d_status,
                                       gmp_batch** out) {
  if (!c || !out || (n_jobs && (!h_jobs || !d_status))) return GMP_EINVAL;
  *out = nullptr;
  HIP_OK(hipSetDevice(c->device));
  std::vector<gmpk::DevJob> dj(n_jobs);
  uint64_t ws_total = 0;
  for (uint32_t i = 0; i < n_jobs; i++) {
    const gmp_job& j = h_jobs[i];
    if (!j.d_comp || !aligned16(j.d_comp) || (!j.d_out && j.out_len) || j.format > 1) return GMP_EINVAL;
    ws_total += gmpk::block_workspace_bytes(j.format, j.n_seq, j.n_lit, j.comp_len);
  }
  gmp_batch* b = new (std::nothrow) gmp_batch();
  if (!b) return GMP_ENOMEM;
  b->device = c->device;
  b->n = n_jobs;
  b->num_cu = c->num_cu;
  b->d_first_err = c->d_first_err;
  if (hipMalloc(&b->d_queue, 256) != hipSuccess || (n_jobs && hipMalloc(&b->d_jobs, n_jobs * sizeof(gmpk::DevJob)) != hipSuccess) ||
      (ws_total && hipMalloc(&b->d_ws, ws_total) != hipSuccess)) {
    gmp_batch_destroy(b);
    return GMP_ENOMEM;
  }
  // largest blocks first: the queue (and the hardware's workgroup order) then
  // hands the long jobs out early and the short ones fill the tail
  std::vector<uint32_t> order(n_jobs);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t x, uint32_t y) { return h_jobs[x].out_len > h_jobs[y].out_len; });
  uint64_t ws_off = 0;
  for (uint32_t k = 0; k < n_jobs; k++) {
    const uint32_t i = order[k];
    const gmp_job& j = h_jobs[i];
    gmpk::DevJob& d = dj[k];
    d.comp = j.d_comp;
    d.comp_len = j.comp_len;
    d.out = j.d_out;
    d.out_len = j.out_len;
    d.ws = b->d_ws + ws_off;
    d.ws_len = gmpk::block_workspace_bytes(j.format, j.n_seq, j.n_lit, j.comp_len);
    d.rounds = j.d_rounds;
    d.times = j.d_times;
    d.status = d_status + i;
    d.stats = j.d_stats;
    d.done = nullptr;
    d.n_seq = j.n_seq;
    d.n_lit = j.n_lit;
    d.spill = nullptr;
    ws_off += d.ws_len;
  }
  if (n_jobs && hipMemcpy(b->d_jobs, dj.data(), n_jobs * sizeof(gmpk::DevJob), hipMemcpyHostToDevice) != hipSuccess) {
    gmp_batch_destroy(b);
    return GMP_EDEVICE;
  }
  b->h_jobs = std::move(dj);
  *out = b;
  return GMP_OK;
}

namespace {

struct Launch {
  uint32_t waves = 1, persistent = 0, workgroups = 0, rounds = 0;
};

gmp_status launch_params(const gmp_batch* b, const gmp_tuning* tuning, Launch* l) {
  Launch x;
  if (tuning) {
    x.waves = tuning->waves_per_block;
    x.persistent = tuning->persistent;
    x.workgroups = tuning->workgroups;
    x.rounds = tuning->rounds_per_launch;
  }
  if (x.waves != 1 && x.waves != 2 && x.waves != 4 && x.waves != 7) return GMP_EINVAL;
  if (x.persistent > 1 || x.rounds > 64) return GMP_EINVAL;
  if (x.persistent && x.workgroups == 0) x.workgroups = (uint32_t)b->num_cu;
  *l = x;
  return GMP_OK;
}

// The spill lists of multi-launch resolution: allocated once, on first use,
// and named in the device job table from then on (a kernel only writes them
// when its launch resolves a bounded number of rounds).
gmp_status batch_spill_areas(gmp_batch* b) {
  if (b->d_spill || b->n == 0) return GMP_OK;
  uint64_t total = 0;
  for (const gmpk::DevJob& j : b->h_jobs) total += (gmpk::spill_bytes(j.n_seq) + 255) / 256 * 256;
  if (hipMalloc(&b->d_spill, total) != hipSuccess) {
    b->d_spill = nullptr;
    return GMP_ENOMEM;
  }
  uint64_t off = 0;
  for (gmpk::DevJob& j : b->h_jobs) {
    j.spill = b->d_spill + off;
    off += (gmpk::spill_bytes(j.n_seq) + 255) / 256 * 256;
  }
  if (hipMemcpy(b->d_jobs, b->h_jobs.data(), b->n * sizeof(gmpk::DevJob), hipMemcpyHostToDevice) != hipSuccess)
    return GMP_EDEVICE;
  return GMP_OK;
}

// One run of the batch: the decoding launch and, with a bounded number of
// rounds per launch, the later launches that resolve the spill lists
// (ceil(64 / R) - 1 of R rounds each, then one that finishes every list).
gmp_status batch_launch(gmp_batch* b, uint32_t flags, const Launch& l, hipStream_t s) {
  const uint32_t rounds = (flags & GMP_MODE_MASK) == GMP_MODE_DE || (flags & GMP_MODE_MASK) == GMP_MODE_SC
                              ? 0u : l.rounds;
  const uint32_t kflags = flags | (rounds << GMPK_ROUNDS_SHIFT);
  if (gmpk_launch(b->d_jobs, b->n, kflags, l.waves, l.persistent, l.workgroups, b->d_queue, b->d_first_err, s) != 0)
    return GMP_EDEVICE;
  if (rounds == 0) return GMP_OK;
  const uint32_t later = (64 + rounds - 1) / rounds - 1;
  for (uint32_t k = 0; k <= later; k++)
    if (gmpk_launch_spills(b->d_jobs, b->n, k < later ? rounds : 0u, k & 1u, nullptr, s) != 0) return GMP_EDEVICE;
  return GMP_OK;
}

void graph_release(gmp_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" gmp_status gmp_batch_run(gmp_ctx* c, gmp_batch* b, uint32_t flags, const gmp_tuning* tuning, void* stream) {
  if (!c || !b || !valid_flags(flags)) return GMP_EINVAL;
  Launch l;
  gmp_status st = launch_params(b, tuning, &l);
  if (st != GMP_OK) return st;
  if (b->n == 0) return GMP_OK;
  HIP_OK(hipSetDevice(b->device));
  if (l.rounds && (st = batch_spill_areas(b)) != GMP_OK) return st;
  return batch_launch(b, flags, l, static_cast<hipStream_t>(stream));
}

extern "C" gmp_status gmp_batch_graph_create(gmp_ctx* c, gmp_batch* b, uint32_t flags, const gmp_tuning* tuning) {
  if (!c || !b || !valid_flags(flags)) return GMP_EINVAL;
  Launch l;
  gmp_status st = launch_params(b, tuning, &l);
  if (st != GMP_OK) return st;
  HIP_OK(hipSetDevice(b->device));
  if (l.rounds && (st = batch_spill_areas(b)) != GMP_OK) return st;
  graph_release(b);
  if (!b->capture) HIP_OK(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
  HIP_OK(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  st = b->n ? batch_launch(b, flags, l, b->capture) : GMP_OK;
  hipGraph_t g = nullptr;
  const hipError_t end = hipStreamEndCapture(b->capture, &g);
  if (st != GMP_OK || end != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return GMP_EDEVICE;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    graph_release(b);
    return GMP_EDEVICE;
  }
  return GMP_OK;
}

extern "C" gmp_status gmp_batch_graph_launch(gmp_ctx* c, gmp_batch* b, void* stream) {
  if (!c || !b || !b->exec) return GMP_EINVAL;
  HIP_OK(hipSetDevice(b->device));
  HIP_OK(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return GMP_OK;
}

extern "C" gmp_status gmp_autotune(gmp_ctx* c, gmp_batch* b, uint32_t flags, uint32_t reps, gmp_tuning* best,
                                   float* best_ms, void* stream) {
  if (!c || !b || !best || !valid_flags(flags) || (flags & GMP_FLAG_STATS) || reps < 1 || reps > 64)
    return GMP_EINVAL;
  HIP_OK(hipSetDevice(b->device));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<Launch> cands;
  for (uint32_t w : {1u, 2u, 4u, 7u}) {
    cands.push_back({w, 0u, 0u, 0u});
    cands.push_back({w, 1u, (uint32_t)b->num_cu, 0u});
    cands.push_back({w, 1u, 2u * (uint32_t)b->num_cu, 0u});
  }
  // launch shapes first (every round in one launch), then rounds per launch
  // on the winning shape
  const size_t n_shapes = cands.size();
  std::vector<hipEvent_t> ev(reps + 1, nullptr);
  gmp_status st = GMP_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = GMP_EDEVICE;
  float best_t = -1.0f;
  Launch win = cands[0];
  const bool mrr_possible = (flags & GMP_MODE_MASK) != GMP_MODE_DE && (flags & GMP_MODE_MASK) != GMP_MODE_SC;
  for (size_t k = 0; st == GMP_OK && k < cands.size(); k++) {
    if (k + 1 == n_shapes && mrr_possible && batch_spill_areas(b) == GMP_OK) {
      // after the last shape: rounds per launch on the winner so far
      for (uint32_t r : {1u, 4u, 16u}) cands.push_back({0u, 0u, 0u, r});
    }
    if (k >= n_shapes) {
      const uint32_t r = cands[k].rounds;
      cands[k] = win;
      cands[k].rounds = r;
    }
    if (b->n && (st = batch_launch(b, flags, cands[k], s)) != GMP_OK) break;  // untimed warm-up
    if (hipEventRecord(ev[0], s) != hipSuccess) st = GMP_EDEVICE;
    for (uint32_t r = 0; st == GMP_OK && r < reps; r++) {
      if (b->n) st = batch_launch(b, flags, cands[k], s);
      if (st == GMP_OK && hipEventRecord(ev[r + 1], s) != hipSuccess) st = GMP_EDEVICE;
    }
    if (st != GMP_OK || hipEventSynchronize(ev[reps]) != hipSuccess) {
      st = st == GMP_OK ? GMP_EDEVICE : st;
      break;
    }
    std::vector<float> t(reps);
    for (uint32_t r = 0; r < reps; r++)
      if (hipEventElapsedTime(&t[r], ev[r], ev[r + 1]) != hipSuccess) st = GMP_EDEVICE;
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    const float med = t[reps / 2];
    if (best_t < 0 || med < best_t) {
      best_t = med;
      win = cands[k];
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != GMP_OK) return st;
  best->waves_per_block = win.waves;
  best->persistent = win.persistent;
  best->workgroups = win.workgroups;
  best->rounds_per_launch = win.rounds;
  if (best_ms) *best_ms = best_t;
  return GMP_OK;
}

extern "C" void gmp_batch_destroy(gmp_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  graph_release(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_spill) (void)hipFree(b->d_spill);
  if (b->d_ws) (void)hipFree(b->d_ws);
  if (b->d_queue) (void)hipFree(b->d_queue);
  delete b;
}

// ---------------------------------------------------------------- compression
extern "C" uint64_t gmp_compress_bound(uint64_t in_len) { return gmpc::bound(in_len); }

extern "C" gmp_status gmp_compress_batch(gmp_ctx* c, const gmp_compress_job* h_jobs, uint32_t n_jobs,
                                         const gmp_compress_params* p, void* stream) {
  if (!c || !p || (n_jobs && !h_jobs)) return GMP_EINVAL;
  if (p->window < 1 || p->window > 32768 || p->max_match < 3 || p->max_match > 258 || p->de > 1) return GMP_EINVAL;
  uint64_t ws_total = 0;
  for (uint32_t i = 0; i < n_jobs; i++) {
    const gmp_compress_job& j = h_jobs[i];
    if ((!j.d_in && j.in_len) || !j.d_out || !aligned16(j.d_out) || !j.d_out_len || !j.d_status ||
        j.in_len > GMP_COMPRESS_MAX_BLOCK || j.out_cap < gmpc::bound(j.in_len))
      return GMP_EINVAL;
    ws_total += (gmpc::workspace_bytes(j.in_len) + 255) / 256 * 256;
  }
  if (n_jobs == 0) return GMP_OK;
  HIP_OK(hipSetDevice(c->device));
  if (c->pending) {
    HIP_OK(hipEventSynchronize(c->done));
    c->pending = false;
  }
  if (n_jobs > c->cjobs_cap) {
    if (c->d_cjobs) (void)hipFree(c->d_cjobs);
    if (c->h_cjobs) (void)hipHostFree(c->h_cjobs);
    c->d_cjobs = nullptr;
    c->h_cjobs = nullptr;
    c->cjobs_cap = 0;
    if (hipMalloc(&c->d_cjobs, n_jobs * sizeof(gmpc::CompressJob)) != hipSuccess ||
        hipHostMalloc(&c->h_cjobs, n_jobs * sizeof(gmpc::CompressJob), hipHostMallocDefault) != hipSuccess)
      return GMP_ENOMEM;
    c->cjobs_cap = n_jobs;
  }
  if (ws_total > c->cws_cap) {
    if (c->d_cws) (void)hipFree(c->d_cws);
    c->d_cws = nullptr;
    c->cws_cap = 0;
    if (hipMalloc(&c->d_cws, ws_total) != hipSuccess) return GMP_ENOMEM;
    c->cws_cap = ws_total;
  }
  uint64_t off = 0;
  for (uint32_t i = 0; i < n_jobs; i++) {
    const gmp_compress_job& j = h_jobs[i];
    gmpc::CompressJob& d = c->h_cjobs[i];
    d.in = j.d_in;
    d.in_len = j.in_len;
    d.out = j.d_out;
    d.out_cap = j.out_cap;
    d.out_len = j.d_out_len;
    d.status = j.d_status;
    d.ws = c->d_cws + off;
    off += (gmpc::workspace_bytes(j.in_len) + 255) / 256 * 256;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_OK(hipMemcpyAsync(c->d_cjobs, c->h_cjobs, n_jobs * sizeof(gmpc::CompressJob), hipMemcpyHostToDevice, s));
  gmpc::CompressParams prm{p->window, p->max_match, p->de, 0u};
  if (gmpc_launch(c->d_cjobs, n_jobs, prm, s) != 0) return GMP_EDEVICE;
  HIP_OK(hipEventRecord(c->done, s));
  c->pending = true;
  return GMP_OK;
}
