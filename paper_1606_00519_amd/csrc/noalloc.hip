// gmp_decompress_block_noalloc: gmp_decompress_block for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The block's token workspace is a fixed
// file-scope device array instead of the context's grown-on-demand buffer,
// and the job descriptor travels in the kernel arguments instead of a device
// job table, so the call allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gompresso.h"
#include "inflate.h"

namespace {

// The workspace of every call on a device.  Each device that runs the library
// holds its own copy until the process ends; calls on one device share it.
static __device__ __align__(256) uint8_t scratch[GMP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device, once resolved

}  // namespace

// Resolves the address of `scratch` on the current device (once per device).
// The array's name in host code is a host-side stand-in, not a device
// address: host code only ever passes this pointer to kernels.
extern "C" gmp_status gmp_noalloc_init(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMP_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return GMP_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[dev]) return GMP_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GMP_EDEVICE;
  g_scratch[dev] = static_cast<uint8_t*>(p);
  return GMP_OK;
}

extern "C" gmp_status gmp_decompress_block_noalloc(const uint8_t* d_block, size_t block_len, const void* h_block,
                                                   size_t h_len, uint8_t* d_out, size_t out_len, int32_t* d_status,
                                                   uint32_t flags, void* stream) {
  if (!d_block || !h_block || !d_status) return GMP_EINVAL;
  if ((flags & ~(GMP_MODE_MASK | GMP_FLAG_VERIFY_DE | GMP_FLAG_PLAIN_MRR)) != 0) return GMP_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_block) & 15) return GMP_EINVAL;
  gmp_block_info info;
  gmp_status st = gmp_block_info_parse(h_block, h_len, &info);
  if (st != GMP_OK) return st;
  if (info.block_bytes > block_len) return GMP_EFORMAT;
  if (out_len != info.raw_len) return GMP_ESIZE;
  if (!d_out && out_len) return GMP_EINVAL;
  const uint64_t ws = gmpk::block_workspace_bytes(info.format, info.n_seq, info.n_lit, block_len);
  if (ws > GMP_NOALLOC_SCRATCH_BYTES) return GMP_ERANGE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMP_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return GMP_EINVAL;
  uint8_t* ptr = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    ptr = g_scratch[dev];
  }
  if (!ptr) {
    if ((st = gmp_noalloc_init()) != GMP_OK) return st;
    std::lock_guard<std::mutex> g(g_mu);
    ptr = g_scratch[dev];
  }
  gmpk::DevJob j{};
  j.comp = d_block;
  j.comp_len = block_len;
  j.out = d_out;
  j.out_len = out_len;
  j.ws = ptr;
  j.ws_len = ws;
  j.status = d_status;
  j.n_seq = info.n_seq;
  j.n_lit = info.n_lit;
  // the kernel writes every workspace byte it reads, so nothing is cleared first
  if (gmpk_launch_single(&j, flags, nullptr, static_cast<hipStream_t>(stream)) != 0) return GMP_EDEVICE;
  return GMP_OK;
}
