// Device job descriptor and launch entry of the Gompresso/Byte compressor.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmpc {

struct CompressJob {
  const uint8_t* in;   // the block's bytes
  uint64_t in_len;
  uint8_t* out;        // the compressed block (capacity bound(in_len), 16-byte aligned)
  uint64_t out_cap;
  uint64_t* out_len;   // the compressed block's size
  int32_t* status;
  uint8_t* ws;         // workspace_bytes(in_len)
};

struct CompressParams {
  uint32_t window;     // 1..32768
  uint32_t max_match;  // 3..258
  uint32_t de;         // 1: Dependency Elimination in groups of 64 sequences
  uint32_t reserved;
};

// Largest compressed size of a block of n bytes: a sequence covers at least
// 3 bytes, or exactly 255 literals, except the block's last.
__host__ __device__ inline uint64_t bound(uint64_t n) {
  const uint64_t seqs = n / 3 + n / 255 + 1;
  return 32 + ((4 * seqs + 15) & ~15ull) + ((n + 15) & ~15ull) + 16;
}
// per-position candidate and match (4 bytes each), padded to 256 positions
__host__ __device__ inline uint64_t workspace_bytes(uint64_t n) { return 8 * ((n + 255) & ~255ull); }

}  // namespace gmpc

extern "C" int gmpc_launch(const gmpc::CompressJob* d_jobs, uint32_t n_jobs, gmpc::CompressParams prm,
                           hipStream_t stream);
