// Device job descriptor and launch entry shared by the kernels and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GMPK_MODE_AUTO 0u
#define GMPK_MODE_MRR 1u
#define GMPK_MODE_DE 2u
#define GMPK_MODE_SC 3u
#define GMPK_MODE_MASK 3u
#define GMPK_FLAG_STATS 0x100u
#define GMPK_FLAG_VERIFY_DE 0x200u
#define GMPK_FLAG_PLAIN_MRR 0x400u
// Multi-round resolution over several launches: the first launch resolves at
// most R rounds per group of 64 sequences (R in bits 16-23 of the kernel's
// flags; 0 = every round), writing the back-references still pending to the
// block's spill list; later launches resolve the list (gmpk_launch_spills).
#define GMPK_ROUNDS_SHIFT 16u
#define GMPK_ROUNDS_MASK 0xFF0000u

namespace gmpk {

constexpr int kMaxDecWaves = 7;  // decoder wavefronts per workgroup: 1, 2, 4 or 7

// One block to decode (device copy of a host job, 96 bytes).
struct DevJob {
  const uint8_t* comp;  // the block: header, index, payload
  uint64_t comp_len;
  uint8_t* out;         // raw_len output bytes
  uint64_t out_len;
  uint8_t* ws;          // token workspace: n_seq 8-byte records, then n_lit bytes + slack
  uint64_t ws_len;
  uint8_t* rounds;      // optional per-group round counts
  uint64_t* times;      // optional phase timestamps (4 per block)
  int32_t* status;      // the block's status word
  uint32_t* stats;      // optional kStatsWords counters (see below)
  uint32_t* done;       // optional counter in host-visible memory: +1 when the block has finished
  uint32_t n_seq, n_lit;
  uint8_t* spill;       // optional spill area (spill_bytes(n_seq)): back-references left for later launches
};
static_assert(sizeof(DevJob) == 104, "DevJob layout");

// A block's spill area: two u32 counts (lists A and B), padding to 16 bytes,
// then lists A and B of up to n_seq entries each {u32 destination, u32
// distance << 9 | length}, in destination order.
__host__ __device__ inline uint64_t spill_bytes(uint32_t n_seq) { return 16 + 16ull * n_seq; }

// Per-block counters written with GMPK_FLAG_STATS when DevJob::stats is set:
//   [0] how the sub-blocks were decoded: 1 segmented, 2 one lane per sub-block
//   [1] decoder lanes whose start was repaired (segmented decoding)
//   [2] groups of 64 sequences, [3] groups resolved in window-sized pieces
//   [4] groups of a DE block resolved by rounds because they break the DE rule
//   [5] the wait that ran out first when the status is ESTALL (0: none)
//   [6] why the last segmented attempt not accepted failed (reason bits; 0: none)
//   [7] further segmented attempts (0-2)
//   [8] back-references the first launch left to later launches (rounds per launch)
//   [16 + r] back-reference bytes copied in round r + 1 (r < 64), all groups
constexpr uint32_t kStatsWords = 80, kStatsRoundBytes = 16;

// Token workspace of one block: the final token stream (n_seq 8-byte records,
// then n_lit literal bytes), then the private areas of the segmented decoder
// (each decoder lane gets room for twice its share of the block's tokens plus
// slack; a lane that overflows makes the block fall back to one lane per
// sub-block, which needs only the final area).
constexpr uint32_t kPrivSlackRec = 64, kPrivSlackLit = 256;
// per-lane extra of the segmented decoder: a log of its first kLogN symbol
// boundaries from its entry.  The tokens of a repair of the lane's start go
// after the lane's own tokens in its area.
constexpr uint32_t kLogN = 128;
constexpr uint32_t kLaneExtra = 4 * kLogN;
__host__ __device__ inline uint64_t final_bytes(uint32_t n_seq, uint32_t n_lit) { return ((8ull * n_seq + n_lit + 64 + 255) / 256) * 256; }
__host__ __device__ inline uint64_t lane_cap_rec(uint32_t n_seq, uint32_t lanes) {
  return ((2ull * n_seq + lanes - 1) / lanes + kPrivSlackRec + 1) / 2 * 2;  // even: areas stay 16-byte aligned
}
__host__ __device__ inline uint64_t lane_cap_lit(uint32_t n_lit, uint64_t comp_len, uint32_t lanes) {
  // a lane's share of the compressed bits, at two bits or more per literal
  // (literal-heavy stretches, such as a block's start, hold far more than
  // the block's average), never more than the block's literals
  const uint64_t by_bits = (4 * comp_len + lanes - 1) / lanes + kPrivSlackLit;
  const uint64_t c = by_bits < (uint64_t)n_lit + kPrivSlackLit ? by_bits : (uint64_t)n_lit + kPrivSlackLit;
  return (c + 15) / 16 * 16;
}
__host__ __device__ inline uint64_t workspace_bytes(uint32_t n_seq, uint32_t n_lit, uint64_t comp_len) {
  const uint32_t lanes = 64 * kMaxDecWaves;
  return final_bytes(n_seq, n_lit) +
         (uint64_t)lanes * (8 * lane_cap_rec(n_seq, lanes) + lane_cap_lit(n_lit, comp_len, lanes) + kLaneExtra) + 256;
}

// Workspace of a block of either format: a byte-level block is resolved
// straight from its records and literals and needs none.
__host__ __device__ inline uint64_t block_workspace_bytes(uint32_t format, uint32_t n_seq, uint32_t n_lit,
                                                          uint64_t comp_len) {
  return format == 1 ? 0 : workspace_bytes(n_seq, n_lit, comp_len);
}

}  // namespace gmpk

// d_first_err (may be null): set to the first non-zero block status of any launch
// that names it, until the host clears it.
extern "C" int gmpk_launch(const gmpk::DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t dec_waves,
                           uint32_t persistent, uint32_t workgroups, uint32_t* d_queue, int32_t* d_first_err,
                           hipStream_t stream);
// Small kernels of the host API (no memset nodes, so graph captures stay plain):
// *word = 0; and *out = *word, *word = 0 in one atomic exchange.
extern "C" int gmpk_clear_word(int32_t* word, hipStream_t stream);
extern "C" int gmpk_take_word(int32_t* word, int32_t* out, hipStream_t stream);
// Later launches of multi-launch resolution: every job's spill list `parity`
// (0: A, 1: B) is resolved, at most `rounds` rounds per group of 64 entries (0 =
// all), what is still pending going to the other list.  d_remaining (may be
// null) receives the number of entries left.
extern "C" int gmpk_launch_spills(const gmpk::DevJob* d_jobs, uint32_t n_jobs, uint32_t rounds, uint32_t parity,
                                  uint32_t* d_remaining, hipStream_t stream);
// One block, seven decoder wavefronts, the job descriptor passed by value in
// the kernel arguments (no device job table).
extern "C" int gmpk_launch_single(const gmpk::DevJob* h_job, uint32_t flags, int32_t* d_first_err,
                                  hipStream_t stream);
