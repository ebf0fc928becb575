// Gompresso/Bit intra-block parallel Inflate for gfx950 (MI355X).
//
// One workgroup decodes one data block (arXiv 1606.00519, section
// "Parallel Decompression").  The workgroup has kDec decoder wavefronts and
// one fetcher wavefront.  The fetcher performs every HBM read of the hot
// loops as asynchronous HBM->LDS copies (global_load_lds_dwordx4) and is the
// only wavefront that waits on the vector-memory counter; the decoder
// wavefronts work out of LDS and only issue stores, which never stall them.
// The two sides hand data over through progress counters in LDS.
//
//   A0  header and sub-block index checks; sub-block offsets by block-wide
//       prefix sums over the sizes stored in the index (section "Huffman
//       Decoding": the decoder locates sub-blocks from their sizes);
//   A1  both canonical Huffman codes expanded into 2^lmax-entry lookup tables
//       in LDS, one lookup per symbol;
//   A2  every decoder lane decodes one sub-block whose bitstream the fetcher
//       streams into a per-lane LDS ring; sequence records and literal bytes
//       go to the block's token workspace (the paper's token stream);
//   A3  decoder wavefront 0 walks the sequences in groups of 64 (one per
//       lane) and computes literal source and output offsets with two DPP
//       prefix sums (section "LZ77 Decompression");
//   A4  literal strings are copied into an on-chip output window (LDS ring);
//   A5  back-references of ordinary streams: Multi-Round Resolution — each
//       round, the high-water mark is the destination of the lowest pending
//       lane (everything below it is written without gaps), found with a
//       ballot; every pending lane whose needed source bytes lie below it
//       copies (section "Multi-Round Resolution (MRR) of Nested
//       back-references");
//   A6  back-references of Dependency-Elimination streams: one pass, no
//       checks (section "Dependency Elimination (DE)");
//   the window is flushed to HBM in coalesced 16-byte-per-lane stores, and
//   during A3-A6 the fetcher streams the token workspace into LDS.
//
// All arithmetic is integer.  No device memory outside the job's output,
// workspace, rounds, times and status words is written.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inflate.h"

namespace gmpk {

// Device-memory pointers are handled as address-space-1 (global) pointers, so
// that every access compiles to a global_* instruction: flat accesses would be
// ordered against LDS traffic and force waits on both counters.
#define GMEM __attribute__((address_space(1)))
// four words at a 16-byte aligned address (one 16-byte access)
struct __attribute__((aligned(16))) Aligned16 {
  uint32_t x, y, z, w;
};
struct __attribute__((packed)) Packed16 {
  uint32_t x, y, z, w;
};
struct __attribute__((packed)) Packed4 {
  uint32_t v;
};
template <typename T>
__device__ __forceinline__ GMEM T* gmem(T* p) {
  return (GMEM T*)p;
}
template <typename T>
__device__ __forceinline__ const GMEM T* gmem(const T* p) {
  return (const GMEM T*)p;
}
__device__ __forceinline__ uint4 gload16(const GMEM uint8_t* p) {
  const GMEM Packed16* t = (const GMEM Packed16*)p;
  return make_uint4(t->x, t->y, t->z, t->w);
}
__device__ __forceinline__ void gstore16(GMEM uint8_t* p, uint4 v) {
  GMEM Packed16* t = (GMEM Packed16*)p;
  t->x = v.x;
  t->y = v.y;
  t->z = v.z;
  t->w = v.w;
}
__device__ __forceinline__ uint32_t gload32(const GMEM uint8_t* p) { return ((const GMEM Packed4*)p)->v; }

constexpr uint32_t kMagicBlock = 0x42504D47u;  // 'GMPB' (Gompresso/Bit)
constexpr uint32_t kMagicByte = 0x59504D47u;   // 'GMPY' (Gompresso/Byte)
constexpr uint32_t kByteHdr = 32;              // a byte-level block's header; its records follow
constexpr uint32_t kHdrBytes = 192;
constexpr uint32_t kIdxBytes = 16;
constexpr uint32_t kNumLL = 286;
constexpr uint32_t kNumD = 30;
constexpr uint32_t kLutBits = 13;  // longest code the on-chip tables hold
constexpr uint32_t kLutSize = 1u << kLutBits;
constexpr uint32_t kRing = 65536;  // on-chip output window
constexpr uint32_t kRingMask = kRing - 1;
constexpr uint32_t kSpanCap = kRing - 32768;  // most output one resolution pass holds (window <= 32768)
constexpr uint32_t kStageBytes = 32768;       // staging area: bit rings, then token rings
constexpr uint32_t kRecRing = 2048;           // staged sequence records (8 bytes each)
constexpr uint32_t kLitRing = 8192;           // staged literal bytes
constexpr uint32_t kLitStagedMax = 4096;      // larger literal groups read HBM directly
constexpr uint32_t kCoopLits = 64;            // longer literal runs are copied by the whole wavefront
constexpr uint32_t kTightPolls = 64;          // polls of a hand-over counter before pausing between polls
constexpr uint32_t kGRing = kRecRing / 64;    // staged group offsets
constexpr uint32_t kSubMax = 512;             // most sub-blocks of a block decoded in segments
constexpr uint32_t kOverlapBits = 768;        // bits a segment decoder reads ahead of its start to synchronise
constexpr uint32_t kOverlapRetry = 8192;      // ... on later attempts, when lanes stayed out of step
constexpr uint32_t kSegAttempts = 3;          // segmented attempts before one lane per sub-block
constexpr uint32_t kSnapBits = 2048;          // segment boundaries this close to a sub-block's end move past it
constexpr bool kSegmentedDecode = true;
constexpr uint32_t kDone = 0xFFFFFFFFu;       // progress value of a finished consumer

// status codes (same values as the public header)
constexpr int kOK = 0, kEINVAL = -1, kEFORMAT = -2, kECODE = -3, kEDIST = -4, kELEN = -5, kESIZE = -6,
              kESUB = -7, kENOSYS = -11, kESTALL = -12;

// Lookup-table entry: bits 0-4 bits consumed by the lookup (0 = invalid
// entry), 5-8 further extra bits to read, 9-10 kind, 16-31 value (literal
// byte, match length or distance; extra bits already folded in when they fit
// inside the lookup width).
constexpr uint32_t kKindLit = 0, kKindLen = 1, kKindEnd = 2, kKindDist = 2;

// RFC 1951 section 3.2.5 length and distance codes, from their closed forms:
// length code i (symbol 257+i): i < 8 -> 3+i, 0 extra bits; 8 <= i < 28 ->
// ((4 + i%4) << e) + 3 with e = i/4 - 1; i = 28 -> 258.
__device__ __forceinline__ void length_code(uint32_t i, uint32_t& base, uint32_t& extra) {
  if (i < 8) {
    base = 3 + i;
    extra = 0;
  } else if (i < 28) {
    extra = i / 4 - 1;
    base = ((4 + (i & 3)) << extra) + 3;
  } else {
    base = 258;
    extra = 0;
  }
}
// distance code i: i < 4 -> 1+i, 0 extra bits; else ((2 + i%2) << e) + 1 with e = i/2 - 1.
__device__ __forceinline__ void dist_code(uint32_t i, uint32_t& base, uint32_t& extra) {
  if (i < 4) {
    base = 1 + i;
    extra = 0;
  } else {
    extra = i / 2 - 1;
    base = ((2 + (i & 1)) << extra) + 1;
  }
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes: row shifts within 16-lane rows,
// then row broadcasts of lanes 15 and 31 (wave64 DPP).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}
__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
// Inclusive prefix maximum over the 64 lanes (same DPP pattern).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
  return x;
}

// LDS progress counters: release after the data they announce, acquire before
// reading that data.
__device__ __forceinline__ uint32_t lds_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int kMaxLanes = 64 * kMaxDecWaves;
// Workgroup shape.  kDec decoder wavefronts (they resolve in phase B) and a
// fetcher, plus a flusher of its own for kDec in {1, 2, 4}.  At kDec = 7 the
// workgroup has eight wavefronts, two per SIMD: phase A decodes on seven; in
// phase B six resolve and the seventh decoder flushes.  With MRR's rounds
// short (sources moved through the group's own copies), a resolver's
// preparation of its next group (scans, literal copies, rounds) takes longer
// than the resolution chain takes for the groups in between, so more
// resolvers beat keeping the chain's copies alone on their SIMD.
template <int kDec>
constexpr uint32_t block_waves() {
  return kDec == 7 ? 8u : (uint32_t)kDec + 2u;
}
template <int kDec>
constexpr uint32_t block_threads() {
  return 64 * block_waves<kDec>();
}
template <int kDec>
constexpr uint32_t flusher_wave() {
  return kDec == 7 ? 6u : (uint32_t)kDec + 1u;
}
template <int kDec>
constexpr int resolver_waves() {
  return kDec == 7 ? 6 : kDec;  // wavefronts 0 .. resolver_waves() - 1
}
// 16-byte rows of each decoder lane's bit ring: the largest power of two
// the staging area holds for all lanes
constexpr uint32_t pow2_floor(uint32_t x) { return x < 2 ? 1u : 2u * pow2_floor(x / 2); }
template <int kDec>
constexpr uint32_t ring_rows() {
  return pow2_floor(kStageBytes / 16 / (64 * kDec));
}

struct Misc {
  uint8_t lens[kNumLL + kNumD];
  uint32_t count[16], first[16];
  uint32_t wave_sum[4][kMaxDecWaves + 2];
  uint32_t sub_woff[kMaxLanes];  // first payload word of each lane's sub-block
  uint32_t sub_nw[kMaxLanes];    // its words, a multiple of 4 (0: nothing to fetch)
  uint32_t rd[kMaxLanes];        // decoder -> fetcher: words taken from the lane's bit ring
  uint32_t avail[kMaxLanes];     // fetcher -> decoder: words present in the lane's bit ring
  uint32_t rec_avail, lit_avail;  // fetcher -> resolvers: records / literal bytes staged
  uint32_t g_out[kGRing], g_lit[kGRing];   // fetcher -> resolvers: offsets of staged groups
  uint32_t next_group[kMaxDecWaves];       // resolver -> fetcher: first group it still reads
  uint32_t coop[kMaxDecWaves][64];         // resolver w: run starts of a cooperative copy pass
  uint32_t done_upto;                      // resolvers: output below this is final
  uint32_t flushed;                        // flusher: output below this is in HBM
  uint32_t next_job;
  uint32_t abort;  // set when a wait exceeded its bound: every wavefront stops waiting
  int err;
  // statistics (GMPK_FLAG_STATS with DevJob::stats): bytes copied per round,
  // groups resolved in pieces, DE groups resolved by rounds
  uint32_t rbytes[64];
  uint32_t n_split, n_de_rounds, a2_path, n_repaired, stall_site, seg_reject, seg_retry;
  uint32_t spill_n;  // back-references written to the block's spill list (groups append in order)
  uint32_t seg_restarts;  // lanes a failed segmented attempt newly gave an exact restart
};

// State of the segmented Huffman decoder (A2 when the block qualifies).
constexpr uint32_t kSegFail = 1, kSegPass = 2, kSegMaybe = 4, kSegMid = 8, kSegRep = 16, kSegOver = 32;
// Why a block's segmented decoding was not accepted (bits of Seg::bad, the
// block's GMPK_FLAG_STATS counter): an index entry out of line, a lane met an
// invalid code, a lane's private area overflowed, a lane's entry is not the
// previous lane's exit and the repair failed, the last lane did not end at
// the payload's end, a literal run stayed open at a sub-block start, the
// tokens counted per sub-block differ from the index.
constexpr uint32_t kRejIndex = 1, kRejCode = 2, kRejOver = 4, kRejMeet = 8, kRejLast = 16, kRejRun = 32,
                   kRejCount = 64, kRejRepair = 128;
struct Seg {
  union {
    struct {
      uint32_t sub_start[kSubMax + 1];  // first payload bit of each sub-block; [n_sub] = payload bits
      uint32_t sub_end[kSubMax];        // bit after each sub-block's end symbol
      uint32_t cnt_seq[kSubMax], cnt_lit[kSubMax], cnt_raw[kSubMax];  // tokens decoded per sub-block, all lanes
    };
    // resolution over several launches (A3-A6 only): one bit per output
    // window position, set while the byte there waits for a later launch
    uint32_t pend[kRing / 32];
  };
  uint32_t entry[kMaxLanes], exit_at[kMaxLanes];  // first / past-last symbol boundary each lane decoded
  uint32_t nrec[kMaxLanes], nlit[kMaxLanes];      // records / literal bytes each lane wrote
  uint32_t tail[kMaxLanes];                       // literals after a lane's last record, run still open
  uint32_t flags[kMaxLanes];                      // kSeg* bits
  uint32_t entry_sub[kMaxLanes];                  // sub-block of the lane's entry
  uint32_t nlog[kMaxLanes];                       // symbol boundaries the lane logged
  uint32_t maybe_idx[kMaxLanes];                  // its record closing its first sub-block (kSegMaybe)
  uint32_t rep_rec[kMaxLanes], rep_lit[kMaxLanes], rep_run[kMaxLanes];     // repair of the lane's start
  uint32_t skip_rec[kMaxLanes], skip_lit[kMaxLanes], skip_run[kMaxLanes];  // own tokens it replaces
  uint32_t eff_tail[kMaxLanes];                   // literals after the lane's last record, after repair
  uint32_t bad;
};

// Workgroup-shared memory.
__shared__ __attribute__((aligned(16))) uint32_t s_big[kRing / 4];     // lookup tables, then the output window
__shared__ __attribute__((aligned(16))) uint4 s_stage[kStageBytes / 16];  // bit rings, then staged tokens
__shared__ Misc s_misc;
__shared__ Seg s_seg;
// exact restarts of the segmented decoder's later attempts (decode_segmented)
__shared__ uint32_t s_xstart[kMaxLanes];

__device__ __forceinline__ uint8_t* ring_ptr() { return reinterpret_cast<uint8_t*>(s_big); }
__device__ __forceinline__ uint2* rec_ring() { return reinterpret_cast<uint2*>(s_stage); }
__device__ __forceinline__ uint8_t* lit_ring() { return reinterpret_cast<uint8_t*>(s_stage) + 8 * kRecRing; }

__device__ __forceinline__ void set_err(int e) { atomicCAS(&s_misc.err, 0, e); }

// Every wait on another wavefront is bounded: a wait that lasts longer than
// about a second (the constant 100 MHz clock), or that sees another
// wavefront give up, ends, and the block reports kESTALL.  A correct
// hand-over never comes near the bound; the bound only guarantees that a
// fault in the hand-over logic ends the kernel instead of hanging it.
constexpr uint64_t kSpinTicks = 100000000ull;
// Which wait ran out first (the block's stall-site counter, GMPK_FLAG_STATS):
// the Huffman-stage fetcher, a decoder lane's bit ring (segmented or one lane
// per sub-block), the token fetcher, the output window, staged records,
// staged literals, the resolution hand-over, the flusher.
constexpr uint32_t kSiteBits = 1, kSiteRingSeg = 2, kSiteRingSub = 3, kSiteTokens = 4, kSiteWindow = 5,
                   kSiteRecs = 6, kSiteLits = 7, kSiteDone = 8, kSiteFlush = 9;
struct Spin {
  uint64_t t0 = 0;
  uint32_t site;
  __device__ explicit Spin(uint32_t s) : site(s) {}
  // one pause of a wait loop; false when the wait must end
  __device__ __forceinline__ bool pause() {
    if (__hip_atomic_load(&s_misc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
    const uint64_t now = (uint64_t)wall_clock64();
    if (t0 == 0) {
      t0 = now;
    } else if (now - t0 > kSpinTicks) {
      atomicCAS(&s_misc.stall_site, 0u, site);
      __hip_atomic_store(&s_misc.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
  }
};

// Asynchronous copy of 1 KiB from HBM into LDS: lane l moves the 16 bytes at
// its src to lds + 16*l (lds is the same for all lanes).
__device__ __forceinline__ void dma16(const GMEM uint8_t* src, void* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
// Wait until every memory operation this wavefront issued has completed.
__device__ __forceinline__ void wait_all_memory() { __builtin_amdgcn_s_waitcnt(0); }

// ---------------------------------------------------------------- A1 tables
// Canonical code of one alphabet -> lookup table.  Codes of each length are
// consecutive in symbol order (RFC 1951 section 3.2.2); a symbol's rank within
// its length comes from ballots over 64-symbol chunks, and its lane writes
// every table entry whose low bits are its (bit-reversed) code.
template <int kThreads>
__device__ void build_table(const uint8_t* lens, uint32_t nsym, uint32_t lmax, uint32_t* lut, bool is_dist) {
  Misc& sh = s_misc;
  const uint32_t t = threadIdx.x;
  const uint32_t lane = t & 63, wave = t >> 6;
  constexpr uint32_t kWaves = kThreads / 64;
  if (t < 16) sh.count[t] = 0;
  __syncthreads();
  for (uint32_t s = t; s < nsym; s += kThreads) {
    uint32_t l = lens[s];
    if (l > lmax) set_err(kECODE);
    if (l) atomicAdd(&sh.count[l], 1u);
  }
  __syncthreads();
  if (t == 0) {
    // Kraft: the codes must exactly fill the code space (or be empty for
    // the distance code of a block without back-references).
    int64_t left = 1;
    uint32_t used = 0;
    for (uint32_t l = 1; l <= 15; l++) {
      left = 2 * left - (int64_t)sh.count[l];
      used += sh.count[l];
      if (left < 0) set_err(kECODE);
    }
    if (used && left != 0) set_err(kECODE);
    if (!used && !is_dist) set_err(kECODE);
    uint32_t code = 0;
    sh.count[0] = 0;
    for (uint32_t l = 1; l <= 15; l++) {
      code = (code + sh.count[l - 1]) << 1;
      sh.first[l] = code;
    }
    sh.count[0] = used;
  }
  __syncthreads();
  if (sh.err) return;
  const uint32_t size = 1u << lmax;
  if (sh.count[0] == 0) {
    for (uint32_t e = t; e < size; e += kThreads) lut[e] = 0;  // no codes: every entry invalid
    return;
  }
  uint32_t first[16];
#pragma unroll
  for (int l = 0; l < 16; l++) first[l] = sh.first[l];
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t run[16];
#pragma unroll
  for (int l = 0; l < 16; l++) run[l] = 0;
  for (uint32_t c = 0, chunk = 0; c < nsym; c += 64, chunk++) {
    const uint32_t s = c + lane;
    const uint32_t l = s < nsym ? lens[s] : 0;
    uint32_t code = 0;
#pragma unroll
    for (uint32_t q = 1; q <= 15; q++) {
      const uint64_t m = __ballot(l == q);
      if (l == q) code = first[q] + run[q] + (uint32_t)__popcll(m & below);
      run[q] += (uint32_t)__popcll(m);
    }
    if (chunk % kWaves != wave || l == 0) continue;
    uint32_t base, extra, kind;
    if (is_dist) {
      kind = kKindDist;
      dist_code(s < kNumD ? s : 0, base, extra);
    } else if (s < 256) {
      kind = kKindLit;
      base = s;
      extra = 0;
    } else if (s == 256) {
      kind = kKindEnd;
      base = 0;
      extra = 0;
    } else {
      kind = kKindLen;
      length_code(s - 257, base, extra);
    }
    const uint32_t rev = __builtin_bitreverse32(code) >> (32 - l);  // first stream bit = code MSB
    const bool fold = l + extra <= lmax;                             // extra bits inside the lookup
    const uint32_t n = fold ? l + extra : l, x = fold ? 0 : extra;
    const uint32_t emask = fold ? (1u << extra) - 1u : 0u;
    for (uint32_t j = 0; j < (size >> l); j++)
      lut[rev | (j << l)] = n | (x << 5) | (kind << 9) | ((base + (j & emask)) << 16);
  }
}

// ---------------------------------------------------------------- block scan
template <int kThreads>
__device__ __forceinline__ void block_excl_scan4(uint32_t v[4], uint32_t tot[4]) {
  Misc& sh = s_misc;
  constexpr int kW = kThreads / 64;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t inc[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    inc[i] = wave_incl_scan(v[i]);
    if (lane == 63) sh.wave_sum[i][w] = inc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; i++) {
    uint32_t pre = 0, all = 0;
    for (int k = 0; k < kW; k++) {
      uint32_t s = sh.wave_sum[i][k];
      if (k < (int)w) pre += s;
      all += s;
    }
    v[i] = pre + inc[i] - v[i];
    tot[i] = all;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- A2 fetch
// Fetcher lane f feeds decoder lanes f, f+64, ...: it copies each lane's
// sub-block into that lane's ring of kRows 16-byte rows (row slot r of all
// lanes forms one contiguous 64-lane strip, so one copy instruction serves a
// whole wavefront), never running more than the ring ahead of what the lane
// has taken, and publishes how many words are present.
template <int kDec>
__device__ void fetch_bitstreams(const GMEM uint8_t* payload) {
  constexpr uint32_t kLanes = 64 * kDec, kRows = ring_rows<kDec>();
  const uint32_t f = lane_id();
  uint32_t total[kDec], woff[kDec], fetched[kDec];
#pragma unroll
  for (int v = 0; v < kDec; v++) {
    total[v] = s_misc.sub_nw[f + 64 * v];
    woff[v] = s_misc.sub_woff[f + 64 * v];
    fetched[v] = 0;
  }
  Spin sp(kSiteBits);
  for (;;) {
    bool left = false, issued = false;
    uint32_t limit[kDec];
#pragma unroll
    for (int v = 0; v < kDec; v++) {
      const uint32_t rd = lds_acquire(&s_misc.rd[f + 64 * v]);
      if (rd == kDone) fetched[v] = total[v];  // the lane stopped: nothing more to deliver
      limit[v] = fetched[v] < total[v] ? min(total[v], (rd & ~3u) + 4 * kRows) : fetched[v];
      left |= fetched[v] < total[v];
    }
    if (!__ballot(left)) break;
#pragma unroll
    for (int v = 0; v < kDec; v++) {
      const uint32_t row0 = fetched[v] / 4, row1 = limit[v] / 4;
      for (uint32_t r = 0; r < kRows; r++) {
        const uint32_t a = row0 + ((r + kRows - row0 % kRows) % kRows);  // the lane's row held in slot r
        const bool go = a < row1;
        if (__ballot(go)) {
          if (go) dma16(payload + 16ull * (woff[v] / 4 + a), &s_stage[r * kLanes + 64 * v]);
          issued = true;
        }
      }
    }
    if (issued) {
      wait_all_memory();
#pragma unroll
      for (int v = 0; v < kDec; v++) {
        fetched[v] = limit[v];
        lds_release(&s_misc.avail[f + 64 * v], fetched[v]);
      }
      sp = Spin(kSiteBits);
    } else if (!sp.pause()) {
      return;
    }
  }
}

// ---------------------------------------------------------------- A2 decode
struct SubBlock {
  uint32_t n_words, bit_len;
  uint32_t n_seq, n_lit, raw_len, raw_off;
  GMEM uint64_t* seq_out;  // records: literal length | (match length | distance << 16) << 32
  GMEM uint8_t* lit_out;
};

// Decode one sub-block's bitstream (lane L of the decoder wavefronts): literal
// bytes to lit_out, one record per sequence to seq_out.
//
// One symbol per step, from either table: a step in the literal/length state
// looks up lut_ll, a step in the distance state lut_d (the two tables are
// adjacent in LDS, so the state is just an index offset).  The stream is seen
// through a window of words w0..w2 at bit offset s (0..31), so every step has
// 64 fresh bits; the window slides by selects, w3 being the word after it and
// nx the word after that, read from the lane's LDS ring a step before it is
// needed.  The step is branch-free apart from the two stores and a stall path
// that is taken only when the fetcher is behind; errors end the lane's loop.
template <int kDec>
__device__ int decode_subblock(const SubBlock& sb, uint32_t L, uint32_t lmax, uint32_t window, uint32_t max_match) {
  constexpr uint32_t kLanes = 64 * kDec, kRows = ring_rows<kDec>();
  static_assert((kRows & (kRows - 1)) == 0, "ring rows must be a power of two");
  if (sb.bit_len == 0) return kESUB;
  const uint32_t lmask = (1u << lmax) - 1u;
  const uint32_t nw = sb.n_words;
  const uint32_t* ring_base = reinterpret_cast<const uint32_t*>(s_stage) + 4 * L;
  uint32_t avail = 0;
  // word k of the lane's stream (zero past its end); waits for the fetcher when needed
  auto ring_word = [&](uint32_t k) -> uint32_t {
    if (k < nw && k >= avail) {
      Spin sp(kSiteRingSub);
      for (;;) {
        avail = lds_acquire(&s_misc.avail[L]);
        if (k < avail) break;
        if (!sp.pause()) {
          avail = kDone;  // give up waiting: the lane decodes to an error and stops
          break;
        }
      }
    }
    const uint32_t w = ring_base[((k >> 2) & (kRows - 1)) * (4 * kLanes) + (k & 3)];
    return k < nw ? w : 0u;
  };
  uint32_t w0 = ring_word(0), w1 = ring_word(1), w2 = ring_word(2), w3 = ring_word(3), nx = ring_word(4);
  uint32_t rd = 4;  // index of the word in nx
  uint32_t s = 0, pos = 0, state = 0;
  uint32_t plen = 0, produced = 0, sc = 0, lc = 0, run = 0;
  int ecode = kOK;
  for (;;) {
    const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, s), hi = __builtin_amdgcn_alignbit(w2, w1, s);
    const uint32_t e = s_big[(state << kLutBits) | (lo & lmask)];
    const uint32_t n = e & 31u, x = (e >> 5) & 15u, kind = (e >> 9) & 3u;
    const uint32_t val = (e >> 16) + __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi, lo, n), 0, x);
    const uint32_t t = n + x;
    pos += t;
    s += t;
    // slide the window by a word when s crossed 32 (t <= 26 and s < 32: at most one word)
    const bool sh = s >= 32;
    s &= 31;
    w0 = sh ? w1 : w0;
    w1 = sh ? w2 : w1;
    w2 = sh ? w3 : w2;
    w3 = sh ? nx : w3;
    rd += sh ? 1u : 0u;
    nx = ring_word(rd);
    s_misc.rd[L] = rd - 4;  // words below rd-4 are out of the window: their ring slots are free
    // what the symbol was
    const bool is_dist = state != 0;
    const bool is_lit = !is_dist && kind == kKindLit;
    const bool is_len = !is_dist && kind == kKindLen;
    const bool is_end = !is_dist && kind == kKindEnd;
    const uint32_t lim = min(window, sb.raw_off + produced);
    int code = n == 0 ? kECODE : kOK;
    code = (code == kOK && is_dist && plen > max_match) ? kELEN : code;
    code = (code == kOK && is_dist && val > lim) ? kEDIST : code;
    code = (code == kOK && ((is_dist && sc >= sb.n_seq) || (is_lit && lc >= sb.n_lit) || pos > sb.bit_len)) ? kESUB
                                                                                                         : code;
    if (is_dist && code == kOK) sb.seq_out[sc] = (uint64_t)run | ((uint64_t)(plen | (val << 16)) << 32);
    if (is_lit && code == kOK) sb.lit_out[lc] = (uint8_t)val;
    sc += is_dist ? 1u : 0u;
    lc += is_lit ? 1u : 0u;
    produced += is_dist ? plen : (is_lit ? 1u : 0u);
    run = is_dist ? 0u : run + (is_lit ? 1u : 0u);
    plen = is_len ? val : plen;
    state = is_len ? 1u : 0u;
    if (code != kOK) {
      ecode = code;
      break;
    }
    if (is_end) break;
  }
  if (ecode != kOK) return ecode;
  if (run) {
    if (sc >= sb.n_seq) return kESUB;
    sb.seq_out[sc++] = (uint64_t)run;
  }
  if (pos != sb.bit_len || sc != sb.n_seq || lc != sb.n_lit || produced != sb.raw_len) return kESUB;
  return kOK;
}

// ---------------------------------------------------------------- A2 segments
// Segmented decoding: the block's payload bits are cut into equal segments,
// one per decoder lane, whatever the sub-block sizes.  A lane whose segment
// starts inside a sub-block does not know where a symbol starts there, so it
// starts decoding up to kOverlapBits earlier (or at the sub-block's start)
// and relies on canonical codes falling back into step within a few symbols
// (a sub-block start is an exact synchronisation point).  It then decodes,
// writing its records and literal bytes to a private area, from the first
// literal/length symbol boundary at or after its segment start (its entry)
// to the first such boundary at or after the next segment's start (its exit),
// across sub-block ends.  The block is accepted when every lane's exit is the
// next lane's entry, no lane failed or overflowed, and the tokens counted
// per sub-block match the index; the private areas are then packed into the
// final token stream.  Otherwise the block is decoded again one lane per
// sub-block.
struct SegLane {
  uint32_t p_begin, p_end;      // segment [p_begin, p_end), payload bits
  uint32_t base_word, n_words;  // the payload words fetched for the lane
  uint32_t cap_rec, cap_lit;
  GMEM uint64_t* rec_out;
  GMEM uint8_t* lit_out;
  GMEM uint32_t* log;           // the first kLogN literal/length symbol boundaries from the entry
  uint32_t overlap;             // bits decoded without output before the segment, to get into step
  uint32_t xstart;              // an exact symbol boundary to start at instead (kDone: none)
};

// The sub-block holding payload bit p, and the first bit a lane whose segment
// starts at p decodes: kOverlapBits before p, but not before that sub-block's
// start (where decoding is exact from the first bit).
__device__ __forceinline__ uint32_t sub_of(uint32_t p, uint32_t n_sub) {
  uint32_t lo = 0, hi = n_sub - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (s_seg.sub_start[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ uint32_t warm_start(uint32_t p, uint32_t sb, uint32_t overlap) {
  return p >= s_seg.sub_start[sb] + overlap ? p - overlap : s_seg.sub_start[sb];
}

template <int kDec>
__device__ void decode_segment(const SegLane& g, uint32_t L, uint32_t n_sub, uint32_t lmax, uint32_t window,
                               uint32_t max_match) {
  constexpr uint32_t kLanes = 64 * kDec, kRows = ring_rows<kDec>();
  const uint32_t lmask = (1u << lmax) - 1u;
  const uint32_t nw = g.n_words;
  const uint32_t* ring_base = reinterpret_cast<const uint32_t*>(s_stage) + 4 * L;
  uint32_t avail = 0;
  auto ring_word = [&](uint32_t k) -> uint32_t {
    if (k < nw && k >= avail) {
      Spin sp(kSiteRingSeg);
      for (;;) {
        avail = lds_acquire(&s_misc.avail[L]);
        if (k < avail) break;
        if (!sp.pause()) {
          avail = kDone;
          break;
        }
      }
    }
    const uint32_t w = ring_base[((k >> 2) & (kRows - 1)) * (4 * kLanes) + (k & 3)];
    return k < nw ? w : 0u;
  };
  uint32_t w0, w1, w2, w3, nx, rd, sbit;
  // window at absolute payload bit p (p >= 32 * base_word, never moving back)
  auto load = [&](uint32_t p) {
    const uint32_t k = p / 32 - g.base_word;
    w0 = ring_word(k);
    w1 = ring_word(k + 1);
    w2 = ring_word(k + 2);
    w3 = ring_word(k + 3);
    nx = ring_word(k + 4);
    rd = k + 4;
    sbit = p & 31;
    s_misc.rd[L] = k;
  };
  // the symbol at the window under `state`: n bits in all (0: no such code)
  auto peek = [&](uint32_t state, uint32_t& n, uint32_t& kind, uint32_t& val) {
    const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, sbit), hi = __builtin_amdgcn_alignbit(w2, w1, sbit);
    const uint32_t e = s_big[(state << kLutBits) | (lo & lmask)];
    n = e & 31u;
    const uint32_t x = (e >> 5) & 15u;
    kind = (e >> 9) & 3u;
    val = (e >> 16) + __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi, lo, n), 0, x);
    n += x;
  };
  // move the window on by b (< 32) bits
  auto advance = [&](uint32_t b) {
    sbit += b;
    const bool sh = sbit >= 32;
    sbit &= 31;
    w0 = sh ? w1 : w0;
    w1 = sh ? w2 : w1;
    w2 = sh ? w3 : w2;
    w3 = sh ? nx : w3;
    rd += sh ? 1u : 0u;
    nx = ring_word(rd);
    s_misc.rd[L] = rd - 4;
  };
  uint32_t sb = sub_of(g.xstart != kDone ? g.xstart : g.p_begin, n_sub);
  // at most 3 words past base_word
  uint32_t pos = g.xstart != kDone ? g.xstart : warm_start(g.p_begin, sb, g.overlap);
  uint32_t sub_end = s_seg.sub_end[sb];
  uint32_t state = 0, n, kind, val;
  load(pos);
  // warm-up: decode without output up to the entry.  The window only ever
  // moves a little at a time (never further than the lane's bit ring holds):
  // an invalid code or an end symbol that does not end the sub-block means
  // the decoder is out of step, and it moves on by one bit.
  for (;;) {
    if (state == 0 && pos >= g.p_begin) break;
    if (pos >= sub_end) {
      // the sub-block's end (or past it, out of step): resume at the next
      // sub-block's start, an exact symbol boundary at most 127 bits on
      sb++;
      pos = s_seg.sub_start[sb];
      state = 0;
      if (sb >= n_sub) break;
      sub_end = s_seg.sub_end[sb];
      load(pos);
      continue;
    }
    peek(state, n, kind, val);
    if (n == 0 || (state == 0 && kind == kKindEnd && pos + n != sub_end)) {
      advance(1);
      pos += 1;
      state = 0;
      continue;
    }
    advance(n);
    pos += n;
    state = (state == 0 && kind == kKindLen) ? 1u : 0u;
  }
  const uint32_t entry = pos, entry_sub = sb;
  uint32_t flags = (sb < n_sub && pos != s_seg.sub_start[sb]) ? kSegMid : 0u;
  // per sub-block tallies: records and literals since the part's start (sc0,
  // lc0), and the match bytes of those records (mlen)
  uint32_t sc = 0, lc = 0, run = 0, plen = 0, sc0 = 0, lc0 = 0, mlen = 0, nlog = 0, maybe_idx = 0, lbuf = 0;
  // records leave two at a time (16 bytes; the area is 16-byte aligned): an
  // even-numbered record waits in rpend for the next one
  uint64_t rpend = 0;
  // literal words likewise wait for the rest of their 16 bytes (lw0..lw2),
  // and log entries for the rest of theirs (lg0..lg2)
  uint32_t lw0 = 0, lw1 = 0, lw2 = 0, lg0 = 0, lg1 = 0, lg2 = 0;
  auto log_push = [&](uint32_t v) {
    const uint32_t wi = nlog & 3;
    if (wi == 3) {
      GMEM Aligned16* d = reinterpret_cast<GMEM Aligned16*>(g.log + (nlog & ~3u));
      d->x = lg0;
      d->y = lg1;
      d->z = lg2;
      d->w = v;
    }
    lg0 = wi == 0 ? v : lg0;
    lg1 = wi == 1 ? v : lg1;
    lg2 = wi == 2 ? v : lg2;
    nlog++;
  };
  auto store_pair = [&](uint32_t i, uint64_t r0, uint64_t r1) {  // records i (even) and i + 1
    GMEM Aligned16* d = reinterpret_cast<GMEM Aligned16*>(g.rec_out + i);
    d->x = (uint32_t)r0;
    d->y = (uint32_t)(r0 >> 32);
    d->z = (uint32_t)r1;
    d->w = (uint32_t)(r1 >> 32);
  };
  bool any_eob = false, fail = false, over_hit = false;
  if (sb < n_sub && pos < g.p_end) {
    log_push(pos);
    for (;;) {
      bool is_end = false;
      // One symbol per step, branch-free apart from the stores.  A bad symbol
      // before the lane's first sub-block end and within its log means the
      // decoder is still out of step: it then moves on by one bit instead
      // (a repair from the previous lane's exit replaces this stretch).
      const bool can_nudge = !any_eob;
      for (;;) {
        peek(state, n, kind, val);
        const bool is_dist = state != 0;
        const bool is_lit = !is_dist && kind == kKindLit;
        const bool is_len = !is_dist && kind == kKindLen;
        is_end = !is_dist && kind == kKindEnd;
        const uint32_t np = pos + n;
        // bitwise, not short-circuit, logic: the compiler keeps it branch-free
        const bool bad = (n == 0) | (np > sub_end) | (is_dist & ((plen > max_match) | (val > window))) |
                         (is_end & (np != sub_end));
        const bool nudge = bad & can_nudge & (nlog < kLogN) & (pos < sub_end);
        const bool over = !bad & ((is_dist & (sc >= g.cap_rec)) | (is_lit & (lc >= g.cap_lit)));
        const bool go = !bad & !over;
        const uint32_t adv = go ? n : 1u;
        advance(adv);
        pos += adv;
        // literal bytes collect in a register, four to a word, and the words
        // leave four at a time (the private area is 16-byte aligned); what
        // is left is written when the lane's decoding ends
        const bool gd = go & is_dist, gl = go & is_lit;
        const uint64_t rec = (uint64_t)run | ((uint64_t)(plen | (val << 16)) << 32);
        if (gd & ((sc & 1) != 0)) store_pair(sc - 1, rpend, rec);
        rpend = (gd & ((sc & 1) == 0)) ? rec : rpend;
        lbuf = gl ? (lbuf | (val << (8 * (lc & 3)))) : lbuf;
        if (gl & ((lc & 3) == 3)) {
          const uint32_t wi = (lc >> 2) & 3;
          if (wi == 3) {
            GMEM Aligned16* d = reinterpret_cast<GMEM Aligned16*>(g.lit_out + (lc & ~15u));
            d->x = lw0;
            d->y = lw1;
            d->z = lw2;
            d->w = lbuf;
          }
          lw0 = wi == 0 ? lbuf : lw0;
          lw1 = wi == 1 ? lbuf : lw1;
          lw2 = wi == 2 ? lbuf : lw2;
          lbuf = 0;
        }
        sc += gd ? 1u : 0u;
        lc += gl ? 1u : 0u;
        mlen += gd ? plen : 0u;
        run = gd ? 0u : run + (gl ? 1u : 0u);
        plen = (go & is_len) ? val : plen;
        state = (go & is_len) ? 1u : 0u;
        if (go & (state == 0) & !is_end & (nlog < kLogN)) log_push(pos);
        // one exit for both ends of the loop (fewer lane masks to track)
        fail = (bad & !nudge) | over;
        over_hit |= over;
        if (fail | (go & (is_end | ((state == 0) & (pos >= g.p_end))))) break;
      }
      if (fail || !is_end) break;  // failed, or reached the segment's end inside sub-block sb
      // sub-block sb ends here.  The literal run the end closes is a sequence
      // without a match.  At the lane's first end such a sequence is always
      // written, even with no literals of its own: trailing literals of
      // earlier lanes (or of a repair) may flow into it; if none do, it is
      // dropped when the tokens are packed.
      uint32_t pseq = sc - sc0;
      if (run || !any_eob) {
        if (sc >= g.cap_rec) {
          fail = over_hit = true;
          break;
        }
        if (sc & 1) store_pair(sc - 1, rpend, (uint64_t)run);
        else rpend = (uint64_t)run;
        if (run) {
          pseq++;
        } else {
          flags |= kSegMaybe;
          maybe_idx = sc;
        }
        sc++;
      }
      any_eob = true;
      atomicAdd(&s_seg.cnt_seq[sb], pseq);
      atomicAdd(&s_seg.cnt_lit[sb], lc - lc0);
      atomicAdd(&s_seg.cnt_raw[sb], lc - lc0 + mlen);
      sc0 = sc;
      lc0 = lc;
      mlen = run = 0;
      sb++;
      pos = s_seg.sub_start[sb];
      state = 0;
      if (sb >= n_sub || pos >= g.p_end) break;
      sub_end = s_seg.sub_end[sb];
      load(pos);
      if (nlog < kLogN) log_push(pos);
    }
    if (!fail && sb < n_sub && (sc - sc0 | lc - lc0)) {
      atomicAdd(&s_seg.cnt_seq[sb], sc - sc0);
      atomicAdd(&s_seg.cnt_lit[sb], lc - lc0);
      atomicAdd(&s_seg.cnt_raw[sb], lc - lc0 + mlen);
    }
  }
  // the last record of an odd count, the last whole literal words of an
  // unfinished 16 bytes, and the last 1-3 literal bytes
  if (sc & 1) g.rec_out[sc - 1] = rpend;
  GMEM uint32_t* lw = reinterpret_cast<GMEM uint32_t*>(g.lit_out + (lc & ~15u));
  const uint32_t nlw = (lc >> 2) & 3;  // whole words since the last 16 bytes left
  if (nlw > 0) lw[0] = lw0;
  if (nlw > 1) lw[1] = lw1;
  if (nlw > 2) lw[2] = lw2;
  GMEM uint32_t* lgw = g.log + (nlog & ~3u);  // the last log entries of an unfinished 16 bytes
  if ((nlog & 3) > 0) lgw[0] = lg0;
  if ((nlog & 3) > 1) lgw[1] = lg1;
  if ((nlog & 3) > 2) lgw[2] = lg2;
  for (uint32_t i = lc & ~3u; i < lc; i++) g.lit_out[i] = (uint8_t)(lbuf >> (8 * (i & 3)));
  if (fail) flags |= kSegFail | (over_hit ? kSegOver : 0u);
  if (sc == 0 && !any_eob) flags |= kSegPass;
  s_seg.entry[L] = entry;
  s_seg.exit_at[L] = fail ? kDone : pos;
  s_seg.nrec[L] = sc;
  s_seg.nlit[L] = lc;
  s_seg.tail[L] = run;
  s_seg.flags[L] = flags;
  s_seg.entry_sub[L] = entry_sub;
  s_seg.nlog[L] = nlog;
  s_seg.maybe_idx[L] = maybe_idx;
  s_seg.rep_rec[L] = s_seg.rep_lit[L] = s_seg.rep_run[L] = 0;
  s_seg.skip_rec[L] = s_seg.skip_lit[L] = s_seg.skip_run[L] = 0;
}

// Repair of lane k's start when its entry is not the previous lane's exit:
// the previous lane's exit is exact, so decoding from there (slowly, straight
// from HBM) follows the true path; the first literal/length boundary on it that
// lane k also passed (its log) is where the two agree, and lane k's tokens
// from there on are correct.  The repair's tokens replace lane k's tokens
// before that point, and the sub-block's counts are corrected to match.
struct SlowBits {
  const GMEM uint8_t* payload;
  uint32_t pw, k0, w0, w1, w2;
  __device__ uint32_t word(uint32_t k) const { return k < pw ? gload32(payload + 4ull * k) : 0u; }
  __device__ void at(uint32_t pos, uint32_t& lo, uint32_t& hi) {
    const uint32_t k = pos >> 5;
    if (k != k0) {
      if (k == k0 + 1) {
        w0 = w1;
        w1 = w2;
        w2 = word(k + 2);
      } else {
        w0 = word(k);
        w1 = word(k + 1);
        w2 = word(k + 2);
      }
      k0 = k;
    }
    lo = __builtin_amdgcn_alignbit(w1, w0, pos & 31);
    hi = __builtin_amdgcn_alignbit(w2, w1, pos & 31);
  }
  __device__ void peek(uint32_t pos, uint32_t state, uint32_t lmask, uint32_t& n, uint32_t& kind, uint32_t& val) {
    uint32_t lo, hi;
    at(pos, lo, hi);
    const uint32_t e = s_big[(state << kLutBits) | (lo & lmask)];
    n = e & 31u;
    const uint32_t x = (e >> 5) & 15u;
    kind = (e >> 9) & 3u;
    val = (e >> 16) + __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(hi, lo, n), 0, x);
    n += x;
  }
};

__device__ void repair_lane(const SegLane& g, uint32_t k, uint32_t n_sub, const GMEM uint8_t* payload, uint32_t pw,
                            uint32_t lmax, uint32_t window, uint32_t max_match) {
  const uint32_t lmask = (1u << lmax) - 1u;
  // the repair's tokens go after the lane's own in its area
  GMEM uint64_t* rep_rec_out = g.rec_out + s_seg.nrec[k];
  GMEM uint8_t* rep_lit_out = g.lit_out + s_seg.nlit[k];
  const uint32_t rep_rec_cap = g.cap_rec - s_seg.nrec[k], rep_lit_cap = g.cap_lit - s_seg.nlit[k];
  const uint32_t X = s_seg.exit_at[k - 1], E = s_seg.entry[k], sb = s_seg.entry_sub[k];
  const uint32_t nlog = s_seg.nlog[k];
  if (sb >= n_sub || nlog == 0 || X < s_seg.sub_start[sb] || X >= s_seg.sub_end[sb]) {
    atomicOr(&s_seg.bad, kRejRepair);
    return;
  }
  const uint32_t sub_end = s_seg.sub_end[sb];
  // the true path from X, until it meets lane k's path
  SlowBits b{payload, pw, 0xFFFFFFFFu, 0u, 0u, 0u};
  uint32_t pos = X, state = 0, plen = 0, rsc = 0, rlc = 0, rraw = 0, run = 0, j = 0;
  uint32_t lg = g.log[0];
  bool met = false;
  // every step moves on by one symbol, and the walk ends once it is past the
  // lane's last logged boundary
  for (uint32_t it = 0; it < (1u << 20); it++) {
    if (state == 0) {
      while (j < nlog && lg < pos) {
        j++;
        lg = j < nlog ? g.log[j] : kDone;
      }
      if (j >= nlog) break;
      if (lg == pos) {
        met = true;
        break;
      }
    }
    uint32_t n, kind, val;
    b.peek(pos, state, lmask, n, kind, val);
    const bool is_dist = state != 0;
    const bool is_lit = !is_dist && kind == kKindLit;
    const bool is_len = !is_dist && kind == kKindLen;
    const bool is_end = !is_dist && kind == kKindEnd;
    if (n == 0 || is_end || pos + n > sub_end || (is_dist && (plen > max_match || val > window))) break;
    if ((is_dist && rsc >= rep_rec_cap) || (is_lit && rlc >= rep_lit_cap)) break;
    if (is_dist) {
      rep_rec_out[rsc++] = (uint64_t)run | ((uint64_t)(plen | (val << 16)) << 32);
      rraw += plen;
      run = 0;
    }
    if (is_lit) {
      rep_lit_out[rlc++] = (uint8_t)val;
      rraw++;
      run++;
    }
    plen = is_len ? val : plen;
    state = is_len ? 1u : 0u;
    pos += n;
  }
  if (!met) {
    atomicOr(&s_seg.bad, kRejRepair);
    return;
  }
  const uint32_t q = pos;
  // lane k's own path from its entry to q, under the same rules as its decoder
  uint32_t p2 = E, st2 = 0, pl2 = 0, sc = 0, lc = 0, raw = 0, run2 = 0;
  for (uint32_t it = 0; p2 < q && it < q - E + 64; it++) {  // each step moves on by one bit or more
    uint32_t n, kind, val;
    b.peek(p2, st2, lmask, n, kind, val);
    const bool is_dist = st2 != 0;
    const bool is_lit = !is_dist && kind == kKindLit;
    const bool is_len = !is_dist && kind == kKindLen;
    const bool is_end = !is_dist && kind == kKindEnd;
    const uint32_t np = p2 + n;
    const bool bad = n == 0 || np > sub_end || (is_dist && (pl2 > max_match || val > window)) ||
                     (is_end && np != sub_end);
    if (bad) {
      if (p2 >= sub_end) break;
      p2 += 1;
      st2 = 0;
      continue;
    }
    if (is_end) break;  // lane k passed a sub-block end before meeting the true path
    if (is_dist) {
      sc++;
      raw += pl2;
      run2 = 0;
    }
    if (is_lit) {
      lc++;
      raw++;
      run2++;
    }
    pl2 = is_len ? val : pl2;
    st2 = is_len ? 1u : 0u;
    p2 = np;
  }
  if (p2 != q || st2 != 0) {
    atomicOr(&s_seg.bad, kRejRepair);
    return;
  }
  atomicAdd(&s_seg.cnt_seq[sb], rsc - sc);
  atomicAdd(&s_seg.cnt_lit[sb], rlc - lc);
  atomicAdd(&s_seg.cnt_raw[sb], rraw - raw);
  s_seg.rep_rec[k] = rsc;
  s_seg.rep_lit[k] = rlc;
  s_seg.rep_run[k] = run;
  s_seg.skip_rec[k] = sc;
  s_seg.skip_lit[k] = lc;
  s_seg.skip_run[k] = run2;
  s_seg.flags[k] |= kSegRep;
}

// ---------------------------------------------------------------- ring helpers
__device__ __forceinline__ uint4 ring_read16(const uint8_t* ring, uint32_t p) {
  const uint32_t a = p & kRingMask;
  uint4 v;
  if (a <= kRing - 16) {
    __builtin_memcpy(&v, ring + a, 16);
  } else {
    // wraps around the end of the window: byte by byte
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; i++) {
      lo |= (uint64_t)ring[(p + i) & kRingMask] << (8 * i);
      hi |= (uint64_t)ring[(p + 8 + i) & kRingMask] << (8 * i);
    }
    v = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
  }
  return v;
}

// write the first n (1..16) bytes of v at window position p
__device__ __forceinline__ void ring_write(uint8_t* ring, uint32_t p, uint4 v, uint32_t n) {
  const uint32_t a = p & kRingMask;
  uint64_t lo = (uint64_t)v.x | ((uint64_t)v.y << 32), hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
  if (a + n <= kRing) {
    uint8_t* d = ring + a;
    if (n == 16) {
      __builtin_memcpy(d, &v, 16);
      return;
    }
    if (n & 8) {
      __builtin_memcpy(d, &lo, 8);
      d += 8;
      lo = hi;
    }
    if (n & 4) {
      uint32_t w = (uint32_t)lo;
      __builtin_memcpy(d, &w, 4);
      d += 4;
      lo >>= 32;
    }
    if (n & 2) {
      uint16_t h = (uint16_t)lo;
      __builtin_memcpy(d, &h, 2);
      d += 2;
      lo >>= 16;
    }
    if (n & 1) *d = (uint8_t)lo;
  } else {
    // wraps around the end of the window: byte by byte
    for (uint32_t i = 0; i < n; i++) {
      const uint64_t w = i < 8 ? lo : hi;
      ring[(p + i) & kRingMask] = (uint8_t)(w >> (8 * (i & 7)));
    }
  }
}

// Copy a back-reference inside the window: len bytes to dst from dst - dist.
// The bytes a copy needs are [src, src + min(len, dist)); an overlapping copy
// (dist < len) repeats them with period dist.
__device__ __forceinline__ void copy_match(uint8_t* ring, uint32_t dst, uint32_t len, uint32_t dist) {
  const uint32_t src = dst - dist;
  if (dist < 16 && dist < len) {
    // short period: the first 16 output bytes are built in registers from the
    // dist bytes before dst (one read), then written every p16 = dist *
    // floor(16 / dist) bytes, a whole number of periods
    const uint4 q = ring_read16(ring, src);
    uint64_t lo = (uint64_t)q.x | ((uint64_t)q.y << 32), hi = (uint64_t)q.z | ((uint64_t)q.w << 32);
    if (dist < 8) {
      lo &= (1ull << (8 * dist)) - 1ull;
      hi = 0;
    } else {
      hi &= (1ull << (8 * (dist - 8))) - 1ull;
    }
    for (uint32_t l = dist; l < 16; l *= 2) {  // append the pattern to itself
      const uint32_t sh = 8 * l;
      if (sh >= 64) {
        hi |= lo << (sh - 64);
      } else {
        hi |= (hi << sh) | (lo >> (64 - sh));
        lo |= lo << sh;
      }
    }
    const uint4 v = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    const uint32_t p16 = dist * (16u / dist);
    for (uint32_t k = 0; k < len; k += p16) ring_write(ring, dst + k, v, min(16u, len - k));
    return;
  }
  if (dist >= len || dist >= 64) {
    // no chunk of a batch of four reads bytes the batch writes: reads first
    for (uint32_t k = 0; k < len; k += 64) {
      uint4 c[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        if (k + 16 * j < len) c[j] = ring_read16(ring, src + k + 16 * j);
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        if (k + 16 * j < len) ring_write(ring, dst + k + 16 * j, c[j], min(16u, len - k - 16 * j));
    }
    return;
  }
  // 16 <= dist < 64, overlapping: each 16-byte chunk ends at or before its destination
  for (uint32_t k = 0; k < len; k += 16) ring_write(ring, dst + k, ring_read16(ring, src + k), min(16u, len - k));
}

__device__ __forceinline__ uint4 lit_read16(uint32_t p) {
  const uint8_t* r = lit_ring();
  const uint32_t a = p & (kLitRing - 1);
  uint4 v;
  if (a <= kLitRing - 16) {
    __builtin_memcpy(&v, r + a, 16);
  } else {
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; i++) {
      lo |= (uint64_t)r[(p + i) & (kLitRing - 1)] << (8 * i);
      hi |= (uint64_t)r[(p + 8 + i) & (kLitRing - 1)] << (8 * i);
    }
    v = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
  }
  return v;
}

// Window/ring accesses that are known not to wrap (the common case).
__device__ __forceinline__ uint4 read16(const uint8_t* p) {
  uint4 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}
// Copy n bytes from q to d, where no byte written is one that is read.
// Any length takes two overlapping stores of one width (16, 8, 4 or 2
// bytes: the first and the last bytes of the span), plus whole 16-byte chunks
// in the middle of a copy longer than 32 bytes; a byte covered twice gets the
// same value both times.  This keeps the lanes of a wavefront, whose lengths
// differ, on few distinct paths.
template <typename T>
__device__ __forceinline__ void copy_pair(uint8_t* d, const uint8_t* q, uint32_t n) {
  T a, b;
  __builtin_memcpy(&a, q, sizeof(T));
  __builtin_memcpy(&b, q + n - sizeof(T), sizeof(T));
  __builtin_memcpy(d, &a, sizeof(T));
  __builtin_memcpy(d + n - sizeof(T), &b, sizeof(T));
}
__device__ __forceinline__ void copy_bytes(uint8_t* d, const uint8_t* q, uint32_t n) {
  if (n >= 16) {
    const uint4 h = read16(q), t = read16(q + n - 16);
    for (uint32_t k = 16; k + 16 < n; k += 16) {
      const uint4 m = read16(q + k);
      __builtin_memcpy(d + k, &m, 16);
    }
    __builtin_memcpy(d, &h, 16);
    __builtin_memcpy(d + n - 16, &t, 16);
  } else if (n >= 8) {
    copy_pair<uint64_t>(d, q, n);
  } else if (n >= 4) {
    copy_pair<uint32_t>(d, q, n);
  } else if (n >= 2) {
    copy_pair<uint16_t>(d, q, n);
  } else if (n) {
    *d = *q;
  }
}
// copy len bytes (dst - src >= len) inside the window, no wrap
__device__ __forceinline__ void copy_nowrap(uint8_t* ring, uint32_t dst, uint32_t src, uint32_t len) {
  copy_bytes(ring + (dst & kRingMask), ring + (src & kRingMask), len);
}

// Rare paths that read literal bytes straight from HBM (literal groups larger
// than the staging ring, literal runs longer than the window).  They are kept
// out of line so that their loads never merge with the registers of the LDS
// path: a merge would make the resolver wait for its own output stores.
__device__ __noinline__ void copy_lits_hbm(const GMEM uint8_t* src, uint32_t pos, uint32_t len) {
  uint8_t* ring = ring_ptr();
  for (uint32_t k = 0; k < len; k += 16) ring_write(ring, pos + k, gload16(src + k), min(16u, len - k));
}
// All lanes together copy n literal bytes from src to window position base.
__device__ __noinline__ void stream_lits_hbm(const GMEM uint8_t* src, uint32_t base, uint32_t n, uint32_t lane) {
  uint8_t* ring = ring_ptr();
  for (uint32_t k = lane * 16; k < n; k += 1024) ring_write(ring, base + k, gload16(src + k), min(16u, n - k));
}

// Cooperative literal copy: lane i's run of n bytes goes from literal-ring
// position lsrc to window position pos.  The runs are cut into 16-byte units
// and the units of all runs are spread over the lanes, 64 per pass, so a
// long run costs its length / 1 KiB passes instead of length / 16 steps of
// one lane.  A unit's owner is found from the run starts marked in a
// 64-entry scratch row and a prefix maximum.
__device__ __forceinline__ uint32_t shfl(uint32_t v, uint32_t src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src_lane << 2), (int)v);
}
__device__ void coop_lits(uint32_t pos, uint32_t lsrc, uint32_t n, uint32_t* scratch) {
  uint8_t* ring = ring_ptr();
  const uint32_t lane = lane_id();
  const uint32_t units = (n + 15) >> 4;
  const uint32_t inc = wave_incl_scan(units);
  const uint32_t first = inc - units, total = readlane(inc, 63);
  uint32_t owner_carry = 0;
  for (uint32_t b = 0; b < total; b += 64) {
    scratch[lane] = 0;
    if (units && first >= b && first < b + 64) scratch[first - b] = lane + 1;
    __builtin_amdgcn_wave_barrier();
    const uint32_t mark = wave_incl_max(scratch[lane]);
    const uint32_t owner = mark ? mark - 1 : owner_carry;
    owner_carry = readlane(owner, 63);
    const uint32_t o_first = shfl(first, owner), o_src = shfl(lsrc, owner), o_pos = shfl(pos, owner),
                   o_n = shfl(n, owner);
    const uint32_t u = b + lane;
    if (u < total) {
      const uint32_t off = (u - o_first) << 4;
      ring_write(ring, o_pos + off, lit_read16(o_src + off), min(16u, o_n - off));
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------- A3-A6
// How a group's back-references are resolved: Multi-Round Resolution, one
// pass (Dependency Elimination streams), or Sequential Copying, the paper's
// baseline in its comparison of resolution strategies (one back-reference
// after another, in sequence order).
constexpr uint32_t kResMRR = 0, kResDE = 1, kResSC = 2;
// Where phase B's sequence records come from: the packed token stream (8-byte
// records, copied into LDS by DMA), the segmented decoder's lane areas, or
// the 4-byte records of a byte-level block (both gathered by the fetcher).
constexpr uint32_t kRecPacked = 0, kRecLanes = 1, kRecByte = 2;
struct LzArgs {
  const GMEM uint8_t* recs;  // kRecPacked: 8-byte records; kRecByte: the block's 4-byte records
  uint64_t recs_len;         // bytes readable at recs (bounds the DMA of kRecPacked)
  const GMEM uint8_t* lits;  // the literal bytes, in sequence order
  uint64_t lits_len;         // bytes readable at lits: at least n_lit + 16
  uint32_t rec_src;          // kRecPacked, kRecLanes or kRecByte
  GMEM uint8_t* out;
  uint32_t n_seq, n_lit, raw_len;
  uint32_t res;      // kResMRR, kResDE (one pass) or kResSC (one back-reference at a time)
  // Multi-round resolution over several launches (kResMRR with a spill area):
  // at most max_rounds rounds per group here, the back-references still
  // pending, and those that read their bytes, go to the spill list
  uint32_t max_rounds;
  GMEM uint32_t* spill;  // list A: {destination, distance << 9 | length} entries (null: no spilling)
  bool verify_de;    // a DE group that breaks the DE rule is an error (it is resolved by rounds either way)
  bool redirect;     // MRR: sources moved through the group's own copies first (see resolve_groups)
  bool stats;        // count bytes per round, split groups and DE groups resolved by rounds
  GMEM uint8_t* rounds;
  // kRecLanes: the segmented decoder's lane areas (priv: the first area)
  const GMEM uint8_t* priv;
  uint64_t lane_bytes;  // an area's size
  uint32_t lanes;
};

// A fetcher lane's view of one lane stream of the segmented decoder: its
// records are its repair's records, then its own from its meeting point,
// less a dropped empty sequence; its first record takes the literal-run
// correction, modulo 2^32 on the literal length (the low word).  The
// parameters stay in registers while the lane's records come from one stream.
struct StreamCursor {
  uint32_t s = 0, begin = 0, end = 0;  // stream s holds final records [begin, end)
  uint32_t rs = 0, first = 0, drop = kDone, fix_rep = 0, fix_own = 0, own = 0;
  const GMEM uint8_t* area = nullptr;
  __device__ __forceinline__ void load(const LzArgs& a, uint32_t k) {
    s = k;
    own = s_seg.nrec[k];  // the lane's own records; its repair's records follow them
    begin = s_seg.entry[k];
    end = k + 1 < a.lanes ? s_seg.entry[k + 1] : a.n_seq;
    rs = s_seg.rep_rec[k];
    first = s_seg.skip_rec[k];
    drop = s_seg.maybe_idx[k];
    fix_rep = s_seg.eff_tail[k];
    fix_own = s_seg.tail[k];
    area = a.priv + a.lane_bytes * k;
  }
  // record o (>= the previous one asked for)
  __device__ __forceinline__ uint64_t record(const LzArgs& a, uint32_t o) {
    while (o >= end && s + 1 < a.lanes) load(a, s + 1);
    const uint32_t j = o - begin;
    uint32_t x = first + (j - rs);
    x += (drop != kDone && x >= drop) ? 1u : 0u;
    const bool rep = j < rs;
    const uint64_t off = rep ? 8ull * (own + j) : 8ull * x;
    const uint32_t fix = rep ? (j == 0 ? fix_rep : 0u) : (x == first ? fix_own : 0u);
    const uint64_t r = *(const GMEM uint64_t*)(area + off);
    return (r & 0xFFFFFFFF00000000ull) | (uint32_t)((uint32_t)r + fix);
  }
  // records o and o + 1: one 16-byte load when both are the stream's own
  // records and lie side by side in its area (the usual case)
  __device__ __forceinline__ void record2(const LzArgs& a, uint32_t o, uint64_t& r0, uint64_t& r1) {
    while (o >= end && s + 1 < a.lanes) load(a, s + 1);
    const uint32_t j = o - begin;
    uint32_t x = first + (j - rs);
    x += (drop != kDone && x >= drop) ? 1u : 0u;
    if (o + 1 < end && j >= rs && x + 1 != drop) {
      const GMEM uint32_t* p = (const GMEM uint32_t*)(area + 8ull * x);
      const uint32_t w0 = p[0], w1 = p[1], w2 = p[2], w3 = p[3];
      const uint32_t fix = x == first ? fix_own : 0u;
      r0 = ((uint64_t)w1 << 32) | (uint32_t)(w0 + fix);
      r1 = ((uint64_t)w3 << 32) | w2;
    } else {
      r0 = record(a, o);
      r1 = o + 1 < a.n_seq ? record(a, o + 1) : 0ull;
    }
  }
};

// A byte-level record (bits 0-7 literal length, 8-15 match length - 3, 16-31
// distance, 0 for no back-reference) in the 8-byte form of the token stream.
__device__ __forceinline__ uint64_t byte_record(uint32_t r) {
  const uint32_t d = r >> 16, m = d ? ((r >> 8) & 0xFFu) + 3u : 0u;
  return (uint64_t)(r & 0xFFu) | ((uint64_t)(m | (d << 16)) << 32);
}
// byte-level records o (even) and o + 1, with one 8-byte load (the record
// area is padded to 16 bytes, so the load stays inside it)
__device__ __forceinline__ void byte_record2(const LzArgs& a, uint32_t o, uint64_t& r0, uint64_t& r1) {
  const GMEM uint64_t* p = (const GMEM uint64_t*)(a.recs + 4ull * o);
  const uint64_t v = *p;
  r0 = byte_record((uint32_t)v);
  r1 = o + 1 < a.n_seq ? byte_record((uint32_t)(v >> 32)) : 0ull;
}

// Resolution runs as a pipeline over groups of 64 sequences.  Resolver
// wavefront w takes groups w, w + kRes, w + 2 kRes, ...; everything a group
// needs that does not depend on earlier groups' output (its records, the two
// prefix sums, its literal strings) is done ahead, and only the copies of its
// back-references wait until every earlier group is final.  Progress is
// handed over through LDS counters:
//   rec_avail / lit_avail  fetcher -> resolvers: records / literal bytes staged
//   g_out / g_lit          fetcher -> resolvers: output and literal offsets of
//                          each staged group (ring of kGRing groups)
//   next_group[w]          resolver w -> fetcher: records, offsets and literals
//                          of w's groups before this index are no longer read
//   done_upto              resolvers: output bytes below are final
//   flushed                flusher: output bytes below are in HBM
// The output window holds positions [low, low + kRing) with
// low = min(done_upto - 32768, flushed): every source a pending copy can
// name lies at or above done_upto - 32768, and slots below flushed are free.

// Fetcher side: stream records (1 KiB = 128 records = 2 groups per copy) and
// literal bytes (1 KiB per copy) into their LDS rings, and compute the offsets
// of each group from its records once they arrive.
template <int kRes, uint32_t kSrc>
__device__ void fetch_tokens(const LzArgs& a) {
  const uint32_t lane = lane_id();
  const uint32_t rec_chunks = (a.n_seq + 127) / 128, lit_chunks = (a.n_lit + 1023) / 1024;
  uint32_t rf = 0, lf = 0, tf = 0, carry_out = 0, carry_lit = 0;
  StreamCursor cur;
  if (kSrc == kRecLanes) cur.load(a, 0);
  Spin sp(kSiteTokens);
  while (rf < rec_chunks || lf < lit_chunks) {
    uint32_t gmin = kDone;
#pragma unroll
    for (int w = 0; w < kRes; w++) gmin = min(gmin, lds_acquire(&s_misc.next_group[w]));
    if (gmin == kDone) break;  // every resolver has finished
    // literal bytes before the first group still being read are consumed
    const uint32_t lit_cons = gmin < 2 * tf ? s_misc.g_lit[gmin % kGRing] : carry_lit;
    uint32_t issued = 0, gathered = 0;
    uint64_t g[8][2];
    if (kSrc != kRecPacked) {
      // records gathered from the lane streams or the byte-level records:
      // lane l takes records 2l and 2l + 1 of up to eight 128-record chunks,
      // loads first, stores after
#pragma unroll
      for (uint32_t c = 0; c < 8; c++) {
        const uint32_t ch = rf + c;
        if (ch < rec_chunks && 128ull * (ch + 1) <= 64ull * gmin + kRecRing && gathered == c) {
          const uint32_t o = 128 * ch + 2 * lane;
          if (o < a.n_seq) {
            if (kSrc == kRecByte) byte_record2(a, o, g[c][0], g[c][1]);
            else cur.record2(a, o, g[c][0], g[c][1]);
          } else {
            g[c][0] = g[c][1] = 0ull;
          }
          gathered++;
        }
      }
      issued = gathered;
    } else {
      while (rf < rec_chunks && 128ull * (rf + 1) <= 64ull * gmin + kRecRing && issued < 8) {
        uint64_t o = 1024ull * rf + 16 * lane;
        if (o + 16 > a.recs_len) o = a.recs_len - 16;
        dma16(a.recs + o, &rec_ring()[128 * (rf % (kRecRing / 128))]);
        rf++;
        issued++;
      }
    }
    while (lf < lit_chunks && 1024ull * (lf + 1) <= (uint64_t)lit_cons + kLitRing && issued < 12) {
      uint64_t o = 1024ull * lf + 16 * lane;
      if (o + 16 > a.lits_len) o = a.lits_len - 16;
      dma16(a.lits + o, &lit_ring()[1024 * (lf % (kLitRing / 1024))]);
      lf++;
      issued++;
    }
    if (!issued) {
      if (!sp.pause()) return;
      continue;
    }
    sp = Spin(kSiteTokens);
    wait_all_memory();
#pragma unroll
    for (uint32_t c = 0; c < 8; c++) {
      if (c < gathered) {
        uint2* row = &rec_ring()[(128 * (rf + c)) % kRecRing];
        row[2 * lane] = make_uint2((uint32_t)g[c][0], (uint32_t)(g[c][0] >> 32));
        row[2 * lane + 1] = make_uint2((uint32_t)g[c][1], (uint32_t)(g[c][1] >> 32));
      }
    }
    rf += gathered;
    // offsets of the two groups of every record chunk that arrived
    for (; tf < rf; tf++) {
      const uint32_t j = 128 * tf + 2 * lane;
      const uint2 r0 = j < a.n_seq ? rec_ring()[j % kRecRing] : make_uint2(0u, 0u);
      const uint2 r1 = j + 1 < a.n_seq ? rec_ring()[(j + 1) % kRecRing] : make_uint2(0u, 0u);
      const uint32_t il = wave_incl_scan(r0.x + r1.x);
      const uint32_t io = wave_incl_scan(r0.x + (r0.y & 0xFFFFu) + r1.x + (r1.y & 0xFFFFu));
      const uint32_t l31 = readlane(il, 31), o31 = readlane(io, 31);
      if (lane == 0) {
        s_misc.g_out[(2 * tf) % kGRing] = carry_out;
        s_misc.g_lit[(2 * tf) % kGRing] = carry_lit;
        s_misc.g_out[(2 * tf + 1) % kGRing] = carry_out + o31;
        s_misc.g_lit[(2 * tf + 1) % kGRing] = carry_lit + l31;
      }
      carry_out += readlane(io, 63);
      carry_lit += readlane(il, 63);
    }
    lds_release(&s_misc.lit_avail, min(a.n_lit, 1024 * lf));
    lds_release(&s_misc.rec_avail, min(a.n_seq, 128 * rf));
  }
}

// Wait until output positions below `end` may be written (see above);
// false if the wait was abandoned.
__device__ __forceinline__ bool wait_window(uint32_t end) {
  Spin sp(kSiteWindow);
  for (uint32_t i = 0;; i++) {
    const uint32_t done = lds_acquire(&s_misc.done_upto), fl = lds_acquire(&s_misc.flushed);
    const uint32_t low = min(done > 32768u ? done - 32768u : 0u, fl);
    if (end <= low + kRing) return true;
    if (i >= kTightPolls && !sp.pause()) return false;
  }
}
// Wait until *p >= v; false if the wait was abandoned.  The first polls are
// back to back: hand-overs between resolver wavefronts are on the critical
// path and usually arrive within a few hundred cycles.
__device__ __forceinline__ bool wait_at_least(const uint32_t* p, uint32_t v, uint32_t& seen, uint32_t site) {
  Spin sp(site);
  for (uint32_t i = 0;; i++) {
    seen = lds_acquire(p);
    if (seen >= v) return true;
    if (i >= kTightPolls && !sp.pause()) return false;
  }
}
__device__ __forceinline__ bool wait_done(uint32_t pos) {
  uint32_t seen;
  return wait_at_least(&s_misc.done_upto, pos, seen, kSiteDone);
}

// Pending-byte bitmap of multi-launch resolution (window positions, like the
// output window).  A group clears its own positions before it writes them; a
// back-reference left pending marks its destination; a back-reference whose
// source holds a marked byte cannot be copied in this launch either.
__device__ __forceinline__ uint32_t pend_mask(uint32_t p, uint32_t hi, uint32_t& n) {
  const uint32_t b = p & 31;
  n = min(32u - b, hi - p);
  return (n == 32 ? ~0u : ((1u << n) - 1u)) << b;
}
__device__ bool pend_any(uint32_t lo, uint32_t hi) {
  for (uint32_t p = lo, n; p < hi; p += n) {
    const uint32_t m = pend_mask(p, hi, n);
    if (s_seg.pend[(p >> 5) & (kRing / 32 - 1)] & m) return true;
  }
  return false;
}
__device__ void pend_mark(uint32_t lo, uint32_t hi) {
  for (uint32_t p = lo, n; p < hi; p += n) atomicOr(&s_seg.pend[(p >> 5) & (kRing / 32 - 1)], pend_mask(p, hi, n));
}
// the whole wavefront clears positions [lo, hi)
__device__ void pend_clear(uint32_t lo, uint32_t hi, uint32_t lane) {
  if (hi <= lo) return;
  for (uint32_t w = (lo >> 5) + lane; w <= ((hi - 1) >> 5); w += 64) {
    const uint32_t p = max(lo, 32 * w), e = min(hi, 32 * w + 32);
    uint32_t n;
    atomicAnd(&s_seg.pend[w & (kRing / 32 - 1)], ~pend_mask(p, e, n));
  }
}
// Append this group's (or piece's) pending back-references to the spill
// list, in sequence order: called once every earlier group is final, so the
// list stays in destination order.
__device__ void spill_append(const LzArgs& a, bool spilled, uint32_t dst, uint32_t D, uint32_t M, uint32_t lane) {
  const uint64_t sv = __ballot(spilled);
  if (!sv) return;
  const uint32_t base = s_misc.spill_n;
  if (spilled) {
    const uint32_t i = base + (uint32_t)__popcll(sv & ((1ull << lane) - 1ull));
    a.spill[2 * i] = dst;
    a.spill[2 * i + 1] = (D << 9) | M;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) s_misc.spill_n = base + (uint32_t)__popcll(sv);
}

// Resolver wavefront w of kRes.
template <int kRes, bool kSpill>
__device__ void resolve_groups(const LzArgs& a, uint32_t w) {
  uint8_t* ring = ring_ptr();
  const uint32_t lane = lane_id();
  const GMEM uint8_t* lits = a.lits;
  uint32_t rec_avail = 0, lit_avail = 0;
  const uint32_t n_groups = (a.n_seq + 63) / 64;
  for (uint32_t g = w; g < n_groups; g += kRes) {
    const uint32_t g0 = g * 64;
    const uint32_t need = min(a.n_seq, g0 + 64);
    if (rec_avail < need && !wait_at_least(&s_misc.rec_avail, need, rec_avail, kSiteRecs)) break;
    const uint32_t j = g0 + lane;
    const bool valid = j < a.n_seq;
    const uint2 rec = valid ? rec_ring()[j % kRecRing] : make_uint2(0u, 0u);
    const uint32_t g_out = s_misc.g_out[g % kGRing], g_lit = s_misc.g_lit[g % kGRing];
    uint32_t L = rec.x;
    const uint32_t M0 = rec.y & 0xFFFFu;
    uint32_t D = rec.y >> 16;
    // A3: two exclusive prefix sums over the group's sequences
    const uint32_t inc_lit = wave_incl_scan(L);
    const uint32_t inc_out = wave_incl_scan(L + M0);
    const uint32_t tot_lit = readlane(inc_lit, 63);
    uint32_t lsrc = g_lit + inc_lit - L;
    uint32_t pos = g_out + inc_out - (L + M0);
    // a distance reaching before the block's start is an error (EDIST); such
    // a copy is dropped so that resolution still ends
    const bool bad_dist = valid && M0 > 0 && D > pos + L;
    if (__ballot(bad_dist)) set_err(kEDIST);
    const uint32_t M = bad_dist ? 0u : M0;
    // end of the bytes the lane writes (a dropped copy writes none)
    const uint32_t end = pos + L + M;
    const uint32_t m_cnt = min(64u, a.n_seq - g0);
    const uint32_t g_end = g_out + readlane(inc_out, 63);
    // literals come from the LDS ring unless the group holds more than half of it
    const bool lits_staged = tot_lit <= kLitStagedMax;
    if (lits_staged && tot_lit && lit_avail < g_lit + tot_lit &&
        !wait_at_least(&s_misc.lit_avail, g_lit + tot_lit, lit_avail, kSiteLits))
      break;
    uint32_t rounds = 0;
    bool split = false;
    // A DE block's group is resolved in one pass only if it keeps the rule its
    // compressor promised: every source ends at or before the destination of
    // the group's first back-reference (the group's frozen high-water mark).
    // A group that breaks it is resolved by rounds, which gives the sequential
    // result; with verify_de it is moreover an error (EDIST, the class the
    // format check gives a DE block that breaks the rule).
    bool one_pass = a.res == kResDE;
    if (one_pass) {
      const uint32_t dst0 = pos + L;
      const uint64_t mv = __ballot(valid && M > 0);
      if (mv) {
        const uint32_t hwm = readlane(dst0, (uint32_t)__builtin_ctzll(mv));
        if (__ballot(valid && M > 0 && dst0 - D + M > hwm)) {
          if (a.verify_de) set_err(kEDIST);
          if (a.stats && lane == 0) atomicAdd(&s_misc.n_de_rounds, 1u);
          one_pass = false;
        }
      }
    }
    // MRR: a back-reference that does not overlap itself and whose bytes all
    // lie inside the destination of an earlier such copy of the group (the
    // last lane whose destination starts at or before its source) reads that
    // copy's source instead: the same bytes, available a round earlier.  Up to
    // kJumps moves, while the source is still inside the group's output; not
    // for groups larger than the on-chip span (their pieces could not reach
    // so far back).  D becomes the distance to the final source.
    if (a.res == kResMRR && a.redirect && g_end - g_out <= kSpanCap) {
      constexpr uint32_t kJumps = 2;
      const uint32_t dst0 = pos + L;
      const bool cand = valid && M > 0 && D >= M;
      uint32_t s = dst0 - D;
      for (uint32_t j = 0; j < kJumps; j++) {
        const bool in_group = cand && s >= g_out;
        if (!__ballot(in_group)) break;
        int idx = -1;  // the last lane whose destination starts at or before s
        for (uint32_t step = 64; step; step >>= 1) {
          const int c = idx + (int)step;
          const uint32_t dc = shfl(dst0, (uint32_t)min(c, 63));
          if (c < 64 && dc <= s) idx = c;
        }
        const uint32_t ii = idx < 0 ? 0u : (uint32_t)idx;
        const uint32_t di = shfl(dst0, ii), mi = shfl(M, ii), Di = shfl(D, ii);
        const bool ok = in_group && idx >= 0 && mi > 0 && Di >= mi && s + M <= di + mi;
        if (!__ballot(ok)) break;
        s = ok ? s - Di : s;
      }
      D = cand ? dst0 - s : D;
    }
    // fast path: the group's literals are staged and its output fits the
    // window; "plain" when moreover no copy wraps around the ring or the
    // literal ring and none overlaps its own output (most groups)
    const bool fast = lits_staged && g_end - g_out <= kSpanCap;
    const uint32_t src0 = pos + L - D;
    const bool lane_plain =
        !valid || ((pos & kRingMask) + L + M0 <= kRing &&
                   (M0 == 0 || (D >= M0 && (src0 & kRingMask) + ((M0 + 15) & ~15u) <= kRing)) &&
                   (L == 0 || (lsrc & (kLitRing - 1)) + ((L + 15) & ~15u) <= kLitRing));
    const bool plain = !__ballot(!lane_plain);
    const bool spill_mode = kSpill && a.res == kResMRR;
    if (fast) {
      if (!wait_window(g_end)) break;
      if (spill_mode) pend_clear(g_out, g_end, lane);
      // A4: literal strings into the window, ahead of earlier groups; long
      // runs are spread over the whole wavefront
      const uint32_t max_l = readlane(wave_incl_max(valid ? L : 0u), 63);
      if (max_l > kCoopLits) {
        coop_lits(pos, lsrc, valid ? L : 0u, s_misc.coop[w]);
      } else if (plain) {
        if (valid && L) copy_bytes(ring + (pos & kRingMask), lit_ring() + (lsrc & (kLitRing - 1)), L);
      } else if (valid && L) {
        // per lane: the plain copy unless this lane's run wraps a ring
        if ((pos & kRingMask) + L <= kRing && (lsrc & (kLitRing - 1)) + ((L + 15) & ~15u) <= kLitRing)
          copy_bytes(ring + (pos & kRingMask), lit_ring() + (lsrc & (kLitRing - 1)), L);
        else
          for (uint32_t k = 0; k < L; k += 16) ring_write(ring, pos + k, lit_read16(lsrc + k), min(16u, L - k));
      }
      lds_release(&s_misc.next_group[w], g + kRes);
      const uint32_t dst = pos + L;
      const bool has = valid && M > 0;
      const uint32_t need_end = dst - D + min(M, D);  // bytes a copy reads that it does not write
      // Round membership depends only on positions.  A6 (DE): every
      // back-reference of the group in the one pass.  A5 (MRR): round r takes
      // the pending lanes whose source ends at or below the destination of the
      // lowest pending lane.  It is worked out first, in registers; the copies
      // then run round after round (a wavefront's LDS accesses stay in order,
      // so each round reads what the earlier ones wrote).
      uint32_t my_round = has ? 1u : 0u;
      if (one_pass) {
        rounds = __ballot(has) ? 1u : 0u;
      } else if (a.res == kResSC) {
        // one back-reference per round, in sequence order
        const uint64_t hv = __ballot(has);
        my_round = has ? 1u + (uint32_t)__popcll(hv & ((1ull << lane) - 1ull)) : 0u;
        rounds = (uint32_t)__popcll(hv);
      } else {
        bool pending = has;
        for (;;) {
          const uint64_t votes = __ballot(pending);
          if (votes == 0) break;
          rounds++;
          const uint32_t hwm = readlane(dst, (uint32_t)__builtin_ctzll(votes));
          const bool can = pending && need_end <= hwm;
          my_round = can ? rounds : my_round;
          pending = pending && !can;
        }
      }
      // The only bytes the group reads that it does not write itself lie
      // below g_out: it copies as soon as those it needs are final, possibly
      // before the groups in front of it have finished.
      const uint32_t need = min(readlane(wave_incl_max(has ? need_end : 0u), 63), g_out);
      uint32_t seen_done = 0;
      if (!wait_at_least(&s_misc.done_upto, need, seen_done, kSiteDone)) break;
      bool spilled = false;
      if (spill_mode) {
        // rounds past max_rounds, and copies whose source holds a byte that
        // waits for a later launch, are left to the spill list
        for (uint32_t r = 1; r <= rounds; r++) {
          if (my_round == r) {
            if ((a.max_rounds && r > a.max_rounds) || pend_any(src0, need_end)) {
              pend_mark(dst, dst + M);
              spilled = true;
            } else if (lane_plain) {
              copy_nowrap(ring, dst, src0, M);
            } else {
              copy_match(ring, dst, M, D);
            }
          }
        }
        if (a.max_rounds) rounds = min(rounds, a.max_rounds);
      } else if (plain) {
        for (uint32_t r = 1; r <= rounds; r++) {
          if (my_round == r) copy_nowrap(ring, dst, src0, M);
        }
      } else {
        // only the copies that wrap or overlap their own output take the
        // general routine; the others keep the plain one
        for (uint32_t r = 1; r <= rounds; r++) {
          if (my_round == r) {
            if (lane_plain) copy_nowrap(ring, dst, src0, M);
            else copy_match(ring, dst, M, D);
          }
        }
      }
      // its output is final once everything in front of it is (often seen
      // by the wait above already)
      if (seen_done < g_out && !wait_done(g_out)) break;
      if (spill_mode) spill_append(a, spilled, dst, D, M, lane);
      lds_release(&s_misc.done_upto, g_end);
      if (a.stats) {
        for (uint32_t r = 1; r <= rounds && r <= 64; r++) {
          const uint32_t b = readlane(wave_incl_scan(my_round == r && !spilled ? M : 0u), 63);
          if (lane == 0) atomicAdd(&s_misc.rbytes[r - 1], b);
        }
      }
    } else {
      // general path, after every earlier group is final: the group is
      // resolved in pieces that fit the window, a literal run longer than the
      // window is streamed through it first
      if (!wait_done(g_out)) break;
      uint32_t lo = 0, released = g_out;
      bool ok = true;
      while (ok && lo < m_cnt) {
        uint32_t base = readlane(pos, lo);
        {
          uint32_t Llo = readlane(L, lo), Mlo = readlane(M, lo), slo = readlane(lsrc, lo);
          while (Llo + Mlo > kSpanCap) {
            const uint32_t P = kSpanCap / 2;
            if (!wait_window(base + P)) {
              ok = false;
              break;
            }
            if (spill_mode) pend_clear(base, base + P, lane);
            stream_lits_hbm(lits + slo, base, P, lane);
            lds_release(&s_misc.done_upto, base + P);
            base += P;
            slo += P;
            Llo -= P;
            split = true;
          }
          if (lane == lo) {
            L = Llo;
            lsrc = slo;
            pos = base;
          }
        }
        const uint64_t fit = __ballot(valid && lane >= lo && end - base <= kSpanCap);
        const uint32_t hi = lo + (uint32_t)__popcll(fit);
        if (hi == lo) {
          // lane lo's literals were cut down to at most kSpanCap above and its
          // copy is at most 258 bytes, so it always fits; this guards the loop
          // against an inconsistent state, which ends the block with an error
          set_err(kEFORMAT);
          ok = false;
          break;
        }
        if (hi < m_cnt) split = true;
        const bool active = lane >= lo && lane < hi;
        const uint32_t piece_end = readlane(end, hi - 1);
        if (!ok || !wait_window(piece_end)) {
          ok = false;
          break;
        }
        if (spill_mode) pend_clear(base, piece_end, lane);
        // A4: literal strings into the window
        if (active && L) {
          if (lits_staged) {
            for (uint32_t k = 0; k < L; k += 16) ring_write(ring, pos + k, lit_read16(lsrc + k), min(16u, L - k));
          } else {
            copy_lits_hbm(lits + lsrc, pos, L);
          }
        }
        const uint32_t dst = pos + L;
        bool pending = active && M > 0;
        if (one_pass) {
          // A6: no back-reference of the group depends on another (DE)
          if (__ballot(pending)) {
            rounds += 1;
            if (a.stats) {
              const uint32_t b = readlane(wave_incl_scan(pending ? M : 0u), 63);
              if (lane == 0) atomicAdd(&s_misc.rbytes[0], b);
            }
          }
          if (pending) copy_match(ring, dst, M, D);
        } else if (a.res == kResSC) {
          // Sequential Copying: one back-reference at a time, in order
          for (uint64_t votes = __ballot(pending); votes; votes &= votes - 1) {
            const uint32_t l = (uint32_t)__builtin_ctzll(votes);
            if (lane == l) copy_match(ring, dst, M, D);
            if (a.stats && lane == 0 && rounds < 64) atomicAdd(&s_misc.rbytes[rounds], readlane(M, l));
            rounds++;
          }
        } else {
          // A5: Multi-Round Resolution
          const uint32_t need_end = dst - D + min(M, D);
          bool spilled = false;
          for (;;) {
            const uint64_t votes = __ballot(pending);
            if (votes == 0) break;
            if (spill_mode && a.max_rounds && rounds >= a.max_rounds) {
              // the rest of the group's back-references wait for a later launch
              if (pending) {
                pend_mark(dst, dst + M);
                spilled = true;
                pending = false;
              }
              break;
            }
            const uint32_t hwm = readlane(dst, (uint32_t)__builtin_ctzll(votes));
            const bool can = pending && need_end <= hwm;
            if (can) {
              if (spill_mode && pend_any(dst - D, need_end)) {
                pend_mark(dst, dst + M);
                spilled = true;
              } else {
                copy_match(ring, dst, M, D);
              }
              pending = false;
            }
            if (a.stats) {
              const uint32_t b = readlane(wave_incl_scan(can ? M : 0u), 63);
              if (lane == 0 && rounds < 64) atomicAdd(&s_misc.rbytes[rounds], b);
            }
            rounds++;
          }
          if (spill_mode) spill_append(a, spilled, dst, D, M, lane);
        }
        lds_release(&s_misc.done_upto, piece_end);
        released = piece_end;
        lo = hi;
      }
      if (!ok) break;
      // a dropped copy (bad distance) at the group's end leaves its bytes
      // unwritten, so the last piece can end before g_end: the group's output
      // still ends there.  Only then is g_end stored here; once a piece has
      // published g_end the next group may already have moved done_upto on,
      // and storing g_end again would move it back.
      if (released != g_end) lds_release(&s_misc.done_upto, g_end);
      lds_release(&s_misc.next_group[w], g + kRes);
    }
    if (a.rounds && lane == 0) a.rounds[g] = (uint8_t)(min(rounds, 127u) | (split ? 0x80u : 0u));
    if (a.stats && split && lane == 0) atomicAdd(&s_misc.n_split, 1u);
  }
  lds_release(&s_misc.next_group[w], kDone);
}

// Flusher wavefront: final window bytes to HBM, 16 bytes per lane per store,
// once at least 1 KiB is final (and the rest at the end).
__device__ void flush_output(const LzArgs& a) {
  const uint8_t* ring = ring_ptr();
  const uint32_t lane = lane_id();
  uint32_t fl = 0;
  Spin sp(kSiteFlush);
  while (fl < a.raw_len) {
    const uint32_t done = min(lds_acquire(&s_misc.done_upto), a.raw_len);
    const uint32_t end = done == a.raw_len ? done : (done & ~15u);
    if (end <= fl || (end - fl < 1024 && end != a.raw_len)) {
      if (!sp.pause()) return;
      continue;
    }
    sp = Spin(kSiteFlush);
    for (uint32_t p = fl + lane * 16; p < end; p += 1024) {
      if (p + 16 <= end) {
        uint4 v;
        __builtin_memcpy(&v, ring + (p & kRingMask), 16);
        gstore16(a.out + p, v);
      } else {
        for (uint32_t q = p; q < end; q++) a.out[q] = ring[q & kRingMask];
      }
    }
    fl = end;
    lds_release(&s_misc.flushed, fl);
  }
}

// ---------------------------------------------------------------- A0/A2 segmented
// A segment boundary that falls close to a sub-block's end moves to the next
// sub-block's start (an exact symbol boundary): a decoder starting there has
// nothing to synchronise, while one starting just before the end could stay
// out of step until the end and then have no symbol boundary to meet.
__device__ __forceinline__ uint32_t snap_boundary(uint32_t p, uint32_t n_sub) {
  const uint32_t lo = sub_of(p, n_sub);
  const uint32_t e = s_seg.sub_end[lo];
  return (p != s_seg.sub_start[lo] && (p >= e || e - p < kSnapBits)) ? s_seg.sub_start[lo + 1] : p;
}

// The segmented form of A2 for a block that qualifies: its index is
// consistent, it has at most kSubMax sub-blocks, its payload gives every lane
// at least two 16-byte rows, and its workspace holds the private areas.
// Returns true when the block's final token stream is in the workspace;
// false leaves the block to the one-lane-per-sub-block decoder (which also
// reports any error).  Called by every thread of the workgroup.
template <int kDec>
__device__ bool decode_segmented(const DevJob& job, const GMEM uint8_t* idx, const GMEM uint8_t* payload_bytes,
                                 uint32_t n_sub, uint32_t n_seq, uint32_t n_lit, uint32_t payload, uint32_t lmax,
                                 uint32_t window, uint32_t max_match, GMEM uint64_t* ws_seq, GMEM uint8_t* ws_lit,
                                 uint32_t overlap, bool second) {
  constexpr uint32_t kThreads = block_threads<kDec>(), kLanes = 64 * kDec;
  Misc& sh = s_misc;
  const uint32_t t = threadIdx.x, wave = t >> 6;
  const uint32_t pw = payload / 4;  // payload words (a multiple of 4)
  const uint64_t fin = final_bytes(n_seq, n_lit);
  const uint64_t cap_rec = lane_cap_rec(n_seq, kLanes), cap_lit = lane_cap_lit(n_lit, job.comp_len, kLanes);
  const uint64_t lane_bytes = 8 * cap_rec + cap_lit + kLaneExtra;
  if (!kSegmentedDecode || n_sub == 0 || n_sub > kSubMax || pw < 8 * kLanes || payload >= (1u << 28) ||
      job.ws_len < fin + kLanes * lane_bytes)
    return false;
  // sub-block table from the index
  if (t == 0) s_seg.bad = 0;
  uint32_t carry[4] = {0, 0, 0, 0};
  for (uint32_t c = 0; c < n_sub; c += kThreads) {
    const uint32_t s = c + t;
    uint32_t bit_len = 0, sseq = 0, slit = 0, sraw = 0;
    if (s < n_sub) {
      const uint4 e = gload16(idx + kIdxBytes * s);
      bit_len = e.x;
      sseq = e.y;
      slit = e.z;
      sraw = e.w;
    }
    const uint32_t nwords = (uint32_t)((((uint64_t)bit_len + 127) >> 7) << 2);
    uint32_t v[4] = {nwords, sseq, slit, sraw}, tot[4];
    block_excl_scan4<kThreads>(v, tot);
    const uint32_t word_off = carry[0] + v[0];
    if (s < n_sub) {
      if (bit_len == 0 || (uint64_t)word_off + nwords > pw) atomicOr(&s_seg.bad, kRejIndex);
      s_seg.sub_start[s] = 32 * word_off;
      s_seg.sub_end[s] = 32 * word_off + bit_len;
      s_seg.cnt_seq[s] = 0;
      s_seg.cnt_lit[s] = 0;
      s_seg.cnt_raw[s] = 0;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) carry[i] += tot[i];
  }
  if (t == 0) {
    s_seg.sub_start[n_sub] = 32 * pw;
    if (carry[0] != pw || carry[1] != n_seq || carry[2] != n_lit) atomicOr(&s_seg.bad, kRejIndex);
  }
  __syncthreads();
  if (s_seg.bad) {
    if (t == 0) sh.seg_reject = s_seg.bad;
    return false;
  }
  // segments: equal runs of 16-byte rows; each lane fetches from where its
  // warm-up may start to a little past its segment's end
  GMEM uint8_t* priv = gmem(job.ws) + fin;
  SegLane g;
  if (t < kLanes) {
    const uint32_t rows = pw / 4;
    g.p_begin = snap_boundary(128 * (uint32_t)((uint64_t)rows * t / kLanes), n_sub);
    g.p_end = t + 1 == kLanes ? 32 * pw : snap_boundary(128 * (uint32_t)((uint64_t)rows * (t + 1) / kLanes), n_sub);
    // the lane's bit ring starts at the row of the first bit it decodes
    g.overlap = overlap;
    // a later attempt restarts a lane that fell out of step exactly where a
    // lane in step before it ended (its first symbol boundary at or after
    // this lane's segment start)
    g.xstart = second && s_xstart[t] < g.p_end ? s_xstart[t] : kDone;
    g.base_word = ((g.xstart != kDone ? g.xstart : warm_start(g.p_begin, sub_of(g.p_begin, n_sub), overlap)) / 32) &
                  ~3u;
    // whole 16-byte rows: the fetcher moves rows, and the ring holds no partial one
    g.n_words = min(pw, (g.p_end / 32 + 8 + 3) & ~3u) - g.base_word;
    g.cap_rec = (uint32_t)cap_rec;
    g.cap_lit = (uint32_t)cap_lit;
    g.rec_out = (GMEM uint64_t*)(priv + lane_bytes * t);
    g.lit_out = priv + lane_bytes * t + 8 * cap_rec;
    g.log = (GMEM uint32_t*)(g.lit_out + cap_lit);
    sh.sub_woff[t] = g.base_word;
    sh.sub_nw[t] = g.n_words;
    sh.rd[t] = 0;
    sh.avail[t] = 0;
  }
  __syncthreads();
  if (wave == kDec) {
    fetch_bitstreams<kDec>(payload_bytes);
  } else if (t < kLanes) {
    decode_segment<kDec>(g, t, n_sub, lmax, window, max_match);
    lds_release(&sh.rd[t], kDone);
  }
  __syncthreads();
  // lanes whose entry is not the previous lane's exit: repair their start
  if (t < kLanes) {
    if (t > 0 && !(s_seg.flags[t] & kSegFail) && !(s_seg.flags[t - 1] & kSegFail) &&
        s_seg.entry[t] != s_seg.exit_at[t - 1])
      repair_lane(g, t, n_sub, payload_bytes, pw, lmax, window, max_match);
  }
  __syncthreads();
  // Each lane's effective token stream: its repair's tokens (if any), then its
  // own tokens from the meeting point.  Literal runs that stay open at a
  // lane's end flow into the next lanes' first sequence.
  uint32_t flags = 0, rsc = 0, rlc = 0, sq = 0, lq = 0, nrec = 0, nlit = 0;
  bool mid = false;
  if (t < kLanes) {
    flags = s_seg.flags[t];
    rsc = s_seg.rep_rec[t];
    rlc = s_seg.rep_lit[t];
    sq = s_seg.skip_rec[t];
    lq = s_seg.skip_lit[t];
    nrec = s_seg.nrec[t];
    nlit = s_seg.nlit[t];
    const uint32_t own_after = nrec - sq;
    s_seg.eff_tail[t] = own_after ? s_seg.tail[t] : s_seg.rep_run[t] + s_seg.tail[t] - s_seg.skip_run[t];
    const uint32_t eb = s_seg.entry_sub[t];
    const uint32_t start = (flags & kSegRep) ? s_seg.exit_at[t - 1] : s_seg.entry[t];
    mid = eb < n_sub && start != s_seg.sub_start[eb];
    const bool meets = t == 0 ? s_seg.entry[0] == 0u : ((flags & kSegRep) || s_seg.entry[t] == s_seg.exit_at[t - 1]);
    if (flags & kSegFail) atomicOr(&s_seg.bad, (flags & kSegOver) ? kRejOver : kRejCode);
    if (!meets) atomicOr(&s_seg.bad, kRejMeet);
    if (t + 1 == kLanes && s_seg.exit_at[t] != 32 * pw) atomicOr(&s_seg.bad, kRejLast);
  }
  __syncthreads();
  uint32_t carry_in = 0, own_fix = 0, drop = kDone;
  if (t < kLanes) {
    if (mid) {
      for (uint32_t j = t; j-- > 0;) {
        carry_in += s_seg.eff_tail[j];
        if (s_seg.rep_rec[j] + s_seg.nrec[j] - s_seg.skip_rec[j] != 0) break;  // j has a sequence: the run starts there
      }
    } else if (t && s_seg.eff_tail[t - 1]) {
      atomicOr(&s_seg.bad, kRejRun);  // an open literal run must continue in the next lane
    }
    own_fix = (rsc ? 0u : carry_in) + s_seg.rep_run[t] - s_seg.skip_run[t];
    if (flags & kSegMaybe) {
      const uint32_t mi = s_seg.maybe_idx[t];
      if (mi == sq && own_fix) atomicAdd(&s_seg.cnt_seq[s_seg.entry_sub[t]], 1u);  // literals flow into it
      else drop = mi;                                                            // an empty sequence: dropped
    }
  }
  __syncthreads();
  for (uint32_t s = t; s < n_sub; s += kThreads) {
    const uint4 e = gload16(idx + kIdxBytes * s);
    if (s_seg.cnt_seq[s] != e.y || s_seg.cnt_lit[s] != e.z || s_seg.cnt_raw[s] != e.w) atomicOr(&s_seg.bad, kRejCount);
  }
  __syncthreads();
  if (s_seg.bad) {
    if (t == 0) {
      sh.seg_reject = s_seg.bad;
      // Which lanes are on the true symbol path from their entry on: lane 0,
      // lanes whose entry is a sub-block start, and lanes that met (or were
      // repaired from) the exit of a lane on it.  A lane that failed or did
      // not meet its predecessor restarts, in a later attempt, exactly at
      // that predecessor's exit when the predecessor is on the path.
      // A restart found once stays: the exit of a lane on the path is the
      // first true boundary at or after the next lane's segment start.
      bool prev_on = false;
      uint32_t prev_exit = kDone, added = 0;
      for (uint32_t k = 0; k < kLanes; k++) {
        const uint32_t f = s_seg.flags[k];
        const bool failed = (f & kSegFail) != 0;
        const bool met = k == 0 ? s_seg.entry[0] == 0u : ((f & kSegRep) || s_seg.entry[k] == s_seg.exit_at[k - 1]);
        const bool exact = second && s_xstart[k] != kDone;
        if (!exact && (failed || !met) && prev_on) {
          s_xstart[k] = prev_exit;
          added++;
        }
        prev_on = !failed && (!(f & kSegMid) || exact || (met && prev_on));
        prev_exit = s_seg.exit_at[k];
      }
      sh.seg_restarts = added;
    }
    return false;
  }
  // pack the effective streams into the final token stream
  uint32_t v[4] = {0, 0, 0, 0}, tot[4];
  if (t < kLanes) {
    v[0] = rsc + (nrec - sq) - (drop != kDone ? 1u : 0u);
    v[1] = rlc + (nlit - lq);
  }
  block_excl_scan4<kThreads>(v, tot);
  if (tot[0] != n_seq || tot[1] != n_lit) return false;  // cannot happen once the counts matched
  // Each lane's stream parameters go to LDS (arrays no longer read).  The
  // records stay in the lane areas: phase B's fetcher gathers them from
  // there (gather_records).  The literals are packed by the whole
  // workgroup: thread i writes the final stream's bytes [16 i, 16 i + 16),
  // then those kThreads further on, finding the lane streams they come from
  // in the offsets, so neighbouring threads read and write neighbouring bytes.
  if (t < kLanes) {
    s_seg.entry[t] = v[0];         // first record of lane t's stream in the final stream
    s_seg.exit_at[t] = v[1];       // its first literal byte there
    s_seg.eff_tail[t] = carry_in;  // literal-run correction of its first repair record
    s_seg.tail[t] = own_fix;       // ... of its first own record
    s_seg.maybe_idx[t] = drop;     // its own record that is dropped (kDone: none)
  }
  __syncthreads();
  // the lane stream holding final-stream index o (starts: its first indexes)
  auto stream_of = [&](const uint32_t* starts, uint32_t o) {
    uint32_t lo = 0, hi = kLanes - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) / 2;
      if (starts[mid] <= o) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  for (uint32_t o = 16 * t; o < n_lit; o += 16 * kThreads) {
    const uint32_t n = min(16u, n_lit - o);
    uint32_t s = stream_of(s_seg.exit_at, o);
    const uint32_t base = s_seg.exit_at[s], end = s + 1 < kLanes ? s_seg.exit_at[s + 1] : n_lit;
    const uint32_t rl = s_seg.rep_lit[s];
    uint4 q;
    if (n == 16 && o >= base + rl && o + 16 <= end) {
      // all 16 bytes are lane s's own literals, in a row
      q = gload16(priv + lane_bytes * s + 8 * cap_rec + s_seg.skip_lit[s] + (o - base - rl));
    } else {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
      for (uint32_t k = 0; k < n; k++) {
        const uint32_t ok = o + k;
        while (s + 1 < kLanes && s_seg.exit_at[s + 1] <= ok) s++;
        const uint32_t j = ok - s_seg.exit_at[s], rj = s_seg.rep_lit[s];
        const GMEM uint8_t* area = priv + lane_bytes * s;
        // the repair's literals follow the lane's own
        const uint8_t b = j < rj ? area[8 * cap_rec + s_seg.nlit[s] + j] : area[8 * cap_rec + s_seg.skip_lit[s] + (j - rj)];
        w[k / 4] |= (uint32_t)b << (8 * (k % 4));
      }
      q = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (n == 16) {
      gstore16(ws_lit + o, q);
    } else {
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
      for (uint32_t k = 0; k < n; k++) ws_lit[o + k] = (uint8_t)(w[k / 4] >> (8 * (k % 4)));
    }
  }
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------- kernel
__device__ __forceinline__ uint32_t ld32(const GMEM uint8_t* p) { return gload32(p); }

__device__ __forceinline__ void stamp(const DevJob& job, int i) {
  if (job.times && threadIdx.x == 0) gmem(job.times)[i] = wall_clock64();
}

// A3-A6 on the workgroup: the resolver wavefronts, the fetcher and the
// flusher of the block's workgroup shape.  Called by every thread.
template <int kDec>
__device__ void resolve_phase(const LzArgs& a) {
  Misc& sh = s_misc;
  const uint32_t t = threadIdx.x, wave = t >> 6;
  if (t == 0) {
    sh.rec_avail = 0;
    sh.lit_avail = 0;
    sh.done_upto = 0;
    sh.flushed = 0;
  }
  constexpr int kRes = resolver_waves<kDec>();
  if (t < kMaxDecWaves) sh.next_group[t] = t < (uint32_t)kRes ? t : kDone;
  __syncthreads();
  if (wave == kDec) {
    if (a.rec_src == kRecLanes) fetch_tokens<kRes, kRecLanes>(a);
    else if (a.rec_src == kRecByte) fetch_tokens<kRes, kRecByte>(a);
    else fetch_tokens<kRes, kRecPacked>(a);
  } else if (wave == flusher_wave<kDec>()) {
    flush_output(a);
  } else if (wave < (uint32_t)kRes) {
    if (a.spill) resolve_groups<kRes, true>(a, wave);
    else resolve_groups<kRes, false>(a, wave);
  }
  __syncthreads();
  // the spill list's length (none after an error: the block has failed)
  if (a.spill && t == 0) a.spill[-4] = (sh.err || sh.abort) ? 0u : sh.spill_n;
}

// ---------------------------------------------------------------- Gompresso/Byte
// Checks of a byte-level block's records before they are resolved, in the
// order the CPU reference decoder checks them: first the totals against the
// header (ESUB), then record by record, the first failing record deciding the
// class: a match field without a distance (EFORMAT), a match longer than
// max_match (ELEN), a distance beyond the window or reaching before the
// block's start (EDIST).  The records are read in chunks of four per thread,
// the output position of each from a workgroup prefix sum, with the next
// chunk's load issued before the current one is checked.
template <int kThreads>
__device__ int check_byte_records(const GMEM uint8_t* recs, uint32_t n_seq, uint32_t n_lit, uint32_t raw_len,
                                  uint32_t window, uint32_t max_match) {
  const uint32_t t = threadIdx.x;
  constexpr uint32_t kChunk = 4 * kThreads;
  __shared__ unsigned long long s_first_bad;
  if (t == 0) s_first_bad = ~0ull;
  uint64_t out_carry = 0, lit_carry = 0, first_bad = ~0ull;
  const uint32_t n_chunks = (n_seq + kChunk - 1) / kChunk;
  // the record area is padded to 16 bytes: every 16-byte load starting below n_seq records stays inside it
  auto load = [&](uint32_t c) -> uint4 {
    const uint64_t i = (uint64_t)c * kChunk + 4ull * t;
    return i < n_seq ? gload16(recs + 4 * i) : make_uint4(0u, 0u, 0u, 0u);
  };
  uint4 next = n_chunks ? load(0) : make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t c = 0; c < n_chunks; c++) {
    const uint4 cur = next;
    if (c + 1 < n_chunks) next = load(c + 1);
    const uint32_t r[4] = {cur.x, cur.y, cur.z, cur.w};
    const uint64_t i0 = (uint64_t)c * kChunk + 4ull * t;
    uint32_t lit[4], m[4], sum_out = 0, sum_lit = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const bool valid = i0 + k < n_seq;
      const uint32_t d = r[k] >> 16;
      lit[k] = valid ? (r[k] & 0xFFu) : 0u;
      m[k] = valid && d ? ((r[k] >> 8) & 0xFFu) + 3u : 0u;
      sum_out += lit[k] + m[k];
      sum_lit += lit[k];
    }
    uint32_t v[4] = {sum_out, sum_lit, 0u, 0u}, tot[4];
    block_excl_scan4<kThreads>(v, tot);
    uint64_t produced = out_carry + v[0];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const bool valid = i0 + k < n_seq;
      const uint32_t d = r[k] >> 16, mf = (r[k] >> 8) & 0xFFu;
      produced += lit[k];
      const int cls = !valid ? kOK
                      : (d == 0 && mf != 0) ? kEFORMAT
                      : (m[k] > max_match) ? kELEN
                      : (d && (d > window || d > produced)) ? kEDIST : kOK;
      if (cls != kOK && first_bad == ~0ull) first_bad = ((i0 + k) << 8) | (uint64_t)(-cls);
      produced += m[k];
    }
    out_carry += tot[0];
    lit_carry += tot[1];
  }
  if (first_bad != ~0ull) atomicMin(&s_first_bad, (unsigned long long)first_bad);
  __syncthreads();
  if (lit_carry != n_lit || out_carry != raw_len) return kESUB;
  return s_first_bad == ~0ull ? kOK : -(int)(s_first_bad & 0xFFu);
}

// A byte-level block (section "Parallel Decompression": its fixed-length
// records are read straight from the compressed block, so decoding and LZ77
// decompression are one pass): header checks, record checks, then A3-A6 with
// the fetcher gathering the records from the block.
// Returns kOK with `a` set for A3-A6, kBlockDone for a block with nothing to
// resolve, or an error.
constexpr int kBlockDone = 1;
template <int kDec, int kMode>
__device__ __forceinline__ int prepare_byte_block(const DevJob& job, uint32_t flags, LzArgs& a) {
  constexpr uint32_t kThreads = block_threads<kDec>();
  Misc& sh = s_misc;
  const GMEM uint8_t* blk = gmem(job.comp);
  if (job.comp_len < kByteHdr) return kEFORMAT;
  const uint32_t w1 = ld32(blk + 4);
  const uint32_t mode = (w1 >> 8) & 0xFF, group = (w1 >> 16) & 0xFF;
  const uint32_t raw_len = ld32(blk + 8), window = ld32(blk + 12), w4 = ld32(blk + 16);
  const uint32_t max_match = w4 & 0xFFFF, n_seq = ld32(blk + 20), n_lit = ld32(blk + 24);
  if ((w1 & 0xFF) != 1 || mode > 1 || group < 1 || (w1 >> 24) != 0 || window < 1 || window > 32768 ||
      max_match < 3 || max_match > 258 || (w4 >> 16) != 0 || ld32(blk + 28) != 0 || n_seq > 0x3FFFFFFFu)
    return kEFORMAT;
  const uint64_t rec_bytes = (4ull * n_seq + 15) & ~15ull, lit_bytes = (((uint64_t)n_lit + 15) & ~15ull) + 16;
  if (kByteHdr + rec_bytes + lit_bytes > job.comp_len) return kEFORMAT;
  if (n_seq != job.n_seq || n_lit != job.n_lit) return kEFORMAT;
  if (raw_len != job.out_len) return kESIZE;
  const bool de_ok = mode == 1 && (group % 64) == 0;
  if (kMode == GMPK_MODE_DE && !de_ok) return kEINVAL;
  const bool single_pass = (kMode == GMPK_MODE_DE) || (kMode == GMPK_MODE_AUTO && de_ok);
  const int e = check_byte_records<kThreads>(blk + kByteHdr, n_seq, n_lit, raw_len, window, max_match);
  if (e != kOK) return e;
  if (threadIdx.x == 0) sh.a2_path = 3;
  stamp(job, 1);
  stamp(job, 2);
  a.rec_src = kRecByte;
  a.recs = blk + kByteHdr;
  a.recs_len = rec_bytes;
  a.lits = blk + kByteHdr + rec_bytes;
  a.lits_len = lit_bytes;
  a.out = gmem(job.out);
  a.n_seq = n_seq;
  a.n_lit = n_lit;
  a.raw_len = raw_len;
  a.res = kMode == GMPK_MODE_SC ? kResSC : (single_pass ? kResDE : kResMRR);
  a.verify_de = (flags & GMPK_FLAG_VERIFY_DE) != 0;
  a.redirect = (flags & GMPK_FLAG_PLAIN_MRR) == 0;
  a.stats = (flags & GMPK_FLAG_STATS) && job.stats;
  a.rounds = (flags & GMPK_FLAG_STATS) && job.rounds ? gmem(job.rounds) : nullptr;
  a.max_rounds = (flags & GMPK_ROUNDS_MASK) >> GMPK_ROUNDS_SHIFT;
  a.spill = a.max_rounds && job.spill ? (GMEM uint32_t*)(gmem(job.spill) + 16) : nullptr;
  a.priv = nullptr;
  return n_seq ? kOK : kBlockDone;
}

// A0-A2 of a Gompresso/Bit block: returns kOK with `a` set for A3-A6,
// kBlockDone for an empty block, or an error.
template <int kDec, int kMode>
__device__ __forceinline__ int prepare_bit_block(const DevJob& job, uint32_t flags, LzArgs& a) {
  constexpr uint32_t kThreads = block_threads<kDec>(), kLanes = 64 * kDec;
  Misc& sh = s_misc;
  const uint32_t t = threadIdx.x, wave = t >> 6;
  const GMEM uint8_t* blk = gmem(job.comp);
  // ---- A0: header
  int err = kOK;
  uint32_t mode = 0, group = 0, lmax = 0, raw_len = 0, window = 0, max_match = 0, n_sub = 0, n_seq = 0,
           n_lit = 0, payload = 0;
  if (job.comp_len < kHdrBytes + 16) {
    err = kEFORMAT;
  } else {
    const uint32_t w1 = ld32(blk + 4);
    mode = (w1 >> 8) & 0xFF;
    group = (w1 >> 16) & 0xFF;
    lmax = w1 >> 24;
    raw_len = ld32(blk + 8);
    window = ld32(blk + 12);
    const uint32_t w4 = ld32(blk + 16);
    max_match = w4 & 0xFFFF;
    n_sub = ld32(blk + 20);
    n_seq = ld32(blk + 24);
    n_lit = ld32(blk + 28);
    if (ld32(blk) != kMagicBlock || (w1 & 0xFF) != 1 || mode > 1 || group < 1 || lmax < 1 || lmax > 15 ||
        window < 1 || window > 32768 || max_match < 3 || max_match > 258 || (w4 >> 16) != 0) {
      err = kEFORMAT;
    } else if (lmax > kLutBits) {
      err = kENOSYS;
    } else if ((uint64_t)kHdrBytes + (uint64_t)kIdxBytes * n_sub + 16 > job.comp_len) {
      err = kEFORMAT;
    } else {
      payload = ld32(blk + kHdrBytes + kIdxBytes * n_sub);
      if ((uint64_t)kHdrBytes + (uint64_t)kIdxBytes * n_sub + 16 + payload > job.comp_len || (payload & 15))
        err = kEFORMAT;
      else if (n_seq != job.n_seq || n_lit != job.n_lit || job.ws_len < 8ull * n_seq + n_lit + 64) err = kEFORMAT;
      else if (raw_len != job.out_len) err = kESIZE;
    }
  }
  const bool de_ok = mode == 1 && (group % 64) == 0;
  if (err == kOK && kMode == GMPK_MODE_DE && !de_ok) err = kEINVAL;
  const bool single_pass = (kMode == GMPK_MODE_DE) || (kMode == GMPK_MODE_AUTO && de_ok);
  if (err != kOK) return err;
  if (n_sub == 0) {
    // an empty block: nothing to decode
    return (raw_len == 0 && n_seq == 0 && n_lit == 0 && payload == 0) ? kBlockDone : kEFORMAT;
  }
  // ---- A1: code lengths and lookup tables
  for (uint32_t i = t; i < kNumLL + kNumD; i += kThreads) sh.lens[i] = (blk[32 + i / 2] >> ((i & 1) * 4)) & 15;
  __syncthreads();
  if (sh.lens[256] == 0) set_err(kECODE);
  uint32_t* lut_ll = s_big;
  uint32_t* lut_d = s_big + kLutSize;
  build_table<kThreads>(sh.lens, kNumLL, lmax, lut_ll, false);
  __syncthreads();
  build_table<kThreads>(sh.lens + kNumLL, kNumD, lmax, lut_d, true);
  __syncthreads();
  if (sh.err) return sh.err;
  stamp(job, 1);
  // ---- A0/A2: sub-block offsets by prefix sums over the index, then decode
  const GMEM uint8_t* idx = blk + kHdrBytes;
  const GMEM uint8_t* payload_bytes = blk + kHdrBytes + kIdxBytes * n_sub + 16;
  GMEM uint64_t* ws_seq = (GMEM uint64_t*)gmem(job.ws);
  GMEM uint8_t* ws_lit = gmem(job.ws) + 8ull * n_seq;
  // Lanes that stayed out of step past what their repair covers (codes that
  // fall into step slowly) get up to two more attempts: a lane that follows a
  // lane on the true path restarts exactly at that lane's exit (and keeps
  // that start), the others warm up far longer.  It costs less than decoding
  // every sub-block in one lane.
  bool segmented = false;
  for (uint32_t k = t; k < kMaxLanes; k += block_threads<kDec>()) s_xstart[k] = kDone;
#pragma nounroll
  for (uint32_t attempt = 0; attempt < kSegAttempts; attempt++) {
    segmented = decode_segmented<kDec>(job, idx, payload_bytes, n_sub, n_seq, n_lit, payload, lmax, window,
                                       max_match, ws_seq, ws_lit, attempt ? kOverlapRetry : kOverlapBits,
                                       attempt != 0);
    __syncthreads();  // the rejection reasons are in LDS for every thread
    // (an invalid code with lanes that did not meet is most often a lane out
    // of step; a corrupt block fails the later attempts too)
    if (segmented || !(sh.seg_reject & (kRejMeet | kRejRepair)) || (sh.seg_reject & kRejIndex) || sh.abort ||
        (attempt > 0 && sh.seg_restarts == 0))
      break;
    if (t == 0 && attempt + 1 < kSegAttempts) sh.seg_retry = attempt + 1;
  }
  uint32_t carry[4] = {0, 0, 0, 0};
  for (uint32_t c = 0; !segmented && c < n_sub; c += kLanes) {
    const uint32_t s = c + t;
    const bool mine = t < kLanes && s < n_sub;
    uint32_t bit_len = 0, sseq = 0, slit = 0, sraw = 0;
    if (mine) {
      const uint4 e = gload16(idx + kIdxBytes * s);
      bit_len = e.x;
      sseq = e.y;
      slit = e.z;
      sraw = e.w;
    }
    const uint32_t nwords = (uint32_t)((((uint64_t)bit_len + 127) >> 7) << 2);  // padded to 16 bytes
    uint32_t v[4] = {nwords, sseq, slit, sraw}, tot[4];
    block_excl_scan4<kThreads>(v, tot);
    // offsets may wrap for corrupt indexes; the sums are checked below
    const uint32_t word_off = carry[0] + v[0], seq_off = carry[1] + v[1], lit_off = carry[2] + v[2],
                   raw_off = carry[3] + v[3];
#pragma unroll
    for (int i = 0; i < 4; i++) carry[i] += tot[i];
    bool ok = false;
    if (t < kLanes) {
      ok = mine && (uint64_t)word_off + nwords <= payload / 4 && (uint64_t)seq_off + sseq <= n_seq &&
           (uint64_t)lit_off + slit <= n_lit && (uint64_t)raw_off + sraw <= raw_len;
      if (mine && !ok) set_err(kEFORMAT);
      sh.sub_woff[t] = word_off;
      sh.sub_nw[t] = ok ? nwords : 0;
      sh.rd[t] = ok ? 0 : kDone;
      sh.avail[t] = 0;
    }
    __syncthreads();
    if (wave == kDec) {
      fetch_bitstreams<kDec>(payload_bytes);
    } else if (ok) {
      SubBlock sb;
      sb.n_words = nwords;
      sb.bit_len = bit_len;
      sb.n_seq = sseq;
      sb.n_lit = slit;
      sb.raw_len = sraw;
      sb.raw_off = raw_off;
      sb.seq_out = ws_seq + seq_off;
      sb.lit_out = ws_lit + lit_off;
      const int e = decode_subblock<kDec>(sb, t, lmax, window, max_match);
      lds_release(&sh.rd[t], kDone);
      if (e != kOK) set_err(e);
    }
    __syncthreads();
  }
  // the index must account for the whole payload and the header counts
  if (!segmented && t == 0 &&
      (carry[0] * 4ull != payload || carry[1] != n_seq || carry[2] != n_lit || carry[3] != raw_len))
    set_err(kEFORMAT);
  if (t == 0) sh.a2_path = segmented ? 1u : 2u;
  if (segmented && t < kLanes && (s_seg.flags[t] & kSegRep)) atomicAdd(&sh.n_repaired, 1u);
  __syncthreads();  // workspace writes of all lanes are visible after this barrier
  if (sh.err || sh.abort) return sh.abort ? kESTALL : sh.err;
  stamp(job, 2);
  // ---- A3-A6 (next): the decoder wavefronts resolve, the fetcher stages
  // tokens, the last wavefront writes the output
  a.rec_src = segmented ? kRecLanes : kRecPacked;
  a.recs = gmem(job.ws);
  a.recs_len = job.ws_len;
  a.lits = gmem(job.ws) + 8ull * n_seq;
  a.lits_len = job.ws_len - 8ull * n_seq;
  a.out = gmem(job.out);
  a.n_seq = n_seq;
  a.n_lit = n_lit;
  a.raw_len = raw_len;
  a.res = kMode == GMPK_MODE_SC ? kResSC : (single_pass ? kResDE : kResMRR);
  a.verify_de = (flags & GMPK_FLAG_VERIFY_DE) != 0;
  a.redirect = (flags & GMPK_FLAG_PLAIN_MRR) == 0;
  a.stats = (flags & GMPK_FLAG_STATS) && job.stats;
  a.rounds = (flags & GMPK_FLAG_STATS) && job.rounds ? gmem(job.rounds) : nullptr;
  a.max_rounds = (flags & GMPK_ROUNDS_MASK) >> GMPK_ROUNDS_SHIFT;
  a.spill = a.max_rounds && job.spill ? (GMEM uint32_t*)(gmem(job.spill) + 16) : nullptr;
  a.priv = nullptr;
  if (segmented) {
    const uint64_t cap_rec = lane_cap_rec(n_seq, kLanes), cap_lit = lane_cap_lit(n_lit, job.comp_len, kLanes);
    a.priv = gmem(job.ws) + final_bytes(n_seq, n_lit);
    a.lane_bytes = 8 * cap_rec + cap_lit + kLaneExtra;
    a.lanes = kLanes;
  }
  return kOK;
}

// Decodes one block and returns its status (the same value in every thread).
// kMode: GMPK_MODE_AUTO (per block from its header), GMPK_MODE_MRR,
// GMPK_MODE_DE or GMPK_MODE_SC.  Both formats meet at one A3-A6 call.
template <int kDec, int kMode>
__device__ int inflate_block(const DevJob& job, uint32_t flags) {
  Misc& sh = s_misc;
  const uint32_t t = threadIdx.x;
  stamp(job, 0);
  if (t == 0) {
    sh.err = 0;
    sh.abort = 0;
    sh.n_split = 0;
    sh.n_de_rounds = 0;
    sh.a2_path = 0;
    sh.n_repaired = 0;
    sh.stall_site = 0;
    sh.seg_reject = 0;
    sh.seg_retry = 0;
    sh.seg_restarts = 0;
    sh.spill_n = 0;
  }
  if (t < 64) sh.rbytes[t] = 0;
  __syncthreads();
  LzArgs a;
  const int st = job.comp_len >= 4 && ld32(gmem(job.comp)) == kMagicByte
                     ? prepare_byte_block<kDec, kMode>(job, flags, a)
                     : prepare_bit_block<kDec, kMode>(job, flags, a);
  if (st != kOK) return st == kBlockDone ? kOK : st;
  resolve_phase<kDec>(a);
  stamp(job, 3);
  return sh.abort ? kESTALL : (sh.err ? sh.err : kOK);
}

// One block from start to end: decode, then its status word, the first-error
// word, its statistics and its completion counter.
template <int kDec, int kMode>
__device__ void run_block(const DevJob& job, uint32_t flags, int32_t* first_err) {
  // an empty spill list unless resolution leaves back-references to later launches
  if (job.spill && threadIdx.x < 2) gmem((uint32_t*)job.spill)[threadIdx.x] = 0;
  const int st = inflate_block<kDec, kMode>(job, flags);
  const uint32_t t = threadIdx.x;
  __syncthreads();
  if (t == 0) {
    *gmem(job.status) = st;
    if (st != kOK && first_err) atomicCAS(first_err, 0, st);
  }
  if ((flags & GMPK_FLAG_STATS) && job.stats) {
    GMEM uint32_t* o = gmem(job.stats);
    if (t < 64) o[kStatsRoundBytes + t] = s_misc.rbytes[t];
    if (t == 0) {
      o[0] = s_misc.a2_path;
      o[1] = s_misc.n_repaired;
      o[2] = (job.n_seq + 63) / 64;
      o[3] = s_misc.n_split;
      o[4] = s_misc.n_de_rounds;
      o[5] = s_misc.stall_site;
      o[6] = s_misc.seg_reject;
      o[7] = s_misc.seg_retry;
      o[8] = s_misc.spill_n;
    }
  }
  if (job.done) {
    // every thread's output stores are made visible beyond the device before
    // the block announces itself finished
    __threadfence_system();
    __syncthreads();
    if (t == 0) __hip_atomic_fetch_add(job.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int kDec, int kMode>
__global__ __launch_bounds__(block_threads<kDec>()) void inflate_kernel(const DevJob* __restrict__ jobs, uint32_t n_jobs,
                                                                  uint32_t flags, int32_t* first_err) {
  if (blockIdx.x >= n_jobs) return;
  DevJob job = jobs[blockIdx.x];
  if (!(flags & GMPK_FLAG_STATS)) job.times = nullptr;
  run_block<kDec, kMode>(job, flags, first_err);
}

// One block whose job descriptor travels in the kernel arguments (the launch
// needs no device job table).
template <int kDec, int kMode>
__global__ __launch_bounds__(block_threads<kDec>()) void inflate_single_kernel(DevJob job, uint32_t flags,
                                                                         int32_t* first_err) {
  if (!(flags & GMPK_FLAG_STATS)) job.times = nullptr;
  run_block<kDec, kMode>(job, flags, first_err);
}

// Persistent form: workgroups take block indices from a device counter until
// the job table is exhausted; every workgroup exits once it draws an index
// past the end.
template <int kDec, int kMode>
__global__ __launch_bounds__(block_threads<kDec>()) void inflate_persistent_kernel(const DevJob* __restrict__ jobs,
                                                                             uint32_t n_jobs, uint32_t flags,
                                                                             uint32_t* __restrict__ queue,
                                                                             int32_t* first_err) {
  for (;;) {
    if (threadIdx.x == 0) s_misc.next_job = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t j = s_misc.next_job;
    __syncthreads();
    if (j >= n_jobs) return;
    DevJob job = jobs[j];
    if (!(flags & GMPK_FLAG_STATS)) job.times = nullptr;
    run_block<kDec, kMode>(job, flags, first_err);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- later launches
// Multi-Round Resolution over several launches (the paper's variant in which
// the back-references still unresolved after a round are written to device
// memory and a later kernel resolves them, section "Performance Impact of
// Nested back-references").  One wavefront per block walks the block's spill
// list, 64 entries at a time, straight in the output in HBM: everything
// outside the destinations still pending is final there.  An entry is copied
// once its source ends at or below the lowest destination still pending (the
// entries are in destination order; with the lowest entry re-spilled in this
// launch that mark covers every pending byte).  At most `rounds` rounds per 64
// entries (0: until none is pending); the rest go to the other list, in order.
// A copy of length n at distance d repeats the d bytes before its destination
// (byte-forward semantics), so it only reads bytes that were final before it.
__global__ __launch_bounds__(64) void resolve_spills_kernel(const DevJob* __restrict__ jobs, uint32_t n_jobs,
                                                            uint32_t rounds, uint32_t parity,
                                                            uint32_t* d_remaining) {
  if (blockIdx.x >= n_jobs) return;
  const DevJob job = jobs[blockIdx.x];
  if (!job.spill) return;
  const uint32_t lane = lane_id();
  GMEM uint32_t* head = gmem((uint32_t*)job.spill);
  GMEM uint32_t* in = head + 4 + 2ull * job.n_seq * parity;
  GMEM uint32_t* out_list = head + 4 + 2ull * job.n_seq * (parity ^ 1u);
  const uint32_t n_in = min(head[parity], job.n_seq);
  uint8_t* out = job.out;
  uint32_t n_out = 0, low_pending = kDone;
  for (uint32_t b = 0; b < n_in; b += 64) {
    const uint32_t i = b + lane;
    const bool valid = i < n_in;
    const uint32_t dst = valid ? in[2 * i] : 0u, dl = valid ? in[2 * i + 1] : 0u;
    const uint32_t D = dl >> 9, M = dl & 511u;
    // entries that do not fit the block's output are dropped (a failed block's list)
    const bool ok = valid && M && D && D <= dst && (uint64_t)dst + M <= job.out_len;
    const uint32_t need_end = dst - D + min(M, D);
    bool pending = ok;
    for (uint32_t r = 0;; r++) {
      const uint64_t votes = __ballot(pending);
      if (!votes || (rounds && r == rounds)) break;
      const uint32_t hwm = min(readlane(dst, (uint32_t)__builtin_ctzll(votes)), low_pending);
      const bool can = pending && need_end <= hwm;
      if (can) {
        const uint32_t src = dst - D, per = min(D, M);
        for (uint32_t k = 0; k < M; k++) out[dst + k] = __hip_atomic_load(out + src + (k % per), __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_AGENT);
      }
      pending = pending && !can;
      // this round's bytes are visible to the next round's loads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const uint64_t left = __ballot(pending);
    if (pending) {
      const uint32_t o = n_out + (uint32_t)__popcll(left & ((1ull << lane) - 1ull));
      out_list[2 * o] = dst;
      out_list[2 * o + 1] = dl;
    }
    if (left) low_pending = min(low_pending, readlane(dst, (uint32_t)__builtin_ctzll(left)));
    n_out += (uint32_t)__popcll(left);
  }
  if (lane == 0) {
    head[parity ^ 1u] = n_out;
    head[parity] = 0;
    if (n_out && d_remaining) atomicAdd(d_remaining, n_out);
  }
}

// resets the persistent queue head (a kernel, so that graph captures hold no memset node)
__global__ void reset_queue_kernel(uint32_t* queue) { *queue = 0; }

template <int kDec, int kMode>
void launch_one(const DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t persistent, uint32_t workgroups,
                uint32_t* d_queue, int32_t* first_err, hipStream_t stream) {
  if (persistent) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, stream, d_queue);
    hipLaunchKernelGGL((inflate_persistent_kernel<kDec, kMode>), dim3(workgroups), dim3(block_threads<kDec>()), 0,
                       stream, d_jobs, n_jobs, flags, d_queue, first_err);
  } else {
    hipLaunchKernelGGL((inflate_kernel<kDec, kMode>), dim3(n_jobs), dim3(block_threads<kDec>()), 0, stream, d_jobs,
                       n_jobs, flags, first_err);
  }
}

template <int kDec>
int launch_mode(const DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t persistent, uint32_t workgroups,
                uint32_t* d_queue, int32_t* first_err, hipStream_t stream) {
  switch (flags & GMPK_MODE_MASK) {
    case GMPK_MODE_AUTO:
      launch_one<kDec, GMPK_MODE_AUTO>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, first_err, stream);
      return 0;
    case GMPK_MODE_MRR:
      launch_one<kDec, GMPK_MODE_MRR>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, first_err, stream);
      return 0;
    case GMPK_MODE_DE:
      launch_one<kDec, GMPK_MODE_DE>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, first_err, stream);
      return 0;
    default:
      launch_one<kDec, GMPK_MODE_SC>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, first_err, stream);
      return 0;
  }
}

}  // namespace gmpk

extern "C" int gmpk_launch(const gmpk::DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t dec_waves,
                           uint32_t persistent, uint32_t workgroups, uint32_t* d_queue, int32_t* d_first_err,
                           hipStream_t stream) {
  using namespace gmpk;
  if (n_jobs == 0) return 0;
  if (persistent && (workgroups == 0 || !d_queue)) return -1;
  int rc;
  switch (dec_waves) {
    case 1: rc = launch_mode<1>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, d_first_err, stream); break;
    case 2: rc = launch_mode<2>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, d_first_err, stream); break;
    case 4: rc = launch_mode<4>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, d_first_err, stream); break;
    case 7: rc = launch_mode<7>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, d_first_err, stream); break;
    default: return -1;
  }
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -8;
}

extern "C" int gmpk_launch_single(const gmpk::DevJob* h_job, uint32_t flags, int32_t* d_first_err,
                                  hipStream_t stream) {
  using namespace gmpk;
  const DevJob job = *h_job;
  const dim3 grid(1), block(block_threads<7>());
  switch (flags & GMPK_MODE_MASK) {
    case GMPK_MODE_AUTO:
      hipLaunchKernelGGL((inflate_single_kernel<7, GMPK_MODE_AUTO>), grid, block, 0, stream, job, flags, d_first_err);
      break;
    case GMPK_MODE_MRR:
      hipLaunchKernelGGL((inflate_single_kernel<7, GMPK_MODE_MRR>), grid, block, 0, stream, job, flags, d_first_err);
      break;
    case GMPK_MODE_DE:
      hipLaunchKernelGGL((inflate_single_kernel<7, GMPK_MODE_DE>), grid, block, 0, stream, job, flags, d_first_err);
      break;
    default:
      hipLaunchKernelGGL((inflate_single_kernel<7, GMPK_MODE_SC>), grid, block, 0, stream, job, flags, d_first_err);
      break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -8;
}

extern "C" int gmpk_launch_spills(const gmpk::DevJob* d_jobs, uint32_t n_jobs, uint32_t rounds, uint32_t parity,
                                  uint32_t* d_remaining, hipStream_t stream) {
  if (n_jobs == 0) return 0;
  hipLaunchKernelGGL(gmpk::resolve_spills_kernel, dim3(n_jobs), dim3(64), 0, stream, d_jobs, n_jobs, rounds,
                     parity & 1u, d_remaining);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}

namespace gmpk {
__global__ void clear_word_kernel(int32_t* word) { *word = 0; }
__global__ void take_word_kernel(int32_t* word, int32_t* out) { *out = atomicExch(word, 0); }
}  // namespace gmpk

extern "C" int gmpk_clear_word(int32_t* word, hipStream_t stream) {
  hipLaunchKernelGGL(gmpk::clear_word_kernel, dim3(1), dim3(1), 0, stream, word);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
extern "C" int gmpk_take_word(int32_t* word, int32_t* out, hipStream_t stream) {
  hipLaunchKernelGGL(gmpk::take_word_kernel, dim3(1), dim3(1), 0, stream, word, out);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
