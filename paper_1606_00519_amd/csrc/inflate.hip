// Gompresso/Bit intra-block parallel Inflate for gfx950 (MI355X).
//
// One workgroup decodes one data block (arXiv 1606.00519, section
// "Parallel Decompression"):
//   A0  header and sub-block index checks; sub-block offsets by block-wide
//       prefix sums over the sizes stored in the index (section "Huffman
//       Decoding": offsets come from the sub-block sizes in the header);
//   A1  both canonical Huffman codes expanded into 2^lmax-entry lookup tables
//       in LDS, one lookup per symbol;
//   A2  every lane decodes one sub-block: sequence records and literal bytes
//       go to a per-block token workspace (the paper's token stream);
//   A3  wavefront 0 walks the sequences in groups of 64 (one per lane) and
//       computes literal source and output offsets with two DPP prefix sums
//       (section "LZ77 Decompression", reading sequences / copying literals);
//   A4  literal strings are copied into an on-chip output window (LDS ring);
//   A5  back-references of ordinary streams: Multi-Round Resolution — each
//       round, the high-water mark is the destination of the lowest pending
//       lane (everything below it is written without gaps), found with a
//       ballot; every pending lane whose needed source bytes lie below it
//       copies (section "Multi-Round Resolution (MRR) of Nested
//       back-references");
//   A6  back-references of Dependency-Elimination streams: one pass, no
//       checks (section "Dependency Elimination (DE)");
//   the window is flushed to HBM in 1 KiB coalesced chunks.
//
// All arithmetic is integer.  No device memory outside the job's output,
// workspace, rounds and status buffers is written.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inflate.h"

namespace gmpk {

constexpr uint32_t kMagicBlock = 0x42504D47u;  // 'GMPB'
constexpr uint32_t kHdrBytes = 192;
constexpr uint32_t kIdxBytes = 16;
constexpr uint32_t kNumLL = 286;
constexpr uint32_t kNumD = 30;
constexpr uint32_t kLutBits = 13;  // longest code the on-chip tables hold
constexpr uint32_t kLutSize = 1u << kLutBits;
constexpr uint32_t kRing = 65536;  // on-chip output window
constexpr uint32_t kRingMask = kRing - 1;
constexpr uint32_t kSpanCap = kRing - 32768;  // most output one resolution pass holds (window <= 32768)
constexpr uint32_t kFlushChunk = 1024;        // 64 lanes x 16 bytes

// status codes (same values as the public header)
constexpr int kOK = 0, kEINVAL = -1, kEFORMAT = -2, kECODE = -3, kEDIST = -4, kELEN = -5, kESIZE = -6,
              kESUB = -7, kENOSYS = -11;

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

struct Shared {
  union {
    uint32_t lut[2 * kLutSize];  // literal/length table, then distance table
    uint8_t ring[kRing];         // output window (after decoding)
  };
  uint8_t lens[kNumLL + kNumD];
  uint16_t sorted[kNumLL];  // symbols of one code in canonical order
  uint32_t count[16], first[16], offs[17];
  uint32_t wave_sum[4][kMaxWaves];
  int err;
};

__device__ __forceinline__ void set_err(Shared& sh, int e) { atomicCAS(&sh.err, 0, e); }

// ---------------------------------------------------------------- A1 tables
// Canonical code of one alphabet -> lookup table (entry-centric fill: the
// lmax stream bits of an index, read MSB-first, fall into exactly one length's
// code range when the code fills the code space).
template <int kThreads>
__device__ void build_table(Shared& sh, const uint8_t* lens, uint32_t nsym, uint32_t lmax, uint32_t* lut,
                            bool is_dist) {
  const uint32_t t = threadIdx.x;
  if (t < 16) sh.count[t] = 0;
  __syncthreads();
  for (uint32_t s = t; s < nsym; s += kThreads) {
    uint32_t l = lens[s];
    if (l > lmax) set_err(sh, kECODE);
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
      if (left < 0) set_err(sh, kECODE);
    }
    if (used && left != 0) set_err(sh, kECODE);
    if (!used && !is_dist) set_err(sh, kECODE);
    uint32_t code = 0;
    sh.offs[1] = 0;
    sh.count[0] = 0;
    for (uint32_t l = 1; l <= 15; l++) {
      code = (code + sh.count[l - 1]) << 1;
      sh.first[l] = code;
      sh.offs[l + 1] = sh.offs[l] + sh.count[l];
    }
  }
  __syncthreads();
  // symbols in canonical order (by length, then symbol), ranks from ballots
  if (t < 64) {
    uint32_t run[16];
#pragma unroll
    for (int l = 0; l < 16; l++) run[l] = 0;
    const uint64_t below = (1ull << t) - 1ull;
    for (uint32_t c = 0; c < nsym; c += 64) {
      uint32_t s = c + t;
      uint32_t l = s < nsym ? lens[s] : 0;
      uint32_t rank = 0;
#pragma unroll
      for (uint32_t q = 1; q <= 15; q++) {
        uint64_t m = __ballot(l == q);
        if (l == q) rank = run[q] + (uint32_t)__popcll(m & below);
        run[q] += (uint32_t)__popcll(m);
      }
      if (l && l <= 15) sh.sorted[sh.offs[l] + rank] = (uint16_t)s;
    }
  }
  __syncthreads();
  if (sh.err) return;
  const uint32_t size = 1u << lmax;
  for (uint32_t e = t; e < size; e += kThreads) {
    uint32_t m = __builtin_bitreverse32(e) >> (32 - lmax);  // first stream bit = code MSB
    uint32_t entry = 0;
    for (uint32_t l = 1; l <= lmax; l++) {
      uint32_t c = m >> (lmax - l);
      uint32_t k = c - sh.first[l];
      if (k < sh.count[l]) {
        uint32_t sym = sh.sorted[sh.offs[l] + k];
        uint32_t base, extra, kind;
        if (is_dist) {
          kind = kKindDist;
          if (sym >= kNumD) break;
          dist_code(sym, base, extra);
        } else if (sym < 256) {
          kind = kKindLit;
          base = sym;
          extra = 0;
        } else if (sym == 256) {
          kind = kKindEnd;
          base = 0;
          extra = 0;
        } else {
          kind = kKindLen;
          length_code(sym - 257, base, extra);
        }
        uint32_t n = l;
        if (l + extra <= lmax) {  // fold the extra bits into the entry
          base += (e >> l) & ((1u << extra) - 1u);
          n = l + extra;
          extra = 0;
        }
        entry = n | (extra << 5) | (kind << 9) | (base << 16);
        break;
      }
    }
    lut[e] = entry;
  }
}

// ---------------------------------------------------------------- block scan
template <int kThreads>
__device__ __forceinline__ void block_excl_scan4(Shared& sh, uint32_t v[4], uint32_t tot[4]) {
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

// ---------------------------------------------------------------- A2 decode
struct SubBlock {
  const uint32_t* words;
  uint32_t n_words, bit_len;
  uint32_t n_seq, n_lit, raw_len, raw_off;
  uint2* seq_out;
  uint8_t* lit_out;
};

// Decode one sub-block's bitstream: literal bytes to lit_out, one record per
// sequence {literal length, match length | distance << 16} to seq_out.
__device__ int decode_subblock(const SubBlock& sb, const uint32_t* __restrict__ lut_ll,
                               const uint32_t* __restrict__ lut_d, uint32_t lmax, uint32_t window,
                               uint32_t max_match) {
  if (sb.bit_len == 0) return kESUB;
  const uint32_t lmask = (1u << lmax) - 1u;
  const uint32_t last = sb.n_words - 1;
  const uint32_t* wp = sb.words;
  // refill queue: words are requested four refills before they are used
  uint64_t buf = (uint64_t)wp[0] | ((uint64_t)wp[min(1u, last)] << 32);
  uint32_t nb = 64;
  uint32_t q0 = wp[min(2u, last)], q1 = wp[min(3u, last)], q2 = wp[min(4u, last)], q3 = wp[min(5u, last)];
  uint32_t next = 6;
#define GMP_REFILL()                                   \
  do {                                                 \
    if (nb <= 32) {                                    \
      buf |= (uint64_t)q0 << nb;                       \
      nb += 32;                                        \
      q0 = q1;                                         \
      q1 = q2;                                         \
      q2 = q3;                                         \
      q3 = wp[min(next, last)];                        \
      next++;                                          \
    }                                                  \
  } while (0)

  uint32_t used = 0, produced = 0, sc = 0, lc = 0, run = 0;
  for (;;) {
    GMP_REFILL();
    const uint32_t e = lut_ll[(uint32_t)buf & lmask];
    const uint32_t n = e & 31u, x = (e >> 5) & 15u;
    const uint32_t val = (e >> 16) + ((uint32_t)(buf >> n) & ((1u << x) - 1u));
    const uint32_t tb = n + x;
    buf >>= tb;
    nb -= tb;
    used += tb;
    if (n == 0) return kECODE;
    if (used > sb.bit_len) return kESUB;
    const uint32_t kind = (e >> 9) & 3u;
    if (kind == kKindLit) {
      if (lc >= sb.n_lit) return kESUB;
      sb.lit_out[lc++] = (uint8_t)val;
      run++;
      produced++;
    } else if (kind == kKindLen) {
      GMP_REFILL();
      const uint32_t d = lut_d[(uint32_t)buf & lmask];
      const uint32_t dn = d & 31u, dx = (d >> 5) & 15u;
      const uint32_t dist = (d >> 16) + ((uint32_t)(buf >> dn) & ((1u << dx) - 1u));
      const uint32_t tdb = dn + dx;
      buf >>= tdb;
      nb -= tdb;
      used += tdb;
      if (dn == 0) return kECODE;
      if (used > sb.bit_len) return kESUB;
      if (val > max_match) return kELEN;
      if (dist > window || dist > sb.raw_off + produced) return kEDIST;
      if (sc >= sb.n_seq) return kESUB;
      sb.seq_out[sc++] = make_uint2(run, val | (dist << 16));
      run = 0;
      produced += val;
    } else if (kind == kKindEnd) {
      if (run) {
        if (sc >= sb.n_seq) return kESUB;
        sb.seq_out[sc++] = make_uint2(run, 0u);
      }
      if (used != sb.bit_len || sc != sb.n_seq || lc != sb.n_lit || produced != sb.raw_len) return kESUB;
      return kOK;
    } else {
      return kECODE;
    }
  }
#undef GMP_REFILL
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
  if (dist >= len || dist >= 16) {
    // each 16-byte source chunk ends at or before its destination chunk
    for (uint32_t k = 0; k < len; k += 16) ring_write(ring, dst + k, ring_read16(ring, src + k), min(16u, len - k));
    return;
  }
  // dist < 16 and overlapping: the first min(len, 16) bytes one at a time,
  // then whole periods: the output repeats with period p16 = dist * (16 / dist).
  const uint32_t head = min(len, 16u);
  for (uint32_t k = 0; k < head; k++) ring[(dst + k) & kRingMask] = ring[(src + k) & kRingMask];
  if (len <= 16) return;
  const uint32_t p16 = dist * (16u / dist);
  const uint4 v = ring_read16(ring, dst);
  for (uint32_t k = p16; k < len; k += p16) ring_write(ring, dst + k, v, min(16u, len - k));
}

__device__ __forceinline__ uint4 gload16(const uint8_t* p) {
  uint4 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

// Flush window bytes [flushed, upto) to HBM: whole 16-byte chunks once a
// full 1 KiB is pending, everything when final.
__device__ __forceinline__ void flush_window(const uint8_t* ring, uint8_t* out, uint32_t& flushed, uint32_t upto,
                                             bool final_flush, uint32_t lane, uint32_t raw_len) {
  upto = min(upto, raw_len);  // never past the block's output
  if (!final_flush && upto - flushed < kFlushChunk) return;
  const uint32_t end = final_flush ? upto : (upto & ~15u);
  for (uint32_t p = flushed + lane * 16; p < end; p += kFlushChunk) {
    if (p + 16 <= end) {
      uint4 v;
      __builtin_memcpy(&v, ring + (p & kRingMask), 16);
      __builtin_memcpy(out + p, &v, 16);
    } else {
      for (uint32_t q = p; q < end; q++) out[q] = ring[q & kRingMask];
    }
  }
  flushed = end;
}

// ---------------------------------------------------------------- A3-A6
struct LzArgs {
  const uint2* seqs;
  const uint8_t* lits;
  uint8_t* out;
  uint32_t n_seq, raw_len;
  bool single_pass;
  uint8_t* rounds;
};

__device__ void resolve_block(uint8_t* ring, const LzArgs& a) {
  const uint32_t lane = lane_id();
  uint32_t carry_lit = 0, carry_out = 0, flushed = 0;
  uint32_t g = 0;
  uint2 rec_next = make_uint2(0u, 0u);
  if (lane < a.n_seq) rec_next = a.seqs[lane];
  for (uint32_t g0 = 0; g0 < a.n_seq; g0 += 64, g++) {
    const uint32_t j = g0 + lane;
    const bool valid = j < a.n_seq;
    uint2 rec = rec_next;
    if (g0 + 64 + lane < a.n_seq) rec_next = a.seqs[g0 + 64 + lane];  // next group's records
    uint32_t L = valid ? rec.x : 0u;
    const uint32_t M = valid ? (rec.y & 0xFFFFu) : 0u;
    const uint32_t D = valid ? (rec.y >> 16) : 0u;
    // A3: two exclusive prefix sums over the group's sequences
    const uint32_t inc_lit = wave_incl_scan(L);
    const uint32_t inc_out = wave_incl_scan(L + M);
    uint32_t lsrc = carry_lit + inc_lit - L;
    uint32_t pos = carry_out + inc_out - (L + M);
    const uint32_t end = pos + L + M;
    const uint32_t m_cnt = min(64u, a.n_seq - g0);
    uint32_t rounds = 0;
    bool split = false;
    uint32_t lo = 0;
    while (lo < m_cnt) {
      uint32_t base = readlane(pos, lo);
      {
        // a literal run too long for the window is streamed through it first
        uint32_t Llo = readlane(L, lo), Mlo = readlane(M, lo), slo = readlane(lsrc, lo);
        while (Llo + Mlo > kSpanCap) {
          const uint32_t P = kSpanCap / 2;
          for (uint32_t k = lane * 16; k < P; k += 1024)
            ring_write(ring, base + k, gload16(a.lits + slo + k), min(16u, P - k));
          flush_window(ring, a.out, flushed, base + P, false, lane, a.raw_len);
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
      if (hi < m_cnt) split = true;
      const bool active = lane >= lo && lane < hi;
      // A4: literal strings into the window
      if (active)
        for (uint32_t k = 0; k < L; k += 16) ring_write(ring, pos + k, gload16(a.lits + lsrc + k), min(16u, L - k));
      const uint32_t dst = pos + L;
      bool pending = active && M > 0;
      if (a.single_pass) {
        // A6: no back-reference of the group depends on another (DE)
        if (__ballot(pending)) rounds += 1;
        if (pending) copy_match(ring, dst, M, D);
      } else {
        // A5: Multi-Round Resolution
        const uint32_t need_end = dst - D + min(M, D);
        for (;;) {
          const uint64_t votes = __ballot(pending);
          if (votes == 0) break;
          const uint32_t hwm = readlane(dst, (uint32_t)__builtin_ctzll(votes));
          if (pending && need_end <= hwm) {
            copy_match(ring, dst, M, D);
            pending = false;
          }
          rounds++;
        }
      }
      const uint32_t sub_end = readlane(end, hi - 1);
      flush_window(ring, a.out, flushed, sub_end, false, lane, a.raw_len);
      lo = hi;
    }
    if (a.rounds && lane == 0) a.rounds[g] = (uint8_t)(min(rounds, 127u) | (split ? 0x80u : 0u));
    carry_lit += readlane(inc_lit, 63);
    carry_out += readlane(inc_out, 63);
  }
  flush_window(ring, a.out, flushed, a.raw_len, true, lane, a.raw_len);
}

// ---------------------------------------------------------------- kernel
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) {
  uint32_t v;
  __builtin_memcpy(&v, p, 4);
  return v;
}

// kMode: GMPK_MODE_AUTO (per block from its header), GMPK_MODE_MRR or GMPK_MODE_DE.
template <int kThreads, int kMode>
__device__ void inflate_block(Shared& sh, const DevJob& job, uint32_t flags) {
  const uint32_t t = threadIdx.x;
  if (t == 0) sh.err = 0;
  __syncthreads();
  const uint8_t* blk = job.comp;
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
      if ((uint64_t)kHdrBytes + (uint64_t)kIdxBytes * n_sub + 16 + payload > job.comp_len) err = kEFORMAT;
      else if (n_seq != job.n_seq || n_lit != job.n_lit) err = kEFORMAT;
      else if (raw_len != job.out_len) err = kESIZE;
    }
  }
  const bool de_ok = mode == 1 && (group % 64) == 0;
  if (err == kOK && kMode == GMPK_MODE_DE && !de_ok) err = kEINVAL;
  const bool single_pass = (kMode == GMPK_MODE_DE) || (kMode == GMPK_MODE_AUTO && de_ok);
  if (err != kOK) {
    if (t == 0) *job.status = err;
    return;
  }
  if (n_sub == 0) {
    // an empty block: nothing to decode
    if (t == 0) *job.status = (raw_len == 0 && n_seq == 0 && n_lit == 0 && payload == 0) ? kOK : kEFORMAT;
    return;
  }
  // ---- A1: code lengths and lookup tables
  for (uint32_t i = t; i < kNumLL + kNumD; i += kThreads) sh.lens[i] = (blk[32 + i / 2] >> ((i & 1) * 4)) & 15;
  __syncthreads();
  if (sh.lens[256] == 0) set_err(sh, kECODE);
  uint32_t* lut_ll = sh.lut;
  uint32_t* lut_d = sh.lut + kLutSize;
  build_table<kThreads>(sh, sh.lens, kNumLL, lmax, lut_ll, false);
  __syncthreads();
  build_table<kThreads>(sh, sh.lens + kNumLL, kNumD, lmax, lut_d, true);
  __syncthreads();
  if (sh.err) {
    if (t == 0) *job.status = sh.err;
    return;
  }
  // ---- A0/A2: sub-block offsets by prefix sums over the index, then decode
  const uint8_t* idx = blk + kHdrBytes;
  const uint32_t* payload_words = reinterpret_cast<const uint32_t*>(blk + kHdrBytes + kIdxBytes * n_sub + 16);
  uint2* ws_seq = reinterpret_cast<uint2*>(job.ws);
  uint8_t* ws_lit = job.ws + 8ull * n_seq;
  uint32_t carry[4] = {0, 0, 0, 0};
  for (uint32_t c = 0; c < n_sub; c += kThreads) {
    const uint32_t s = c + t;
    uint32_t bit_len = 0, sseq = 0, slit = 0, sraw = 0;
    if (s < n_sub) {
      uint4 e;
      __builtin_memcpy(&e, idx + kIdxBytes * s, 16);
      bit_len = e.x;
      sseq = e.y;
      slit = e.z;
      sraw = e.w;
    }
    const uint32_t nwords = (uint32_t)(((uint64_t)bit_len + 31) >> 5);
    uint32_t v[4] = {nwords, sseq, slit, sraw}, tot[4];
    block_excl_scan4<kThreads>(sh, v, tot);
    // offsets may wrap for corrupt indexes; the sums are checked below
    const uint32_t word_off = carry[0] + v[0], seq_off = carry[1] + v[1], lit_off = carry[2] + v[2],
                   raw_off = carry[3] + v[3];
#pragma unroll
    for (int i = 0; i < 4; i++) carry[i] += tot[i];
    if (s < n_sub) {
      int e = kOK;
      const uint64_t words_end = (uint64_t)word_off + nwords;
      if (words_end * 4 > payload || (uint64_t)seq_off + sseq > n_seq || (uint64_t)lit_off + slit > n_lit ||
          (uint64_t)raw_off + sraw > raw_len) {
        e = kEFORMAT;
      } else {
        SubBlock sb;
        sb.words = payload_words + word_off;
        sb.n_words = nwords;
        sb.bit_len = bit_len;
        sb.n_seq = sseq;
        sb.n_lit = slit;
        sb.raw_len = sraw;
        sb.raw_off = raw_off;
        sb.seq_out = ws_seq + seq_off;
        sb.lit_out = ws_lit + lit_off;
        e = decode_subblock(sb, lut_ll, lut_d, lmax, window, max_match);
      }
      if (e != kOK) set_err(sh, e);
    }
  }
  // the index must account for the whole payload and the header counts
  if (t == 0 && (carry[0] * 4ull != payload || carry[1] != n_seq || carry[2] != n_lit || carry[3] != raw_len))
    set_err(sh, kEFORMAT);
  __syncthreads();  // workspace writes of all lanes are visible after this barrier
  if (sh.err) {
    if (t == 0) *job.status = sh.err;
    return;
  }
  if (t >= 64) return;
  // ---- A3-A6 on wavefront 0
  LzArgs a;
  a.seqs = ws_seq;
  a.lits = ws_lit;
  a.out = job.out;
  a.n_seq = n_seq;
  a.raw_len = raw_len;
  a.single_pass = single_pass;
  a.rounds = (flags & GMPK_FLAG_STATS) ? job.rounds : nullptr;
  resolve_block(sh.ring, a);
  if (t == 0) *job.status = kOK;
}

template <int kThreads, int kMode>
__global__ __launch_bounds__(kThreads) void inflate_kernel(const DevJob* __restrict__ jobs, uint32_t n_jobs,
                                                           uint32_t flags) {
  __shared__ Shared sh;
  if (blockIdx.x >= n_jobs) return;
  const DevJob job = jobs[blockIdx.x];
  inflate_block<kThreads, kMode>(sh, job, flags);
}

// Persistent form: workgroups take block indices from a device counter until
// the job table is exhausted; every workgroup exits once it draws an index
// past the end.
template <int kThreads, int kMode>
__global__ __launch_bounds__(kThreads) void inflate_persistent_kernel(const DevJob* __restrict__ jobs,
                                                                      uint32_t n_jobs, uint32_t flags,
                                                                      uint32_t* __restrict__ queue) {
  __shared__ Shared sh;
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t j = next;
    __syncthreads();
    if (j >= n_jobs) return;
    const DevJob job = jobs[j];
    inflate_block<kThreads, kMode>(sh, job, flags);
    __syncthreads();
  }
}

// resets the persistent queue head (a kernel, so that graph captures hold no memset node)
__global__ void reset_queue_kernel(uint32_t* queue) { *queue = 0; }

}  // namespace gmpk

namespace gmpk {

template <int kThreads, int kMode>
void launch_one(const DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t persistent, uint32_t workgroups,
                uint32_t* d_queue, hipStream_t stream) {
  if (persistent) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, stream, d_queue);
    hipLaunchKernelGGL((inflate_persistent_kernel<kThreads, kMode>), dim3(workgroups), dim3(kThreads), 0, stream,
                       d_jobs, n_jobs, flags, d_queue);
  } else {
    hipLaunchKernelGGL((inflate_kernel<kThreads, kMode>), dim3(n_jobs), dim3(kThreads), 0, stream, d_jobs, n_jobs,
                       flags);
  }
}

template <int kThreads>
int launch_mode(const DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t persistent, uint32_t workgroups,
                uint32_t* d_queue, hipStream_t stream) {
  switch (flags & GMPK_MODE_MASK) {
    case GMPK_MODE_AUTO: launch_one<kThreads, GMPK_MODE_AUTO>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); return 0;
    case GMPK_MODE_MRR: launch_one<kThreads, GMPK_MODE_MRR>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); return 0;
    case GMPK_MODE_DE: launch_one<kThreads, GMPK_MODE_DE>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); return 0;
    default: return -1;
  }
}

}  // namespace gmpk

extern "C" int gmpk_launch(const gmpk::DevJob* d_jobs, uint32_t n_jobs, uint32_t flags, uint32_t waves,
                           uint32_t persistent, uint32_t workgroups, uint32_t* d_queue, hipStream_t stream) {
  using namespace gmpk;
  if (n_jobs == 0) return 0;
  if (persistent && workgroups == 0) return -1;
  int rc;
  switch (waves) {
    case 1: rc = launch_mode<64>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); break;
    case 2: rc = launch_mode<128>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); break;
    case 4: rc = launch_mode<256>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); break;
    case 8: rc = launch_mode<512>(d_jobs, n_jobs, flags, persistent, workgroups, d_queue, stream); break;
    default: return -1;
  }
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
