// Gompresso/Byte compression on the GPU, with optional Dependency Elimination.
//
// The paper compresses each data block with a group of threads that find
// matches in parallel, then writes the tokens in a byte-level encoding
// (section "Parallel Compression"); with Dependency Elimination the matches
// of each group of sequences only read bytes that precede the group's first
// back-reference (section "Dependency Elimination (DE)" and its compression
// algorithm).  One workgroup compresses one block:
//
//   W  the first eight of the workgroup's sixteen wavefronts each walk one
//      eighth of the block, 64 positions at a time, through a hash table of
//      3-byte keys in LDS (preceded by the window before their eighth, so
//      every position sees up to the window's history): every position gets
//      the most recent position with its key's hash in an earlier group of
//      64, its candidate (the candidates form hash chains);
//   L  the workgroup takes 1024 positions at a time; each thread walks its
//      position's chain (up to kChain candidates within the window) in an
//      LDS ring of the candidates' links, then loads the eight bytes at every
//      candidate and at distances 1-4 at once, extends the candidates that
//      agree on all eight together, eight bytes a round, and keeps the
//      longest match (the first of equals);
//   P  each wavefront parses one sixteenth of the block greedily (a block
//      under 64 KiB: wavefront 0 all of it): a literal run ends at the first
//      position whose match (cut at the part's end, and under the DE rule) is
//      at least 3 bytes long, found 64 positions at a time with a ballot; a
//      run that reaches 255 bytes becomes a sequence of its own.  Under DE a
//      part's records are padded with empty ones to a multiple of 64, so the
//      next part starts a group.  The parts' records are then put in order;
//   A  the whole workgroup writes the literal bytes after the records, from
//      prefix sums over the records, then the header and zero padding.
//
// The output is the byte-level block format the decoder reads.  All
// arithmetic is integer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "compress.h"

namespace gmpc {

#define GMEM __attribute__((address_space(1)))

constexpr uint32_t kWaves = 8;                                    // W's walkers
constexpr uint32_t kBlockWaves = 16, kThreads = 64 * kBlockWaves;  // the workgroup
constexpr uint32_t kParts = kBlockWaves;                           // P's parts
constexpr uint32_t kHashBits = 12, kHashSize = 1u << kHashBits;  // per walker
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kChain = 8;                  // candidates measured per position
constexpr uint32_t kSegMin = 65536;             // blocks at least this long are parsed in kParts parts
constexpr uint32_t kMagicByte = 0x59504D47u;    // 'GMPY'
constexpr int kOK = 0;

__shared__ __attribute__((aligned(16))) uint32_t s_lds[kWaves * kHashSize];  // hash tables, then the match ring
struct CMisc {
  uint32_t seg_seq[kParts], seg_lit[kParts];  // records and literal bytes of each part's parse
  uint32_t wave_sum[2][kBlockWaves];
};
__shared__ CMisc s_cm;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}
// exclusive prefix sums of two values over the workgroup
__device__ void block_excl_scan2(uint32_t& a, uint32_t& b, uint32_t& tot_a, uint32_t& tot_b) {
  const uint32_t w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  if (lane == 63) {
    s_cm.wave_sum[0][w] = ia;
    s_cm.wave_sum[1][w] = ib;
  }
  __syncthreads();
  uint32_t pa = 0, pb = 0, ta = 0, tb = 0;
  for (uint32_t k = 0; k < kBlockWaves; k++) {
    const uint32_t x = s_cm.wave_sum[0][k], y = s_cm.wave_sum[1][k];
    if (k < w) {
      pa += x;
      pb += y;
    }
    ta += x;
    tb += y;
  }
  a = pa + ia - a;
  b = pb + ib - b;
  tot_a = ta;
  tot_b = tb;
  __syncthreads();
}

// Loads of 4 and 8 bytes at any byte address (the target reads global
// memory unaligned).
typedef uint32_t __attribute__((aligned(1))) u32u;
typedef uint64_t __attribute__((aligned(1))) u64u;

// the 3-byte key at p (p + 3 <= n)
__device__ __forceinline__ uint32_t key3(const GMEM uint8_t* in, uint32_t p, uint32_t n) {
  if (p + 4 <= n) return *(const GMEM u32u*)(in + p) & 0xFFFFFFu;
  return (uint32_t)in[p] | ((uint32_t)in[p + 1] << 8) | ((uint32_t)in[p + 2] << 16);
}
__device__ __forceinline__ uint32_t hash_key(uint32_t k) { return (k * 2654435761u) >> (32 - kHashBits); }

// ---------------------------------------------------------------- W
// Wavefront w's walk: the window before its eighth only fills its table;
// over its eighth every position also records its candidate.
__device__ void walk(const GMEM uint8_t* in, uint32_t n, uint32_t window, GMEM uint32_t* cand, uint32_t w) {
  const uint32_t lane = lane_id();
  uint32_t* table = s_lds + w * kHashSize;
  for (uint32_t i = lane; i < kHashSize; i += 64) table[i] = 0;  // buckets hold position + 1 (0: empty)
  const uint32_t part = ((n + kWaves - 1) / kWaves + 63) & ~63u;
  const uint32_t lo = min(n, w * part), hi = min(n, lo + part);
  const uint32_t start = lo > window ? ((lo - window) & ~63u) : 0u;
  for (uint32_t c = start; c < hi; c += 64) {
    const uint32_t p = c + lane;
    const bool has = p + 3 <= n;
    const uint32_t h = has ? hash_key(key3(in, p, n)) : 0u;
    const uint32_t b = has ? table[h] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (has) atomicMax(&table[h], p + 1);  // the most recent position of the 64 holds the bucket
    if (p >= lo && p < hi) cand[p] = b ? b - 1 : kNone;
  }
}

// ---------------------------------------------------------------- L
// Candidates' links, for the chain walks of L, live in an LDS ring (the hash
// tables' space) of the last kRingC positions, as distances back (16 bits;
// 0: none).  The workgroup measures kStep positions at a time (kPer per
// thread).  A wavefront may store the next positions' links while another
// still walks chains of the current ones, so a chain reaches back at most
// kRingC - 2 kStep positions: the slots being overwritten are never read.
constexpr uint32_t kPer = 1;
constexpr uint32_t kStep = kPer * kThreads;
constexpr uint32_t kRingC = 2 * kWaves * kHashSize;
constexpr uint32_t kReach = kRingC - 2 * kStep;
constexpr uint32_t kCand = 4 + kChain;  // distances 1-4, then the chain
static_assert(kRingC * sizeof(uint16_t) <= sizeof(s_lds), "the ring fits the hash tables' space");
static_assert(kReach >= 32768, "a chain reaches a 32 KiB window");
__device__ __forceinline__ uint16_t* link_ring() { return reinterpret_cast<uint16_t*>(s_lds); }

// The best matches at kPer positions: length | distance << 9 (0 when none of
// 3 bytes or more).  Distances 1-4 first (runs and short periods), then up to
// kChain candidates of the hash chain; the longest wins, the first of
// equals.  The chains are walked in LDS first; then the eight bytes at every
// candidate of every position are loaded at once, so the loads overlap.  The
// candidates whose eight bytes all agree are then extended together, eight
// bytes a round with every such candidate's load in flight at once, so a
// wavefront waits for one load per round, not one per candidate and round.
__device__ __forceinline__ void best_matches(const GMEM uint8_t* in, uint32_t n, uint32_t window,
                                             uint32_t max_match, const uint32_t (&p)[kPer],
                                             uint32_t (&res)[kPer]) {
  const uint32_t reach = min(window, kReach);
  uint32_t cs[kPer][kCand], cap[kPer];
  bool ok[kPer][kCand], live[kPer];
  uint32_t c[kPer];
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const bool has = p[i] + 3 <= n;
    cap[i] = has ? min(max_match, n - p[i]) : 0u;
#pragma unroll
    for (uint32_t d = 1; d <= 4; d++) {
      ok[i][d - 1] = has && d <= p[i] && d <= window;
      cs[i][d - 1] = ok[i][d - 1] ? p[i] - d : p[i];
    }
    const uint32_t l = has ? link_ring()[p[i] % kRingC] : 0u;
    c[i] = l ? p[i] - l : kNone;
    live[i] = has;
  }
#pragma unroll
  for (uint32_t k = 0; k < kChain; k++) {
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
      live[i] = live[i] && c[i] != kNone && c[i] < p[i] && p[i] - c[i] <= reach;
      ok[i][4 + k] = live[i] && p[i] - c[i] > 4;
      cs[i][4 + k] = ok[i][4 + k] ? c[i] : p[i];
      const uint32_t l = live[i] ? link_ring()[c[i] % kRingC] : 0u;
      c[i] = l ? c[i] - l : kNone;
    }
  }
  uint64_t head[kPer], v[kPer][kCand];
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const bool wide = cap[i] >= 8;  // then every candidate's eight bytes lie inside the block
    head[i] = wide ? *(const GMEM u64u*)(in + p[i]) : 0ull;
    // distances 1-4 from the eight bytes before p and the eight at p
    const bool near = wide && p[i] >= 8;
    const uint64_t before = near ? *(const GMEM u64u*)(in + p[i] - 8) : 0ull;
#pragma unroll
    for (uint32_t k = 0; k < kCand; k++) {
      const bool from_regs = k < 4 && near;  // distance k + 1
      v[i][k] = !(wide && ok[i][k]) ? 0ull
                : from_regs        ? (before >> (8 * (7 - k))) | (head[i] << (8 * (k + 1)))
                                   : *(const GMEM u64u*)(in + cs[i][k]);
    }
  }
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    uint32_t len[kCand];
    if (cap[i] >= 8) {
      uint32_t more = 0;  // bit k: candidate k agrees on every byte so far
#pragma unroll
      for (uint32_t k = 0; k < kCand; k++) {
        const uint64_t x = v[i][k] ^ head[i];
        len[k] = !ok[i][k] ? 0u : x ? (uint32_t)__builtin_ctzll(x) >> 3 : 8u;
        more |= (ok[i][k] && !x ? 1u : 0u) << k;
      }
      for (uint32_t off = 8; more && off < cap[i]; off += 8) {
        if (p[i] + off + 8 <= n) {
          // eight bytes at p + off and at every candidate still agreeing
          // (candidates lie before p, so all of them are inside the block)
          const uint64_t h = *(const GMEM u64u*)(in + p[i] + off);
          uint64_t w[kCand];
#pragma unroll
          for (uint32_t k = 0; k < kCand; k++)
            w[k] = (more >> k) & 1u ? *(const GMEM u64u*)(in + cs[i][k] + off) : 0ull;
#pragma unroll
          for (uint32_t k = 0; k < kCand; k++) {
            const uint64_t y = w[k] ^ h;
            if ((more >> k) & 1u) {
              len[k] = y ? off + ((uint32_t)__builtin_ctzll(y) >> 3) : off + 8;
              if (y) more &= ~(1u << k);
            }
          }
        } else {
          // the block's last bytes, one at a time
#pragma unroll
          for (uint32_t k = 0; k < kCand; k++) {
            if (!((more >> k) & 1u)) continue;
            uint32_t L = off;
            while (L < cap[i] && in[cs[i][k] + L] == in[p[i] + L]) L++;
            len[k] = L;
          }
          more = 0;
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < kCand; k++) len[k] = min(len[k], cap[i]);
    } else {
#pragma unroll
      for (uint32_t k = 0; k < kCand; k++) {
        uint32_t L = 0;
        if (ok[i][k])
          while (L < cap[i] && in[cs[i][k] + L] == in[p[i] + L]) L++;
        len[k] = L;
      }
    }
    uint32_t bl = 0, bd = 0;
#pragma unroll
    for (uint32_t k = 0; k < kCand; k++) {
      if (ok[i][k] && len[k] > bl) {
        bl = len[k];
        bd = p[i] - cs[i][k];
      }
    }
    res[i] = bl >= 3 ? (bl | (bd << 9)) : 0u;
  }
}
// best[p] for every position, kStep positions at a time: each thread stores
// its position's link (its candidate was loaded during the previous
// positions' walks), then, after one barrier, measures it.
__device__ void measure(const GMEM uint8_t* in, uint32_t n, uint32_t window, uint32_t max_match,
                        const GMEM uint32_t* cand, GMEM uint32_t* best) {
  static_assert(kPer == 1, "one position per thread");
  const uint32_t t = threadIdx.x;
  uint32_t next = t < n ? cand[t] : kNone;  // the candidate of the thread's next position (before it)
  for (uint32_t P = 0; P < n; P += kStep) {
    const uint32_t p = P + t;
    if (p < n) link_ring()[p % kRingC] = (uint16_t)(next != kNone && p - next < 65536u ? p - next : 0u);
    __syncthreads();
    next = p + kStep < n ? cand[p + kStep] : kNone;
    uint32_t q[kPer] = {p}, res[kPer];
    best_matches(in, n, window, max_match, q, res);
    if (p < n) best[p] = res[0];
  }
}

// ---------------------------------------------------------------- P
// The greedy parse of positions [lo, hi) by one wavefront, from best[]: a
// literal run ends at the first position whose match (cut to end at hi, and
// under the DE rule) is at least 3 bytes long; a run that reaches 255 bytes
// becomes a sequence of its own.  DE: every match of a group of 64 sequences
// must end at or before the group's high-water mark, which is the cursor
// while the group has no back-reference yet, then the destination of its
// first one (a match is cut to end there; under 3 bytes it is no match).
// The records go to rec[0 ..); with pad the count is rounded up to a
// multiple of 64 with empty records, so that the next part starts a group.
__device__ void parse(const GMEM uint32_t* best, uint32_t lo, uint32_t hi, uint32_t de, bool pad,
                      GMEM uint32_t* rec, uint32_t& n_seq_out, uint32_t& n_lit_out) {
  const uint32_t lane = lane_id();
  uint32_t pos = lo, lit_start = lo, n_seq = 0, n_lit = 0, hwm = 0;
  bool frozen = false;
  // records collect one per lane and leave 64 at a time (256 bytes)
  uint32_t rbuf = 0;
  auto emit = [&](uint32_t lit, uint32_t m, uint32_t d) {
    const uint32_t r = lit | ((m ? m - 3 : 0u) << 8) | (d << 16);
    rbuf = lane == (n_seq & 63u) ? r : rbuf;
    if ((n_seq & 63u) == 63u) rec[n_seq - 63 + lane] = rbuf;
    n_seq++;
    n_lit += lit;
    if (n_seq % 64 == 0) frozen = false;
  };
  while (pos < hi) {
    // the positions this step looks at: up to 64, not past the point where
    // the literal run reaches 255 bytes
    const uint32_t end = min(min(pos + 64, hi), lit_start + 255);
    const uint32_t q = pos + lane;
    uint32_t L = 0, d = 0;
    if (q < end) {
      const uint32_t b = best[q];
      L = min(b & 511u, hi - q);
      d = b >> 9;
    }
    // every sequence whose match starts in [pos, end), from these 64 entries:
    // the next match is the first position at or after the cursor whose
    // match is at least 3 bytes long.  The lanes that hold such a match are
    // one mask, worked out again only when the DE state changes (a group's
    // first match, a group's end).
    uint32_t cap = 0;
    auto matches = [&]() -> uint64_t {
      cap = L;
      if (de && L) {
        const uint32_t lim = frozen ? hwm : q;  // the cursor would be at q
        const uint32_t src = q - d;
        cap = lim > src ? min(L, lim - src) : 0u;
      }
      return __ballot(cap >= 3);
    };
    uint64_t ok = matches();
    uint32_t cur = pos;
    for (;;) {
      const uint64_t from = ok & (~0ull << (cur - pos));  // cur - pos < 64 here
      if (!from) {
        cur = end;
        break;
      }
      const uint32_t f = (uint32_t)__builtin_ctzll(from);
      const uint32_t qm = pos + f, m = readlane(cap, f), dm = readlane(d, f);
      bool changed = false;
      if (de && !frozen) {
        frozen = true;
        hwm = qm;
        changed = true;
      }
      emit(qm - lit_start, m, dm);
      changed = changed || (de && !frozen);
      cur = qm + m;
      lit_start = cur;
      if (cur >= end) break;
      if (changed) ok = matches();
    }
    pos = cur;
    if (pos - lit_start == 255) {
      emit(255, 0, 0);
      lit_start = pos;
    }
  }
  if (pos > lit_start) emit(pos - lit_start, 0, 0);
  while (pad && (n_seq & 63u)) emit(0, 0, 0);
  if (lane < (n_seq & 63u)) rec[(n_seq & ~63u) + lane] = rbuf;
  n_seq_out = n_seq;
  n_lit_out = n_lit;
}

// ---------------------------------------------------------------- kernel
__global__ __launch_bounds__(kThreads) void compress_kernel(const CompressJob* __restrict__ jobs, uint32_t n_jobs,
                                                            CompressParams prm) {
  if (blockIdx.x >= n_jobs) return;
  const CompressJob job = jobs[blockIdx.x];
  const uint32_t t = threadIdx.x, wave = t >> 6, lane = lane_id();
  const GMEM uint8_t* in = (const GMEM uint8_t*)job.in;
  GMEM uint8_t* out = (GMEM uint8_t*)job.out;
  GMEM uint32_t* cand = (GMEM uint32_t*)job.ws;
  GMEM uint32_t* best = cand + ((job.in_len + 255) & ~255ull);
  const uint32_t n = (uint32_t)job.in_len;
  __syncthreads();
  // W
  if (wave < kWaves) walk(in, n, prm.window, cand, wave);
  __threadfence();
  __syncthreads();
  // L
  measure(in, n, prm.window, prm.max_match, cand, best);
  for (uint32_t p = n + t; p < ((n + 255) & ~255u); p += kThreads) best[p] = 0;  // staging reads whole KiBs
  __threadfence();
  __syncthreads();
  // P: a block of at least kSegMin bytes is parsed in kParts parts at once
  // (one per wavefront, into the candidate area, free after L; a match does
  // not cross a part's end), a shorter one by wavefront 0 alone; then the
  // parts' records go to the output, in order
  GMEM uint32_t* rec = (GMEM uint32_t*)(out + 32);
  const uint32_t parts = n >= kSegMin ? kParts : 1u;
  const uint32_t part = parts == 1 ? n : ((n + kParts - 1) / kParts + 63) & ~63u;
  const uint32_t lo = wave < parts ? min(n, wave * part) : n, hi = wave < parts ? min(n, lo + part) : n;
  if (wave < kParts) {
    uint32_t ns = 0, nl = 0;
    parse(best, lo, hi, prm.de, prm.de && wave + 1 < parts, cand + lo, ns, nl);
    if (lane == 0) {
      s_cm.seg_seq[wave] = ns;
      s_cm.seg_lit[wave] = nl;
    }
  }
  __threadfence();
  __syncthreads();
  uint32_t n_seq = 0, n_lit = 0;
  for (uint32_t w = 0; w < kParts; w++) {
    const uint32_t ns = s_cm.seg_seq[w];
    const GMEM uint32_t* src = cand + (w < parts ? min(n, w * part) : n);
    for (uint32_t i = t; i < ns; i += kThreads) rec[n_seq + i] = src[i];
    n_seq += ns;
    n_lit += s_cm.seg_lit[w];
  }
  __threadfence();
  __syncthreads();
  // A: literals after the records; the records' positions from prefix sums
  const uint64_t rec_bytes = (4ull * n_seq + 15) & ~15ull;
  GMEM uint8_t* lit_out = out + 32 + rec_bytes;
  uint32_t carry_pos = 0, carry_lit = 0;
  for (uint32_t c = 0; c < n_seq; c += kThreads) {
    const uint32_t i = c + t;
    const uint32_t r = i < n_seq ? rec[i] : 0u;
    const uint32_t lit = r & 0xFFu, d = r >> 16;
    const uint32_t m = d ? ((r >> 8) & 0xFFu) + 3 : 0u;
    uint32_t p = lit + m, l = lit, tp, tl;
    block_excl_scan2(p, l, tp, tl);
    const uint32_t src = carry_pos + p, dst = carry_lit + l;
    for (uint32_t k = 0; k < lit; k++) lit_out[dst + k] = in[src + k];
    carry_pos += tp;
    carry_lit += tl;
  }
  // zero padding after the records and after the literals (16 more bytes)
  for (uint64_t k = 4ull * n_seq + t; k < rec_bytes; k += kThreads) out[32 + k] = 0;
  const uint64_t lit_pad = ((n_lit + 15ull) & ~15ull) + 16;
  for (uint64_t k = n_lit + t; k < lit_pad; k += kThreads) lit_out[k] = 0;
  if (t == 0) {
    GMEM uint32_t* h = (GMEM uint32_t*)out;
    h[0] = kMagicByte;
    h[1] = 1u | ((prm.de ? 1u : 0u) << 8) | (64u << 16);  // version, mode, group 64, reserved 0
    h[2] = n;
    h[3] = prm.window;
    h[4] = prm.max_match;  // max_match, reserved 0
    h[5] = n_seq;
    h[6] = n_lit;
    h[7] = 0;
    *job.out_len = 32 + rec_bytes + lit_pad;
    *job.status = kOK;
  }
}

}  // namespace gmpc

extern "C" int gmpc_launch(const gmpc::CompressJob* d_jobs, uint32_t n_jobs, gmpc::CompressParams prm,
                           hipStream_t stream) {
  if (n_jobs == 0) return 0;
  hipLaunchKernelGGL(gmpc::compress_kernel, dim3(n_jobs), dim3(gmpc::kThreads), 0, stream, d_jobs, n_jobs, prm);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
