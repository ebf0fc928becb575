// Gompresso/Byte compression on the GPU, with optional Dependency Elimination.
//
// The paper compresses each data block with a group of threads that find
// matches in parallel, then writes the tokens in a byte-level encoding
// (section "Parallel Compression"); with Dependency Elimination the matches
// of each group of sequences only read bytes that precede the group's first
// back-reference (section "Dependency Elimination (DE)" and its compression
// algorithm).  One workgroup compresses one block:
//
//   W  eight wavefronts each walk one eighth of the block, 64 positions at a
//      time, through a hash table of 3-byte keys in LDS (preceded by the
//      window before their eighth, so every position sees up to the window's
//      history): every position gets the most recent earlier position with
//      its key's hash, its candidate (the candidates form hash chains);
//   L  every thread takes positions and measures the match at each candidate
//      of the chain (up to kChain of them, within the window) and at
//      distances 1-4, keeping the longest (the nearest on a tie);
//   P  one wavefront parses greedily from the block's start: a literal run
//      ends at the first position whose match (truncated under the DE rule)
//      is at least 3 bytes long, found 64 positions at a time with a ballot;
//      a run that reaches 255 bytes becomes a sequence of its own.  Another
//      wavefront streams the per-position matches into an LDS ring ahead of
//      it;
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

constexpr uint32_t kWaves = 8, kThreads = 64 * kWaves;
constexpr uint32_t kHashBits = 12, kHashSize = 1u << kHashBits;  // per walker
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kChain = 8;                  // candidates measured per position
constexpr uint32_t kRingEnt = 16384;            // staged per-position matches (64 KiB)
constexpr uint32_t kStageEnt = 256;             // entries per staging copy (1 KiB)
constexpr uint32_t kMagicByte = 0x59504D47u;    // 'GMPY'
constexpr uint64_t kSpinTicks = 100000000ull;   // about one second of the 100 MHz clock
constexpr int kOK = 0, kESTALL = -12;

__shared__ __attribute__((aligned(16))) uint32_t s_lds[kWaves * kHashSize];  // hash tables, then the match ring
struct CMisc {
  uint32_t staged;      // stager -> parser: entries of best[] present in the ring (absolute position)
  uint32_t consumed;    // parser -> stager: positions below this are no longer read
  uint32_t n_seq, n_lit;
  uint32_t abort;
  uint32_t wave_sum[2][kWaves];
};
__shared__ CMisc s_cm;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint32_t lds_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// a bounded wait: false once it has lasted about a second (or the block gave up)
struct Spin {
  uint64_t t0 = 0;
  __device__ bool pause() {
    if (__hip_atomic_load(&s_cm.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
    const uint64_t now = (uint64_t)wall_clock64();
    if (t0 == 0) t0 = now;
    else if (now - t0 > kSpinTicks) {
      __hip_atomic_store(&s_cm.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
  }
};

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
  for (uint32_t k = 0; k < kWaves; k++) {
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

__device__ __forceinline__ uint32_t key3(const GMEM uint8_t* in, uint32_t p) {
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
    const uint32_t h = has ? hash_key(key3(in, p)) : 0u;
    const uint32_t b = has ? table[h] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (has) atomicMax(&table[h], p + 1);  // the most recent position of the 64 holds the bucket
    if (p >= lo && p < hi) cand[p] = b ? b - 1 : kNone;
  }
}

// ---------------------------------------------------------------- L
__device__ __forceinline__ uint32_t match_len(const GMEM uint8_t* in, uint32_t p, uint32_t s, uint32_t cap) {
  uint32_t L = 0;
  while (L < cap && in[s + L] == in[p + L]) L++;
  return L;
}
// best[p] = length | distance << 9 (0 when no match of 3 bytes or more)
__device__ void measure(const GMEM uint8_t* in, uint32_t n, uint32_t window, uint32_t max_match,
                        const GMEM uint32_t* cand, GMEM uint32_t* best) {
  for (uint32_t p = threadIdx.x; p < n; p += kThreads) {
    uint32_t bl = 0, bd = 0;
    if (p + 3 <= n) {
      const uint32_t cap = min(max_match, n - p);
      // short distances first (runs and short periods), then the hash chain
      for (uint32_t d = 1; d <= 4 && d <= p && d <= window; d++) {
        if (bl >= cap) break;
        const uint32_t L = match_len(in, p, p - d, cap);
        if (L > bl) {
          bl = L;
          bd = d;
        }
      }
      uint32_t c = cand[p];
      for (uint32_t k = 0; k < kChain && c != kNone && c < p && p - c <= window && bl < cap; k++) {
        if (p - c > 4) {
          const uint32_t L = match_len(in, p, c, cap);
          if (L > bl) {
            bl = L;
            bd = p - c;
          }
        }
        c = cand[c];
      }
    }
    best[p] = bl >= 3 ? (bl | (bd << 9)) : 0u;
  }
}

// ---------------------------------------------------------------- P
// The stager wavefront keeps best[] entries [consumed, consumed + kRingEnt)
// in the LDS ring, 1 KiB per copy.
__device__ void stage_matches(const GMEM uint32_t* best, uint32_t n) {
  const uint32_t lane = lane_id();
  uint32_t staged = 0;
  Spin sp;
  while (staged < n) {
    const uint32_t cons = lds_acquire(&s_cm.consumed);
    if (cons == kNone) return;  // the parser has finished
    // up to four copies of 256 entries: lane l moves entries 4l..4l+3 of
    // each (16 bytes; best[] is padded to 256 entries); loads first
    uint32_t k = 0;
    uint4 v[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
      const uint32_t s0 = staged + j * kStageEnt;
      if (k == j && s0 < n && s0 + kStageEnt <= cons + kRingEnt) {
        const GMEM uint32_t* q = best + s0 + 4 * lane;
        v[j] = make_uint4(q[0], q[1], q[2], q[3]);
        k++;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; j++)
      if (j < k) *(uint4*)&s_lds[(staged + j * kStageEnt + 4 * lane) % kRingEnt] = v[j];
    staged += k * kStageEnt;
    const bool issued = k > 0;
    if (issued) {
      __builtin_amdgcn_s_waitcnt(0);
      lds_release(&s_cm.staged, min(staged, n));
      sp = Spin();
    } else if (!sp.pause()) {
      return;
    }
  }
}

struct ParseOut {
  GMEM uint32_t* rec;  // records, one u32 each
  uint32_t n_seq, n_lit;
};

// The greedy parse (wavefront 0).  DE: every match of a group of 64
// sequences must end at or before the group's high-water mark, which is the
// cursor while the group has no back-reference yet, then the destination of
// its first one (a match is cut to end there; under 3 bytes it is no match).
__device__ bool parse(uint32_t n, uint32_t de, GMEM uint32_t* rec, uint32_t& n_seq_out, uint32_t& n_lit_out) {
  const uint32_t lane = lane_id();
  uint32_t pos = 0, lit_start = 0, n_seq = 0, n_lit = 0, hwm = 0, staged = 0;
  bool frozen = false;
  Spin sp;
  auto emit = [&](uint32_t lit, uint32_t m, uint32_t d) {
    if (lane == 0) rec[n_seq] = lit | ((m ? m - 3 : 0u) << 8) | (d << 16);
    n_seq++;
    n_lit += lit;
    if (n_seq % 64 == 0) frozen = false;
  };
  while (pos < n) {
    // the positions this step looks at: up to 64, not past the point where
    // the literal run reaches 255 bytes (a sequence of its own)
    const uint32_t end = min(min(pos + 64, n), lit_start + 255);
    while (staged < end) {
      staged = lds_acquire(&s_cm.staged);
      if (staged >= end) break;
      if (!sp.pause()) return false;
    }
    sp = Spin();
    const uint32_t q = pos + lane;
    uint32_t cap = 0, d = 0;
    if (q < end) {
      const uint32_t b = s_lds[q % kRingEnt];
      const uint32_t L = b & 511u;
      d = b >> 9;
      cap = L;
      if (de && L) {
        const uint32_t lim = frozen ? hwm : q;  // the cursor would be at q
        const uint32_t src = q - d;
        cap = lim > src ? min(L, lim - src) : 0u;
      }
    }
    const uint64_t ok = __ballot(cap >= 3);
    if (!ok) {
      pos = end;
      if (pos - lit_start == 255) {
        emit(255, 0, 0);
        lit_start = pos;
      }
      lds_release(&s_cm.consumed, pos);
      continue;
    }
    const uint32_t f = (uint32_t)__builtin_ctzll(ok);
    const uint32_t qm = pos + f, m = readlane(cap, f), dm = readlane(d, f);
    if (de && !frozen) {
      frozen = true;
      hwm = qm;
    }
    emit(qm - lit_start, m, dm);
    pos = qm + m;
    lit_start = pos;
    lds_release(&s_cm.consumed, pos);
  }
  if (pos > lit_start) emit(pos - lit_start, 0, 0);
  n_seq_out = n_seq;
  n_lit_out = n_lit;
  return true;
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
  if (t == 0) {
    s_cm.staged = 0;
    s_cm.consumed = 0;
    s_cm.abort = 0;
    s_cm.n_seq = 0;
    s_cm.n_lit = 0;
  }
  __syncthreads();
  // W
  walk(in, n, prm.window, cand, wave);
  __threadfence();
  __syncthreads();
  // L
  measure(in, n, prm.window, prm.max_match, cand, best);
  for (uint32_t p = n + t; p < ((n + 255) & ~255u); p += kThreads) best[p] = 0;  // staging reads whole KiBs
  __threadfence();
  __syncthreads();
  // P
  GMEM uint32_t* rec = (GMEM uint32_t*)(out + 32);
  bool ok = true;
  if (wave == 0) {
    uint32_t ns = 0, nl = 0;
    ok = parse(n, prm.de, rec, ns, nl);
    if (lane == 0) {
      s_cm.n_seq = ns;
      s_cm.n_lit = nl;
      if (!ok) s_cm.abort = 1;
    }
    lds_release(&s_cm.consumed, kNone);
  } else if (wave == 1) {
    stage_matches(best, n);
  }
  __threadfence();
  __syncthreads();
  if (s_cm.abort) {
    if (t == 0) {
      *job.status = kESTALL;
      *job.out_len = 0;
    }
    return;
  }
  // A: literals after the records; the records' positions from prefix sums
  const uint32_t n_seq = s_cm.n_seq, n_lit = s_cm.n_lit;
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
