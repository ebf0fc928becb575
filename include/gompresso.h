/*
 * gompresso.h — C ABI of the MI355X (gfx950) Gompresso decompressor: Gompresso/Bit
 * (Huffman-coded sub-blocks) and Gompresso/Byte (byte-level records).
 *
 * Decompresses the block format of arXiv 1606.00519 (section "Gompresso
 * Overview"): independently compressed data blocks, each carrying two
 * canonical Huffman codes (literal/length and offset) and a token stream cut
 * into sub-blocks whose compressed sizes in bits are stored in the block
 * (section "Parallel Compression").  Per block, one workgroup decodes every
 * sub-block in its own lane (section "Huffman Decoding"), then one 64-lane
 * wavefront resolves the sequences group by group (section "LZ77
 * Decompression"): back-references of ordinary streams by Multi-Round
 * Resolution (section "Multi-Round Resolution (MRR) of Nested
 * back-references"), those of streams written with Dependency Elimination in
 * a single pass (section "Dependency Elimination (DE)").
 *
 * Block layout (little-endian; the paper's format figure is not available,
 * so this is the project's own concrete layout):
 *   0   u32 magic 'GMPB'      4 u8 version(1)  5 u8 mode(0 ordinary, 1 DE)
 *   6   u8 group G            7 u8 lmax (max code length)
 *   8   u32 raw_len          12 u32 window (max distance, <= 32768)
 *   16  u16 max_match (3..258)  18 u16 reserved(0)
 *   20  u32 n_sub            24 u32 n_seq            28 u32 n_lit
 *   32  u8 lens[160]  nibbles, low first: 286 literal/length then 30 distance
 *   192 index: n_sub x {u32 bit_len, u32 n_seq, u32 n_lit, u32 raw_len}
 *   then u32 payload_bytes, 12 zero bytes, payload (sub-block bitstreams,
 *   each padded to 128 bits; sub-block i starts at 16*sum_{j<i} ceil(bit_len_j/128)).
 * Byte-level block (Gompresso/Byte, sections "Parallel Compression" and
 * "Parallel Decompression": the tokens are written with a direct byte-level
 * encoding, no Huffman stage, and read straight from the block):
 *   0   u32 magic 'GMPY'      4 u8 version(1)  5 u8 mode(0 ordinary, 1 DE)
 *   6   u8 group G            7 u8 reserved(0)
 *   8   u32 raw_len          12 u32 window (<= 32768)
 *   16  u16 max_match (3..258)  18 u16 reserved(0)
 *   20  u32 n_seq            24 u32 n_lit            28 u32 reserved(0)
 *   32  n_seq records, u32 each: bits 0-7 literal length, 8-15 match length - 3,
 *       16-31 distance (0: no back-reference, and then bits 8-15 are 0);
 *       zero bytes to a multiple of 16; then the n_lit literal bytes, zero
 *       bytes to a multiple of 16, and 16 more zero bytes.
 *   Blocks of both formats may be mixed in one stream, batch or request.
 * Bit order and alphabets follow RFC 1951 (LSB-first packing, codes MSB-first,
 * length codes 257..285 and distance codes 0..29 with their extra bits);
 * symbol 256 ends every sub-block.
 * Stream layout: 'GMPF', u16 version, u16 flags, u32 block_size, u32 n_blocks,
 *   u64 raw_total, u64 reserved, u64 block_off[n_blocks+1]; block b decodes to
 *   output bytes [b*block_size, b*block_size + raw_len_b).
 *
 * Conventions for every call:
 *   - "d_" pointers are device pointers (hipMalloc / torch CUDA tensors),
 *     "h_" pointers are host pointers.  The caller owns every buffer it
 *     passes; the library keeps no caller pointer after the call's stream
 *     work completes.  Device input blocks must be 16-byte aligned.
 *   - Calls that take a hipStream_t are asynchronous on that stream.
 *   - Return value: host-detected errors synchronously (GMP_E*).  Errors
 *     found on the device are written to a per-block status word (0 = OK,
 *     otherwise a GMP_E* code) that the caller reads after synchronising.
 *   - On any error, output contents are unspecified, but nothing is ever
 *     written outside [out, out + out_len) of each block.
 */
#ifndef GOMPRESSO_H
#define GOMPRESSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gmp_status;
#define GMP_OK 0
#define GMP_EINVAL -1   /* bad argument */
#define GMP_EFORMAT -2  /* magic, version, header field, index or payload layout */
#define GMP_ECODE -3    /* code lengths over lmax or not filling the code space; invalid symbol */
#define GMP_EDIST -4    /* distance 0, beyond the bytes produced in the block, or beyond window */
#define GMP_ELEN -5     /* match length outside [3, max_match] */
#define GMP_ESIZE -6    /* out_len differs from the block's raw_len */
#define GMP_ESUB -7     /* sub-block bit overrun, missing end symbol, count mismatch with the index */
#define GMP_EDEVICE -8  /* HIP runtime error */
#define GMP_ENOMEM -9   /* device or host allocation failed */
#define GMP_EBUSY -10   /* no capacity (serving back-pressure) */
#define GMP_ENOSYS -11  /* valid format feature this decoder does not implement (lmax > 13) */
#define GMP_ESTALL -12  /* a device-side wait exceeded its time bound (about 1 s); the block's
                           output is incomplete.  An internal error: the kernel bounds every
                           wait so that a fault in its hand-over logic ends instead of hanging */
/* Error classes on the device follow the order in which the decoder meets the
 * problem, which is the order of the CPU reference decoder's checks for header,
 * code-length and index errors.  Inside a bitstream the two decoders can meet
 * different first errors, because the GPU decodes all sub-blocks at once: a
 * corrupt bitstream always fails, with ECODE, EDIST, ELEN or ESUB. */

/* flags */
#define GMP_MODE_AUTO 0u  /* single pass if the block says DE and its group is a multiple of 64, else MRR */
#define GMP_MODE_MRR 1u   /* Multi-Round Resolution for every block (valid for any stream) */
#define GMP_MODE_DE 2u    /* single pass; blocks whose header is not DE with group % 64 == 0 fail EINVAL */
#define GMP_MODE_SC 3u    /* Sequential Copying: the back-references of a group one after another, in
                             sequence order (the baseline of the paper's section "Performance Impact of
                             Nested back-references"; valid for any stream) */
#define GMP_MODE_MASK 3u
#define GMP_FLAG_STATS 0x100u /* record MRR rounds per 64-sequence group (gmp_job.d_rounds), phase times
                                 (d_times) and counters (d_stats); batched calls only */
#define GMP_FLAG_VERIFY_DE 0x200u /* check the Dependency Elimination rule (section "Dependency Elimination
                                 (DE)") in every group of a DE block: every source must end at or before the
                                 destination of the group's first back-reference.  Without the flag a group
                                 that breaks the rule is still decoded correctly (by rounds); with it the
                                 block's status is GMP_EDIST, as the CPU format check reports */
#define GMP_FLAG_PLAIN_MRR 0x400u /* MRR exactly as section "Multi-Round Resolution (MRR)" states it.  By
                                 default a back-reference that does not overlap its own output and reads
                                 only bytes that an earlier such back-reference of its group writes first
                                 reads that one's source instead (at most two such moves, groups of at most
                                 32 KiB of output): the same bytes, available in an earlier round.  Output
                                 is identical either way; only the round counts differ */

typedef struct gmp_ctx gmp_ctx;
typedef struct gmp_batch gmp_batch;

/* Header fields of one block, parsed on the host.  format 0: Gompresso/Bit
 * ('GMPB'); format 1: Gompresso/Byte ('GMPY', lmax = n_sub = 0). */
typedef struct {
  uint32_t mode, group, lmax, raw_len, window, max_match;
  uint32_t n_sub, n_seq, n_lit, payload_bytes;
  uint64_t block_bytes; /* header + index + payload (Byte: header + records + literals) */
  uint32_t format;
  uint32_t reserved;
} gmp_block_info;

/* One block to decode.  The host fills n_seq / n_lit from gmp_block_info;
 * they size the token workspace.  With GMP_FLAG_STATS, d_rounds (may be NULL)
 * receives one byte per 64-sequence group: the rounds taken (MRR rounds; 1
 * for a single pass; the number of back-references under GMP_MODE_SC; 0 for
 * a group without back-references; bit 7 set when the group was split
 * because its output exceeded the on-chip window), d_times (may be NULL)
 * four device wall-clock stamps (100 MHz ticks): start, tables built,
 * sub-blocks decoded, back-references resolved, and d_stats (may be NULL)
 * GMP_STATS_WORDS counters, laid out as the GMP_STAT_* indexes say. */
typedef struct {
  const uint8_t* d_comp; /* device: the block (header, index, payload), 16-byte aligned */
  uint64_t comp_len;     /* bytes readable at d_comp */
  uint8_t* d_out;        /* device: where the block's raw_len bytes go */
  uint64_t out_len;      /* must equal raw_len */
  uint32_t n_seq, n_lit; /* from the block header */
  uint8_t* d_rounds;     /* optional, ceil(n_seq/64) bytes */
  uint64_t* d_times;     /* optional, 4 x uint64 */
  uint32_t* d_stats;     /* optional, GMP_STATS_WORDS x uint32 */
  uint32_t format;       /* gmp_block_info.format: 1 (byte-level) needs no token workspace */
  uint32_t reserved;
} gmp_job;

/* Counters of one block (gmp_job.d_stats, GMP_FLAG_STATS). */
#define GMP_STATS_WORDS 80
#define GMP_STAT_A2_PATH 0      /* how the Huffman stage ran: 1 segmented (the block's bits cut into equal
                                   segments, one per decoder lane), 2 one lane per sub-block, 3 none
                                   (a byte-level block) */
#define GMP_STAT_REPAIRED 1     /* segmented: decoder lanes whose start had to be repaired */
#define GMP_STAT_GROUPS 2       /* groups of 64 sequences */
#define GMP_STAT_SPLIT 3        /* groups resolved in pieces (output larger than the on-chip window) */
#define GMP_STAT_DE_ROUNDS 4    /* groups of a DE block that broke the DE rule and were resolved by rounds */
#define GMP_STAT_STALL_SITE 5   /* 0, or (status GMP_ESTALL) the wait that ran out first: 1 Huffman-stage
                                   fetcher, 2/3 a decoder lane's bit ring (segmented / one lane per
                                   sub-block), 4 token fetcher, 5 output window, 6 staged records, 7 staged
                                   literals, 8 resolution hand-over, 9 output flusher */
#define GMP_STAT_SEG_REJECT 6   /* why segmented decoding was not accepted (then GMP_STAT_A2_PATH is 2), bits:
                                   1 index, 2 invalid code in a lane, 4 a lane's area overflowed, 8 lanes did
                                   not meet, 16 last lane's end, 32 open literal run, 64 per-sub-block counts,
                                   128 repair failed; those of the last attempt that was not accepted (0
                                   when the first attempt was accepted or none was made) */
#define GMP_STAT_SEG_RETRY 7    /* further segmented attempts (0, 1 or 2) because lanes stayed out of step:
                                   a lane after a lane on the true symbol path restarts exactly at that
                                   lane's exit, the others warm up longer before their segment */
#define GMP_STAT_SPILLED 8      /* back-references the decoding launch left to later launches
                                   (gmp_tuning.rounds_per_launch) */
#define GMP_STAT_ROUND_BYTES 16 /* [16 + r]: back-reference bytes copied in round r + 1, over all groups
                                   (r < 64): the numerator of the paper's bytes-per-round measure */

/* Tuning of the batched kernel (section "Dependency on Data Block Size":
 * sub-block count sets the Huffman parallelism per block). */
typedef struct {
  uint32_t waves_per_block; /* decoder wavefronts per workgroup: 1, 2, 4 or 7 (Huffman lanes = 64 x waves);
                               they also resolve back-references, groups round-robin.  Each workgroup adds
                               a fetcher wavefront (HBM -> LDS) and, for 1, 2 or 4, a flusher wavefront
                               (output -> HBM); with 7 (eight wavefronts, two per SIMD) four of the
                               decoders resolve and the seventh flushes */
  uint32_t persistent;      /* 1: persistent workgroups pull blocks from a device queue; 0: one workgroup per block */
  uint32_t workgroups;      /* persistent grid size (0 = one per compute unit) */
  uint32_t rounds_per_launch; /* Multi-Round Resolution over several launches (the variant of section
                               "Performance Impact of Nested back-references" that writes unresolved
                               back-references to device memory for later kernels): 0 = every round in the
                               decoding launch; R in 1..64 = at most R rounds per group of 64 sequences there,
                               the back-references still pending (and those reading their bytes) go to a
                               per-block list in device memory, which later launches resolve R rounds per 64
                               entries at a time, ceil(64 / R) - 1 of them, then one launch finishes the
                               list.  MRR blocks only (DE and Sequential Copying ignore it); batches only.
                               The batch allocates the lists (16 bytes per sequence) on first use */
} gmp_tuning;

/* ---- context ------------------------------------------------------------------ */
/* Creates a context on `device`: it owns the token workspace (grown on demand),
 * job tables, status words and tuning.  Not thread-safe; use one per host thread. */
gmp_status gmp_ctx_create(int device, gmp_ctx** out);
void gmp_ctx_destroy(gmp_ctx* ctx);
const char* gmp_strerror(gmp_status s);
/* First device-side error (section "Parallel Decompression": every block is
 * decoded on the device, so its errors surface there).  Waits until the work
 * queued on `stream` has finished, then moves to *h_first_error the first
 * non-zero block status that any launch of this context recorded since the
 * previous gmp_poll (its block, stream and batch calls, and its servers'
 * launches), and clears it; GMP_OK there means none.  The per-block status
 * words keep every block's own result.  Returns EDEVICE on a HIP error. */
gmp_status gmp_poll(gmp_ctx* ctx, void* stream, int32_t* h_first_error);

/* ---- host-side parsing ---------------------------------------------------------- */
/* Parse a block header from a host copy of at least its first 208 + 16*n_sub bytes
 * (len = bytes available).  Fails EFORMAT on bad magic/version/fields. */
gmp_status gmp_block_info_parse(const void* h_block, size_t len, gmp_block_info* out);
/* Device token workspace one Gompresso/Bit block needs (a byte-level block needs
 * none), from its header's n_seq and n_lit: the
 * token stream between the Huffman and the LZ77 stages (section "Gompresso
 * Overview": sequences and literal strings) plus the segmented decoder's
 * per-lane areas, which depend on the block's compressed bytes (comp_len).  Contexts, batches and servers allocate it themselves; a
 * server's budget counts it per request. */
uint64_t gmp_workspace_bytes(uint32_t n_seq, uint32_t n_lit, uint64_t comp_len);
/* Stream header: number of blocks, block size and total raw bytes. */
gmp_status gmp_stream_info(const void* h_stream, size_t len, uint32_t* n_blocks, uint32_t* block_size,
                           uint64_t* raw_total);

/* ---- single block (sections "Huffman Decoding" and "LZ77 Decompression") ---------- */
/* Decode one block.  d_block: the block on the device, 16-byte aligned (EINVAL
 * otherwise).  h_block: host copy of the block's header and index (the same
 * bytes as d_block, at least gmp_block_info.block_bytes - payload_bytes long), used
 * only to size the workspace.  d_status: device int32 that receives the block's
 * status.  flags: GMP_MODE_*, GMP_FLAG_VERIFY_DE.  Asynchronous on `stream`.  This call and gmp_decompress_stream launch one
 * workgroup per block with seven decoder wavefronts (see gmp_tuning). */
gmp_status gmp_decompress_block(gmp_ctx* ctx, const uint8_t* d_block, size_t block_len, const void* h_block,
                                size_t h_len, uint8_t* d_out, size_t out_len, int32_t* d_status, uint32_t flags,
                                void* stream);

/* ---- single block without allocation ----------------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results as gmp_decompress_block, without a context, on the current device: the
 * block's token workspace is a fixed device array of GMP_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends, and
 * the job descriptor travels in the kernel arguments.  The call makes no
 * hipMalloc, hipFree or other allocating call.  GMP_ERANGE if the block's
 * workspace (gmp_workspace_bytes) exceeds the array: 32 MiB holds every block
 * of up to 4 MiB of Zipf text or CSV rows.  Calls on one device share the
 * array, so calls that overlap on one device (other streams, other threads)
 * race and must not be made; the array keeps the last call's contents, and the
 * kernel writes every byte of it that it reads.  gmp_noalloc_init resolves the
 * array's device address on the current device; the first call does it by
 * itself, so call gmp_noalloc_init (or the entry point once) before capturing.
 * Device-side errors go to *d_status only (no context, so no gmp_poll word). */
#define GMP_NOALLOC_SCRATCH_BYTES (32u << 20)
#define GMP_ERANGE -13 /* the block is larger than gmp_decompress_block_noalloc's fixed workspace */
gmp_status gmp_noalloc_init(void);
gmp_status gmp_decompress_block_noalloc(const uint8_t* d_block, size_t block_len, const void* h_block,
                                        size_t h_len, uint8_t* d_out, size_t out_len, int32_t* d_status,
                                        uint32_t flags, void* stream);

/* ---- whole stream (blocks in parallel, section "Parallel Decompression") ----------- */
/* Decode a stream.  h_stream: host copy of the whole stream (for the block table and
 * block headers); d_stream: the same bytes on the device, 16-byte aligned, with
 * every block at a 16-byte aligned offset (EINVAL / EFORMAT otherwise).  d_status: n_blocks int32
 * on the device.  out_len must equal the stream's raw_total. */
gmp_status gmp_decompress_stream(gmp_ctx* ctx, const uint8_t* d_stream, const void* h_stream, size_t len,
                                 uint8_t* d_out, size_t out_len, int32_t* d_status, uint32_t flags, void* stream);

/* ---- batch of independent blocks (one launch over a device job table) ------------ */
/* Upload a job table once; run it any number of times.  d_status: n_jobs int32 on
 * the device; job i's status goes to d_status[i].  The batch owns its device job
 * table and workspace.  Jobs are dispatched largest first (by out_len), which
 * evens out the finish times of uneven blocks. */
gmp_status gmp_batch_create(gmp_ctx* ctx, const gmp_job* h_jobs, uint32_t n_jobs, int32_t* d_status,
                            gmp_batch** out);
gmp_status gmp_batch_run(gmp_ctx* ctx, gmp_batch* batch, uint32_t flags, const gmp_tuning* tuning, void* stream);
void gmp_batch_destroy(gmp_batch* batch);

/* ---- graph-captured batch (one launch decodes the whole batch) ------------------- */
/* Capture the batch's launch with these flags and tuning into a HIP graph owned by
 * the batch (blocks are independent, section "Gompresso Overview", so a single
 * launch serves any number of them).  The graph holds a small kernel that resets
 * the persistent queue (no memset node) and the decode kernel.  A new capture
 * replaces the previous graph.  EINVAL on bad flags or tuning; EDEVICE if capture
 * or instantiation fails. */
gmp_status gmp_batch_graph_create(gmp_ctx* ctx, gmp_batch* batch, uint32_t flags, const gmp_tuning* tuning);
/* Replay the captured graph on `stream`; EINVAL if none was captured. */
gmp_status gmp_batch_graph_launch(gmp_ctx* ctx, gmp_batch* batch, void* stream);

/* ---- autotuner ---------------------------------------------------------------- */
/* Choose launch parameters for a batch by timing candidates on the device
 * (section "Dependency on Data Block Size": parallelism per block against
 * per-block overheads): wavefronts per block in {1, 2, 4, 7} x {one workgroup per
 * job, persistent with one or two workgroups per compute unit}, all rounds in
 * one launch; then, on the winning shape, rounds per launch in {1, 4, 16}
 * (section "Performance Impact of Nested back-references").  Each candidate
 * runs once untimed, then `reps` (1..64) timed runs on `stream`; the least
 * median wins.  The batch's outputs are overwritten (with the same bytes, for
 * valid input).  *best receives the winner, *best_ms (may be NULL) its median
 * time.  Synchronous. */
gmp_status gmp_autotune(gmp_ctx* ctx, gmp_batch* batch, uint32_t flags, uint32_t reps, gmp_tuning* best,
                        float* best_ms, void* stream);

/* ---- compression on the GPU (Gompresso/Byte) ------------------------------------ */
/* Compress independent data blocks into byte-level blocks (the format above),
 * one workgroup per block (section "Parallel Compression": each block is
 * compressed by a group of threads that find matches in parallel; the byte
 * level encoding needs no Huffman stage).  With de = 1 every group of 64
 * sequences obeys the Dependency Elimination rule (section "Dependency
 * Elimination (DE)"): each of its back-references ends at or before the
 * destination of the group's first one, so the decoder resolves the group in
 * one pass.  Matches come from hash chains of 3-byte keys (the most recent
 * positions first, a bounded number of them) and from distances 1-4; the
 * parse is greedy.  Several compressed forms of a block are valid: the output
 * is checked by decoding, not against another compressor's bytes. */
typedef struct {
  uint32_t window;     /* longest distance, 1..32768 */
  uint32_t max_match;  /* 3..258 */
  uint32_t de;         /* 0: ordinary LZ77 stream, 1: Dependency Elimination (group of 64) */
  uint32_t reserved;
} gmp_compress_params;
typedef struct {
  const uint8_t* d_in;  /* device: the block's bytes */
  uint64_t in_len;      /* at most GMP_COMPRESS_MAX_BLOCK */
  uint8_t* d_out;       /* device, 16-byte aligned: the compressed block */
  uint64_t out_cap;     /* at least gmp_compress_bound(in_len) */
  uint64_t* d_out_len;  /* device: receives the compressed block's size */
  int32_t* d_status;    /* device: GMP_OK once the block is written */
} gmp_compress_job;
#define GMP_COMPRESS_MAX_BLOCK (64u << 20)
/* Largest compressed size of a block of in_len bytes. */
uint64_t gmp_compress_bound(uint64_t in_len);
/* Compress n_jobs blocks, asynchronously on `stream`.  The context holds the job
 * table and a workspace of 8 bytes per input byte (grown on demand; the call
 * waits for the context's previous single call first).  EINVAL on bad
 * parameters, a misaligned output, a capacity below the bound or a block over
 * GMP_COMPRESS_MAX_BLOCK. */
gmp_status gmp_compress_batch(gmp_ctx* ctx, const gmp_compress_job* h_jobs, uint32_t n_jobs,
                              const gmp_compress_params* params, void* stream);

/* ---- request loop (continuous batching on one GPU) ------------------------------ */
/* A server admits decompression requests of mixed sizes as they arrive and runs
 * them concurrently.  A scheduler thread admits requests first come first served
 * while the bytes of everything in flight (compressed + decompressed + token
 * workspace) stay within `budget_bytes`; whenever one of its `n_slots` launch
 * slots (a HIP stream each, default priority) is free, it launches every
 * admitted request that is not running yet as one kernel over all their blocks
 * (one workgroup per block, largest first; one kernel per distinct request
 * flags; blocks are independent, section "Gompresso Overview").  Requests that
 * arrive while others run join the next launch, and launches of different
 * slots overlap on the device.  Each request completes on its own: its blocks
 * count themselves done in host-visible memory, and the request is reported,
 * and its budget released, as soon as the last of them has finished.  Every
 * block is decoded with its request's flags (GMP_MODE_*, GMP_FLAG_VERIFY_DE).
 * Compressed input, output and status words belong to the caller and stay
 * resident on the device; the server owns a token-workspace arena of
 * `workspace_bytes` (0 = budget / 2), handed out first-fit.  A request whose
 * bytes exceed the budget, or whose workspace exceeds the arena, can never be
 * admitted and is refused by gmp_server_submit with GMP_EBUSY.  At most 4096
 * requests are admitted at once. */
typedef struct gmp_server gmp_server;

typedef struct {
  const uint8_t* d_stream; /* device: a whole stream (gmp_decompress_stream's input) */
  const void* h_stream;    /* host copy of the stream's header, block table and block headers/indexes */
  uint64_t len;            /* stream bytes (at d_stream and h_stream) */
  uint8_t* d_out;          /* device output, out_len = the stream's raw_total */
  uint64_t out_len;
  int32_t* d_status;       /* device: one int32 per block */
  uint32_t flags;          /* GMP_MODE_* */
  uint32_t reserved;
  uint64_t tag;            /* caller's identifier, returned in the completion */
} gmp_request;

typedef struct {
  uint64_t tag;
  int32_t status;          /* GMP_OK once every block of the request has finished (per-block results
                              are in d_status); else the host-side or HIP error that ended it */
  uint32_t reserved;
  uint64_t bytes;          /* decompressed bytes of the request */
  uint64_t t_submit_ns, t_admit_ns, t_done_ns; /* host steady clock: submitted, launched, seen complete */
} gmp_completion;

typedef struct {
  uint64_t submitted, finished, pending;
  uint64_t in_flight_bytes, peak_in_flight_bytes, budget;
  uint64_t launches;        /* kernel launches so far (each covers every request admitted since the last) */
  uint32_t peak_slots;      /* most launches in flight at once */
  uint32_t reserved;
} gmp_server_info;

gmp_status gmp_server_create(gmp_ctx* ctx, uint64_t budget_bytes, uint64_t workspace_bytes, uint32_t n_slots,
                             const gmp_tuning* tuning, gmp_server** out);
/* Queue a request (thread-safe).  The header and block table are checked here:
 * EFORMAT / ESIZE / EINVAL as for gmp_decompress_stream (a d_stream that is not
 * 16-byte aligned, or GMP_MODE_DE on a block whose header is not DE with a group
 * that is a multiple of 64, is EINVAL); EBUSY if the request alone exceeds the
 * budget or its workspace the arena. */
gmp_status gmp_server_submit(gmp_server* srv, const gmp_request* req);
/* Move up to `max` completions (in completion order) to `out`; returns how many. */
uint32_t gmp_server_poll(gmp_server* srv, gmp_completion* out, uint32_t max);
/* Wait until every submitted request has completed (EBUSY on timeout). */
gmp_status gmp_server_drain(gmp_server* srv, uint32_t timeout_ms);
gmp_status gmp_server_stats(gmp_server* srv, gmp_server_info* out);
/* Drops requests not yet admitted, waits for the admitted ones, frees everything. */
void gmp_server_destroy(gmp_server* srv);

#ifdef __cplusplus
}
#endif
#endif
