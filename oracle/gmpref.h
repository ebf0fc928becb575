/*
 * gmpref — the CPU ORACLE for the Gompresso/Bit format (arXiv 1606.00519).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the GPU decoder is checked against, plus the CPU
 * compressor that produces every compressed input.  Only the test suite,
 * the smoke check and the benchmark's input-generation / CPU-baseline leg
 * may load it.  The GPU library never links, loads or calls it, and the two
 * share no code: no headers, tables, helpers or constants.
 *
 * What it computes (paper section "Gompresso Overview"):
 *   - compression: equal-sized data blocks, each LZ77-parsed (optionally with
 *     Dependency Elimination, section "Dependency Elimination (DE)" and the
 *     DE compression algorithm figure), the token stream cut into sub-blocks,
 *     two canonical Huffman codes per block (literal/length and offset) built
 *     from the block's token frequencies, each sub-block stored with its
 *     compressed size in bits;
 *   - decompression: the plain sequential Inflate-like decode of that format
 *     (bit-serial canonical decoding, then byte-by-byte LZ77 copying);
 *   - validation of the format invariants and of the DE rule;
 *   - the Multi-Round Resolution round count per group of sequences
 *     (section "Multi-Round Resolution (MRR) of Nested back-references").
 *
 * Functions whose result has no independent pin are marked "parity
 * unpinned" in their comment; all others are pinned by the CPU test suite.
 *
 * ---------------------------------------------------------------------------
 * Concrete format (the paper's format figure is lost; this is our layout).
 * All integers little-endian.
 *
 * Block (one independently decodable data block):
 *   off   0  u32 magic 'GMPB' (0x42504D47)
 *   off   4  u8  version (1)
 *   off   5  u8  mode     0 = ordinary LZ77 stream, 1 = DE stream
 *   off   6  u8  group    G: sequences per resolution group (DE guarantee)
 *   off   7  u8  lmax     maximum Huffman code length, 1..15
 *   off   8  u32 raw_len  decompressed bytes of this block
 *   off  12  u32 window   maximum back-reference distance, 1..32768
 *   off  16  u16 max_match  longest match, 3..258
 *   off  18  u16 reserved (0)
 *   off  20  u32 n_sub    number of sub-blocks
 *   off  24  u32 n_seq    number of sequences in the block
 *   off  28  u32 n_lit    number of literal bytes in the block
 *   off  32  u8  lens[160]  code lengths, two per byte, low nibble first:
 *                           286 literal/length codes then 30 distance codes
 *                           (316 nibbles = 158 bytes, 2 zero pad bytes)
 *   off 192  sub-block index, n_sub entries of 16 bytes:
 *              u32 bit_len   compressed size of the sub-block in bits
 *              u32 n_seq     sequences in the sub-block
 *              u32 n_lit     literal bytes in the sub-block
 *              u32 raw_len   decompressed bytes of the sub-block
 *   off 192 + 16*n_sub   u32 payload_bytes
 *   then 12 zero bytes (payload starts 16-byte aligned)
 *   payload: the sub-block bitstreams, each padded to a multiple of 128 bits,
 *            so sub-block i starts at byte 16 * sum_{j<i} ceil(bit_len_j/128).
 *
 * Bitstream of a sub-block (RFC 1951 section 3.1.1 packing): bits are read
 * least-significant first from consecutive bytes; Huffman codes are stored
 * most-significant code bit first; extra bits least-significant first.
 * Symbols: literal/length alphabet 0..255 literal, 256 end of sub-block,
 * 257..285 length codes with RFC 1951 extra bits; distance alphabet 0..29
 * with RFC 1951 extra bits.  Every sub-block ends with symbol 256.
 *
 * Sequences: a sequence is a (possibly empty) run of literals followed by one
 * back-reference (section "LZ77 Decompression").  A literal run that is
 * closed by the end of a sub-block forms a sequence with match length 0.
 *
 * Byte-level block (Gompresso/Byte, section "Gompresso Overview": the token
 * streams are written with a direct byte-level encoding and no Huffman stage,
 * so the decoder reads them straight from the compressed block):
 *   off   0  u32 magic 'GMPY' (0x59504D47)
 *   off   4  u8  version (1)
 *   off   5  u8  mode     0 = ordinary LZ77 stream, 1 = DE stream
 *   off   6  u8  group    G
 *   off   7  u8  reserved (0)
 *   off   8  u32 raw_len
 *   off  12  u32 window   1..32768
 *   off  16  u16 max_match 3..258
 *   off  18  u16 reserved (0)
 *   off  20  u32 n_seq    sequences (4-byte records)
 *   off  24  u32 n_lit    literal bytes
 *   off  28  u32 reserved (0)
 *   off  32  n_seq records, one u32 each, little-endian:
 *              bits 0-7   literal length 0..255
 *              bits 8-15  match length - 3 (0 when the sequence has no match)
 *              bits 16-31 distance 1..32768, 0 = no back-reference
 *            then zero bytes up to a multiple of 16
 *   then the n_lit literal bytes, zero bytes up to a multiple of 16, and 16
 *   more zero bytes.  Literal runs longer than 255 bytes are split into
 *   literal-only sequences, which may appear anywhere.
 *
 * Stream (a whole input):
 *   off 0  u32 magic 'GMPF' (0x46504D47), u16 version (1), u16 flags (0),
 *          u32 block_size, u32 n_blocks, u64 raw_total, u64 reserved
 *   off 32 u64 block_off[n_blocks + 1]  (byte offsets from stream start;
 *          the last entry is the stream length; blocks are 16-byte aligned)
 *   Block b decompresses to [b*block_size, b*block_size + raw_len_b).
 * ---------------------------------------------------------------------------
 */
#ifndef GMPREF_H
#define GMPREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (negative = error) */
#define GMPREF_OK        0
#define GMPREF_EINVAL   -1  /* bad argument */
#define GMPREF_EFORMAT  -2  /* magic, version, header field or index layout */
#define GMPREF_ECODE    -3  /* code lengths (> lmax, Kraft sum != 1) or invalid symbol */
#define GMPREF_EDIST    -4  /* distance 0, beyond bytes produced in block, or beyond window */
#define GMPREF_ELEN     -5  /* match length out of [3, max_match] or output overrun */
#define GMPREF_ESIZE    -6  /* output capacity differs from the decompressed size */
#define GMPREF_ESUB     -7  /* sub-block bit overrun, missing end symbol, count mismatch */
#define GMPREF_ENOMEM   -9

typedef struct {
  uint32_t lit_len;    /* literal bytes before the back-reference */
  uint32_t match_len;  /* 0 (literal-only sequence) or 3..max_match */
  uint32_t dist;       /* back-reference distance (1..window), 0 when match_len is 0 */
} gmpref_seq;

typedef struct {
  uint32_t block_size;     /* bytes per data block */
  uint32_t window;         /* maximum distance, <= 32768 */
  uint32_t max_match;      /* maximum match length, 3..258 */
  uint32_t lmax;           /* maximum code length, 1..15 (must fit the alphabets) */
  uint32_t sub_target_raw; /* close a sub-block at the first token end >= this many bytes; 0 = off */
  uint32_t sub_target_seq; /* or after this many sequences (used when sub_target_raw == 0) */
  uint32_t de;             /* 1 = Dependency Elimination */
  uint32_t group;          /* G, sequences per group (1..255) */
  uint32_t chain;          /* maximum match candidates examined per position */
  uint32_t hash_mode;      /* 0 = hash chains, 1 = single-entry table with minimal staleness */
  uint32_t staleness;      /* hash_mode 1: replace an entry only if it is more than this many bytes old */
  uint32_t format;         /* 0 = Gompresso/Bit (Huffman-coded sub-blocks), 1 = Gompresso/Byte (byte-level
                              records; literal runs of at most 255 bytes; no sub-blocks) */
} gmpref_params;

typedef struct {
  uint32_t version, mode, group, lmax, raw_len, window, max_match;
  uint32_t n_sub, n_seq, n_lit, payload_bytes;
  uint64_t block_bytes;    /* total bytes of the block including header, index and payload */
  uint32_t format;         /* 0 = Bit ('GMPB'), 1 = Byte ('GMPY'; lmax and n_sub are 0) */
  uint32_t reserved;
} gmpref_block_info;

void gmpref_default_params(gmpref_params* p);

/* ---- compressor (input generator) ------------------------------------- */
int gmpref_compress(const uint8_t* in, size_t n, const gmpref_params* p,
                    uint8_t** out, size_t* out_len);
int gmpref_compress_block(const uint8_t* in, size_t n, const gmpref_params* p,
                          uint8_t** out, size_t* out_len);
/* LZ77 parse only: sequences, literal stream and sequences per sub-block. */
int gmpref_parse_block(const uint8_t* in, size_t n, const gmpref_params* p,
                       gmpref_seq** seqs, size_t* n_seq, uint8_t** lits, size_t* n_lits,
                       uint32_t** sub_seqs, size_t* n_sub);
/* Byte-level block of a given token stream (every lit_len <= 255; sequences
 * without a match have dist 0).  mode/group/window/max_match come from p. */
int gmpref_encode_byte_block(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits,
                             const gmpref_params* p, uint8_t** out, size_t* out_len);
/* Encode a given token stream (tests build adversarial streams with it).
 * sub_seqs[i] = sequences in sub-block i; mode/group/window/max_match/lmax
 * come from p and are written to the header unchecked. */
int gmpref_encode_block(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits,
                        const uint32_t* sub_seqs, size_t n_sub, const gmpref_params* p,
                        uint8_t** out, size_t* out_len);

/* ---- decoder (the definition) ----------------------------------------- */
int gmpref_block_info_parse(const uint8_t* blk, size_t len, gmpref_block_info* info);
int gmpref_decompress_block(const uint8_t* blk, size_t len, uint8_t* out, size_t cap, size_t* out_len);
int gmpref_decompress(const uint8_t* comp, size_t len, uint8_t* out, size_t cap, size_t* out_len);
/* Decode a block's token stream (sequences and literal bytes) without LZ77. */
int gmpref_block_tokens(const uint8_t* blk, size_t len, gmpref_seq** seqs, size_t* n_seq,
                        uint8_t** lits, size_t* n_lits);
/* Plain LZ77 expansion of a token stream (byte-by-byte copies). */
int gmpref_lz77_expand(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits,
                       uint32_t window, uint32_t max_match, uint8_t* out, size_t cap, size_t* out_len);

/* ---- checks ----------------------------------------------------------- */
/* Full check of a block: everything the decoder checks, plus (mode 1) the DE
 * rule: in every group of G sequences, every source interval ends at or before
 * the destination of the group's first back-reference. */
int gmpref_validate_block(const uint8_t* blk, size_t len);
/* DE rule on a token stream for group width G (returns 1 if it holds). */
int gmpref_de_holds(const gmpref_seq* seqs, size_t n_seq, uint32_t G);
/* MRR rounds per group of G sequences and bytes copied in each round.
 * rounds[g] for g < ceil(n_seq/G); bytes_per_round[r] for r in 0..G-1 (round r+1). */
int gmpref_mrr_rounds(const gmpref_seq* seqs, size_t n_seq, uint32_t G,
                      uint32_t* rounds, uint64_t* bytes_per_round);
/* MRR rounds where each back-reference that does not overlap itself first moves
 * its source, up to `jumps` times, through an earlier non-overlapping copy of
 * its own group whose destination holds every byte it reads (groups whose
 * output exceeds span_limit bytes are not redirected; 0 = no limit).
 * seq_round / seq_dist may be NULL; else n_seq entries each: the round of each
 * sequence's back-reference (0 if it has none) and the distance it reads from. */
int gmpref_mrr_rounds_redirect(const gmpref_seq* seqs, size_t n_seq, uint32_t G, uint32_t jumps,
                               uint64_t span_limit, uint32_t* rounds, uint64_t* bytes_per_round,
                               uint32_t* seq_round, uint32_t* seq_dist);

/* ---- Huffman helpers exposed for pinning ------------------------------ */
/* Optimal code lengths limited to lmax (package-merge); zero weight -> 0. */
int gmpref_limited_lengths(const uint64_t* w, int n, int lmax, uint8_t* lens);
/* Canonical codes from lengths (RFC 1951 section 3.2.2); codes are MSB-first values. */
int gmpref_canonical_codes(const uint8_t* lens, int n, uint32_t* codes);
/* Length / distance symbol tables (RFC 1951 section 3.2.5). */
void gmpref_length_table(uint16_t base[29], uint8_t extra[29]);
void gmpref_dist_table(uint16_t base[30], uint8_t extra[30]);

void gmpref_free(void* p);

#ifdef __cplusplus
}
#endif
#endif
