/*
 * gmpref.c — CPU ORACLE (test infrastructure only; see gmpref.h).
 *
 * Plain C, no threads, no vector tricks.  Every step follows the paper's
 * description (arXiv 1606.00519, sections "Gompresso Overview", "Parallel
 * Compression", "Huffman Decoding", "LZ77 Decompression", "Data Dependencies
 * in Nested back-references") and, for the coding conventions the paper
 * adopts from DEFLATE, RFC 1951 sections 3.1.1, 3.2.2 and 3.2.5.
 */
#include "gmpref.h"

#include <stdlib.h>
#include <string.h>

/* ======================================================================== */
/* RFC 1951 section 3.2.5: length codes 257..285 and distance codes 0..29.   */
/* ======================================================================== */
static const uint16_t LEN_BASE[29] = {3,   4,   5,   6,   7,   8,   9,   10,  11, 13,
                                      15,  17,  19,  23,  27,  31,  35,  43,  51, 59,
                                      67,  83,  99,  115, 131, 163, 195, 227, 258};
static const uint8_t LEN_EXTRA[29] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2,
                                      2, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 5, 0};
static const uint16_t DIST_BASE[30] = {1,    2,    3,    4,    5,    7,     9,     13,    17,    25,
                                       33,   49,   65,   97,   129,  193,   257,   385,   513,   769,
                                       1025, 1537, 2049, 3073, 4097, 6145,  8193,  12289, 16385, 24577};
static const uint8_t DIST_EXTRA[30] = {0, 0, 0, 0, 1, 1, 2, 2,  3,  3,  4,  4,  5,  5,  6,
                                       6, 7, 7, 8, 8, 9, 9, 10, 10, 11, 11, 12, 12, 13, 13};

#define N_LL 286   /* literal/length alphabet size (0..255 literal, 256 end, 257..285 lengths) */
#define N_D 30     /* distance alphabet size */
#define SYM_END 256
#define HDR_BYTES 192
#define IDX_ENTRY 16
#define MAX_BITS 15

void gmpref_length_table(uint16_t base[29], uint8_t extra[29]) {
  memcpy(base, LEN_BASE, sizeof LEN_BASE);
  memcpy(extra, LEN_EXTRA, sizeof LEN_EXTRA);
}
void gmpref_dist_table(uint16_t base[30], uint8_t extra[30]) {
  memcpy(base, DIST_BASE, sizeof DIST_BASE);
  memcpy(extra, DIST_EXTRA, sizeof DIST_EXTRA);
}

/* Length symbol index 0..28 for a match length 3..258. */
static int len_index(uint32_t len) {
  if (len == 258) return 28;
  int i = 27;
  while (LEN_BASE[i] > len) i--;
  return i;
}
/* Distance symbol 0..29 for a distance 1..32768. */
static int dist_index(uint32_t d) {
  int i = 29;
  while (DIST_BASE[i] > d) i--;
  return i;
}

void gmpref_free(void* p) { free(p); }

void gmpref_default_params(gmpref_params* p) {
  p->block_size = 1u << 20;
  p->window = 32768;
  p->max_match = 258;
  p->lmax = 12;
  p->sub_target_raw = 16384;
  p->sub_target_seq = 0;
  p->de = 0;
  p->group = 64;
  p->chain = 64;
  p->hash_mode = 0;
  p->staleness = 1024;
  p->format = 0;
}

/* ======================================================================== */
/* little-endian helpers                                                    */
/* ======================================================================== */
static uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint64_t rd64(const uint8_t* p) { return (uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32); }
static void wr32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
static void wr16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void wr64(uint8_t* p, uint64_t v) { wr32(p, (uint32_t)v); wr32(p + 4, (uint32_t)(v >> 32)); }

/* ======================================================================== */
/* Huffman code lengths: package-merge (length-limited, optimal).           */
/* The paper limits code lengths (section "Dependency on Data Block Size")  */
/* but names no method; package-merge (Larmore & Hirschberg) is used.       */
/* ======================================================================== */
typedef struct {
  uint64_t w;
  int a, b;   /* children for a package, -1 for a leaf */
  int sym;    /* symbol for a leaf */
} pm_node;

static const uint64_t* pm_weights;
static int cmp_by_weight(const void* x, const void* y) {
  int i = *(const int*)x, j = *(const int*)y;
  if (pm_weights[i] != pm_weights[j]) return pm_weights[i] < pm_weights[j] ? -1 : 1;
  return i - j;
}

int gmpref_limited_lengths(const uint64_t* w, int n, int lmax, uint8_t* lens) {
  if (n <= 0 || lmax < 1 || lmax > MAX_BITS) return GMPREF_EINVAL;
  memset(lens, 0, (size_t)n);
  int* used = (int*)malloc(sizeof(int) * (size_t)n);
  if (!used) return GMPREF_ENOMEM;
  int m = 0;
  for (int i = 0; i < n; i++)
    if (w[i] > 0) used[m++] = i;
  if (m == 0) { free(used); return GMPREF_OK; }
  if (m == 1) {
    /* a single used symbol: give it and the lowest-numbered unused symbol
       length 1 so that the code is complete (Kraft sum exactly 1) */
    if (n < 2) { free(used); return GMPREF_EINVAL; }
    lens[used[0]] = 1;
    lens[used[0] == 0 ? 1 : 0] = 1;
    free(used);
    return GMPREF_OK;
  }
  if (lmax < 31 && (uint64_t)m > ((uint64_t)1 << lmax)) { free(used); return GMPREF_EINVAL; }
  pm_weights = w;
  qsort(used, (size_t)m, sizeof(int), cmp_by_weight);

  size_t cap = (size_t)m * 2 * (size_t)lmax + (size_t)m + 8;
  pm_node* pool = (pm_node*)malloc(sizeof(pm_node) * cap);
  int* cur = (int*)malloc(sizeof(int) * (size_t)(2 * m + 2));
  int* nxt = (int*)malloc(sizeof(int) * (size_t)(2 * m + 2));
  int* stack = (int*)malloc(sizeof(int) * cap);
  if (!pool || !cur || !nxt || !stack) {
    free(used); free(pool); free(cur); free(nxt); free(stack);
    return GMPREF_ENOMEM;
  }
  size_t np = 0;
  /* leaves, sorted by weight */
  for (int i = 0; i < m; i++) {
    pool[np].w = w[used[i]]; pool[np].a = pool[np].b = -1; pool[np].sym = used[i];
    np++;
  }
  /* the list for the deepest level is the leaves alone */
  int ncur = m;
  for (int i = 0; i < m; i++) cur[i] = i;
  /* for each shallower level: package adjacent pairs of the deeper list and
     merge the packages with the leaves, by weight */
  for (int level = lmax - 1; level >= 1; level--) {
    int npk = ncur / 2;
    int pk0 = (int)np;
    for (int k = 0; k < npk; k++) {
      pool[np].w = pool[cur[2 * k]].w + pool[cur[2 * k + 1]].w;
      pool[np].a = cur[2 * k]; pool[np].b = cur[2 * k + 1]; pool[np].sym = -1;
      np++;
    }
    int i = 0, k = 0, t = 0;
    while (i < m || k < npk) {
      if (k >= npk || (i < m && pool[i].w <= pool[pk0 + k].w)) nxt[t++] = i++;
      else nxt[t++] = pk0 + k++;
    }
    int* tmp = cur; cur = nxt; nxt = tmp;
    ncur = t;
  }
  /* the first 2m-2 items of the shallowest list form the optimal solution;
     a symbol's code length is the number of its leaf occurrences */
  int take = 2 * m - 2;
  int sp = 0;
  for (int i = 0; i < take; i++) stack[sp++] = cur[i];
  int ok = GMPREF_OK;
  while (sp > 0) {
    int x = stack[--sp];
    if (pool[x].a < 0) {
      if (lens[pool[x].sym] >= lmax) ok = GMPREF_EINVAL;
      lens[pool[x].sym]++;
    } else {
      stack[sp++] = pool[x].a;
      stack[sp++] = pool[x].b;
    }
  }
  free(used); free(pool); free(cur); free(nxt); free(stack);
  return ok;
}

/* RFC 1951 section 3.2.2: consecutive code values per length, in symbol order. */
int gmpref_canonical_codes(const uint8_t* lens, int n, uint32_t* codes) {
  uint32_t bl_count[MAX_BITS + 1] = {0};
  uint32_t next_code[MAX_BITS + 2] = {0};
  for (int i = 0; i < n; i++) {
    if (lens[i] > MAX_BITS) return GMPREF_ECODE;
    bl_count[lens[i]]++;
  }
  bl_count[0] = 0;
  uint32_t code = 0;
  for (int bits = 1; bits <= MAX_BITS; bits++) {
    code = (code + bl_count[bits - 1]) << 1;
    next_code[bits] = code;
  }
  for (int i = 0; i < n; i++) {
    codes[i] = 0;
    if (lens[i]) codes[i] = next_code[lens[i]]++;
  }
  return GMPREF_OK;
}

/* ======================================================================== */
/* growable byte buffer and LSB-first bit writer                            */
/* ======================================================================== */
typedef struct {
  uint8_t* p;
  size_t len, cap;
} buf_t;

static int buf_reserve(buf_t* b, size_t extra) {
  if (b->len + extra <= b->cap) return 0;
  size_t nc = b->cap ? b->cap : 4096;
  while (nc < b->len + extra) nc *= 2;
  uint8_t* q = (uint8_t*)realloc(b->p, nc);
  if (!q) return -1;
  b->p = q;
  b->cap = nc;
  return 0;
}
static int buf_push(buf_t* b, uint8_t v) {
  if (buf_reserve(b, 1)) return -1;
  b->p[b->len++] = v;
  return 0;
}

typedef struct {
  buf_t* out;
  uint64_t nbits;   /* bits written into the current sub-block */
  int err;
} bitw;

/* append one bit (bit position nbits within the sub-block, LSB-first) */
static void bw_bit(bitw* w, int bit) {
  if ((w->nbits & 7) == 0)
    if (buf_push(w->out, 0)) { w->err = 1; return; }
  if (bit) w->out->p[w->out->len - 1] |= (uint8_t)(1u << (w->nbits & 7));
  w->nbits++;
}
/* extra bits: least-significant bit first */
static void bw_value(bitw* w, uint32_t v, int n) {
  for (int i = 0; i < n; i++) bw_bit(w, (int)((v >> i) & 1));
}
/* Huffman code: most-significant code bit first */
static void bw_code(bitw* w, uint32_t code, int len) {
  for (int i = len - 1; i >= 0; i--) bw_bit(w, (int)((code >> i) & 1));
}

/* ======================================================================== */
/* encoder: token stream -> block                                           */
/* ======================================================================== */
static int seq_codable(const gmpref_seq* s) {
  if (s->match_len == 0) return s->dist == 0;
  return s->match_len >= 3 && s->match_len <= 258 && s->dist >= 1 && s->dist <= 32768;
}

int gmpref_encode_block(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits,
                        const uint32_t* sub_seqs, size_t n_sub, const gmpref_params* p,
                        uint8_t** out, size_t* out_len) {
  if (!p || !out || !out_len) return GMPREF_EINVAL;
  if (p->lmax < 1 || p->lmax > MAX_BITS || p->group < 1 || p->group > 255) return GMPREF_EINVAL;
  /* structural consistency of the given tokens */
  uint64_t sum_seq = 0, sum_lit = 0, raw = 0;
  for (size_t i = 0; i < n_sub; i++) sum_seq += sub_seqs[i];
  if (sum_seq != n_seq) return GMPREF_EINVAL;
  for (size_t i = 0; i < n_seq; i++) {
    if (!seq_codable(&seqs[i])) return GMPREF_EINVAL;
    sum_lit += seqs[i].lit_len;
    raw += (uint64_t)seqs[i].lit_len + seqs[i].match_len;
  }
  if (sum_lit != n_lits || raw > 0xFFFFFFFFu) return GMPREF_EINVAL;

  /* token frequencies of the block (section "Parallel Compression": both
     codes are built from the token frequencies of the block) */
  uint64_t ll_freq[N_LL] = {0}, d_freq[N_D] = {0};
  size_t li = 0;
  for (size_t i = 0; i < n_seq; i++) {
    for (uint32_t k = 0; k < seqs[i].lit_len; k++) ll_freq[lits[li++]]++;
    if (seqs[i].match_len) {
      ll_freq[257 + len_index(seqs[i].match_len)]++;
      d_freq[dist_index(seqs[i].dist)]++;
    }
  }
  ll_freq[SYM_END] += n_sub; /* one end symbol per sub-block */
  uint8_t lens[N_LL + N_D];
  memset(lens, 0, sizeof lens);
  int rc;
  if (n_sub > 0) {
    if ((rc = gmpref_limited_lengths(ll_freq, N_LL, (int)p->lmax, lens)) != GMPREF_OK) return rc;
    if ((rc = gmpref_limited_lengths(d_freq, N_D, (int)p->lmax, lens + N_LL)) != GMPREF_OK) return rc;
  }
  uint32_t ll_code[N_LL], d_code[N_D];
  gmpref_canonical_codes(lens, N_LL, ll_code);
  gmpref_canonical_codes(lens + N_LL, N_D, d_code);

  /* payload: each sub-block separately, padded to 128 bits */
  buf_t pay = {0, 0, 0};
  uint32_t* sub_bits = (uint32_t*)calloc(n_sub ? n_sub : 1, sizeof(uint32_t));
  uint32_t* sub_nlit = (uint32_t*)calloc(n_sub ? n_sub : 1, sizeof(uint32_t));
  uint32_t* sub_raw = (uint32_t*)calloc(n_sub ? n_sub : 1, sizeof(uint32_t));
  if (!sub_bits || !sub_nlit || !sub_raw) {
    free(sub_bits); free(sub_nlit); free(sub_raw);
    return GMPREF_ENOMEM;
  }
  size_t si = 0;
  li = 0;
  int err = 0;
  for (size_t s = 0; s < n_sub && !err; s++) {
    bitw w = {&pay, 0, 0};
    uint64_t nlit = 0, nraw = 0;
    for (uint32_t q = 0; q < sub_seqs[s]; q++, si++) {
      const gmpref_seq* sq = &seqs[si];
      for (uint32_t k = 0; k < sq->lit_len; k++) {
        uint8_t c = lits[li++];
        bw_code(&w, ll_code[c], lens[c]);
      }
      nlit += sq->lit_len;
      nraw += sq->lit_len + sq->match_len;
      if (sq->match_len) {
        int lx = len_index(sq->match_len), dx = dist_index(sq->dist);
        bw_code(&w, ll_code[257 + lx], lens[257 + lx]);
        bw_value(&w, sq->match_len - LEN_BASE[lx], LEN_EXTRA[lx]);
        bw_code(&w, d_code[dx], lens[N_LL + dx]);
        bw_value(&w, sq->dist - DIST_BASE[dx], DIST_EXTRA[dx]);
      }
    }
    bw_code(&w, ll_code[SYM_END], lens[SYM_END]);
    while (w.nbits & 127) bw_bit(&w, 0); /* pad to a 128-bit boundary */
    /* the recorded size excludes the padding */
    err = w.err;
    sub_nlit[s] = (uint32_t)nlit;
    sub_raw[s] = (uint32_t)nraw;
    sub_bits[s] = 0; /* filled below */
  }
  if (err) {
    free(pay.p); free(sub_bits); free(sub_nlit); free(sub_raw);
    return GMPREF_ENOMEM;
  }
  /* recompute exact bit lengths (without padding): re-walk sizes */
  si = 0;
  li = 0;
  for (size_t s = 0; s < n_sub; s++) {
    uint64_t bits = 0;
    for (uint32_t q = 0; q < sub_seqs[s]; q++, si++) {
      const gmpref_seq* sq = &seqs[si];
      for (uint32_t k = 0; k < sq->lit_len; k++) bits += lens[lits[li++]];
      if (sq->match_len) {
        int lx = len_index(sq->match_len), dx = dist_index(sq->dist);
        bits += lens[257 + lx] + LEN_EXTRA[lx] + lens[N_LL + dx] + DIST_EXTRA[dx];
      }
    }
    bits += lens[SYM_END];
    if (bits > 0xFFFFFFFFu) { free(pay.p); free(sub_bits); free(sub_nlit); free(sub_raw); return GMPREF_EINVAL; }
    sub_bits[s] = (uint32_t)bits;
  }

  size_t idx_bytes = IDX_ENTRY * n_sub;
  size_t total = HDR_BYTES + idx_bytes + 16 + pay.len;
  uint8_t* blk = (uint8_t*)calloc(total, 1);
  if (!blk) { free(pay.p); free(sub_bits); free(sub_nlit); free(sub_raw); return GMPREF_ENOMEM; }
  wr32(blk + 0, 0x42504D47u);
  blk[4] = 1;
  blk[5] = (uint8_t)(p->de ? 1 : 0);
  blk[6] = (uint8_t)p->group;
  blk[7] = (uint8_t)p->lmax;
  wr32(blk + 8, (uint32_t)raw);
  wr32(blk + 12, p->window);
  wr16(blk + 16, (uint16_t)p->max_match);
  wr16(blk + 18, 0);
  wr32(blk + 20, (uint32_t)n_sub);
  wr32(blk + 24, (uint32_t)n_seq);
  wr32(blk + 28, (uint32_t)n_lits);
  for (int i = 0; i < N_LL + N_D; i++) blk[32 + i / 2] |= (uint8_t)(lens[i] << ((i & 1) * 4));
  for (size_t s = 0; s < n_sub; s++) {
    uint8_t* e = blk + HDR_BYTES + IDX_ENTRY * s;
    wr32(e + 0, sub_bits[s]);
    wr32(e + 4, sub_seqs[s]);
    wr32(e + 8, sub_nlit[s]);
    wr32(e + 12, sub_raw[s]);
  }
  wr32(blk + HDR_BYTES + idx_bytes, (uint32_t)pay.len);
  if (pay.len) memcpy(blk + HDR_BYTES + idx_bytes + 16, pay.p, pay.len);
  free(pay.p); free(sub_bits); free(sub_nlit); free(sub_raw);
  *out = blk;
  *out_len = total;
  return GMPREF_OK;
}

/* ======================================================================== */
/* compressor: greedy LZ77 with hash chains, Dependency Elimination, and    */
/* sub-block cutting at sequence boundaries                                  */
/* ======================================================================== */
#define HASH_BITS 15
static uint32_t hash3(const uint8_t* s) {
  uint32_t v = (uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16);
  return (v * 2654435761u) >> (32 - HASH_BITS);
}

typedef struct {
  gmpref_seq* v;
  size_t n, cap;
} seqvec;
static int seq_push(seqvec* s, uint32_t lit, uint32_t len, uint32_t dist) {
  if (s->n == s->cap) {
    size_t nc = s->cap ? s->cap * 2 : 1024;
    gmpref_seq* q = (gmpref_seq*)realloc(s->v, nc * sizeof(gmpref_seq));
    if (!q) return -1;
    s->v = q;
    s->cap = nc;
  }
  s->v[s->n].lit_len = lit;
  s->v[s->n].match_len = len;
  s->v[s->n].dist = dist;
  s->n++;
  return 0;
}
typedef struct {
  uint32_t* v;
  size_t n, cap;
} u32vec;
static int u32_push(u32vec* s, uint32_t x) {
  if (s->n == s->cap) {
    size_t nc = s->cap ? s->cap * 2 : 64;
    uint32_t* q = (uint32_t*)realloc(s->v, nc * sizeof(uint32_t));
    if (!q) return -1;
    s->v = q;
    s->cap = nc;
  }
  s->v[s->n++] = x;
  return 0;
}

int gmpref_parse_block(const uint8_t* in, size_t n, const gmpref_params* p,
                       gmpref_seq** seqs_out, size_t* n_seq_out, uint8_t** lits_out, size_t* n_lits_out,
                       uint32_t** sub_out, size_t* n_sub_out) {
  if (!p || p->window < 1 || p->window > 32768 || p->max_match < 3 || p->max_match > 258 || p->group < 1 ||
      p->group > 255 || p->format > 1 || (p->format == 0 && p->sub_target_raw == 0 && p->sub_target_seq == 0) ||
      n > 0xFFFFFFF0u)
    return GMPREF_EINVAL;
  /* Byte-level blocks have no sub-blocks (the decoder reads the fixed-size
     records directly) and keep literal runs within one byte's count */
  const int byte_fmt = p->format == 1;
  int32_t* head = (int32_t*)malloc(sizeof(int32_t) << HASH_BITS);
  int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));
  uint8_t* lits = (uint8_t*)malloc(n ? n : 1);
  if (!head || !prev || !lits) { free(head); free(prev); free(lits); return GMPREF_ENOMEM; }
  for (size_t i = 0; i < ((size_t)1 << HASH_BITS); i++) head[i] = -1;
  seqvec sv = {0, 0, 0};
  u32vec subs = {0, 0, 0};
  size_t nl = 0;
  size_t pos = 0, lit_start = 0, sub_start = 0;
  uint32_t sub_nseq = 0;
  size_t seq_count = 0;   /* sequences emitted in this block */
  int frozen = 0;         /* DE: has the current group's high-water mark been fixed? */
  size_t hwm = 0;         /* DE: the group's high-water mark once frozen */
  int err = 0;
  const uint32_t G = p->group;

  /* insert position q into the dictionary */
#define INSERT(q)                                                                     \
  do {                                                                                \
    if ((q) + 3 <= n) {                                                               \
      uint32_t h_ = hash3(in + (q));                                                  \
      if (p->hash_mode == 0) {                                                        \
        prev[(q)] = head[h_];                                                         \
        head[h_] = (int32_t)(q);                                                      \
      } else if (head[h_] < 0 || (size_t)(q) - (size_t)head[h_] > p->staleness) {     \
        head[h_] = (int32_t)(q);                                                      \
      }                                                                               \
    }                                                                                 \
  } while (0)

  /* close the current sequence; a new group starts every G sequences */
#define CLOSE_SEQ(lit_, len_, dist_)                                                  \
  do {                                                                                \
    if (seq_push(&sv, (uint32_t)(lit_), (len_), (dist_))) err = 1;                     \
    seq_count++;                                                                      \
    sub_nseq++;                                                                       \
    if (seq_count % G == 0) frozen = 0;                                               \
  } while (0)

  while (pos < n && !err) {
    /* DE: matches must end at or before the group's high-water mark: the
       cursor position while the group has not yet emitted a back-reference,
       then frozen at the destination of the group's first back-reference */
    size_t limit = p->de ? (frozen ? hwm : pos) : (size_t)-1;
    uint32_t best = 0, best_dist = 0;
    if (pos + 3 <= n) {
      size_t maxlen = n - pos;
      if (maxlen > p->max_match) maxlen = p->max_match;
      size_t lo = pos > p->window ? pos - p->window : 0;
      int32_t cand = head[hash3(in + pos)];
      uint32_t tries = 0;
      while (cand >= 0 && (size_t)cand >= lo && tries < p->chain) {
        size_t s = (size_t)cand;
        tries++;
        size_t cap = maxlen;
        if (p->de) cap = (limit > s) ? (limit - s < cap ? limit - s : cap) : 0;
        if (cap >= 3 && cap > best) {
          size_t L = 0;
          while (L < cap && in[s + L] == in[pos + L]) L++;
          if (L > best) { best = (uint32_t)L; best_dist = (uint32_t)(pos - s); }
          if (best == maxlen) break;
        }
        if (p->hash_mode != 0) break;
        cand = prev[s];
      }
    }
    if (best >= 3) {
      if (p->de && !frozen) { hwm = pos; frozen = 1; }
      for (size_t q = 0; q < best; q++) INSERT(pos + q);
      CLOSE_SEQ(pos - lit_start, best, best_dist);
      pos += best;
      lit_start = pos;
      int cut = p->sub_target_raw ? (pos - sub_start >= p->sub_target_raw) : (sub_nseq >= p->sub_target_seq);
      if (cut && !byte_fmt) {
        if (u32_push(&subs, sub_nseq)) err = 1;
        sub_nseq = 0;
        sub_start = pos;
      }
    } else {
      lits[nl++] = in[pos];
      INSERT(pos);
      pos++;
      if (byte_fmt && pos - lit_start == 255) {
        /* a literal run as long as a record can hold becomes a sequence of its own */
        CLOSE_SEQ(255, 0, 0);
        lit_start = pos;
      } else if (!byte_fmt && p->sub_target_raw && pos - sub_start >= p->sub_target_raw) {
        /* the sub-block ends inside a literal run: the run becomes a
           sequence without a back-reference */
        CLOSE_SEQ(pos - lit_start, 0, 0);
        lit_start = pos;
        if (u32_push(&subs, sub_nseq)) err = 1;
        sub_nseq = 0;
        sub_start = pos;
      }
    }
  }
  if (!err && pos > lit_start) CLOSE_SEQ(pos - lit_start, 0, 0);
  if (!err && sub_nseq > 0 && !byte_fmt)
    if (u32_push(&subs, sub_nseq)) err = 1;
#undef INSERT
#undef CLOSE_SEQ
  free(head);
  free(prev);
  if (err) { free(sv.v); free(subs.v); free(lits); return GMPREF_ENOMEM; }
  *seqs_out = sv.v ? sv.v : (gmpref_seq*)malloc(sizeof(gmpref_seq));
  *n_seq_out = sv.n;
  *lits_out = lits;
  *n_lits_out = nl;
  *sub_out = subs.v ? subs.v : (uint32_t*)malloc(sizeof(uint32_t));
  *n_sub_out = subs.n;
  return GMPREF_OK;
}


/* ======================================================================== */
/* Gompresso/Byte: the token stream written with a direct byte-level        */
/* encoding (section "Gompresso Overview"), one fixed-size record per       */
/* sequence and the literal bytes after the records.                        */
/* ======================================================================== */
#define BYTE_MAGIC 0x59504D47u
#define BYTE_HDR 32

static size_t pad16(size_t x) { return (x + 15) & ~(size_t)15; }

int gmpref_encode_byte_block(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits,
                             const gmpref_params* p, uint8_t** out, size_t* out_len) {
  if (!p || n_seq > 0x3FFFFFFFu || n_lits > 0xFFFFFFFFu) return GMPREF_EINVAL;
  uint64_t raw = 0, lit_sum = 0;
  for (size_t i = 0; i < n_seq; i++) {
    const gmpref_seq* q = &seqs[i];
    if (q->lit_len > 255 || q->dist > 65535) return GMPREF_EINVAL;
    if (q->match_len == 0 ? q->dist != 0 : (q->match_len < 3 || q->match_len > 258 || q->dist == 0))
      return GMPREF_EINVAL;
    raw += q->lit_len + q->match_len;
    lit_sum += q->lit_len;
  }
  if (lit_sum != n_lits || raw > 0xFFFFFFFFu) return GMPREF_EINVAL;
  const size_t rec_bytes = pad16(4 * n_seq), total = BYTE_HDR + rec_bytes + pad16(n_lits) + 16;
  uint8_t* b = (uint8_t*)calloc(total, 1);
  if (!b) return GMPREF_ENOMEM;
  wr32(b, BYTE_MAGIC);
  b[4] = 1;
  b[5] = (uint8_t)(p->de ? 1 : 0);
  b[6] = (uint8_t)p->group;
  wr32(b + 8, (uint32_t)raw);
  wr32(b + 12, p->window);
  wr16(b + 16, (uint16_t)p->max_match);
  wr32(b + 20, (uint32_t)n_seq);
  wr32(b + 24, (uint32_t)n_lits);
  for (size_t i = 0; i < n_seq; i++) {
    const gmpref_seq* q = &seqs[i];
    const uint32_t m = q->match_len ? q->match_len - 3 : 0;
    wr32(b + BYTE_HDR + 4 * i, q->lit_len | (m << 8) | (q->dist << 16));
  }
  if (n_lits) memcpy(b + BYTE_HDR + rec_bytes, lits, n_lits);
  *out = b;
  *out_len = total;
  return GMPREF_OK;
}

static int byte_info_parse(const uint8_t* blk, size_t len, gmpref_block_info* info) {
  if (len < BYTE_HDR || rd32(blk) != BYTE_MAGIC || blk[4] != 1) return GMPREF_EFORMAT;
  memset(info, 0, sizeof(*info));
  info->format = 1;
  info->version = 1;
  info->mode = blk[5];
  info->group = blk[6];
  info->raw_len = rd32(blk + 8);
  info->window = rd32(blk + 12);
  info->max_match = rd16(blk + 16);
  info->n_seq = rd32(blk + 20);
  info->n_lit = rd32(blk + 24);
  if (info->mode > 1 || info->group < 1 || blk[7] != 0 || info->window < 1 || info->window > 32768 ||
      info->max_match < 3 || info->max_match > 258 || rd16(blk + 18) != 0 || rd32(blk + 28) != 0 ||
      info->n_seq > 0x3FFFFFFFu)
    return GMPREF_EFORMAT;
  const uint64_t payload = pad16(4 * (size_t)info->n_seq) + pad16(info->n_lit) + 16;
  if (payload > 0xFFFFFFFFu) return GMPREF_EFORMAT;
  info->payload_bytes = (uint32_t)payload;
  info->block_bytes = BYTE_HDR + payload;
  if (info->block_bytes > len) return GMPREF_EFORMAT;
  return GMPREF_OK;
}

/* The records of a byte-level block, checked: first the totals against the
   header (ESUB), then each record in order, with the first failing check of
   the first failing record deciding the class: a distance field of 0 with a
   nonzero match field (EFORMAT), a match longer than max_match (ELEN), a
   distance beyond the window or before the block's start (EDIST). */
static int byte_tokens(const uint8_t* blk, size_t len, gmpref_block_info* info, seqvec* sv, uint8_t** lits_out,
                       size_t* nl_out) {
  int rc = byte_info_parse(blk, len, info);
  if (rc) return rc;
  const uint8_t* rec = blk + BYTE_HDR;
  uint64_t lit_sum = 0, out_sum = 0;
  for (uint32_t i = 0; i < info->n_seq; i++) {
    const uint32_t r = rd32(rec + 4 * (size_t)i);
    const uint32_t d = r >> 16;
    lit_sum += r & 0xFF;
    out_sum += (r & 0xFF) + (d ? ((r >> 8) & 0xFF) + 3 : 0);
  }
  if (lit_sum != info->n_lit || out_sum != info->raw_len) return GMPREF_ESUB;
  uint64_t produced = 0;
  for (uint32_t i = 0; i < info->n_seq; i++) {
    const uint32_t r = rd32(rec + 4 * (size_t)i);
    const uint32_t lit = r & 0xFF, mf = (r >> 8) & 0xFF, d = r >> 16;
    const uint32_t m = d ? mf + 3 : 0;
    produced += lit;
    if (d == 0 && mf != 0) return GMPREF_EFORMAT;
    if (m > info->max_match) return GMPREF_ELEN;
    if (d && (d > info->window || d > produced)) return GMPREF_EDIST;
    if (seq_push(sv, lit, m, d)) return GMPREF_ENOMEM;
    produced += m;
  }
  uint8_t* lits = (uint8_t*)malloc(info->n_lit ? info->n_lit : 1);
  if (!lits) return GMPREF_ENOMEM;
  if (info->n_lit) memcpy(lits, rec + pad16(4 * (size_t)info->n_seq), info->n_lit);
  *lits_out = lits;
  *nl_out = info->n_lit;
  return GMPREF_OK;
}

int gmpref_compress_block(const uint8_t* in, size_t n, const gmpref_params* p, uint8_t** out, size_t* out_len) {
  gmpref_seq* seqs = NULL;
  uint8_t* lits = NULL;
  uint32_t* subs = NULL;
  size_t ns = 0, nl = 0, nsub = 0;
  int rc = gmpref_parse_block(in, n, p, &seqs, &ns, &lits, &nl, &subs, &nsub);
  if (rc) return rc;
  if (p->format == 1)
    rc = gmpref_encode_byte_block(seqs, ns, lits, nl, p, out, out_len);
  else
    rc = gmpref_encode_block(seqs, ns, lits, nl, subs, nsub, p, out, out_len);
  free(seqs);
  free(lits);
  free(subs);
  return rc;
}

int gmpref_compress(const uint8_t* in, size_t n, const gmpref_params* p, uint8_t** out, size_t* out_len) {
  if (!p || p->block_size == 0) return GMPREF_EINVAL;
  size_t nb = (n + p->block_size - 1) / p->block_size;
  size_t head_bytes = 32 + 8 * (nb + 1);
  head_bytes = (head_bytes + 15) & ~(size_t)15;
  buf_t b = {0, 0, 0};
  if (buf_reserve(&b, head_bytes)) return GMPREF_ENOMEM;
  memset(b.p, 0, head_bytes);
  b.len = head_bytes;
  uint64_t* offs = (uint64_t*)malloc(sizeof(uint64_t) * (nb + 1));
  if (!offs) { free(b.p); return GMPREF_ENOMEM; }
  for (size_t i = 0; i < nb; i++) {
    size_t len_i = (i + 1 < nb) ? p->block_size : n - i * p->block_size;
    uint8_t* blk = NULL;
    size_t bl = 0;
    int rc = gmpref_compress_block(in + i * p->block_size, len_i, p, &blk, &bl);
    if (rc) { free(b.p); free(offs); return rc; }
    offs[i] = b.len;
    if (buf_reserve(&b, bl + 16)) { free(blk); free(b.p); free(offs); return GMPREF_ENOMEM; }
    memcpy(b.p + b.len, blk, bl);
    b.len += bl;
    while (b.len & 15) b.p[b.len++] = 0;
    free(blk);
  }
  offs[nb] = b.len;
  wr32(b.p + 0, 0x46504D47u);
  wr16(b.p + 4, 1);
  wr16(b.p + 6, 0);
  wr32(b.p + 8, p->block_size);
  wr32(b.p + 12, (uint32_t)nb);
  wr64(b.p + 16, (uint64_t)n);
  wr64(b.p + 24, 0);
  for (size_t i = 0; i <= nb; i++) wr64(b.p + 32 + 8 * i, offs[i]);
  free(offs);
  *out = b.p;
  *out_len = b.len;
  return GMPREF_OK;
}

/* ======================================================================== */
/* decoder                                                                  */
/* ======================================================================== */
int gmpref_block_info_parse(const uint8_t* blk, size_t len, gmpref_block_info* info) {
  if (!blk || !info) return GMPREF_EINVAL;
  if (len >= 4 && rd32(blk) == BYTE_MAGIC) return byte_info_parse(blk, len, info);
  if (len < HDR_BYTES) return GMPREF_EFORMAT;
  if (rd32(blk) != 0x42504D47u || blk[4] != 1) return GMPREF_EFORMAT;
  info->format = 0;
  info->reserved = 0;
  info->version = blk[4];
  info->mode = blk[5];
  info->group = blk[6];
  info->lmax = blk[7];
  info->raw_len = rd32(blk + 8);
  info->window = rd32(blk + 12);
  info->max_match = rd16(blk + 16);
  info->n_sub = rd32(blk + 20);
  info->n_seq = rd32(blk + 24);
  info->n_lit = rd32(blk + 28);
  if (info->mode > 1 || info->group < 1 || info->lmax < 1 || info->lmax > MAX_BITS || info->window < 1 ||
      info->window > 32768 || info->max_match < 3 || info->max_match > 258 || rd16(blk + 18) != 0)
    return GMPREF_EFORMAT;
  uint64_t idx_end = HDR_BYTES + (uint64_t)IDX_ENTRY * info->n_sub;
  if (idx_end + 16 > len) return GMPREF_EFORMAT;
  info->payload_bytes = rd32(blk + idx_end);
  info->block_bytes = idx_end + 16 + info->payload_bytes;
  if (info->block_bytes > len) return GMPREF_EFORMAT;
  return GMPREF_OK;
}

/* A canonical code in the form needed for bit-serial decoding: the number of
   codes of each length and the symbols ordered by (length, symbol). */
typedef struct {
  uint16_t count[MAX_BITS + 1];
  uint16_t symbol[N_LL];
  int lmax;
} canon_t;

/* returns 0 complete, 1 empty, <0 error */
static int canon_build(canon_t* h, const uint8_t* lens, int n, int lmax) {
  memset(h, 0, sizeof *h);
  h->lmax = lmax;
  for (int i = 0; i < n; i++) {
    if (lens[i] > lmax) return GMPREF_ECODE;
    h->count[lens[i]]++;
  }
  if (h->count[0] == n) return 1;
  /* Kraft: the codes must exactly fill the code space */
  int64_t left = 1;
  for (int l = 1; l <= MAX_BITS; l++) {
    left <<= 1;
    left -= h->count[l];
    if (left < 0) return GMPREF_ECODE;
  }
  if (left != 0) return GMPREF_ECODE;
  uint16_t offs[MAX_BITS + 2];
  offs[1] = 0;
  for (int l = 1; l <= MAX_BITS; l++) offs[l + 1] = (uint16_t)(offs[l] + h->count[l]);
  for (int i = 0; i < n; i++)
    if (lens[i]) h->symbol[offs[lens[i]]++] = (uint16_t)i;
  return 0;
}

typedef struct {
  const uint8_t* p;
  uint64_t nbits, pos;
} bitr;

static int br_bit(bitr* r) {
  if (r->pos >= r->nbits) return -1;
  int b = (r->p[r->pos >> 3] >> (r->pos & 7)) & 1;
  r->pos++;
  return b;
}
static int br_value(bitr* r, int n, uint32_t* v) {
  uint32_t x = 0;
  for (int i = 0; i < n; i++) {
    int b = br_bit(r);
    if (b < 0) return -1;
    x |= (uint32_t)b << i;
  }
  *v = x;
  return 0;
}
/* one symbol, one bit at a time: a code of length l is the (l)-bit value read
   MSB-first; it is valid when it falls inside the range of length-l codes */
static int canon_decode(const canon_t* h, bitr* r) {
  int code = 0, first = 0, index = 0;
  for (int l = 1; l <= h->lmax; l++) {
    int b = br_bit(r);
    if (b < 0) return GMPREF_ESUB;
    code |= b;
    int cnt = h->count[l];
    if (code - first < cnt) return h->symbol[index + (code - first)];
    index += cnt;
    first += cnt;
    first <<= 1;
    code <<= 1;
  }
  return GMPREF_ECODE;
}

/* Decode all sub-blocks of a block into sequences and literal bytes, checking
   every format rule (section "Huffman Decoding": each sub-block is located by
   the sizes in the header and decoded with the block's two codes). */
static int decode_tokens(const uint8_t* blk, size_t len, gmpref_block_info* info, seqvec* sv, uint8_t** lits_out,
                         size_t* nl_out) {
  if (len >= 4 && rd32(blk) == BYTE_MAGIC) return byte_tokens(blk, len, info, sv, lits_out, nl_out);
  int rc = gmpref_block_info_parse(blk, len, info);
  if (rc) return rc;
  uint8_t lens[N_LL + N_D];
  for (int i = 0; i < N_LL + N_D; i++) lens[i] = (uint8_t)((blk[32 + i / 2] >> ((i & 1) * 4)) & 15);
  if (blk[32 + 158] != 0 || blk[32 + 159] != 0) return GMPREF_EFORMAT;
  const uint8_t* idx = blk + HDR_BYTES;
  const uint8_t* payload = blk + HDR_BYTES + (size_t)IDX_ENTRY * info->n_sub + 16;
  /* index sums must match the header and the payload size */
  uint64_t words = 0, s_seq = 0, s_lit = 0, s_raw = 0;
  for (uint32_t s = 0; s < info->n_sub; s++) {
    const uint8_t* e = idx + IDX_ENTRY * s;
    words += 4 * (((uint64_t)rd32(e) + 127) / 128);
    s_seq += rd32(e + 4);
    s_lit += rd32(e + 8);
    s_raw += rd32(e + 12);
  }
  if (words * 4 != info->payload_bytes || s_seq != info->n_seq || s_lit != info->n_lit || s_raw != info->raw_len)
    return GMPREF_EFORMAT;
  canon_t ll, dd;
  if (info->n_sub > 0) {
    rc = canon_build(&ll, lens, N_LL, (int)info->lmax);
    if (rc < 0) return rc;
    if (rc == 1 || lens[SYM_END] == 0) return GMPREF_ECODE;
    rc = canon_build(&dd, lens + N_LL, N_D, (int)info->lmax);
    if (rc < 0) return rc;
  } else {
    dd.count[0] = N_D;
  }
  int dist_empty = (dd.count[0] == N_D);
  uint8_t* lits = (uint8_t*)malloc(info->n_lit ? info->n_lit : 1);
  if (!lits) return GMPREF_ENOMEM;
  size_t nl = 0;
  uint64_t produced = 0; /* bytes produced in the block so far */
  uint64_t byte_off = 0;
  for (uint32_t s = 0; s < info->n_sub; s++) {
    const uint8_t* e = idx + IDX_ENTRY * s;
    uint32_t bit_len = rd32(e), want_seq = rd32(e + 4), want_lit = rd32(e + 8), want_raw = rd32(e + 12);
    bitr r = {payload + byte_off, bit_len, 0};
    byte_off += 16 * (((uint64_t)bit_len + 127) / 128);
    uint64_t got_seq = 0, got_lit = 0, sub_raw0 = produced;
    uint32_t run = 0;
    for (;;) {
      int sym = canon_decode(&ll, &r);
      if (sym < 0) { free(lits); return sym; }
      if (sym < 256) {
        if (nl >= info->n_lit || got_lit >= want_lit) { free(lits); return GMPREF_ESUB; }
        lits[nl++] = (uint8_t)sym;
        got_lit++;
        run++;
        produced++;
        continue;
      }
      if (sym == SYM_END) {
        if (run > 0) {
          if (seq_push(sv, run, 0, 0)) { free(lits); return GMPREF_ENOMEM; }
          got_seq++;
          run = 0;
        }
        break;
      }
      int lx = sym - 257;
      if (lx >= 29) { free(lits); return GMPREF_ECODE; }
      uint32_t ex = 0;
      if (br_value(&r, LEN_EXTRA[lx], &ex)) { free(lits); return GMPREF_ESUB; }
      uint32_t mlen = LEN_BASE[lx] + ex;
      if (dist_empty) { free(lits); return GMPREF_ECODE; }
      int dx = canon_decode(&dd, &r);
      if (dx < 0) { free(lits); return dx; }
      if (dx >= 30) { free(lits); return GMPREF_ECODE; }
      if (br_value(&r, DIST_EXTRA[dx], &ex)) { free(lits); return GMPREF_ESUB; }
      uint32_t dist = DIST_BASE[dx] + ex;
      if (mlen < 3 || mlen > info->max_match) { free(lits); return GMPREF_ELEN; }
      if (dist > info->window || dist > produced) { free(lits); return GMPREF_EDIST; }
      if (seq_push(sv, run, mlen, dist)) { free(lits); return GMPREF_ENOMEM; }
      got_seq++;
      run = 0;
      produced += mlen;
    }
    if (r.pos != bit_len || got_seq != want_seq || got_lit != want_lit || produced - sub_raw0 != want_raw) {
      free(lits);
      return GMPREF_ESUB;
    }
  }
  if (produced != info->raw_len || nl != info->n_lit) { free(lits); return GMPREF_ESUB; }
  *lits_out = lits;
  *nl_out = nl;
  return GMPREF_OK;
}

int gmpref_block_tokens(const uint8_t* blk, size_t len, gmpref_seq** seqs, size_t* n_seq, uint8_t** lits,
                        size_t* n_lits) {
  gmpref_block_info info;
  seqvec sv = {0, 0, 0};
  uint8_t* l = NULL;
  size_t nl = 0;
  int rc = decode_tokens(blk, len, &info, &sv, &l, &nl);
  if (rc) { free(sv.v); return rc; }
  *seqs = sv.v ? sv.v : (gmpref_seq*)malloc(sizeof(gmpref_seq));
  *n_seq = sv.n;
  *lits = l;
  *n_lits = nl;
  return GMPREF_OK;
}

/* Sequential LZ77 (section "LZ77 Compression"): append the literals of each
   sequence, then copy its back-reference one byte at a time from dist bytes
   back, so that overlapping copies repeat the pattern. */
int gmpref_lz77_expand(const gmpref_seq* seqs, size_t n_seq, const uint8_t* lits, size_t n_lits, uint32_t window,
                       uint32_t max_match, uint8_t* out, size_t cap, size_t* out_len) {
  size_t o = 0, li = 0;
  for (size_t i = 0; i < n_seq; i++) {
    const gmpref_seq* s = &seqs[i];
    if (li + s->lit_len > n_lits) return GMPREF_ESUB;
    if (o + s->lit_len > cap) return GMPREF_ELEN;
    for (uint32_t k = 0; k < s->lit_len; k++) out[o++] = lits[li++];
    if (s->match_len == 0) continue;
    if (s->match_len < 3 || s->match_len > max_match) return GMPREF_ELEN;
    if (s->dist == 0 || s->dist > window || s->dist > o) return GMPREF_EDIST;
    if (o + s->match_len > cap) return GMPREF_ELEN;
    for (uint32_t k = 0; k < s->match_len; k++, o++) out[o] = out[o - s->dist];
  }
  if (li != n_lits) return GMPREF_ESUB;
  *out_len = o;
  return GMPREF_OK;
}

int gmpref_decompress_block(const uint8_t* blk, size_t len, uint8_t* out, size_t cap, size_t* out_len) {
  gmpref_block_info info;
  seqvec sv = {0, 0, 0};
  uint8_t* lits = NULL;
  size_t nl = 0;
  int rc = decode_tokens(blk, len, &info, &sv, &lits, &nl);
  if (rc) { free(sv.v); return rc; }
  if (cap != info.raw_len) { free(sv.v); free(lits); return GMPREF_ESIZE; }
  rc = gmpref_lz77_expand(sv.v, sv.n, lits, nl, info.window, info.max_match, out, cap, out_len);
  free(sv.v);
  free(lits);
  return rc;
}

int gmpref_decompress(const uint8_t* comp, size_t len, uint8_t* out, size_t cap, size_t* out_len) {
  if (len < 32 || rd32(comp) != 0x46504D47u || rd16(comp + 4) != 1) return GMPREF_EFORMAT;
  uint32_t bs = rd32(comp + 8), nb = rd32(comp + 12);
  uint64_t raw_total = rd64(comp + 16);
  if (bs == 0) return GMPREF_EFORMAT;
  if ((uint64_t)32 + 8 * ((uint64_t)nb + 1) > len) return GMPREF_EFORMAT;
  if (nb != (raw_total + bs - 1) / bs) return GMPREF_EFORMAT;
  if (cap != raw_total) return GMPREF_ESIZE;
  for (uint32_t b = 0; b < nb; b++) {
    uint64_t o0 = rd64(comp + 32 + 8 * (size_t)b), o1 = rd64(comp + 32 + 8 * ((size_t)b + 1));
    if (o0 > o1 || o1 > len || (o0 & 15)) return GMPREF_EFORMAT;
    uint64_t want = (b + 1 < nb) ? bs : raw_total - (uint64_t)b * bs;
    size_t got = 0;
    gmpref_block_info info;
    int rc = gmpref_block_info_parse(comp + o0, (size_t)(o1 - o0), &info);
    if (rc) return rc;
    if (info.raw_len != want) return GMPREF_ESIZE;
    rc = gmpref_decompress_block(comp + o0, (size_t)(o1 - o0), out + (size_t)b * bs, (size_t)want, &got);
    if (rc) return rc;
  }
  *out_len = (size_t)raw_total;
  return GMPREF_OK;
}

/* ======================================================================== */
/* checks                                                                   */
/* ======================================================================== */
/* DE rule (section "Dependency Elimination (DE)"), read as: in each group of
   G sequences, counted from the block start, every back-reference's source
   interval ends at or before the destination of the group's first
   back-reference. */
int gmpref_de_holds(const gmpref_seq* seqs, size_t n_seq, uint32_t G) {
  if (G == 0) return 0;
  uint64_t pos = 0;
  for (size_t g0 = 0; g0 < n_seq; g0 += G) {
    size_t g1 = g0 + G < n_seq ? g0 + G : n_seq;
    int have = 0;
    uint64_t hwm = 0;
    for (size_t i = g0; i < g1; i++) {
      pos += seqs[i].lit_len;
      if (seqs[i].match_len) {
        if (!have) { have = 1; hwm = pos; }
        uint64_t src = pos - seqs[i].dist;
        if (src + seqs[i].match_len > hwm) return 0;
      }
      pos += seqs[i].match_len;
    }
  }
  return 1;
}

int gmpref_validate_block(const uint8_t* blk, size_t len) {
  gmpref_block_info info;
  seqvec sv = {0, 0, 0};
  uint8_t* lits = NULL;
  size_t nl = 0;
  int rc = decode_tokens(blk, len, &info, &sv, &lits, &nl);
  if (rc) { free(sv.v); return rc; }
  if (info.format == 1) {
    /* byte-level block: every padding byte is zero */
    const size_t r_end = BYTE_HDR + 4 * (size_t)info.n_seq, l0 = BYTE_HDR + pad16(4 * (size_t)info.n_seq);
    for (size_t k = r_end; k < l0 && rc == 0; k++)
      if (blk[k]) rc = GMPREF_ESUB;
    for (size_t k = l0 + info.n_lit; k < info.block_bytes && rc == 0; k++)
      if (blk[k]) rc = GMPREF_ESUB;
    info.n_sub = 0;
  }
  /* padding bits after each sub-block are zero */
  const uint8_t* idx = blk + HDR_BYTES;
  const uint8_t* payload = blk + HDR_BYTES + (size_t)IDX_ENTRY * info.n_sub + 16;
  uint64_t byte_off = 0;
  for (uint32_t s = 0; s < info.n_sub && rc == 0; s++) {
    uint32_t bit_len = rd32(idx + IDX_ENTRY * s);
    uint64_t padded = 128 * (((uint64_t)bit_len + 127) / 128);
    for (uint64_t b = bit_len; b < padded; b++)
      if ((payload[byte_off + b / 8] >> (b % 8)) & 1) rc = GMPREF_ESUB;
    byte_off += padded / 8;
  }
  /* (A sequence without a back-reference carries literals and ends its
     sub-block: decode_tokens only forms one at a sub-block's end symbol, from
     a non-empty literal run, and checks the index's sequence counts, so the
     rule needs no separate check here.) */
  if (rc == 0 && info.mode == 1 && !gmpref_de_holds(sv.v, sv.n, info.group)) rc = GMPREF_EDIST;
  if (rc == 0) {
    uint8_t* out = (uint8_t*)malloc(info.raw_len ? info.raw_len : 1);
    size_t got = 0;
    if (!out) rc = GMPREF_ENOMEM;
    else rc = gmpref_lz77_expand(sv.v, sv.n, lits, nl, info.window, info.max_match, out, info.raw_len, &got);
    free(out);
  }
  free(sv.v);
  free(lits);
  return rc;
}

/* Multi-Round Resolution round count (section "Multi-Round Resolution (MRR)
   of Nested back-references").  Per group of G sequences: all literal runs are
   written first (not a round); then, in each round, the high-water mark is the
   destination of the lowest-numbered sequence whose back-reference is still
   pending (everything below it is written, with no gaps), and every pending
   back-reference whose needed source bytes lie below the mark is copied.  The
   needed source bytes of a copy of length L at distance D are the first
   min(L, D) bytes after its source position, since an overlapping copy reads
   its own output after that.  Returns rounds per group and bytes per round. */
int gmpref_mrr_rounds(const gmpref_seq* seqs, size_t n_seq, uint32_t G, uint32_t* rounds,
                      uint64_t* bytes_per_round) {
  return gmpref_mrr_rounds_redirect(seqs, n_seq, G, 0, 0, rounds, bytes_per_round, NULL, NULL);
}

/* The same, where each back-reference that does not overlap itself first
   moves its source, up to `jumps` times, through the group's own copies: if
   the bytes it reads all lie inside the destination of an earlier sequence k
   of the group (the last one whose destination starts at or before them)
   whose back-reference does not overlap itself either, those bytes equal the
   ones dist_k further back, so the source moves there (while it still lies
   inside the group's output).  Only groups whose output is at most
   span_limit bytes (0: any) are redirected.  Byte output is unchanged; the
   rounds can only fall.  seq_round / seq_dist (optional) receive each
   sequence's round (0: no back-reference) and the distance it reads from. */
int gmpref_mrr_rounds_redirect(const gmpref_seq* seqs, size_t n_seq, uint32_t G, uint32_t jumps,
                               uint64_t span_limit, uint32_t* rounds, uint64_t* bytes_per_round,
                               uint32_t* seq_round, uint32_t* seq_dist) {
  if (G == 0 || G > 1024) return GMPREF_EINVAL;
  uint64_t* dst = (uint64_t*)malloc(sizeof(uint64_t) * G);
  uint64_t* src = (uint64_t*)malloc(sizeof(uint64_t) * G);
  int* pend = (int*)malloc(sizeof(int) * G);
  int* done_now = (int*)malloc(sizeof(int) * G);
  if (!dst || !src || !pend || !done_now) {
    free(dst); free(src); free(pend); free(done_now);
    return GMPREF_ENOMEM;
  }
  for (uint32_t r = 0; r < G; r++) bytes_per_round[r] = 0;
  uint64_t pos = 0;
  size_t g = 0;
  for (size_t g0 = 0; g0 < n_seq; g0 += G, g++) {
    size_t m = (g0 + G < n_seq) ? G : n_seq - g0;
    int npend = 0;
    const uint64_t g_start = pos;
    for (size_t i = 0; i < m; i++) {
      pos += seqs[g0 + i].lit_len;
      dst[i] = pos;
      src[i] = pos - seqs[g0 + i].dist;
      pos += seqs[g0 + i].match_len;
      pend[i] = seqs[g0 + i].match_len > 0;
      npend += pend[i];
    }
    if (jumps && (span_limit == 0 || pos - g_start <= span_limit)) {
      for (size_t i = 0; i < m; i++) {
        const uint64_t L = seqs[g0 + i].match_len;
        if (L == 0 || seqs[g0 + i].dist < L) continue;
        for (uint32_t j = 0; j < jumps && src[i] >= g_start; j++) {
          size_t k = m;  /* the last sequence whose destination starts at or before the source */
          for (size_t q = 0; q < m; q++)
            if (dst[q] <= src[i]) k = q;
          if (k == m) break;
          const uint64_t Lk = seqs[g0 + k].match_len, dk = seqs[g0 + k].dist;
          if (Lk == 0 || dk < Lk || src[i] + L > dst[k] + Lk) break;
          src[i] -= dk;
        }
      }
    }
    uint32_t nr = 0;
    while (npend > 0) {
      size_t lowest = 0;
      while (!pend[lowest]) lowest++;
      uint64_t hwm = dst[lowest];
      for (size_t i = 0; i < m; i++) {
        done_now[i] = 0;
        if (!pend[i]) continue;
        uint64_t d = dst[i] - src[i], L = seqs[g0 + i].match_len;
        uint64_t need_end = src[i] + (L < d ? L : d);
        if (need_end <= hwm) done_now[i] = 1;
      }
      for (size_t i = 0; i < m; i++)
        if (done_now[i]) {
          pend[i] = 0;
          npend--;
          bytes_per_round[nr] += seqs[g0 + i].match_len;
          if (seq_round) seq_round[g0 + i] = nr + 1;
        }
      nr++;
    }
    for (size_t i = 0; i < m; i++) {
      if (seq_round && seqs[g0 + i].match_len == 0) seq_round[g0 + i] = 0;
      if (seq_dist) seq_dist[g0 + i] = (uint32_t)(dst[i] - src[i]);
    }
    rounds[g] = nr;
  }
  free(dst);
  free(src);
  free(pend);
  free(done_now);
  return GMPREF_OK;
}
